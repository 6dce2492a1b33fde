"""The NTT and MAC schedule tables and the launches they dispatch to (host only).

An NTT schedule id indexes both the table that the library reports and tunes
over (ring degree, threads per polynomial, stages per pass, launch form) and
the switch that instantiates the kernel for it. The two are separate lists in
csrc/ntt.hip; these tests read the source and check that entry i of the
table and case i of the switch name the same template arguments and launch
form, that every ring degree's schedules are contiguous (the library reports
them as a range), that the default schedule of each degree is one of its
own, and that the built library reports the same ranges. Likewise every row
of the MAC schedule table (csrc/conv.hip) has an instantiated per-layer
kernel and, if it uses LDS, a persistent one (csrc/batch.hip), and the
default MAC schedules have the block tiles their comments state.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2311_12519_amd", "csrc", "ntt.hip")
FORMS = {"sched": 0, "persist": 1, "stream": 2}


def _source():
    with open(SRC) as f:
        return f.read()


def _table(s):
    body = s[s.index("const NttSched kNtt[] = {"):s.index("const int kNumNtt")]
    return [tuple(int(v) for v in m.split(",")) for m in re.findall(r"\{([\d, ]+)\}", body)]


def _switch(s):
    body = s[s.index("hipError_t launch_idx(int i"):]
    body = body[:body.index("default:")]
    return [(int(c), f, tuple(int(v) for v in a.split(",")))
            for c, f, a in re.findall(r"case (\d+): return launch_(\w+)<([\d, ]+)>", body)]


def _defaults(s):
    body = s[s.index("int ntt_default_schedule(uint32_t logN)"):]
    body = body[:body.index("default:")]
    return {int(n): int(i) for n, i in re.findall(r"case (\d+): return (\d+);", body)}


def test_table_and_switch_agree():
    s = _source()
    table, switch = _table(s), _switch(s)
    assert len(table) == len(switch) > 0
    for i, (entry, (case, form, args)) in enumerate(zip(table, switch)):
        assert case == i, (i, case)
        assert entry[:6] == args, (i, entry, args)
        assert entry[6] == FORMS[form], (i, entry, form)
        logn, logt, e0, e1, e2, e3, _ = entry
        assert e0 + e1 + e2 + e3 == logn and e0 == logn - logt, (i, entry)


def test_degrees_contiguous_and_defaults_their_own():
    s = _source()
    table = _table(s)
    logns = [e[0] for e in table]
    assert logns == sorted(logns)
    for logn, sid in _defaults(s).items():
        assert table[sid][0] == logn, (logn, sid)
        assert table[sid][6] == 0, "a default schedule launches one block per limb-polynomial"


def test_library_reports_the_table_ranges():
    hy = pytest.importorskip("paper_2311_12519_amd")
    table = _table(_source())
    for logn in sorted({e[0] for e in table}):
        ids = [i for i, e in enumerate(table) if e[0] == logn]
        assert hy.hyena_ntt_schedules(1 << logn) == ids, logn


# ---------------------------------------------------------------- MAC

CONV = os.path.join(ROOT, "paper_2311_12519_amd", "csrc", "conv.hip")
BATCH = os.path.join(ROOT, "paper_2311_12519_amd", "csrc", "batch.hip")


def _mac_table():
    with open(CONV) as f:
        s = f.read()
    body = s[s.index("static const MacSched kScheds[] = {"):s.index("static const int kNumScheds")]
    return s, [tuple(int(v) for v in m.split(",")) for m in re.findall(r"\{([\d, ]+)\}", body)]


def _macro_args(s, name):
    return {tuple(int(v) for v in a.split(",")) for a in re.findall(name + r"\(([\d, ]+)\)", s)
            if "M" not in a}


def test_every_mac_schedule_has_a_launch():
    """Every row of the MAC schedule table is instantiated for per-layer
    launches (register-only, LDS-pipelined or synthesizing form) and, when it
    uses LDS, for the persistent launch of the batched step."""
    s, table = _mac_table()
    with open(BATCH) as f:
        b = f.read()
    reg, lds, syn, pers = (_macro_args(s, "HY_CASE"), _macro_args(s, "HY_L"), _macro_args(s, "HY_S"),
                           _macro_args(b, "HY_P"))
    assert table
    for i, (uses_lds, mt, ot, wr, wo, ns, taps) in enumerate(table):
        if not uses_lds:
            assert (mt, ot) in reg, i
        elif taps:
            assert (mt, ot, wr, wo, ns, taps) in syn, i
        else:
            assert (mt, ot, wr, wo, ns) in lds, i
        if uses_lds:
            assert (mt, ot, wr, wo, ns, taps) in pers, i


def test_default_mac_schedules_have_their_tiles():
    """The default schedule ids name the block tiles (rows x outputs) that
    their comments give."""
    s, table = _mac_table()
    body = s[s.index("static int default_sched(const hyena_conv_desc *d)"):]
    body = body[:body.index("static bool sched_valid")]
    found = re.findall(r"return (\d+);\s+// LDS (\d+) x (\d+)", body)
    assert len(found) == 4
    for sid, rows, outs in found:
        uses_lds, mt, ot, wr, wo, ns, taps = table[int(sid)]
        assert uses_lds == 1 and taps == 0 and (wr * mt, wo * ot) == (int(rows), int(outs)), sid
