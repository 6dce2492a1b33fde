"""The host C++ of the library (parameters, keys, encryption, decryption,
planning, packing) under AddressSanitizer and UndefinedBehaviorSanitizer: the
CPU tests of the C ABI run against a sanitizer build of those sources in a
child process. Host code only; no GPU is touched."""
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_abi_under_address_and_ub_sanitizers():
    if not os.path.exists(os.path.join(ROOT, "paper_2311_12519_amd", "sanitize_build.py")):
        pytest.skip("sanitizer build script not present")
    from paper_2311_12519_amd import sanitize_build as sb
    sb.build()
    r = sb.run_tests()
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
