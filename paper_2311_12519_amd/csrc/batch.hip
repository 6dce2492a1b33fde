// Batched execution of many convolution layers (and images) per step.
//
// One step is: forward NTT of every layer's input ciphertexts (segmented
// launches over all layers), the multiply-accumulate of every layer, and the
// inverse NTT of every layer's outputs. Layers whose multiply-accumulate uses
// the same LDS schedule share one persistent launch: a grid sized to the
// chip's occupancy pulls (layer, tile) work items from eight per-XCD queues,
// each holding one eighth of every layer (contiguous per layer, so the tiles
// of one slot chunk stay in one L2); uneven layers are balanced by
// construction, every XCD doing the same share of each. The step can be
// captured once into a hipGraph and replayed. An autotuner times the
// candidate MAC schedules per layer, the persistent launch against per-layer
// launches and the NTT schedules per direction, and keeps the choices in a
// text cache (HYENA_TUNE_CACHE) so later runs reuse them.
//
// Every layer's inputs are independent here: the nonlinear layers between
// convolutions run under MPC in the paper's protocol and are not part of this
// server-side computation.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>

#include "mac.h"

// schedule table and validity (conv.hip)
int conv_launch(const hyena_ctx *c, const hyena_conv_desc *d, const uint32_t *ct, const uint32_t *w,
                const int32_t *taps, uint32_t *out, int sched, bool per_channel, hipStream_t s);
int conv_sched_info(int sched, int *info);
int conv_num_scheds();
bool conv_sched_valid(const hyena_conv_desc *d, int sched);
int conv_default_sched(const hyena_conv_desc *d);
MacArgs conv_make_args(const hyena_ctx *c, const hyena_conv_desc *d, const uint32_t *ct, const uint32_t *w,
                       const int32_t *taps, uint32_t *out, int sched, bool per_channel, bool *needs_wht);
int conv_sched_syn(int sched);
int conv_default_synth_sched(const hyena_conv_desc *d);
hipError_t conv_launch_wht(const hyena_ctx *c, uint32_t cn, const uint32_t *in, uint32_t *out, size_t G,
                           hipStream_t s);

namespace {

// Work queues of the persistent launch: queue x (drained by the blocks of
// XCD x: blocks are dealt to the XCDs round robin) holds the x-th eighth of
// every layer's items, a contiguous slice per layer, layers in order. Each XCD
// thus does the same share of every layer, in order: tiles that share input
// rows are in flight together in one L2, and no XCD runs dry early, so there
// is no stealing (a stolen tile would fetch its rows into a second L2).
// Table: lfirst[n_layers + 1] (first item of each layer) followed by
// qfirst[8][n_layers + 1] (position of each layer's slice within queue x).
__device__ __forceinline__ uint32_t slice_start(uint32_t n, uint32_t x) { return (uint32_t)(((uint64_t)n * x) >> 3); }

// Thread 0 claims the next item of its XCD's queue; `total` once it is empty.
// `l` is the layer of the previous claim (claims only move forward).
__device__ __forceinline__ uint32_t draw_item(uint32_t *counters, const uint32_t *lfirst, uint32_t n_layers,
                                              uint32_t total, uint32_t x, uint32_t &l) {
    const uint32_t *qf = lfirst + (n_layers + 1) * (1 + x);
    const uint32_t c = atomicAdd(&counters[x], 1u);
    if (c >= qf[n_layers]) return total;
    while (c >= qf[l + 1]) l++;
    return lfirst[l] + slice_start(lfirst[l + 1] - lfirst[l], x) + (c - qf[l]);
}

// resident blocks per CU as the per-layer kernel (three, at most 168 VGPRs,
// where the LDS stages allow)
template <int MT, int OT, int WR, int WO, int NS, int TM>
__global__ void __launch_bounds__(256, (MacLdsShape<MT, OT, WR, WO, NS, TM>::MIN_BLOCKS))
mac_persistent_kernel(const MacArgs *__restrict__ layers, const uint32_t *__restrict__ first, uint32_t n_layers,
                      uint32_t *__restrict__ counters, uint32_t total) {
    __shared__ __attribute__((aligned(16))) uint32_t lds[MacLdsShape<MT, OT, WR, WO, NS, TM>::LDS_WORDS];
    __shared__ uint32_t item_s[2], layer_s[2];  // claimed item and its layer, double buffered
    const uint32_t x = blockIdx.x & 7u;  // this block's XCD and queue
    uint32_t lq = 0;                     // layer of thread 0's last claim
    if (threadIdx.x == 0) {
        item_s[0] = draw_item(counters, first, n_layers, total, x, lq);
        layer_s[0] = lq;
    }
    __syncthreads();
    for (uint32_t round = 0;; round ^= 1) {
        // uniform across the block: lets the layer's arguments load as scalars
        const uint32_t it = __builtin_amdgcn_readfirstlane(item_s[round]);
        if (it >= total) break;
        const uint32_t l = __builtin_amdgcn_readfirstlane(layer_s[round]);
        // the following item is claimed when this one's accumulation is done:
        // items then start in queue order, as the hardware dispatcher would
        // start blocks, and the claim's latency hides behind the epilogue
        auto claim = [&]() {
            if (threadIdx.x == 0) {
                item_s[round ^ 1] = draw_item(counters, first, n_layers, total, x, lq);
                layer_s[round ^ 1] = lq;
            }
        };
        mac_lds_block<MT, OT, WR, WO, NS, TM>(layers[l], it - first[l], lds, claim);
        __syncthreads();  // LDS stages and the next claim ready for the next round
    }
}

__global__ void zero_words_kernel(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

typedef void (*PersistentFn)(const MacArgs *, const uint32_t *, uint32_t, uint32_t *, uint32_t);

PersistentFn persistent_fn(const int *info, int syn) {
#define HY_P(M, O, R, W, S, T)                                                                    \
    if (info[1] == M && info[2] == O && info[3] == R && info[4] == W && info[5] == S && syn == T) \
        return mac_persistent_kernel<M, O, R, W, S, T>;
    HY_P(8, 8, 2, 2, 4, 0) HY_P(8, 8, 2, 2, 3, 0) HY_P(4, 8, 2, 2, 4, 0) HY_P(8, 8, 1, 4, 4, 0)
    HY_P(2, 16, 1, 4, 4, 0) HY_P(4, 16, 1, 4, 3, 0) HY_P(8, 4, 4, 1, 4, 0) HY_P(4, 8, 1, 4, 4, 0)
    HY_P(8, 8, 2, 2, 5, 0) HY_P(8, 8, 2, 2, 6, 0)
    HY_P(8, 8, 2, 2, 4, 9) HY_P(8, 8, 4, 1, 4, 9) HY_P(8, 8, 2, 2, 4, 18) HY_P(8, 8, 4, 1, 4, 18)
#undef HY_P
    return nullptr;
}

uint32_t mac_blocks(const MacArgs &a) { return a.n_ot * a.n_mt * a.kchunks * a.L; }

// ------------------------------------------------------------------ tuning cache

std::string cache_path() {
    const char *p = std::getenv("HYENA_TUNE_CACHE");
    return p ? std::string(p) : std::string();
}

std::map<std::string, int> load_cache() {
    std::map<std::string, int> m;
    const std::string path = cache_path();
    if (path.empty()) return m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos) continue;
        m[line.substr(0, tab)] = std::atoi(line.c_str() + tab + 1);
    }
    return m;
}

void save_cache(const std::map<std::string, int> &m) {
    const std::string path = cache_path();
    if (path.empty()) return;
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        for (auto &kv : m) f << kv.first << '\t' << kv.second << '\n';
    }
    std::rename(tmp.c_str(), path.c_str());
}

std::string arch_name(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string s = p.gcnArchName;
    return s.substr(0, s.find(':'));
}

}  // namespace

struct hyena_batch {
    const hyena_ctx *ctx = nullptr;
    uint32_t flags = 0;
    std::vector<hyena_conv_desc> desc;
    std::vector<hyena_layer_io> io;
    std::vector<int> mac_sched;
    int ntt_fwd = -1, ntt_inv = -1;
    // persistent groups
    struct Group {
        int sched;
        std::vector<uint32_t> layers;
        MacArgs *d_args = nullptr;
        uint32_t *d_first = nullptr;
        uint32_t total = 0;
        uint32_t grid = 0;
    };
    std::vector<Group> groups;
    bool mac_solo = false;  // autotuner: per-layer launches beat the persistent ones
    // autotuner: inverse-NTT schedules within 5% of the fastest when timed on
    // their own, and the cache key of the choice (settled in step context)
    std::vector<int> inv_cands;
    std::string inv_key;
    int per_cu = 0;  // persistent blocks per CU
    std::vector<uint32_t> solo;   // layers launched on their own
    uint32_t *d_counters = nullptr;  // per persistent launch: 8 queue counters
    uint32_t n_counters = 0;
    // one graph for the whole step, or one per phase when timing (events
    // between graph launches; event nodes inside a graph cannot be timed)
    hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    int launches = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // phase boundaries (HYENA_BATCH_TIMING)
};

// Enqueue phase `phase` of a step (0: forward NTTs, 1: multiply-accumulate,
// 2: inverse NTTs) or all of them (phase < 0).
static int issue_mac_phase(hyena_batch *b, hipStream_t s, int &launches) {
    const hyena_ctx *c = b->ctx;
    if (b->mac_solo) {
        for (uint32_t l = 0; l < b->desc.size(); l++) {
            const int rc = conv_launch(c, &b->desc[l], b->io[l].d_ct, b->io[l].d_wntt, b->io[l].d_taps,
                                       b->io[l].d_out, b->mac_sched[l], true, s);
            if (rc) return rc;
            launches++;
        }
        return HYENA_OK;
    }
    if (b->n_counters) {
        hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, b->d_counters, b->n_counters);
        launches++;
    }
    for (size_t gi = 0; gi < b->groups.size(); gi++) {
        auto &g = b->groups[gi];
        int info[6];
        conv_sched_info(g.sched, info);
        PersistentFn fn = persistent_fn(info, conv_sched_syn(g.sched));
        hipLaunchKernelGGL(fn, dim3(g.grid), dim3(256), 0, s, (const MacArgs *)g.d_args,
                           (const uint32_t *)g.d_first, (uint32_t)g.layers.size(), b->d_counters + 8 * gi, g.total);
        launches++;
        // layers whose Walsh group is wider than the fused epilogue
        for (uint32_t l : g.layers) {
            bool wht = false;
            conv_make_args(c, &b->desc[l], b->io[l].d_ct, b->io[l].d_wntt, b->io[l].d_taps, b->io[l].d_out, g.sched,
                           true, &wht);
            if (wht) {
                const hyena_conv_desc &d = b->desc[l];
                const hipError_t e = conv_launch_wht(c, d.c_n, b->io[l].d_out, b->io[l].d_out,
                                                     (size_t)d.batch * d.tiles * d.Co / d.c_n, s);
                if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_batch_run: ") + hipGetErrorString(e));
                launches++;
            }
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(HYENA_EHIP, std::string("hyena_batch_run: ") + hipGetErrorString(e));
    for (uint32_t l : b->solo) {
        const int rc = conv_launch(c, &b->desc[l], b->io[l].d_ct, b->io[l].d_wntt, b->io[l].d_taps, b->io[l].d_out,
                                   b->mac_sched[l], true, s);
        if (rc) return rc;
        launches++;
    }
    return HYENA_OK;
}

static int issue_step(hyena_batch *b, hipStream_t s, int phase = -1) {
    const hyena_ctx *c = b->ctx;
    std::vector<uint32_t *> in_ptrs, out_ptrs;
    std::vector<size_t> in_P, out_P;
    for (size_t l = 0; l < b->io.size(); l++) {
        const hyena_conv_desc &d = b->desc[l];
        in_ptrs.push_back(b->io[l].d_ct);
        in_P.push_back((size_t)d.batch * d.n_in * 2);
        out_ptrs.push_back(b->io[l].d_out);
        out_P.push_back((size_t)d.batch * d.n_out * 2);
    }
    int launches = 0, rc = HYENA_OK;
    if (phase < 0 || phase == 0) {
        rc = launch_ntt_segs(c, in_ptrs.data(), in_P.data(), (uint32_t)in_ptrs.size(), false, b->ntt_fwd, s);
        if (rc) return rc;
        launches += (int)((in_ptrs.size() + HYENA_MAX_SEGS - 1) / HYENA_MAX_SEGS);
    }
    if (phase < 0 || phase == 1) {
        rc = issue_mac_phase(b, s, launches);
        if (rc) return rc;
    }
    if (phase < 0 || phase == 2) {
        rc = launch_ntt_segs(c, out_ptrs.data(), out_P.data(), (uint32_t)out_ptrs.size(), true, b->ntt_inv, s);
        if (rc) return rc;
        launches += (int)((out_ptrs.size() + HYENA_MAX_SEGS - 1) / HYENA_MAX_SEGS);
    }
    // launches per step (summed over the three phase calls when run phase by phase)
    if (phase <= 0) b->launches = launches;
    else b->launches += launches;
    return HYENA_OK;
}

// time `fn` (enqueued on s) with events: best of `reps` after one warm-up
template <class F>
static float time_best(hipStream_t s, int reps, F fn) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    fn();
    float best = 1e30f;
    for (int r = 0; r < reps; r++) {
        (void)hipEventRecord(e0, s);
        fn();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

static std::string layer_key(const hyena_ctx *c, const std::string &arch, const hyena_conv_desc &d,
                             const hyena_layer_io &io) {
    std::ostringstream k;
    k << arch << "|mac|N" << c->N << "|L" << c->L << "|lazy" << c->lazy_ntt << "|" << d.H << "x" << d.W << "|"
      << d.Ci << ">" << d.Co << "|k" << d.k << "|dw" << d.depthwise << "|cn" << d.c_n << "|ci" << d.ci << "|b"
      << d.batch << "|t" << d.tiles << "|w" << (io.d_wntt ? 1 : 0) << "|taps" << (io.d_taps ? 1 : 0);
    return k.str();
}

// a schedule the layer can run: valid for its shape, and its weights in the
// form the schedule reads (NTT-domain words, or integer taps)
static bool sched_usable(const hyena_conv_desc &d, const hyena_layer_io &io, int sid) {
    if (!conv_sched_valid(&d, sid)) return false;
    return conv_sched_syn(sid) ? io.d_taps != nullptr : io.d_wntt != nullptr;
}

static int tune(hyena_batch *b) {
    const hyena_ctx *c = b->ctx;
    const std::string arch = arch_name(c->device);
    auto cache = load_cache();
    bool dirty = false;
    hipStream_t s;
    HIP_TRY(hipStreamCreate(&s));
    const int ns = conv_num_scheds();
    const bool persistent = (b->flags & HYENA_BATCH_PERSISTENT) != 0;
    std::vector<std::vector<float>> times(b->desc.size(), std::vector<float>(ns, -1.f));
    bool all_cached = true;
    for (size_t l = 0; l < b->desc.size(); l++) {
        const hyena_conv_desc &d = b->desc[l];
        const std::string key = layer_key(c, arch, d, b->io[l]) + (persistent ? "|persistent" : "");
        auto it = cache.find(key);
        if (it != cache.end() && it->second >= 0 && it->second < ns && sched_usable(d, b->io[l], it->second)) {
            b->mac_sched[l] = it->second;
            continue;
        }
        all_cached = false;
        float best = 1e30f;
        int best_s = b->mac_sched[l];
        for (int sid = 0; sid < ns; sid++) {
            if (!sched_usable(d, b->io[l], sid)) continue;
            int info[6];
            conv_sched_info(sid, info);
            if (!d.depthwise && !info[0] && info[1] * info[2] < 16) continue;  // tiny register tiles
            int rc = HYENA_OK;
            const float ms = time_best(s, 2, [&] {
                if (!rc) rc = conv_launch(c, &d, b->io[l].d_ct, b->io[l].d_wntt, b->io[l].d_taps, b->io[l].d_out, sid,
                                          true, s);
            });
            if (rc) continue;
            times[l][sid] = ms;
            if (ms < best) {
                best = ms;
                best_s = sid;
            }
        }
        b->mac_sched[l] = best_s;
        dirty = true;
    }
    if (persistent && !all_cached) {
        // one persistent launch covers the layers of one LDS schedule: use a
        // common schedule when it costs at most 5% over the per-layer optimum
        float opt = 0.f;
        std::vector<size_t> lds_layers;
        for (size_t l = 0; l < b->desc.size(); l++) {
            int info[6];
            conv_sched_info(b->mac_sched[l], info);
            if (!info[0]) continue;
            lds_layers.push_back(l);
            opt += times[l][b->mac_sched[l]];
        }
        int common = -1;
        float common_t = 1e30f;
        for (int sid = 0; sid < ns && !lds_layers.empty(); sid++) {
            int info[6];
            conv_sched_info(sid, info);
            if (!info[0]) continue;
            float t = 0.f;
            for (size_t l : lds_layers) {
                if (times[l][sid] < 0) { t = 1e30f; break; }
                t += times[l][sid];
            }
            if (t < common_t) { common_t = t; common = sid; }
        }
        if (common >= 0 && common_t <= 1.05f * opt)
            for (size_t l : lds_layers) b->mac_sched[l] = common;
    }
    for (size_t l = 0; l < b->desc.size(); l++)
        cache[layer_key(c, arch, b->desc[l], b->io[l]) + (persistent ? "|persistent" : "")] = b->mac_sched[l];
    // NTT schedules per direction, each timed alone on the arrays it
    // transforms in a step: the forward on every layer's inputs (an untimed
    // default inverse after each timed forward restores them), the inverse on
    // every layer's outputs (overwritten by every step anyway)
    std::vector<uint32_t *> pin, pout;
    std::vector<size_t> Pin, Pout;
    size_t polys_in = 0, polys_out = 0;
    for (size_t l = 0; l < b->desc.size(); l++) {
        pin.push_back(b->io[l].d_ct);
        Pin.push_back((size_t)b->desc[l].batch * b->desc[l].n_in * 2);
        polys_in += Pin.back();
        pout.push_back(b->io[l].d_out);
        Pout.push_back((size_t)b->desc[l].batch * b->desc[l].n_out * 2);
        polys_out += Pout.back();
    }
    std::ostringstream nk;
    nk << arch << "|ntt|N" << c->N << "|L" << c->L << "|lazy" << c->lazy_ntt;
    const std::string kf = nk.str() + "|polys" + std::to_string(std::min<size_t>(polys_in, 4096)) + "|fwd";
    const std::string ki = nk.str() + "|polys" + std::to_string(std::min<size_t>(polys_out, 4096)) + "|inv";
    int nfirst = 0, ncount = 0;
    hyena_ntt_schedules(c->N, &nfirst, &ncount);
    auto valid_ntt = [&](const std::string &k) {
        return cache.count(k) && cache[k] >= nfirst && cache[k] < nfirst + ncount;
    };
    if (valid_ntt(kf) && valid_ntt(ki)) {
        b->ntt_fwd = cache[kf];
        b->ntt_inv = cache[ki];
    } else {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            (void)hipStreamDestroy(s);
            return set_error(HYENA_EHIP, "hyena_batch_create: event");
        }
        // best of 3 timed runs of `timed` after one warm-up; `after` (untimed)
        // follows every run
        auto best_of = [&](auto timed, auto after) {
            float best = 1e30f;
            for (int r = 0; r < 4; r++) {
                (void)hipEventRecord(e0, s);
                timed();
                (void)hipEventRecord(e1, s);
                after();
                (void)hipEventSynchronize(e1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (r > 0) best = std::min(best, ms);
            }
            return best;
        };
        float bf = 1e30f, bi = 1e30f;
        std::vector<std::pair<float, int>> inv_times;
        for (int sid = nfirst; sid < nfirst + ncount; sid++) {
            const float tf = best_of(
                [&] { launch_ntt_segs(c, pin.data(), Pin.data(), (uint32_t)pin.size(), false, sid, s); },
                [&] { launch_ntt_segs(c, pin.data(), Pin.data(), (uint32_t)pin.size(), true, -1, s); });
            const float ti = best_of(
                [&] { launch_ntt_segs(c, pout.data(), Pout.data(), (uint32_t)pout.size(), true, sid, s); },
                [] {});
            if (tf < bf) { bf = tf; b->ntt_fwd = sid; }
            if (ti < bi) { bi = ti; b->ntt_inv = sid; }
            inv_times.emplace_back(ti, sid);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        std::sort(inv_times.begin(), inv_times.end());
        for (const auto &t : inv_times)
            if (t.first <= 1.05f * bi) b->inv_cands.push_back(t.second);
        b->inv_key = ki;
        cache[kf] = b->ntt_fwd;
        cache[ki] = b->ntt_inv;
        dirty = true;
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (dirty) save_cache(cache);
    return HYENA_OK;
}

static int build_groups(hyena_batch *b) {
    const hyena_ctx *c = b->ctx;
    std::map<int, std::vector<uint32_t>> by_sched;
    for (uint32_t l = 0; l < b->desc.size(); l++) {
        int info[6];
        conv_sched_info(b->mac_sched[l], info);
        if ((b->flags & HYENA_BATCH_PERSISTENT) && info[0] && persistent_fn(info, conv_sched_syn(b->mac_sched[l])))
            by_sched[b->mac_sched[l]].push_back(l);
        else
            b->solo.push_back(l);
    }
    int n_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
    b->n_counters = 8 * (uint32_t)by_sched.size();
    if (b->n_counters) HIP_TRY(hipMalloc((void **)&b->d_counters, sizeof(uint32_t) * b->n_counters));
    for (auto &kv : by_sched) {
        hyena_batch::Group g;
        g.sched = kv.first;
        // biggest layers first so the tail of the queue holds the short items
        g.layers = kv.second;
        std::vector<MacArgs> args;
        std::vector<uint32_t> first;
        uint32_t total = 0;
        for (uint32_t l : g.layers) {
            bool wht = false;
            MacArgs a = conv_make_args(c, &b->desc[l], b->io[l].d_ct, b->io[l].d_wntt, b->io[l].d_taps,
                                       b->io[l].d_out, g.sched, true, &wht);
            args.push_back(a);
            first.push_back(total);
            total += mac_blocks(a);
        }
        first.push_back(total);
        g.total = total;
        // per-queue slice table (see draw_item): qfirst[x][j] = items of the
        // layers before j in queue x
        {
            const size_t nl = g.layers.size();
            std::vector<uint32_t> qf(8 * (nl + 1), 0);
            for (uint32_t x = 0; x < 8; x++)
                for (size_t j = 0; j < nl; j++) {
                    const uint64_t n = first[j + 1] - first[j];
                    const uint32_t sz = (uint32_t)((n * (x + 1)) >> 3) - (uint32_t)((n * x) >> 3);
                    qf[x * (nl + 1) + j + 1] = qf[x * (nl + 1) + j] + sz;
                }
            first.insert(first.end(), qf.begin(), qf.end());
        }
        int info[6];
        conv_sched_info(g.sched, info);
        int per_cu = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void *)persistent_fn(info, conv_sched_syn(g.sched)), 256, 0));
        b->per_cu = per_cu;
        // every XCD queue needs its own blocks: a multiple of 8, at least 8
        g.grid = (uint32_t)std::max(1, per_cu) * (uint32_t)n_cu;
        if (g.grid > total) g.grid = std::max<uint32_t>(total, 1);
        g.grid = std::max<uint32_t>(8, (g.grid + 7) & ~7u);
        // owned by the batch before allocating, so hyena_batch_destroy frees
        // whatever was allocated if a later call fails
        b->groups.push_back(g);
        hyena_batch::Group &G = b->groups.back();
        HIP_TRY(hipMalloc((void **)&G.d_args, sizeof(MacArgs) * args.size()));
        HIP_TRY(hipMalloc((void **)&G.d_first, sizeof(uint32_t) * first.size()));
        HIP_TRY(hipMemcpy(G.d_args, args.data(), sizeof(MacArgs) * args.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(G.d_first, first.data(), sizeof(uint32_t) * first.size(), hipMemcpyHostToDevice));
    }
    return HYENA_OK;
}

// Autotuner, second stage: time the whole multiply-accumulate phase as the
// persistent launches and as one launch per layer, and keep the faster.
static int tune_mac_phase(hyena_batch *b) {
    const hyena_ctx *c = b->ctx;
    const std::string arch = arch_name(c->device);
    std::ostringstream all;
    for (size_t l = 0; l < b->desc.size(); l++)
        all << layer_key(c, arch, b->desc[l], b->io[l]) << "#" << b->mac_sched[l] << ";";
    std::ostringstream k;
    k << arch << "|macphase|" << std::hex << std::hash<std::string>()(all.str());
    auto cache = load_cache();
    auto it = cache.find(k.str());
    if (it != cache.end()) {
        b->mac_solo = it->second == 1;
        return HYENA_OK;
    }
    hipStream_t s;
    HIP_TRY(hipStreamCreate(&s));
    int rc = HYENA_OK;
    auto phase = [&](bool solo) {
        b->mac_solo = solo;
        int n = 0;
        if (!rc) rc = issue_mac_phase(b, s, n);
    };
    const float tp = time_best(s, 3, [&] { phase(false); });
    const float ts = time_best(s, 3, [&] { phase(true); });
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (rc) return rc;
    // the persistent launch unless per-layer launches are clearly faster (the
    // two are often within timing noise)
    b->mac_solo = ts < 0.97f * tp;
    cache[k.str()] = b->mac_solo ? 1 : 0;
    save_cache(cache);
    return HYENA_OK;
}

// Autotuner, third stage: in a step the inverse transforms run right after
// the multiply-accumulate, whose output writes they then read; schedules that
// time alike on their own can differ there by several percent. Time each
// close candidate after an untimed multiply-accumulate phase and keep the
// fastest.
static int tune_inv_in_step(hyena_batch *b) {
    const hyena_ctx *c = b->ctx;
    std::vector<uint32_t *> pout;
    std::vector<size_t> Pout;
    for (size_t l = 0; l < b->desc.size(); l++) {
        pout.push_back(b->io[l].d_out);
        Pout.push_back((size_t)b->desc[l].batch * b->desc[l].n_out * 2);
    }
    hipStream_t s;
    HIP_TRY(hipStreamCreate(&s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = HYENA_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = set_error(HYENA_EHIP, "hyena_batch_create: event");
    float best = 1e30f;
    int best_sid = b->ntt_inv;
    for (int sid : b->inv_cands) {
        float t = 1e30f;
        for (int r = 0; r < 4 && !rc; r++) {
            int n = 0;
            rc = issue_mac_phase(b, s, n);
            if (rc) break;
            (void)hipEventRecord(e0, s);
            rc = launch_ntt_segs(c, pout.data(), Pout.data(), (uint32_t)pout.size(), true, sid, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) t = std::min(t, ms);
        }
        if (rc) break;
        if (t < best) { best = t; best_sid = sid; }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (rc) return rc;
    b->ntt_inv = best_sid;
    auto cache = load_cache();
    cache[b->inv_key] = best_sid;
    save_cache(cache);
    return HYENA_OK;
}

extern "C" void hyena_batch_destroy(hyena_batch *b) {
    if (!b) return;
    for (int i = 0; i < 3; i++) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
    }
    for (auto &g : b->groups) {
        if (g.d_args) (void)hipFree(g.d_args);
        if (g.d_first) (void)hipFree(g.d_first);
    }
    if (b->d_counters) (void)hipFree(b->d_counters);
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    delete b;
}

extern "C" int hyena_batch_create(const hyena_ctx *c, const hyena_layer_io *layers, uint32_t n_layers,
                                  uint32_t flags, hyena_batch **out) {
    if (!c || !layers || !out || n_layers == 0) return set_error(HYENA_EINVAL, "hyena_batch_create: bad argument");
    if (!c->d_fw) return set_error(HYENA_EINVAL, "hyena_batch_create: context was created host-only");
    *out = nullptr;
    auto *b = new (std::nothrow) hyena_batch();
    if (!b) return set_error(HYENA_ENOMEM, "hyena_batch_create: out of host memory");
    b->ctx = c;
    b->flags = flags;
    for (uint32_t l = 0; l < n_layers; l++) {
        const hyena_layer_io &io = layers[l];
        if (!io.desc || !io.d_ct || (!io.d_wntt && !io.d_taps) || !io.d_out || !io.desc->Bt) {
            delete b;
            return set_error(HYENA_EINVAL, "hyena_batch_create: layer " + std::to_string(l) +
                                               " has a NULL buffer or an unplanned descriptor");
        }
        if (((uintptr_t)io.d_ct | (uintptr_t)io.d_wntt | (uintptr_t)io.d_out) & 15u || ((uintptr_t)io.d_taps & 3u)) {
            delete b;
            return set_error(HYENA_EINVAL, "hyena_batch_create: layer " + std::to_string(l) +
                                               " has a misaligned buffer");
        }
        b->desc.push_back(*io.desc);
        if (b->desc.back().batch == 0) b->desc.back().batch = 1;
        b->io.push_back(io);
        // streamed weights by default; the synthesizing schedule when only
        // the integer taps are given
        const int def = io.d_wntt ? conv_default_sched(&b->desc.back()) : conv_default_synth_sched(&b->desc.back());
        if (def < 0 || !sched_usable(b->desc.back(), io, def)) {
            delete b;
            return set_error(HYENA_EINVAL, "hyena_batch_create: layer " + std::to_string(l) +
                                               " has only integer taps but cannot synthesize its weights "
                                               "(depthwise, or more than 18 taps per word)");
        }
        b->mac_sched.push_back(def);
    }
    b->ntt_fwd = b->ntt_inv = ntt_default_schedule(c->logN);
    int rc = HYENA_OK;
    if (flags & HYENA_BATCH_TIMING)
        for (auto &e : b->ev)
            if (!rc && hipEventCreate(&e) != hipSuccess) rc = set_error(HYENA_EHIP, "hyena_batch_create: event");
    if (flags & HYENA_BATCH_TUNE) rc = tune(b);
    if (!rc) rc = build_groups(b);
    if (!rc && (flags & HYENA_BATCH_TUNE) && !b->groups.empty()) rc = tune_mac_phase(b);
    if (!rc && (flags & HYENA_BATCH_TUNE) && b->inv_cands.size() > 1) rc = tune_inv_in_step(b);
    if (rc) {
        hyena_batch_destroy(b);
        return rc;
    }
    *out = b;
    return HYENA_OK;
}

static int capture(hyena_batch *b, int phase, int slot) {
    // capture on a private stream (the null stream cannot be captured)
    hipStream_t cs;
    HIP_TRY(hipStreamCreate(&cs));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = HYENA_OK;
    if (e == hipSuccess) rc = issue_step(b, cs, phase);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return set_error(HYENA_EHIP, std::string("hyena_batch_run: capture failed: ") +
                                         hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph[slot] = g;
    HIP_TRY(hipGraphInstantiate(&b->exec[slot], g, nullptr, nullptr, 0));
    return HYENA_OK;
}

extern "C" int hyena_batch_run(hyena_batch *b, hyena_stream_t stream) {
    if (!b) return set_error(HYENA_EINVAL, "hyena_batch_run: NULL batch");
    const hipStream_t s = (hipStream_t)stream;
    const bool timing = b->ev[0] != nullptr;
    if (!(b->flags & HYENA_BATCH_GRAPH)) {
        if (!timing) return issue_step(b, s);
        for (int p = 0; p < 3; p++) {
            HIP_TRY(hipEventRecord(b->ev[p], s));
            const int rc = issue_step(b, s, p);
            if (rc) return rc;
        }
        HIP_TRY(hipEventRecord(b->ev[3], s));
        return HYENA_OK;
    }
    if (!timing) {
        if (!b->exec[0]) {
            const int rc = capture(b, -1, 0);
            if (rc) return rc;
        }
        HIP_TRY(hipGraphLaunch(b->exec[0], s));
        return HYENA_OK;
    }
    for (int p = 0; p < 3; p++)
        if (!b->exec[p]) {
            const int rc = capture(b, p, p);
            if (rc) return rc;
        }
    for (int p = 0; p < 3; p++) {
        HIP_TRY(hipEventRecord(b->ev[p], s));
        HIP_TRY(hipGraphLaunch(b->exec[p], s));
    }
    HIP_TRY(hipEventRecord(b->ev[3], s));
    return HYENA_OK;
}

extern "C" int hyena_batch_phase_ms(const hyena_batch *b, float *ms) {
    if (!b || !ms) return set_error(HYENA_EINVAL, "hyena_batch_phase_ms: NULL argument");
    if (!b->ev[0]) return set_error(HYENA_EINVAL, "hyena_batch_phase_ms: batch built without HYENA_BATCH_TIMING");
    HIP_TRY(hipEventSynchronize(b->ev[3]));
    for (int i = 0; i < 3; i++) HIP_TRY(hipEventElapsedTime(&ms[i], b->ev[i], b->ev[i + 1]));
    return HYENA_OK;
}

extern "C" int hyena_batch_info(const hyena_batch *b, int *info, size_t n_info) {
    if (!b || !info) return set_error(HYENA_EINVAL, "hyena_batch_info: NULL argument");
    std::vector<int> v = {b->ntt_fwd, b->ntt_inv, b->launches, (int)b->desc.size(),
                          b->mac_solo ? 0 : (int)b->groups.size()};
    for (int s : b->mac_sched) v.push_back(s);
    for (size_t i = 0; i < n_info; i++) info[i] = i < v.size() ? v[i] : -1;
    return HYENA_OK;
}
