// Host side of the counting path: k <= 2, the directed-graph check, the work schedule
// (root sort by tier and cost, expansion into items) and the tier launches.
#include <string.h>

#include <mutex>
#include <vector>

#include "count_kernels.h"

namespace arb {

// ------------------------------------------------------------------ small k, checks

__global__ void k_count_k1(int64_t n, unsigned long long *total, unsigned long long *pv) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0) *total = (unsigned long long)n;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (pv) pv[i] = 1ull;
}

__global__ void k_count_k2(int64_t n, const int64_t *off, const int32_t *idx, unsigned long long *total,
                           unsigned long long *pv) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0) *total = (unsigned long long)off[n];
    if (!pv) return;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t s = off[i], e = off[i + 1];
        if (e > s) atomicAdd(&pv[i], (unsigned long long)(e - s));
        for (int64_t p = s; p < e; ++p) atomicAdd(&pv[idx[p]], 1ull);
    }
}

__global__ void k_root_outdeg(int64_t n, const int64_t *off, unsigned long long *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (unsigned long long)(off[i + 1] - off[i]);
}

__global__ void k_check_oriented(int64_t n, const int64_t *off, const int32_t *idx, int64_t m, int32_t *err) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int32_t bad = 0;
    if (wave == 0 && lane == 0 && (off[0] != 0 || off[n] != m)) bad = 1;
    for (int64_t v = wave; v < n; v += nwaves) {
        int64_t s = off[v], e = off[v + 1];
        if (e < s || s < 0 || e > m) { bad = 1; continue; }
        for (int64_t p = s + lane; p < e; p += 64) {
            int32_t u = idx[p];
            if (u <= v || u >= n) bad = 1;
            if (p > s && idx[p - 1] >= u) bad = 1;
        }
    }
    if (bad) atomicOr(err, 1);
}

__global__ void k_u64_fill(unsigned long long *p, unsigned long long v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_count_reset(unsigned long long *total, int *err, int *heads, int64_t *seg,
                              unsigned long long *ovf_count) {
    const int t = threadIdx.x;
    if (t == 0) {
        *total = 0ull;
        *ovf_count = 0ull;
    }
    if (t < 4) err[t] = 0;
    if (t < 16) {
        heads[t] = 0;
        seg[t] = 0;
    }
}

__global__ void k_finish(const int32_t *err, unsigned long long *total) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *err) *total = ~0ull;
}

// ------------------------------------------------------------------ schedule
//
// Roots are sorted by (tier, cost descending) -- heavy first, the longest-processing-
// time rule -- then expanded into items: a whole root is one item, a split root one item
// per out-neighbour (edge parallelism, Sec. 3.4), placed where the root sorted.  Items of
// a split root stay in the root's tier (|S| <= d+(root)); roots too large for any tier
// are always split and use the largest tier.

constexpr int kCostBits = 13;                 // schedule key: tier (3 bits) above the cost
constexpr uint32_t kCostMax = (1u << kCostBits) - 1;
constexpr int kBigTier = kNumTiers;        // roots above the LDS tiers, d+ <= dbig
constexpr int kDeadTier = 7;
constexpr int kMaxParts = 64;
constexpr int64_t kOvfCap = 1 << 20;          // overflowed pair items the big kernel can take

// Parts of a root: degree schedule P = ceil(d / split_deg); learned schedule
// P = ceil(2^(y - split_cost)) with y the predicted log2(1 + work); at most 64 and at
// most d.  Roots too large for LDS (d > ARB_MAX_LOCAL) are split per out-neighbour.
__device__ __forceinline__ int root_parts(int64_t d, int split_deg, const float *lcost, float split_cost, int64_t v) {
    int64_t P = 1;
    if (lcost) {
        if (split_cost > 0.f && lcost[v] >= split_cost)
            P = (int64_t)ceilf(exp2f(fminf(lcost[v] - split_cost, 7.f)));
    } else if (split_deg > 0 && d >= split_deg) {
        P = (d + split_deg - 1) / split_deg;
    }
    if (P > kMaxParts) P = kMaxParts;
    if (P > d) P = d;
    return (int)(P < 1 ? 1 : P);
}

// Tier of an item with a set of d vertices: the first tier whose capacity times fill / 100
// holds d (larger tiles and teams for lower fill), -1 above the largest tier.
__device__ __forceinline__ int tier_of_fill(int64_t d, int fill) {
    constexpr int cap[kNumTiers] = {64, 128, 256, 384, 512, 768};
    const int t0 = tier_of(d);
    if (t0 < 0) return -1;
    for (int t = t0; t < kNumTiers; ++t)
        if (d * 100 <= (int64_t)cap[t] * fill) return t;
    return kNumTiers - 1;
}

__global__ void k_root_keys(int64_t n, const int64_t *off, int k, const float *lcost, int split_deg, float split_cost,
                            int dbig, int fill, uint32_t *key, int32_t *val, int32_t *parts) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = off[v + 1] - off[v];
        uint32_t kk;
        int P = 0;
        if (d < k - 1) {
            kk = ((uint32_t)kDeadTier << kCostBits) | kCostMax;
        } else {
            int t = tier_of_fill(d, fill);
            // the learned cost is evaluated for roots above the 64-tier only (its light
            // roots balance under any order); the 64-tier keeps the degree cost
            const float *lc = t == 0 ? nullptr : lcost;
            if (t < 0 && d <= dbig) {
                t = kBigTier;                  // whole root, bit rows in global scratch
                P = 1;
            } else if (t < 0) {                // per-out-neighbour items in the largest tier
                t = kNumTiers - 1;
                P = -1;
            } else {
                P = root_parts(d, split_deg, lc, split_cost, v);
            }
            const float per = P > 0 ? (float)P : (float)d;
            // degree cost: out-degree per item; learned: predicted log2 work per item in
            // steps of 1/64
            float c = lc ? fmaxf(lc[v] - log2f(per), 0.f) * 64.f : (float)d / per;
            uint32_t cq = (uint32_t)fminf(c, (float)kCostMax);
            kk = ((uint32_t)t << kCostBits) | (kCostMax - cq);
        }
        key[v] = kk;
        val[v] = (int32_t)v;
        parts[v] = P;
    }
}

// items of the root at sorted position p: 0 (dead), P (parts) or d (per out-neighbour)
__global__ void k_sorted_units(int64_t n, const int64_t *off, const uint32_t *key, const int32_t *val,
                               const int32_t *parts, int64_t *ucnt) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        int64_t u = 0;
        if ((key[p] >> kCostBits) != (uint32_t)kDeadTier) {
            const int32_t v = val[p];
            const int P = parts[v];
            u = P > 0 ? P : off[v + 1] - off[v];
        }
        ucnt[p] = u;
    }
}

// item i of the root v with P parts (P == 1 whole root, P > 1 parts, else one item per
// out-neighbour)
__device__ __forceinline__ void put_item(const int64_t *off, const int32_t *idx, int32_t *iroot, int32_t *ichild,
                                         int64_t at, int32_t v, int P, int64_t i) {
    iroot[at] = v;
    ichild[at] = P == 1 ? -1 : (P > 1 ? (int32_t)(-2 - (i * 128 + P)) : idx[off[v] + i]);
}

// Writes the items of every sorted root: a lane per root, and the whole wave for the
// roots with more than a few items.
__global__ void k_expand(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *val, const int32_t *parts,
                         const int64_t *uoff, int32_t *iroot, int32_t *ichild) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
        const int64_t p = base + lane;
        int64_t b = 0, c = 0;
        int32_t v = 0;
        int P = 0;
        if (p < n) {
            b = uoff[p];
            c = uoff[p + 1] - b;
            if (c) {
                v = val[p];
                P = parts[v];
            }
        }
        const bool big = c > 4;
        if (!big)
            for (int64_t i = 0; i < c; ++i) put_item(off, idx, iroot, ichild, b + i, v, P, i);
        uint64_t m = __ballot(big);
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const int64_t bb = __shfl(b, src, 64), cc = __shfl(c, src, 64);
            const int32_t vv = __shfl(v, src, 64);
            const int PP = __shfl(P, src, 64);
            for (int64_t i = lane; i < cc; i += 64) put_item(off, idx, iroot, ichild, bb + i, vv, PP, i);
        }
    }
}

// seg[t] = first item of tier t (t = 0..8); items of dead roots are none.
__global__ void k_segments(int64_t n, const uint32_t *key, const int64_t *uoff, int64_t *seg) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(key[p] >> kCostBits);
        const int tp = p > 0 ? (int)(key[p - 1] >> kCostBits) : -1;
        for (int tt = tp + 1; tt <= t; ++tt) seg[tt] = uoff[p];
        if (p == n - 1)
            for (int tt = t + 1; tt <= 8; ++tt) seg[tt] = uoff[n];
    }
}

struct CountWs {
    int64_t *ucnt;        // n+1, scanned in place
    int64_t *seg;         // 16
    int *heads;           // 16
    int32_t *err;         // 4
    uint32_t *key, *key_alt;
    int32_t *val, *val_alt;
    int32_t *iroot, *ichild;
    int32_t *parts;       // n
    float *lcost;         // n
    unsigned long long *tot;  // total of the synchronous arb_count
    uint32_t *big_rows;       // big-item bit rows: big_teams slices of big_words words
    int64_t big_teams, big_words;
    int64_t *ovf_items;       // pair items overflowing the LDS tiers (ovf_cap entries)
    unsigned long long *ovf_count;
    int64_t ovf_cap;
    int dbig;
    void *scan_ws, *radix_ws;
};

static size_t carve_count(Carver &c, int64_t n, int64_t m, int k, CountWs *w) {
    const int64_t nn = n > 0 ? n : 1;
    const int64_t U = nn + (m > 0 ? m : 1);
    w->ucnt = c.take<int64_t>(nn + 1);
    w->seg = c.take<int64_t>(16);
    w->heads = c.take<int>(16);
    w->err = c.take<int32_t>(4);
    w->key = c.take<uint32_t>(nn);
    w->key_alt = c.take<uint32_t>(nn);
    w->val = c.take<int32_t>(nn);
    w->val_alt = c.take<int32_t>(nn);
    w->iroot = c.take<int32_t>(U);
    w->ichild = c.take<int32_t>(U);
    w->parts = c.take<int32_t>(nn);
    w->lcost = c.take<float>(nn);
    w->tot = c.take<unsigned long long>(4);
    w->scan_ws = c.take<char>(scan_workspace(nn + 1));
    w->radix_ws = c.take<char>(radix_workspace(nn));
    w->dbig = k >= 3 ? big_dmax(m) : 0;
    w->big_teams = w->dbig ? big_teams(m) : 0;
    w->big_words = w->dbig ? big_team_words(w->dbig) : 0;
    w->big_rows = c.take<uint32_t>(w->big_teams * w->big_words > 0 ? w->big_teams * w->big_words : 1);
    w->ovf_cap = w->dbig ? (m < kOvfCap ? (m > 0 ? m : 1) : kOvfCap) : 0;
    w->ovf_items = c.take<int64_t>(w->ovf_cap > 0 ? w->ovf_cap : 1);
    w->ovf_count = c.take<unsigned long long>(1);
    return c.used;
}

// learned cost (mlp.hip): predicted log2(1 + work) per root
int learned_cost(const arb_ocsr *dg, int k, const uint16_t *w, const float *feat, float *cost, hipStream_t s);

// Optional launch timing: while enabled, every counting-kernel launch is bracketed by
// two HIP events on the stream it runs on; arb_profile_read folds the pending pairs into
// per-(tier, k, per-vertex, instrumented) totals.
struct ProfKey {
    int tier, k, pv, instr;
    bool operator==(const ProfKey &o) const { return tier == o.tier && k == o.k && pv == o.pv && instr == o.instr; }
};
struct ProfPending {
    ProfKey key;
    hipEvent_t a, b;
};
struct ProfTotal {
    ProfKey key;
    int64_t launches;
    double ms;
};
struct Profile {
    bool enabled = false;
    std::vector<ProfPending> pending;
    std::vector<hipEvent_t> pool;
    std::vector<ProfTotal> totals;
};
static Profile g_prof;
// set while arb_count_noalloc runs: no launch-timing events are created
static thread_local bool g_no_events = false;

static int prof_event(hipEvent_t *e) {
    if (!g_prof.pool.empty()) {
        *e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return ARB_OK;
    }
    ARB_HIP(hipEventCreate(e));
    return ARB_OK;
}

static int prof_fold() {
    for (auto &p : g_prof.pending) {
        ARB_HIP(hipEventSynchronize(p.b));
        float ms = 0.f;
        ARB_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        bool found = false;
        for (auto &t : g_prof.totals)
            if (t.key == p.key) { t.launches += 1; t.ms += ms; found = true; break; }
        if (!found) g_prof.totals.push_back(ProfTotal{p.key, 1, (double)ms});
        g_prof.pool.push_back(p.a);
        g_prof.pool.push_back(p.b);
    }
    g_prof.pending.clear();
    return ARB_OK;
}

// Streams on which the tier kernels of one call run side by side (fork/join through
// events from the caller's stream; default priority).  One set per host thread.
struct TierStreams {
    bool ready = false;
    hipStream_t st[kNumTiers + 1];          // the tiers, then the global-scratch kernel
    hipEvent_t fork, join[kNumTiers + 1];
};
static thread_local TierStreams g_ts;

static int tier_streams_init() {
    if (g_ts.ready) return ARB_OK;
    for (int t = 0; t <= kNumTiers; ++t) {
        ARB_HIP(hipStreamCreateWithFlags(&g_ts.st[t], hipStreamNonBlocking));
        ARB_HIP(hipEventCreateWithFlags(&g_ts.join[t], hipEventDisableTiming));
    }
    ARB_HIP(hipEventCreateWithFlags(&g_ts.fork, hipEventDisableTiming));
    g_ts.ready = true;
    return ARB_OK;
}

static int launch_count(int depth, int tier, bool pv, bool instr, const CountArgs &a, unsigned grid, hipStream_t s) {
    switch (depth < 1 ? 1 : depth) {
        case 1: return launch_count_depth1(tier, pv, instr, a, grid, s);
        case 2: return launch_count_depth2(tier, pv, instr, a, grid, s);
        case 3: return launch_count_depth3(tier, pv, instr, a, grid, s);
        case 4: return launch_count_depth4(tier, pv, instr, a, grid, s);
        case 5: return launch_count_depth5(tier, pv, instr, a, grid, s);
        case 6: return launch_count_depth6(tier, pv, instr, a, grid, s);
        case 7: return launch_count_depth7(tier, pv, instr, a, grid, s);
        default: return launch_count_depth8(tier, pv, instr, a, grid, s);     // any deeper walk
    }
}

static int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return 256;
        cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
    }
    return cus;
}

}  // namespace arb

using namespace arb;

extern "C" void arb_count_default_opts(arb_count_opts *o) {
    if (!o) return;
    o->schedule = ARB_SCHED_PERSISTENT;
    o->split_min_degree = 0;
    o->split_min_cost = 0.f;
    o->persist_blocks_per_cu = 8;
    o->chunk_small = 16;
    o->bitmap_max_span = 1 << 30;
    o->concurrent_tiers = 1;
    o->tier_fill = 100;
    o->big_max_degree = -1;
    o->mlp_weights = nullptr;
    o->features = nullptr;
}

extern "C" size_t arb_count_workspace(int64_t n, int64_t m, int k) {
    (void)k;
    Carver c(nullptr);
    CountWs w;
    return carve_count(c, n, m, k, &w) + 256;
}

static bool ocsr_ok(const arb_ocsr *dg) {
    return dg && dg->n >= 0 && dg->m >= 0 && dg->n < (int64_t(1) << 31) && dg->offsets &&
           (dg->m == 0 || dg->indices);
}

extern "C" int arb_check_oriented(const arb_ocsr *dg, void *ws, size_t ws_bytes, void *stream) {
    hipStream_t s = as_stream(stream);
    int rc = ARB_OK;
    if (!ocsr_ok(dg) || !ws) rc = ARB_EINVAL;
    else if (ws_bytes < 1024) rc = ARB_EWORKSPACE;
    if (rc) { set_error(rc); return rc; }
    int32_t *err = static_cast<int32_t *>(ws);
    if ((rc = fill_i32(err, 0, 1, s))) { set_error(rc); return rc; }
    k_check_oriented<<<grid_for(dg->n * 64 + 64, 256, 8192), 256, 0, s>>>(dg->n, dg->offsets, dg->indices, dg->m, err);
    int32_t h = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&h, err, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error(ARB_EHIP);
        return ARB_EHIP;
    }
    rc = h ? ARB_EGRAPH : ARB_OK;
    set_error(rc);
    return rc;
}

// roff/ridx (nullable): the candidate set of each root in place of N+(v) -- any sorted
// set of vertices whose every (k-1)-clique, with the root, is a k-clique to count
// (arb-peel's updates); the workspace must then be sized for max(m, rnnz) arcs.
// root_ids (nullable, device): the roots are the nroots vertices listed there, root i with
// candidate set ridx[roff[i] .. roff[i + 1]) (roff then has nroots + 1 entries); only they
// are scheduled.  pv_zeroed: per_vertex already holds zeros (it is added to, not cleared).
int arb::count_with_roots(const arb_ocsr *dg, int k, uint64_t *total_dev, uint64_t *per_vertex, uint64_t *per_root_out,
                     uint64_t *work_out, const arb_count_opts *opts_in, void *ws, size_t ws_bytes, hipStream_t s,
                     const int64_t *roff, const int32_t *ridx, int64_t rnnz, uint64_t *cycles_out,
                     const int32_t *root_ids, int64_t nroots, bool pv_zeroed) {
    if (!ocsr_ok(dg) || !total_dev || !ws) return ARB_EINVAL;
    if (k < 1 || k > ARB_MAX_K) return ARB_EINVAL;
    if (roff && (!ridx || k < 3)) return ARB_EINVAL;
    if (root_ids && (!roff || nroots < 0 || nroots > dg->n || work_out || cycles_out)) return ARB_EINVAL;
    const int64_t mw = roff && rnnz > dg->m ? rnnz : dg->m;     // arcs the item arrays must hold
    if (!roff) {
        roff = dg->offsets;
        ridx = dg->indices;
    }
    arb_count_opts opts;
    arb_count_default_opts(&opts);
    if (opts_in) opts = *opts_in;
    if (opts.schedule < 0 || opts.schedule > 2) return ARB_EINVAL;
    if (opts.schedule == ARB_SCHED_LEARNED && (!opts.mlp_weights || !opts.features || root_ids)) return ARB_EINVAL;
    if (opts.persist_blocks_per_cu < 1 || opts.persist_blocks_per_cu > 8) return ARB_EINVAL;
    if (opts.chunk_small < 1 || opts.chunk_small > 256) return ARB_EINVAL;
    if (opts.bitmap_max_span < 0) return ARB_EINVAL;
    if (opts.split_min_degree < 0 || !(opts.split_min_cost >= 0.f)) return ARB_EINVAL;
    if (opts.tier_fill < 10 || opts.tier_fill > 100 || opts.big_max_degree < -1) return ARB_EINVAL;
    const int64_t n = dg->n, m = dg->m;
    if (ws_bytes < arb_count_workspace(n, mw, k)) return ARB_EWORKSPACE;
    unsigned long long *total = reinterpret_cast<unsigned long long *>(total_dev);
    unsigned long long *pv = reinterpret_cast<unsigned long long *>(per_vertex);
    unsigned long long *work = reinterpret_cast<unsigned long long *>(work_out);
    unsigned long long *cycles = work ? reinterpret_cast<unsigned long long *>(cycles_out) : nullptr;
    unsigned long long *per_root = reinterpret_cast<unsigned long long *>(per_root_out);
    int rc;
    const unsigned gb = grid_for(n, 256, 4096);
    if (pv && !pv_zeroed) { k_u64_fill<<<gb, 256, 0, s>>>(pv, 0ull, n); ARB_CHECK_LAUNCH(); }
    if (work) { k_u64_fill<<<gb, 256, 0, s>>>(work, 0ull, n); ARB_CHECK_LAUNCH(); }
    if (cycles) { k_u64_fill<<<gb, 256, 0, s>>>(cycles, 0ull, n); ARB_CHECK_LAUNCH(); }
    if (per_root) { k_u64_fill<<<gb, 256, 0, s>>>(per_root, 0ull, n); ARB_CHECK_LAUNCH(); }
    if (per_root && k <= 2) {
        if (k == 1) k_u64_fill<<<gb, 256, 0, s>>>(per_root, 1ull, n);
        else k_root_outdeg<<<gb, 256, 0, s>>>(n, dg->offsets, per_root);
        ARB_CHECK_LAUNCH();
    }
    if (k == 1) { k_count_k1<<<gb, 256, 0, s>>>(n, total, pv); ARB_CHECK_LAUNCH(); return ARB_OK; }
    if (k == 2) { k_count_k2<<<gb, 256, 0, s>>>(n, dg->offsets, dg->indices, total, pv); ARB_CHECK_LAUNCH(); return ARB_OK; }
    // roots scheduled: every vertex, or the listed ones
    const int64_t ns = root_ids ? nroots : n;
    const unsigned gs = grid_for(ns, 256, 4096);
    if (ns == 0) {
        k_u64_fill<<<1, 64, 0, s>>>(total, 0ull, 1);
        ARB_CHECK_LAUNCH();
        return ARB_OK;
    }

    Carver cv(ws);
    CountWs w;
    carve_count(cv, n, mw, k, &w);
    // the total, error flags, queue heads, segments and overflow count, in one launch
    k_count_reset<<<1, 64, 0, s>>>(total, w.err, w.heads, w.seg, w.ovf_count);
    ARB_CHECK_LAUNCH();

    const bool learned = opts.schedule == ARB_SCHED_LEARNED && !work;
    const float *lcost = nullptr;
    if (learned) {
        if ((rc = learned_cost(dg, k, opts.mlp_weights, opts.features, w.lcost, s))) return rc;
        lcost = w.lcost;
    }
    const int split_deg = work ? 0 : opts.split_min_degree;
    const float split_cost = work ? 0.f : opts.split_min_cost;
    const int dbig_whole = opts.big_max_degree < 0 ? w.dbig : (opts.big_max_degree < w.dbig ? opts.big_max_degree : w.dbig);
    k_root_keys<<<gs, 256, 0, s>>>(ns, roff, k, lcost, split_deg, split_cost, dbig_whole, opts.tier_fill, w.key,
                                   w.val, w.parts);
    ARB_CHECK_LAUNCH();
    if ((rc = radix_sort_u32(w.key, w.val, w.key_alt, w.val_alt, ns, kCostBits + 3, w.radix_ws, s))) return rc;
    k_sorted_units<<<gs, 256, 0, s>>>(ns, roff, w.key, w.val, w.parts, w.ucnt);
    ARB_CHECK_LAUNCH();
    if ((rc = exclusive_scan_i64(w.ucnt, w.ucnt, ns, w.scan_ws, s))) return rc;
    k_expand<<<gs, 256, 0, s>>>(ns, roff, ridx, w.val, w.parts, w.ucnt, w.iroot, w.ichild);
    ARB_CHECK_LAUNCH();
    k_segments<<<gs, 256, 0, s>>>(ns, w.key, w.ucnt, w.seg);
    ARB_CHECK_LAUNCH();

    const bool pvm = pv != nullptr;
    const bool instr = work != nullptr;
    int64_t hseg[16] = {0};
    const bool plain = opts.schedule == ARB_SCHED_PLAIN;
    if (plain) {
        ARB_HIP(hipMemcpyAsync(hseg, w.seg, sizeof(int64_t) * 9, hipMemcpyDeviceToHost, s));
        ARB_HIP(hipStreamSynchronize(s));
    }
    const int cus = device_cus();
    const bool prof = g_prof.enabled && !g_no_events;
    if (prof && g_prof.pending.size() > 2048 && (rc = prof_fold())) return rc;
    const bool conc = opts.concurrent_tiers && !plain;
    if (conc) {
        if ((rc = tier_streams_init())) return rc;
        ARB_HIP(hipEventRecord(g_ts.fork, s));
    }
    // Items above the LDS tiers (global-scratch kernel).  Its schedule items do not depend
    // on the tier kernels, so with the tiers side by side it starts first, on a stream of
    // its own (one 16-wave team per CU beside the tiers' teams); the pair items that the
    // tier kernels overflow follow in a second launch after them.
    auto launch_big_part = [&](int parts, hipStream_t bs) -> int {
        CountArgs a;
        a.off = dg->offsets;
        a.idx = dg->indices;
        a.roff = roff;
        a.ridx = ridx;
        a.n = n;
        a.m = m;
        a.k = k;
        a.item_root = w.iroot;
        a.item_child = w.ichild;
        a.seg = w.seg + kBigTier;
        a.head = w.heads + (parts & kBigSegment ? kBigTier : kBigTier + 1);
        a.total = total;
        a.pv = pv;
        a.per_root = per_root;
        a.work = work;
        a.cycles = cycles;
        a.root_ids = root_ids;
        a.err = w.err;
        a.chunk = 1;
        a.span_max = 0;
        a.persistent = 1;
        a.one_item_per_team = 0;
        a.ovf_items = w.ovf_items;
        a.ovf_count = w.ovf_count;
        a.ovf_cap = w.ovf_cap;
        const BigArgs b{w.big_rows, w.big_words, w.dbig, parts};
        int64_t bteams = w.big_teams < cus ? w.big_teams : cus;
        if (parts & kBigSegment && ns * 64 < bteams) bteams = ns * 64;      // as for the tiers
        const unsigned grid = (unsigned)(bteams > 0 ? bteams : 1);
        const int ptier = parts & kBigSegment ? kBigTier : kBigTier + 1;
        ProfPending pp{ProfKey{ptier, k, pvm ? 1 : 0, instr ? 1 : 0}, nullptr, nullptr};
        if (prof) {
            if (prof_event(&pp.a) || prof_event(&pp.b)) return ARB_EHIP;
            if (hipEventRecord(pp.a, bs) != hipSuccess) return ARB_EHIP;
        }
        const int r = launch_count_big(pvm, instr, a, b, grid, bs);
        if (r) return r;
        if (prof) {
            if (hipEventRecord(pp.b, bs) != hipSuccess) return ARB_EHIP;
            g_prof.pending.push_back(pp);
        }
        return ARB_OK;
    };
    if (conc && w.big_teams > 0) {
        hipStream_t bs = g_ts.st[kNumTiers];
        ARB_HIP(hipStreamWaitEvent(bs, g_ts.fork, 0));
        if ((rc = launch_big_part(kBigSegment, bs))) return rc;
        ARB_HIP(hipEventRecord(g_ts.join[kNumTiers], bs));
    }
    for (int t = kNumTiers - 1; t >= 0; --t) {
        CountArgs a;
        a.off = dg->offsets;
        a.idx = dg->indices;
        a.roff = roff;
        a.ridx = ridx;
        a.n = n;
        a.m = m;
        a.k = k;
        a.item_root = w.iroot;
        a.item_child = w.ichild;
        a.seg = w.seg + t;
        a.head = w.heads + t;
        a.total = total;
        a.pv = pv;
        a.per_root = per_root;
        a.work = work;
        a.cycles = cycles;
        a.root_ids = root_ids;
        a.err = w.err;
        a.chunk = t == 0 ? opts.chunk_small : 1;
        a.span_max = opts.bitmap_max_span;
        a.persistent = plain ? 0 : 1;
        a.one_item_per_team = plain ? 1 : 0;
        a.ovf_items = w.big_teams > 0 ? w.ovf_items : nullptr;
        a.ovf_count = w.ovf_count;
        a.ovf_cap = w.ovf_cap;
        const int tpb = tier_teams_per_block(t);
        unsigned grid;
        if (plain) {
            const int64_t cnt = hseg[t + 1] - hseg[t];
            if (cnt <= 0) continue;
            grid = (unsigned)((cnt + tpb - 1) / tpb);
        } else {
            const size_t lds = tier_block_lds(t, pvm, k - 3 < 1 ? 1 : k - 3);
            int per_cu = (int)((160 * 1024) / (lds > 0 ? lds : 1));
            if (per_cu > opts.persist_blocks_per_cu) per_cu = opts.persist_blocks_per_cu;
            if (per_cu < 1) per_cu = 1;
            grid = (unsigned)(cus * per_cu);
            // a few scheduled roots (the peels' rounds) need few teams: a persistent grid
            // of empty teams costs ~0.1 ms a launch.  A root gives at most 64 items here
            // (split parts) unless it becomes pair items, which the teams still drain.
            const int64_t cap = (ns * 64 + tpb - 1) / tpb;
            if (cap < (int64_t)grid) grid = (unsigned)(cap > 0 ? cap : 1);
        }
        hipStream_t ls = s;
        if (conc) {
            ls = g_ts.st[t];
            ARB_HIP(hipStreamWaitEvent(ls, g_ts.fork, 0));
        }
        ProfPending pp{ProfKey{t, k, pvm ? 1 : 0, instr ? 1 : 0}, nullptr, nullptr};
        if (prof) {
            if ((rc = prof_event(&pp.a)) || (rc = prof_event(&pp.b))) return rc;
            ARB_HIP(hipEventRecord(pp.a, ls));
        }
        rc = launch_count(k - 3, t, pvm, instr, a, grid, ls);
        if (rc) return rc;
        if (prof) {
            ARB_HIP(hipEventRecord(pp.b, ls));
            g_prof.pending.push_back(pp);
        }
        if (conc) {
            ARB_HIP(hipEventRecord(g_ts.join[t], ls));
            ARB_HIP(hipStreamWaitEvent(s, g_ts.join[t], 0));
        }
    }
    if (w.big_teams > 0) {
        if (conc) {
            // the overflowed pair items, which the tier kernels appended
            ARB_HIP(hipStreamWaitEvent(s, g_ts.join[kNumTiers], 0));
            if ((rc = launch_big_part(kBigOverflow, s))) return rc;
        } else {
            // roots above the LDS tiers, then the overflowed pair items, after the tiers
            if ((rc = launch_big_part(kBigSegment | kBigOverflow, s))) return rc;
        }
    }
    k_finish<<<1, 64, 0, s>>>(w.err, total);
    ARB_CHECK_LAUNCH();
    return ARB_OK;
}

static int count_impl(const arb_ocsr *dg, int k, uint64_t *total_dev, uint64_t *per_vertex, uint64_t *per_root_out,
                      uint64_t *work_out, const arb_count_opts *opts_in, void *ws, size_t ws_bytes, hipStream_t s) {
    return count_with_roots(dg, k, total_dev, per_vertex, per_root_out, work_out, opts_in, ws, ws_bytes, s, nullptr,
                            nullptr, 0);
}

extern "C" int arb_count_async(const arb_ocsr *dg, int k, uint64_t *total_dev, uint64_t *per_vertex,
                               uint64_t *per_root, uint64_t *work_out, const arb_count_opts *opts, void *ws,
                               size_t ws_bytes, void *stream) {
    int rc = count_impl(dg, k, total_dev, per_vertex, per_root, work_out, opts, ws, ws_bytes, as_stream(stream));
    set_error(rc);
    return rc;
}

extern "C" int arb_count_instrumented(const arb_ocsr *dg, int k, uint64_t *work_out, uint64_t *cycles_out,
                                      const arb_count_opts *opts, void *ws, size_t ws_bytes, void *stream) {
    int rc = ARB_OK;
    if (!work_out || !ws) rc = ARB_EINVAL;
    else if (ws_bytes < 64) rc = ARB_EWORKSPACE;
    if (!rc) {
        // the total goes to the workspace's own slot (the workspace is sized with room for it)
        Carver cv(ws);
        CountWs w;
        carve_count(cv, dg && dg->n >= 0 ? dg->n : 0, dg && dg->m >= 0 ? dg->m : 0, k, &w);
        rc = count_with_roots(dg, k, reinterpret_cast<uint64_t *>(w.tot), nullptr, nullptr, work_out, opts, ws,
                              ws_bytes, as_stream(stream), nullptr, nullptr, 0, cycles_out);
    }
    set_error(rc);
    return rc;
}

extern "C" uint64_t arb_count(const arb_ocsr *dg, int k, uint64_t *per_vertex, const arb_count_opts *opts,
                              void *ws, size_t ws_bytes, void *stream) {
    hipStream_t s = as_stream(stream);
    if (!ocsr_ok(dg) || !ws) { set_error(ARB_EINVAL); return 0; }
    if (ws_bytes < arb_count_workspace(dg->n, dg->m, k)) { set_error(ARB_EWORKSPACE); return 0; }
    if (arb_check_oriented(dg, ws, ws_bytes, stream)) return 0;
    Carver cv(ws);
    CountWs w;
    carve_count(cv, dg->n, dg->m, k, &w);
    int rc = count_impl(dg, k, reinterpret_cast<uint64_t *>(w.tot), per_vertex, nullptr, nullptr, opts, ws, ws_bytes, s);
    if (rc) { set_error(rc); return 0; }
    uint64_t h = 0;
    if (hipMemcpyAsync(&h, w.tot, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error(ARB_EHIP);
        return 0;
    }
    if (h == ~0ull) {         // k_finish: an item did not fit the largest tier
        set_error(ARB_ELIMIT);
        return 0;
    }
    set_error(ARB_OK);
    return h;
}

// ------------------------------------------------------------------ allocation-free entry point
//
// arb_count_noalloc takes its workspace from this file-scope device array instead of a
// caller buffer.  Each device holds its own copy for the life of the process; host code
// reaches it only through the address hipGetSymbolAddress returns on that device (the
// array's name in host code is not a device address).
constexpr size_t kNoAllocScratch = ARB_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];
constexpr int kNoAllocDevices = 64;
static void *g_scratch_ptr[kNoAllocDevices];
static std::mutex g_scratch_mu;

static int noalloc_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ARB_EHIP;
    if (dev < 0 || dev >= kNoAllocDevices) return ARB_ELIMIT;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ARB_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ARB_OK;
}

extern "C" int arb_count_noalloc(const arb_ocsr *dg, int k, uint64_t *total_dev, uint64_t *per_vertex,
                                 const arb_count_opts *opts, void *stream) {
    int rc = ARB_OK;
    void *ws = nullptr;
    if (!ocsr_ok(dg) || !total_dev || k < 1 || k > ARB_MAX_K) rc = ARB_EINVAL;
    else if (arb_count_workspace(dg->n, dg->m, k) > kNoAllocScratch) rc = ARB_ELIMIT;
    else rc = noalloc_scratch(&ws);
    if (rc) { set_error(rc); return rc; }
    arb_count_opts o;
    arb_count_default_opts(&o);
    if (opts) o = *opts;
    o.concurrent_tiers = 0;          // the caller's stream only: no library streams or events
    g_no_events = true;
    rc = count_impl(dg, k, total_dev, per_vertex, nullptr, nullptr, &o, ws, kNoAllocScratch, as_stream(stream));
    g_no_events = false;
    set_error(rc);
    return rc;
}

extern "C" int arb_profile_enable(int on) {
    int rc = ARB_OK;
    if (on) {
        rc = prof_fold();
        g_prof.totals.clear();
    } else {
        rc = prof_fold();
    }
    g_prof.enabled = on != 0;
    set_error(rc);
    return rc;
}

extern "C" int arb_profile_read(int max_entries, int32_t *tier, int32_t *k, int32_t *per_vertex,
                                int32_t *instrumented, int64_t *launches, double *total_ms) {
    if (max_entries < 0 || (max_entries > 0 && (!tier || !k || !per_vertex || !instrumented || !launches ||
                                                !total_ms))) {
        set_error(ARB_EINVAL);
        return -1;
    }
    int rc = prof_fold();
    if (rc) { set_error(rc); return -1; }
    int nout = 0;
    for (auto &t : g_prof.totals) {
        if (nout < max_entries) {
            tier[nout] = t.key.tier;
            k[nout] = t.key.k;
            per_vertex[nout] = t.key.pv;
            instrumented[nout] = t.key.instr;
            launches[nout] = t.launches;
            total_ms[nout] = t.ms;
        }
        ++nout;
    }
    set_error(ARB_OK);
    return nout;
}

// ------------------------------------------------------------------ autotuner

namespace {

struct TuneSpace {
    std::vector<int> split_deg{0, 32, 64, 128, 256};
    std::vector<float> split_cost{0.f, 14.f, 17.f, 20.f, 23.f, 26.f};
    std::vector<int> conc{0, 1};
    std::vector<int> blocks{2, 4, 8};
    std::vector<int> chunk{4, 16, 64};
    std::vector<int> span{0, 1 << 30};
    std::vector<int> fill{100, 75, 50};
    std::vector<int> bigmax{-1, 768};
};

}  // namespace

extern "C" int arb_autotune_space(int dim, int max_values, double *values) {
    TuneSpace sp;
    std::vector<double> v;
    switch (dim) {
        case ARB_TUNE_SPLIT_MIN_DEGREE: v.assign(sp.split_deg.begin(), sp.split_deg.end()); break;
        case ARB_TUNE_SPLIT_MIN_COST: v.assign(sp.split_cost.begin(), sp.split_cost.end()); break;
        case ARB_TUNE_BLOCKS_PER_CU: v.assign(sp.blocks.begin(), sp.blocks.end()); break;
        case ARB_TUNE_CHUNK_SMALL: v.assign(sp.chunk.begin(), sp.chunk.end()); break;
        case ARB_TUNE_BITMAP_MAX_SPAN: v.assign(sp.span.begin(), sp.span.end()); break;
        case ARB_TUNE_CONCURRENT_TIERS: v.assign(sp.conc.begin(), sp.conc.end()); break;
        case ARB_TUNE_TIER_FILL: v.assign(sp.fill.begin(), sp.fill.end()); break;
        case ARB_TUNE_BIG_MAX_DEGREE: v.assign(sp.bigmax.begin(), sp.bigmax.end()); break;
        default: set_error(ARB_EINVAL); return -1;
    }
    if (max_values < 0 || (max_values > 0 && !values)) { set_error(ARB_EINVAL); return -1; }
    for (int i = 0; i < (int)v.size() && i < max_values; ++i) values[i] = v[i];
    set_error(ARB_OK);
    return (int)v.size();
}

extern "C" int arb_autotune(const arb_ocsr *dg, int k, arb_count_opts *opts, int trials, float *best_ms,
                            void *ws, size_t ws_bytes, void *stream) {
    hipStream_t s = as_stream(stream);
    auto fail = [](int rc) { set_error(rc); return rc; };
    if (!ocsr_ok(dg) || !opts || !ws || trials < 1 || trials > 100) return fail(ARB_EINVAL);
    if (ws_bytes < arb_count_workspace(dg->n, dg->m, k)) return fail(ARB_EWORKSPACE);
    Carver cv(ws);
    CountWs w;
    carve_count(cv, dg->n, dg->m, k, &w);
    uint64_t *tot = reinterpret_cast<uint64_t *>(w.tot);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(ARB_EHIP);
    uint64_t ref_total = 0;
    bool have_ref = false;
    int rc = ARB_OK;
    // time one configuration: one warm-up, then the best of `trials`; totals must agree.
    // A candidate whose warm-up run takes more than twice the best time so far is not
    // timed further (its time is the warm-up's)
    float cur_ms = 0.f;
    auto measure = [&](const arb_count_opts &o, float *ms_out) -> int {
        float best = 1e30f;
        for (int t = 0; t <= trials; ++t) {
            if (hipEventRecord(e0, s) != hipSuccess) return ARB_EHIP;
            int r = count_impl(dg, k, tot, nullptr, nullptr, nullptr, &o, ws, ws_bytes, s);
            if (r) return r;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return ARB_EHIP;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return ARB_EHIP;
            if (t > 0 && ms < best) best = ms;
            if (t == 0 && have_ref && ms > 2.f * cur_ms) {
                best = ms;
                break;
            }
        }
        uint64_t h = 0;
        if (hipMemcpy(&h, tot, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return ARB_EHIP;
        if (h == ~0ull) return ARB_ELIMIT;
        if (!have_ref) { ref_total = h; have_ref = true; }
        else if (h != ref_total) return ARB_EMISMATCH;
        *ms_out = best;
        return ARB_OK;
    };
    TuneSpace sp;
    arb_count_opts cur = *opts;
    if (cur.schedule == ARB_SCHED_PLAIN) cur.schedule = ARB_SCHED_PERSISTENT;
    const bool learned = cur.schedule == ARB_SCHED_LEARNED;
    if ((rc = measure(cur, &cur_ms))) goto out;
    for (int pass = 0; pass < 2; ++pass) {
        for (int param = 0; param < 7; ++param) {
            const int nv = param == 0 ? (learned ? (int)sp.split_cost.size() : (int)sp.split_deg.size())
                         : param == 1 ? (int)sp.blocks.size() : param == 2 ? (int)sp.chunk.size()
                         : param == 3 ? (int)sp.span.size() : param == 4 ? (int)sp.conc.size()
                         : param == 5 ? (int)sp.fill.size() : (int)sp.bigmax.size();
            for (int i = 0; i < nv; ++i) {
                arb_count_opts o = cur;
                if (param == 0) {
                    if (learned) o.split_min_cost = sp.split_cost[i];
                    else o.split_min_degree = sp.split_deg[i];
                } else if (param == 1) o.persist_blocks_per_cu = sp.blocks[i];
                else if (param == 2) o.chunk_small = sp.chunk[i];
                else if (param == 3) o.bitmap_max_span = sp.span[i];
                else if (param == 4) o.concurrent_tiers = sp.conc[i];
                else if (param == 5) o.tier_fill = sp.fill[i];
                else o.big_max_degree = sp.bigmax[i];
                if (memcmp(&o, &cur, sizeof(o)) == 0) continue;
                float ms = 0.f;
                if ((rc = measure(o, &ms))) goto out;
                if (ms < cur_ms) { cur = o; cur_ms = ms; }
            }
        }
    }
    *opts = cur;
    if (best_ms) *best_ms = cur_ms;
out:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return fail(rc);
}
