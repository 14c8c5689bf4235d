// Low out-degree orientation on the GPU (Sec. 3.1 of Shi, Dhulipala, Shun; appendix Alg. 4
// with the threshold (2+eps) x the average degree of the vertices still present) and
// directing of the CSR into rank space (Sec. 3.1, last paragraph).
//
// Per round r (all on the device, no host round trip, so the sequence can be captured):
//   k_peel_reduce     c_r = #present, S_r = sum of present degrees
//   k_peel_threshold  T_r = floor(((2+eps) * S_r) / c_r) in IEEE double
//   k_peel_mark       present v with deg <= T_r: round = r, deg_at_peel = deg (start of round)
//   k_peel_decrement  each vertex removed in round r lowers each still-present neighbour
//                     (push), or each vertex still present counts its neighbours removed
//                     in round r (pull): whichever walks fewer arcs, chosen on the device
//                     from the arc totals k_peel_mark adds up; both leave the same degrees
// A round with c_r = 0 does nothing, so the host enqueues the proven maximum number of
// rounds, ceil(log_{2+eps} n): every round leaves fewer than c_r/(2+eps) vertices.
#include <math.h>

#include "common.h"

namespace arb {

constexpr int32_t kPresent = -1;
constexpr int kDegBits = 26;   // degree at removal packed below the round in the sort key

enum : int32_t {
    kErrOffsets = 1, kErrRange = 2, kErrSelf = 4, kErrOrder = 8, kErrAsym = 16,
    kErrDegree = 32, kErrRowLong = 64, kErrLeft = 128, kErrBatch = 256
};

// rows of at most this many entries are walked by a group of 16 lanes, longer ones by a
// whole wave
constexpr int kGroupRow = 64;
static_assert(kGroupRow <= 4 * 16, "a short row is four loads per lane of its 16-lane group");

// ------------------------------------------------------------------ validation

// One wave per vertex: offsets monotone, ids in range, no self-loop, strictly ascending
// rows, and every entry u of row v has v in row u (binary search).
__global__ void k_validate(int64_t n, const int64_t *off, const int32_t *idx, int64_t nnz, int32_t *err) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int32_t bad = 0;
    for (int64_t v = wave; v < n; v += nwaves) {
        int64_t s = off[v], e = off[v + 1];
        if (e < s || s < 0 || e > nnz) { bad |= kErrOffsets; continue; }
        for (int64_t p = s + lane; p < e; p += 64) {
            int32_t u = idx[p];
            if (u < 0 || u >= n) { bad |= kErrRange; continue; }
            if (u == v) bad |= kErrSelf;
            if (p > s && idx[p - 1] >= u) bad |= kErrOrder;
            int64_t lo = off[u], hi = off[u + 1];
            if (hi < lo || lo < 0 || hi > nnz) { bad |= kErrOffsets; continue; }
            while (lo < hi) {
                int64_t mid = lo + ((hi - lo) >> 1);
                if (idx[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo >= off[u + 1] || idx[lo] != v) bad |= kErrAsym;
        }
    }
    if (bad) atomicOr(err, bad);
}

__global__ void k_check_offsets_ends(int64_t n, const int64_t *off, int64_t nnz, int32_t *err) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        if (off[0] != 0 || off[n] != nnz) atomicOr(err, (int32_t)kErrOffsets);
}

// ------------------------------------------------------------------ peel rounds

__global__ void k_orient_init(int64_t n, const int64_t *off, int32_t *deg, int32_t *rnd, int32_t *err) {
    int32_t bad = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        int64_t d = off[v + 1] - off[v];
        if (d >= (int64_t(1) << kDegBits)) bad = kErrDegree;
        deg[v] = (int32_t)d;
        rnd[v] = kPresent;
    }
    if (bad) atomicOr(err, bad);
}

// rs[2r] = number present at the start of round r, rs[2r+1] = sum of their degrees.
__global__ void k_peel_reduce(int64_t n, const int32_t *deg, const int32_t *rnd, int r, int64_t *rs) {
    if (r > 0 && rs[2 * (r - 1)] == 0) return;          // graph already empty
    __shared__ int64_t sc[4], ss[4];
    int64_t c = 0, s = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (rnd[v] == kPresent) { c += 1; s += deg[v]; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_down(c, off, 64);
        s += __shfl_down(s, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sc[wid] = c; ss[wid] = s; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tc = 0, ts = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { tc += sc[w]; ts += ss[w]; }
        if (tc) {
            atomicAdd((unsigned long long *)&rs[2 * r], (unsigned long long)tc);
            atomicAdd((unsigned long long *)&rs[2 * r + 1], (unsigned long long)ts);
        }
    }
}

// thr[r] = T_r, or -1 when nothing is present.  stats[0] counts the rounds that peeled.
__global__ void k_peel_threshold(int r, double eps, const int64_t *rs, int64_t *thr, int64_t *stats) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t c = rs[2 * r], S = rs[2 * r + 1];
    if (c == 0) { thr[r] = -1; return; }
    double num = (2.0 + eps) * (double)S;     // product, then quotient: no contraction
    double t = num / (double)c;
    int64_t T = (int64_t)floor(t);
    thr[r] = T;
    if (stats) {
        stats[0] = r + 1;
        if (r < ARB_MAX_ROUNDS) stats[2 + r] = T;
    }
}

// arcs[2r] += row lengths of the vertices removed in round r, arcs[2r+1] += those of the
// vertices still present after it (the arcs a push or a pull decrement would walk)
__global__ void k_peel_mark(int64_t n, const int64_t *off, const int32_t *deg, int32_t *rnd, int32_t *dap, int r,
                            const int64_t *thr, int64_t *arcs) {
    int64_t T = thr[r];
    if (T < 0) return;
    __shared__ int64_t sa[4], sb[4];
    int64_t out = 0, stay = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (rnd[v] == kPresent) {
            const int64_t len = off[v + 1] - off[v];
            if ((int64_t)deg[v] <= T) {
                rnd[v] = r;
                dap[v] = deg[v];
                out += len;
            } else {
                stay += len;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        out += __shfl_down(out, o, 64);
        stay += __shfl_down(stay, o, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sa[wid] = out; sb[wid] = stay; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t to = 0, ts = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { to += sa[w]; ts += sb[w]; }
        if (to) atomicAdd((unsigned long long *)&arcs[2 * r], (unsigned long long)to);
        if (ts) atomicAdd((unsigned long long *)&arcs[2 * r + 1], (unsigned long long)ts);
    }
}

// true when round r's decrement is cheaper pulled: the vertices still present have fewer
// arcs than the vertices removed (null arcs: always push)
__device__ __forceinline__ bool peel_pulls(const int64_t *arcs) {
    return arcs != nullptr && arcs[1] < arcs[0];
}

// Vertices are taken by groups of 16 lanes (four per wave); a vertex removed in round r
// lowers each neighbour still present by one, its row walked by its group when it has at
// most kGroupRow entries, else by the whole wave after the groups' short rows.
// act[0] < 0: nothing was present at the start of round r (the round is a no-op).
// arcs (this round's pair of arc totals, or null): the push runs unless peel_pulls says
// the pull is cheaper.  A short row's up to four arcs per lane are loaded side by side.
__global__ void k_peel_decrement(int64_t n, const int64_t *off, const int32_t *idx, int32_t *deg,
                                 const int32_t *rnd, int r, const int64_t *act, const int64_t *arcs) {
    if (act[0] < 0 || peel_pulls(arcs)) return;
    const int lane = threadIdx.x & 63, sl = lane & 15;
    int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) >> 4;
    for (; grp - (lane >> 4) < n; grp += ngrp) {      // while the wave's first group has a vertex
        int64_t b = 0, e = 0;
        bool heavy = false;
        if (grp < n && rnd[grp] == r) {
            b = off[grp];
            e = off[grp + 1];
            heavy = e - b > kGroupRow;
            if (!heavy && e > b) {
                int32_t u[4], ru[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = idx[b + sl + 16 * q < e ? b + sl + 16 * q : b];
#pragma unroll
                for (int q = 0; q < 4; ++q) ru[q] = rnd[u[q]];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (b + sl + 16 * q < e && ru[q] == kPresent) atomicSub(&deg[u[q]], 1);
            }
        }
        uint64_t hm = __ballot(heavy && sl == 0);
        while (hm) {
            const int src = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            const int64_t hb = __shfl(b, src, 64), he = __shfl(e, src, 64);
            for (int64_t p0 = hb + lane; p0 < he; p0 += 256) {     // four loads in flight per lane
                int32_t u[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = p0 + 64 * q < he ? idx[p0 + 64 * q] : -1;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (u[q] >= 0 && rnd[u[q]] == kPresent) atomicSub(&deg[u[q]], 1);
            }
        }
    }
}

// Pull form of round r's decrement: every vertex still present lowers its own degree by
// the number of its neighbours removed in round r (the same degrees the push leaves).
// Runs only when peel_pulls(arcs); short rows by groups of 16 lanes, long ones by a wave.
__global__ void k_peel_pull(int64_t n, const int64_t *off, const int32_t *idx, int32_t *deg, const int32_t *rnd,
                            int r, const int64_t *act, const int64_t *arcs) {
    if (act[0] < 0 || !peel_pulls(arcs)) return;
    const int lane = threadIdx.x & 63, sl = lane & 15;
    int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) >> 4;
    for (; grp - (lane >> 4) < n; grp += ngrp) {      // while the wave's first group has a vertex
        int64_t b = 0, e = 0;
        bool light = false, heavy = false;
        if (grp < n && rnd[grp] == kPresent) {
            b = off[grp];
            e = off[grp + 1];
            heavy = e - b > kGroupRow;
            light = !heavy && e > b;
        }
        int32_t c = 0;
        if (light) {
            int32_t u[4], ru[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) u[q] = idx[b + sl + 16 * q < e ? b + sl + 16 * q : b];
#pragma unroll
            for (int q = 0; q < 4; ++q) ru[q] = rnd[u[q]];
#pragma unroll
            for (int q = 0; q < 4; ++q) c += (b + sl + 16 * q < e && ru[q] == r) ? 1 : 0;
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) c += __shfl_xor(c, o, 16);
        if (light && sl == 0 && c) deg[grp] -= c;
        uint64_t hm = __ballot(heavy && sl == 0);
        while (hm) {
            const int src = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            const int64_t hb = __shfl(b, src, 64), he = __shfl(e, src, 64);
            const int64_t hv = __shfl(grp, src, 64);
            int32_t hc = 0;
            for (int64_t p0 = hb + lane; p0 < he; p0 += 256) {     // four loads in flight per lane
                int32_t u[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = p0 + 64 * q < he ? idx[p0 + 64 * q] : -1;
#pragma unroll
                for (int q = 0; q < 4; ++q) hc += (u[q] >= 0 && rnd[u[q]] == r) ? 1 : 0;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) hc += __shfl_xor(hc, o, 64);
            if (lane == 0 && hc) deg[hv] -= hc;
        }
    }
}

__global__ void k_count_left(int64_t n, const int32_t *rnd, int32_t *err) {
    int32_t bad = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        if (rnd[v] == kPresent) bad = kErrLeft;
    if (bad) atomicOr(err, bad);
}

__global__ void k_copy_rounds(int64_t n, const int32_t *src, int32_t *dst) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        dst[v] = src[v];
}

// ------------------------------------------------------------------ batches
// A disjoint union of G graphs, graph g on the vertex range vo[g] .. vo[g+1]-1, is peeled
// with each graph's own n_r, S_r and T_r, so that every graph is oriented exactly as on
// its own; ranks stay inside each graph's range.

// gid was zero-filled first; ranges are clamped to [0, n), so malformed offsets (caught
// by the range check when validating) cannot write outside gid or leave an id >= G
__global__ void k_gid_fill(int64_t n, int64_t G, const int64_t *vo, int32_t *gid) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t g = wave; g < G; g += nwaves) {
        const int64_t lo = vo[g] < 0 ? 0 : vo[g], hi = vo[g + 1] > n ? n : vo[g + 1];
        for (int64_t v = lo + lane; v < hi; v += 64) gid[v] = (int32_t)g;
    }
}

// vertex ranges: vo[0] = 0, vo[G] = n, non-decreasing
__global__ void k_check_ranges(int64_t n, int64_t G, const int64_t *vo, int32_t *err) {
    int32_t bad = 0;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x)
        if (vo[g + 1] < vo[g]) bad = kErrBatch;
    if (blockIdx.x == 0 && threadIdx.x == 0 && (vo[0] != 0 || vo[G] != n)) bad = kErrBatch;
    if (bad) atomicOr(err, bad);
}

// every edge stays inside its graph
__global__ void k_check_batch_edges(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *gid,
                                    int32_t *err) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int32_t bad = 0;
    for (int64_t v = wave; v < n; v += nwaves)
        for (int64_t p = off[v] + lane; p < off[v + 1]; p += 64)
            if (gid[idx[p]] != gid[v]) bad = kErrBatch;
    if (bad) atomicOr(err, bad);
}

// rs[2g], rs[2g+1] = number present in graph g and the sum of their degrees (rs zeroed
// before each round).  A wave whose 64 vertices share one graph adds its sums once.
__global__ void k_bpeel_reduce(int64_t n, const int32_t *deg, const int32_t *rnd, const int32_t *gid, int64_t *rs) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
        const int64_t v = base + lane;
        const bool in = v < n;
        const bool present = in && rnd[v] == kPresent;
        int64_t c = present ? 1 : 0, sd = present ? deg[v] : 0;
        const int32_t g = in ? gid[v] : -1;
        const int32_t g0 = __shfl(g, 0, 64);
        if (__all(!in || g == g0)) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                c += __shfl_xor(c, o, 64);
                sd += __shfl_xor(sd, o, 64);
            }
            if (lane == 0 && c) {
                atomicAdd((unsigned long long *)&rs[2 * g0], (unsigned long long)c);
                atomicAdd((unsigned long long *)&rs[2 * g0 + 1], (unsigned long long)sd);
            }
        } else if (present) {
            atomicAdd((unsigned long long *)&rs[2 * g], 1ull);
            atomicAdd((unsigned long long *)&rs[2 * g + 1], (unsigned long long)sd);
        }
    }
}

// thr[g] = T_r of graph g (-1 when it is empty); any[r] = the largest of them, so that
// rounds with nothing left skip their work; stats[0] = rounds that peeled.
__global__ void k_bpeel_threshold(int64_t G, int r, double eps, const int64_t *rs, int64_t *thr, int64_t *any,
                                  int64_t *stats) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = rs[2 * g], S = rs[2 * g + 1];
        if (c == 0) {
            thr[g] = -1;
            continue;
        }
        double num = (2.0 + eps) * (double)S;
        double t = num / (double)c;
        const int64_t T = (int64_t)floor(t);
        thr[g] = T;
        atomicMax((long long *)&any[r], (long long)T);
        if (stats) atomicMax((long long *)&stats[0], (long long)(r + 1));
    }
}

__global__ void k_bpeel_mark(int64_t n, const int32_t *deg, int32_t *rnd, int32_t *dap, const int32_t *gid, int r,
                             const int64_t *thr, const int64_t *any) {
    if (any[r] < 0) return;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (rnd[v] == kPresent && (int64_t)deg[v] <= thr[gid[v]]) {
            rnd[v] = r;
            dap[v] = deg[v];
        }
    }
}

// second sort key: the graph of the vertex at each position
__global__ void k_gid_keys(int64_t n, const int32_t *vals, const int32_t *gid, uint32_t *keys) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        keys[p] = (uint32_t)gid[vals[p]];
}

// ------------------------------------------------------------------ other orderings
// (the orientations the paper compares, Sec. 3.1, 5: degree ordering, Goodrich-Pszona
// (Alg. 3), k-core ordering); all end in the same (round, degree at removal, id) ranking

// degree ordering: every vertex in round 0 with its degree, so the rank orders by (degree, id)
__global__ void k_all_round0(int64_t n, const int32_t *deg, int32_t *rnd, int32_t *dap) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        rnd[v] = 0;
        dap[v] = deg[v];
    }
}

__global__ void k_present_flags(int64_t n, const int32_t *rnd, int64_t *flag) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flag[v] = rnd[v] == kPresent ? 1 : 0;
}

// present vertices in id order: keys = degree, vals = id
__global__ void k_present_compact(int64_t n, const int32_t *rnd, const int32_t *deg, const int64_t *pos,
                                  uint32_t *keys, int32_t *vals) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (rnd[v] == kPresent) {
            keys[pos[v]] = (uint32_t)deg[v];
            vals[pos[v]] = (int32_t)v;
        }
}

// Goodrich-Pszona round r: the s present vertices of lowest (degree, id) are removed
__global__ void k_gp_mark(int64_t s, const int32_t *vals, const int32_t *deg, int32_t *rnd, int32_t *dap, int r) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = vals[i];
        rnd[v] = r;
        dap[v] = deg[v];
    }
}

// k-core round: st[0] = least degree present, st[1] = number present (st reset by the
// threshold kernel)
__global__ void k_kcore_reduce(int64_t n, const int32_t *deg, const int32_t *rnd, int64_t *st) {
    int64_t c = 0, mn = INT64_MAX;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (rnd[v] == kPresent) {
            c += 1;
            mn = deg[v] < mn ? deg[v] : mn;
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o, 64);
        const int64_t y = __shfl_xor(mn, o, 64);
        mn = y < mn ? y : mn;
    }
    if ((threadIdx.x & 63) == 0 && c) {
        atomicAdd((unsigned long long *)&st[1], (unsigned long long)c);
        atomicMin((long long *)&st[0], (long long)mn);
    }
}

// T[0] = max(T[0], least degree present), or -1 once nothing is present; st[2] counts
// the rounds that peeled
__global__ void k_kcore_threshold(int64_t *st, int64_t *T) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (st[1] == 0) {
        T[0] = -1;
    } else {
        T[0] = st[0] > T[0] ? st[0] : T[0];
        st[2] += 1;
    }
    st[0] = INT64_MAX;
    st[1] = 0;
}

__global__ void k_kcore_mark(int64_t n, const int32_t *deg, int32_t *rnd, int32_t *dap, int r, const int64_t *T) {
    const int64_t t = T[0];
    if (t < 0) return;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (rnd[v] == kPresent && (int64_t)deg[v] <= t) {
            rnd[v] = r;
            dap[v] = deg[v];
        }
}

// second rank key when rounds do not fit beside the degree: the round of each position
__global__ void k_round_keys(int64_t n, const int32_t *vals, const int32_t *rnd, uint32_t *keys) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        keys[p] = (uint32_t)rnd[vals[p]];
}

__global__ void k_set_stat(int64_t *stats, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) stats[0] = v;
}

// ------------------------------------------------------------------ rank

__global__ void k_rank_keys(int64_t n, const int32_t *rnd, const int32_t *dap, uint32_t *keys, int32_t *vals) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        keys[v] = ((rnd ? (uint32_t)rnd[v] : 0u) << kDegBits) | (uint32_t)dap[v];
        vals[v] = (int32_t)v;
    }
}

__global__ void k_rank_scatter(int64_t n, const int32_t *inv, int32_t *rank) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        rank[inv[p]] = (int32_t)p;
}

// ------------------------------------------------------------------ directing

// Vertices of degree <= 64 are taken by groups of 16 lanes (four per wave): most rows are
// short, and a whole wave per row would leave most lanes idle and only one row's chain of
// dependent loads per wave in flight.  A longer row is taken by the whole wave after its
// groups' short rows.
// Number of neighbours of higher rank, stored at the vertex's rank.
__global__ void k_dir_count(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *rank,
                            int64_t *outdeg, int32_t *arc_rank) {
    const int lane = threadIdx.x & 63, sl = lane & 15;
    int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) >> 4;
    for (; grp - (lane >> 4) < n; grp += ngrp) {      // while the wave's first group has a vertex
        int32_t rv = 0;
        int64_t b = 0, e = 0, c = 0;
        bool light = false, heavy = false;
        if (grp < n) {
            b = off[grp];
            e = off[grp + 1];
            rv = rank[grp];
            light = e - b <= kGroupRow;
            heavy = !light;
        }
        if (light && e > b) {          // up to four arcs per lane, their loads side by side
            int32_t u[4], ru[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) u[q] = idx[b + sl + 16 * q < e ? b + sl + 16 * q : b];
#pragma unroll
            for (int q = 0; q < 4; ++q) ru[q] = rank[u[q]];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t p = b + sl + 16 * q;
                if (p < e) {
                    arc_rank[p] = ru[q];
                    c += ru[q] > rv;
                }
            }
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) c += __shfl_xor(c, o, 16);
        if (light && sl == 0) outdeg[rv] = c;
        uint64_t hm = __ballot(heavy && sl == 0);
        while (hm) {
            const int src = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            const int64_t hb = __shfl(b, src, 64), he = __shfl(e, src, 64);
            const int32_t hr = __shfl(rv, src, 64);
            int64_t hc = 0;
            for (int64_t p0 = hb + lane; p0 < he; p0 += 256) {     // four loads in flight per lane
                int32_t u[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = p0 + 64 * q < he ? idx[p0 + 64 * q] : -1;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (u[q] >= 0) {
                        const int32_t r = rank[u[q]];
                        arc_rank[p0 + 64 * q] = r;
                        hc += r > hr;
                    }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) hc += __shfl_xor(hc, o, 64);
            if (lane == 0) outdeg[hr] = hc;
        }
    }
}

// Write the higher-ranked neighbours' ranks into the row of the vertex's rank: sorted for
// input rows of at most kGroupRow entries, in the input row's order for longer ones
// (sorted afterwards).
__global__ void k_dir_fill(int64_t n, const int64_t *off, const int32_t *arc_rank, const int32_t *rank,
                           const int64_t *ooff, int32_t *oidx) {
    const int lane = threadIdx.x & 63, sl = lane & 15;
    const uint64_t below = lanes_below_mask();
    int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) >> 4;
    for (; grp - (lane >> 4) < n; grp += ngrp) {      // while the wave's first group has a vertex
        int32_t rv = 0;
        int64_t w = 0, b = 0, len = 0;
        bool heavy = false;
        if (grp < n) {
            b = off[grp];
            len = off[grp + 1] - b;
            rv = rank[grp];
            w = ooff[rv];
            heavy = len > kGroupRow;
        }
        // short rows (at most four entries per lane): each kept entry goes straight to its
        // sorted place, the number of the row's kept entries below it (entries are
        // distinct ranks; a dropped entry reads as INT32_MAX and counts for none).  The
        // wave takes as many of the four slots as its longest short row needs
        const int64_t ll = heavy ? 0 : len;
        int64_t lmax = ll;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int64_t y = __shfl_xor(lmax, o, 64);
            lmax = y > lmax ? y : lmax;
        }
        int32_t v[4];
        int pos[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t ru = (16 * q + sl < ll) ? arc_rank[b + 16 * q + sl] : -1;
            v[q] = ru > rv ? ru : INT32_MAX;
            pos[q] = 0;
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            if (16 * qq >= lmax) break;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int32_t y = __shfl(v[qq], j, 16);
#pragma unroll
                for (int q = 0; q < 4; ++q) pos[q] += y < v[q] ? 1 : 0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (v[q] != INT32_MAX) oidx[w + pos[q]] = v[q];
        uint64_t hm = __ballot(heavy && sl == 0);
        while (hm) {
            const int src = __ffsll((unsigned long long)hm) - 1;
            hm &= hm - 1;
            const int64_t hb = __shfl(b, src, 64), he = hb + __shfl(len, src, 64);
            const int32_t hr = __shfl(rv, src, 64);
            int64_t hw = __shfl(w, src, 64);
            for (int64_t q0 = hb; q0 < he; q0 += 256) {            // four loads in flight per lane
                int32_t ru[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t p = q0 + 64 * q + lane;
                    ru[q] = p < he ? arc_rank[p] : -1;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool keep = ru[q] > hr;
                    const uint64_t m = __ballot(keep);
                    if (keep) oidx[hw + __popcll(m & below)] = ru[q];
                    hw += __popcll(m);
                }
            }
        }
    }
}

constexpr int kMidRow = 2048;

// Rows of at most 16 entries: one group of 16 lanes per row, each lane's destination is
// the number of smaller entries (entries are distinct); rows of 17..64 entries: the same
// by the whole wave after its groups' short rows, unless the row is already sorted.  Longer rows are listed for the kernels
// below (mid: 65..kMidRow entries, big: longer; cnt[0], cnt[1] entries), with one global
// atomic per block and round.  Also reduces the largest row length.
__global__ void __launch_bounds__(256) k_row_sort_small(int64_t n, const int64_t *ooff, int32_t *oidx,
                                                        int64_t *stats, int32_t *mid, int32_t *big, int32_t *cnt) {
    __shared__ int32_t lcnt[2], lbase[2];
    const int lane = threadIdx.x & 63, sl = lane & 15;
    int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) >> 4;
    const int64_t first = ((int64_t)blockIdx.x * blockDim.x) >> 4;
    int64_t dmax = 0;
    for (int64_t base = first; base < n; base += ngrp, grp += ngrp) {   // uniform over the block
        if (threadIdx.x < 2) lcnt[threadIdx.x] = 0;
        __syncthreads();
        int d = 0;
        int64_t s = 0;
        int slot = -1, which = 0;
        if (grp < n) {
            s = ooff[grp];
            d = (int)min<int64_t>(ooff[grp + 1] - s, 0x7fffffff);
            dmax = d > dmax ? d : dmax;
            if (d > 64 && sl == 0) {
                which = d <= kMidRow ? 0 : 1;
                slot = atomicAdd(&lcnt[which], 1);
            }
        }
        const bool mine = d >= 2 && d <= 16;
        const int32_t x = (mine && sl < d) ? oidx[s + sl] : 0x7fffffff;
        int pos = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) pos += __shfl(x, j, 16) < x;
        if (mine && sl < d) oidx[s + pos] = x;
        uint64_t wm = __ballot(d > 16 && d <= 64 && sl == 0);
        while (wm) {
            const int src = __ffsll((unsigned long long)wm) - 1;
            wm &= wm - 1;
            const int64_t ws = __shfl(s, src, 64);
            const int wd = __shfl(d, src, 64);
            const int32_t y = lane < wd ? oidx[ws + lane] : 0x7fffffff;
            const int32_t ynext = __shfl_down(y, 1, 64);
            if (__ballot(lane + 1 < wd && ynext < y) == 0) continue;     // sorted by the fill
            int wpos = 0;
            for (int j = 0; j < wd; ++j) wpos += __shfl(y, j, 64) < y;
            if (lane < wd) oidx[ws + wpos] = y;
        }
        __syncthreads();
        if (threadIdx.x < 2 && lcnt[threadIdx.x] > 0)
            lbase[threadIdx.x] = atomicAdd(&cnt[threadIdx.x], lcnt[threadIdx.x]);
        __syncthreads();
        if (slot >= 0) (which ? big : mid)[lbase[which] + slot] = (int32_t)grp;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t y = __shfl_xor(dmax, o, 64);
        dmax = y > dmax ? y : dmax;
    }
    if (stats && lane == 0 && dmax > 0) atomicMax((unsigned long long *)&stats[1], (unsigned long long)dmax);
}

// Ascending bitonic sort of buf[0 .. p2) in LDS by the whole block (p2 a power of two).
__device__ void block_bitonic(int32_t *buf, int p2) {
    for (int size = 2; size <= p2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < (p2 >> 1); i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int32_t a = buf[lo], b = buf[hi];
                if ((a > b) == up) {
                    buf[lo] = b;
                    buf[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

// One block per listed row (rows[0 .. *cnt)), bitonic sort in LDS padded to a power of
// two: rows of 65..kMidRow entries in a static buffer, longer ones (up to
// ARB_MAX_ROW_SORT) in dynamic LDS.
template <bool BIG>
__global__ void __launch_bounds__(256) k_row_sort_lds(const int32_t *rows, const int32_t *cnt, const int64_t *ooff,
                                                      int32_t *oidx, int32_t *err) {
    __shared__ int32_t mid_buf[BIG ? 1 : kMidRow];
    extern __shared__ int32_t big_buf[];
    int32_t *buf = BIG ? big_buf : mid_buf;
    const int32_t nl = *cnt;
    for (int32_t l = blockIdx.x; l < nl; l += gridDim.x) {
        const int32_t r = rows[l];
        const int64_t s = ooff[r];
        const int64_t d64 = ooff[r + 1] - s;
        if (d64 > ARB_MAX_ROW_SORT) {
            if (threadIdx.x == 0) atomicOr(err, (int32_t)kErrRowLong);
            continue;
        }
        const int d = (int)d64;
        int p2 = 128;
        while (p2 < d) p2 <<= 1;
        for (int i = threadIdx.x; i < p2; i += blockDim.x) buf[i] = i < d ? oidx[s + i] : 0x7fffffff;
        __syncthreads();
        block_bitonic(buf, p2);
        for (int i = threadIdx.x; i < d; i += blockDim.x) oidx[s + i] = buf[i];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side

static int max_rounds(int64_t n, double eps) {
    // each round leaves fewer than c/(2+eps) vertices: c_{r+1} <= ceil(c_r/(2+eps)) - 1
    double b = 2.0 + eps;
    int64_t c = n;
    int r = 0;
    while (c > 0) {
        double q = (double)c / b;
        int64_t nc = (int64_t)ceil(q) - 1;
        if (nc >= c) nc = c - 1;
        c = nc < 0 ? 0 : nc;
        ++r;
    }
    return r < 1 ? 1 : r;
}

struct OrientWs {
    int32_t *deg, *rnd, *dap, *err;
    uint32_t *keys, *keys_alt;
    int32_t *vals, *vals_alt;
    int64_t *rs, *thr, *outdeg;
    int64_t *arcs;           // per round: arcs of the removed and of the remaining vertices
    int32_t *arc_rank;       // rank of each arc's head, written by the counting pass of the
                             // directing and read by the filling pass (one gather per arc)
    void *scan_ws, *radix_ws;
    int32_t *gid;            // batches: graph of each vertex
    int64_t *rs_g, *thr_g;   // batches: per-graph round sums and thresholds
};

static size_t carve_orient(Carver &c, int64_t n, int64_t nnz, OrientWs *w, int64_t G = 0) {
    int64_t nn = n > 0 ? n : 1;
    if (G > 0) {
        w->gid = c.take<int32_t>(nn);
        w->rs_g = c.take<int64_t>(2 * G);
        w->thr_g = c.take<int64_t>(G);
    } else {
        w->gid = nullptr;
        w->rs_g = w->thr_g = nullptr;
    }
    w->deg = c.take<int32_t>(nn);
    w->rnd = c.take<int32_t>(nn);
    w->dap = c.take<int32_t>(nn);
    w->err = c.take<int32_t>(4);      // [0] error flags, [1], [2] list counters
    w->keys = c.take<uint32_t>(nn);
    w->keys_alt = c.take<uint32_t>(nn);
    w->vals = c.take<int32_t>(nn);
    w->vals_alt = c.take<int32_t>(nn);
    w->rs = c.take<int64_t>(2 * 128);
    w->thr = c.take<int64_t>(128);
    w->arcs = c.take<int64_t>(2 * 128);
    w->outdeg = c.take<int64_t>(nn + 1);
    w->arc_rank = c.take<int32_t>(nnz > 0 ? nnz : 1);
    w->scan_ws = c.take<char>(scan_workspace(nn + 1));
    w->radix_ws = c.take<char>(radix_workspace(nn));
    return c.used;
}

}  // namespace arb

using namespace arb;

extern "C" size_t arb_orient_workspace(int64_t n, int64_t nnz) {
    Carver c(nullptr);
    OrientWs w;
    return carve_orient(c, n, nnz, &w) + 256;
}

static int validate_impl(const arb_csr *g, int32_t *err, hipStream_t s) {
    ARB_CHECK_LAUNCH();
    int rc = fill_i32(err, 0, 1, s);
    if (rc) return rc;
    k_check_offsets_ends<<<1, 64, 0, s>>>(g->n, g->offsets, g->nnz, err);
    ARB_CHECK_LAUNCH();
    if (g->n > 0) {
        k_validate<<<grid_for(g->n * 64, 256, 8192), 256, 0, s>>>(g->n, g->offsets, g->indices, g->nnz, err);
        ARB_CHECK_LAUNCH();
    }
    int32_t h = 0;
    ARB_HIP(hipMemcpyAsync(&h, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ARB_HIP(hipStreamSynchronize(s));
    return h ? ARB_EGRAPH : ARB_OK;
}

extern "C" int arb_validate(const arb_csr *g, void *ws, size_t ws_bytes, void *stream) {
    int rc = ARB_OK;
    if (!g || !ws || g->n < 0 || g->nnz < 0 || (g->n > 0 && !g->offsets) || (g->nnz > 0 && !g->indices))
        rc = ARB_EINVAL;
    else if (ws_bytes < 512)
        rc = ARB_EWORKSPACE;
    else
        rc = validate_impl(g, static_cast<int32_t *>(ws), as_stream(stream));
    set_error(rc);
    return rc;
}

struct BatchDesc {
    const int64_t *vo;       // device, G + 1 vertex offsets
    int64_t G;
    int64_t max_n;           // largest graph (bounds the number of rounds)
};

static int orient_impl(const arb_csr *g, double eps, int validate, arb_ocsr *out, int32_t *rank,
                       int32_t *round_out, int32_t *dap_out, int64_t *stats, void *ws, size_t ws_bytes,
                       hipStream_t s, const BatchDesc *b, int method = ARB_ORIENT_PEEL) {
    if (!g || !out || !rank || !ws) return ARB_EINVAL;
    if (!(eps >= 0.0 && eps <= 64.0)) return ARB_EINVAL;
    if (method < ARB_ORIENT_PEEL || method > ARB_ORIENT_KCORE || (b && method != ARB_ORIENT_PEEL)) return ARB_EINVAL;
    if (method == ARB_ORIENT_GOODRICH_PSZONA && !(eps > 0.0)) return ARB_EINVAL;
    const int64_t n = g->n, nnz = g->nnz;
    if (n < 0 || nnz < 0 || (nnz & 1)) return ARB_EINVAL;
    if (n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 40)) return ARB_ELIMIT;
    if (!g->offsets || (nnz > 0 && !g->indices) || !out->offsets || (nnz > 0 && !out->indices))
        return ARB_EINVAL;
    if (out->n != n || out->m != nnz / 2) return ARB_EINVAL;
    const int64_t G = b ? b->G : 0;
    if (b && (G < 1 || G > n + 1 || !b->vo || b->max_n < 0 || b->max_n > n)) return ARB_EINVAL;
    const size_t need = b ? arb_orient_batch_workspace(n, nnz, G) : arb_orient_workspace(n, nnz);
    if (ws_bytes < need) return ARB_EWORKSPACE;

    Carver cv(ws);
    OrientWs w;
    carve_orient(cv, n, nnz, &w, G);
    int rc;
    if (validate) {
        rc = validate_impl(g, w.err, s);
        if (rc) return rc;
    }
    if ((rc = fill_i32(w.err, 0, 1, s))) return rc;
    if ((rc = fill_i64(w.rs, 0, 2 * 128, s))) return rc;
    if ((rc = fill_i64(w.thr, -1, 128, s))) return rc;
    if ((rc = fill_i64(w.arcs, 0, 2 * 128, s))) return rc;
    if (stats && (rc = fill_i64(stats, 0, 2 + ARB_MAX_ROUNDS, s))) return rc;
    int32_t *dap = dap_out ? dap_out : w.dap;
    int32_t *rnd = w.rnd;

    const unsigned gb = grid_for(n, 256, 2048);
    const unsigned gw = grid_for(n, 256, 4096);
    if (b) {
        k_check_ranges<<<grid_for(G, 256, 1024), 256, 0, s>>>(n, G, b->vo, w.err);
        if ((rc = fill_i32(w.gid, 0, n > 0 ? n : 1, s))) return rc;
        k_gid_fill<<<grid_for(G * 64, 256, 4096), 256, 0, s>>>(n, G, b->vo, w.gid);
        if (hipGetLastError() != hipSuccess) return ARB_EHIP;
        if (validate) {
            if (n > 0)
                k_check_batch_edges<<<grid_for(n * 64, 256, 8192), 256, 0, s>>>(n, g->offsets, g->indices, w.gid,
                                                                               w.err);
            int32_t h = 0;
            if (hipMemcpyAsync(&h, w.err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return ARB_EHIP;
            if (h) return ARB_EGRAPH;
        }
    }
    k_orient_init<<<gb, 256, 0, s>>>(n, g->offsets, w.deg, rnd, w.err);
    if (hipGetLastError() != hipSuccess) return ARB_EHIP;
    int64_t R = 0;                                  // rounds the rank key must hold
    if (method == ARB_ORIENT_PEEL) {
        R = max_rounds(b ? b->max_n : n, eps);
        if (R > 120) return ARB_ELIMIT;
        for (int r = 0; r < R; ++r) {
            if (b) {
                if ((rc = fill_i64(w.rs_g, 0, 2 * G, s))) return rc;
                k_bpeel_reduce<<<gw, 256, 0, s>>>(n, w.deg, rnd, w.gid, w.rs_g);
                k_bpeel_threshold<<<grid_for(G, 256, 1024), 256, 0, s>>>(G, r, eps, w.rs_g, w.thr_g, w.thr, stats);
                k_bpeel_mark<<<gb, 256, 0, s>>>(n, w.deg, rnd, dap, w.gid, r, w.thr_g, w.thr);
            } else {
                k_peel_reduce<<<gb, 256, 0, s>>>(n, w.deg, rnd, r, w.rs);
                k_peel_threshold<<<1, 64, 0, s>>>(r, eps, w.rs, w.thr, stats);
                k_peel_mark<<<gb, 256, 0, s>>>(n, g->offsets, w.deg, rnd, dap, r, w.thr, w.arcs);
            }
            const int64_t *arcs = b ? nullptr : w.arcs + 2 * r;
            k_peel_decrement<<<gw, 256, 0, s>>>(n, g->offsets, g->indices, w.deg, rnd, r, w.thr + r, arcs);
            if (!b) k_peel_pull<<<gw, 256, 0, s>>>(n, g->offsets, g->indices, w.deg, rnd, r, w.thr + r, arcs);
        }
    } else if (method == ARB_ORIENT_DEGREE) {
        k_all_round0<<<gb, 256, 0, s>>>(n, w.deg, rnd, dap);
        R = 1;
        if (stats) k_set_stat<<<1, 64, 0, s>>>(stats, n > 0 ? 1 : 0);
    } else if (method == ARB_ORIENT_GOODRICH_PSZONA) {
        // Alg. 3: each round removes the ceil(eps c / (2 + eps)) present vertices of lowest
        // (degree, id), c = number present (host loop: one synchronisation per round)
        int64_t *act = w.rs;                         // >= 0: the decrement runs
        if ((rc = fill_i64(act, 0, 1, s))) return rc;
        int r = 0;
        while (true) {
            k_present_flags<<<gb, 256, 0, s>>>(n, rnd, w.outdeg);
            if ((rc = exclusive_scan_i64(w.outdeg, w.outdeg, n, w.scan_ws, s))) return rc;
            int64_t c = 0;
            ARB_HIP(hipMemcpyAsync(&c, w.outdeg + n, sizeof(c), hipMemcpyDeviceToHost, s));
            ARB_HIP(hipStreamSynchronize(s));
            if (c == 0) break;
            if (r >= (1 << 20)) return ARB_ELIMIT;
            int64_t sr = (int64_t)ceil((eps * (double)c) / (2.0 + eps));
            if (sr < 1) sr = 1;
            if (sr > c) sr = c;
            k_present_compact<<<gb, 256, 0, s>>>(n, rnd, w.deg, w.outdeg, w.keys, w.vals);
            if ((rc = radix_sort_u32(w.keys, w.vals, w.keys_alt, w.vals_alt, c, kDegBits, w.radix_ws, s))) return rc;
            k_gp_mark<<<grid_for(sr, 256, 4096), 256, 0, s>>>(sr, w.vals, w.deg, rnd, dap, r);
            k_peel_decrement<<<gw, 256, 0, s>>>(n, g->offsets, g->indices, w.deg, rnd, r, act, nullptr);
            ++r;
        }
        R = r;
        if (stats) k_set_stat<<<1, 64, 0, s>>>(stats, r);
    } else {
        // k-core ordering: round r removes every present vertex of degree <= T_r,
        // T_r = max(T_{r-1}, least degree present); launched 64 rounds at a time
        int64_t *st = w.rs, *T = w.rs + 4;
        if ((rc = fill_i64(st, INT64_MAX, 1, s)) || (rc = fill_i64(st + 1, 0, 2, s)) || (rc = fill_i64(T, 0, 1, s)))
            return rc;
        int r = 0;
        while (true) {
            for (int i = 0; i < 64; ++i, ++r) {
                k_kcore_reduce<<<gb, 256, 0, s>>>(n, w.deg, rnd, st);
                k_kcore_threshold<<<1, 64, 0, s>>>(st, T);
                k_kcore_mark<<<gb, 256, 0, s>>>(n, w.deg, rnd, dap, r, T);
                k_peel_decrement<<<gw, 256, 0, s>>>(n, g->offsets, g->indices, w.deg, rnd, r, T, nullptr);
            }
            int64_t h[2] = {0, 0};
            ARB_HIP(hipMemcpyAsync(&h[0], T, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            ARB_HIP(hipMemcpyAsync(&h[1], st + 2, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            ARB_HIP(hipStreamSynchronize(s));
            if (h[0] < 0) {
                R = h[1];
                break;
            }
            if (r > n + 64) return ARB_ELIMIT;       // every round with a vertex present removes one
        }
        if (stats) k_set_stat<<<1, 64, 0, s>>>(stats, R);
    }
    k_count_left<<<gb, 256, 0, s>>>(n, rnd, w.err);
    if (hipGetLastError() != hipSuccess) return ARB_EHIP;
    // rank: stable sort of ids by (round, degree at removal); in a batch then stably by
    // graph, which keeps every graph's ranks inside its own vertex range
    int round_bits = 1;
    while ((int64_t(1) << round_bits) <= R) ++round_bits;
    if (kDegBits + round_bits <= 32) {
        k_rank_keys<<<gb, 256, 0, s>>>(n, rnd, dap, w.keys, w.vals);
        if (hipGetLastError() != hipSuccess) return ARB_EHIP;
        if ((rc = radix_sort_u32(w.keys, w.vals, w.keys_alt, w.vals_alt, n, kDegBits + round_bits, w.radix_ws, s)))
            return rc;
    } else {
        // many rounds: by degree at removal first, then stably by round
        k_rank_keys<<<gb, 256, 0, s>>>(n, nullptr, dap, w.keys, w.vals);
        if (hipGetLastError() != hipSuccess) return ARB_EHIP;
        if ((rc = radix_sort_u32(w.keys, w.vals, w.keys_alt, w.vals_alt, n, kDegBits, w.radix_ws, s))) return rc;
        k_round_keys<<<gb, 256, 0, s>>>(n, w.vals, rnd, w.keys);
        if ((rc = radix_sort_u32(w.keys, w.vals, w.keys_alt, w.vals_alt, n, round_bits, w.radix_ws, s))) return rc;
    }
    if (b && G > 1) {
        k_gid_keys<<<gb, 256, 0, s>>>(n, w.vals, w.gid, w.keys);
        if (hipGetLastError() != hipSuccess) return ARB_EHIP;
        int gbits = 1;
        while ((int64_t(1) << gbits) < G) ++gbits;
        if ((rc = radix_sort_u32(w.keys, w.vals, w.keys_alt, w.vals_alt, n, gbits, w.radix_ws, s))) return rc;
    }
    k_rank_scatter<<<gb, 256, 0, s>>>(n, w.vals, rank);
    // directing
    const unsigned g16 = grid_for(n * 16, 256, 8192);
    k_dir_count<<<g16, 256, 0, s>>>(n, g->offsets, g->indices, rank, w.outdeg, w.arc_rank);
    if (hipGetLastError() != hipSuccess) return ARB_EHIP;
    if ((rc = exclusive_scan_i64(w.outdeg, out->offsets, n, w.scan_ws, s))) return rc;
    k_dir_fill<<<g16, 256, 0, s>>>(n, g->offsets, w.arc_rank, rank, out->offsets, out->indices);
    // rows longer than 64 are listed by the small-row sort (the rank-sort buffers are free
    // by now; counters in err[1], err[2])
    int32_t *mid_rows = w.vals_alt, *big_rows = reinterpret_cast<int32_t *>(w.keys_alt), *row_cnt = w.err + 1;
    if ((rc = fill_i32(row_cnt, 0, 2, s))) return rc;
    k_row_sort_small<<<g16, 256, 0, s>>>(n, out->offsets, out->indices, stats, mid_rows, big_rows, row_cnt);
    k_row_sort_lds<false><<<grid_for(n, 1, 8192), 256, 0, s>>>(mid_rows, row_cnt, out->offsets, out->indices, w.err);
    k_row_sort_lds<true><<<grid_for(n, 64, 256), 256, ARB_MAX_ROW_SORT * sizeof(int32_t), s>>>(
        big_rows, row_cnt + 1, out->offsets, out->indices, w.err);
    if (hipGetLastError() != hipSuccess) return ARB_EHIP;
    if (round_out) {
        k_copy_rounds<<<gb, 256, 0, s>>>(n, rnd, round_out);
        if (hipGetLastError() != hipSuccess) return ARB_EHIP;
    }
    if (validate) {
        int32_t h = 0;
        if (hipMemcpyAsync(&h, w.err, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return ARB_EHIP;
        if (h & kErrBatch) return ARB_EGRAPH;
        if (h) return ARB_ELIMIT;
    }
    return ARB_OK;
}

extern "C" size_t arb_orient_batch_workspace(int64_t n, int64_t nnz, int64_t G) {
    Carver c(nullptr);
    OrientWs w;
    return carve_orient(c, n, nnz, &w, G > 0 ? G : 1) + 256;
}

extern "C" int arb_orient(const arb_csr *g, double eps, int validate, arb_ocsr *out, int32_t *rank,
                          int32_t *round_out, int32_t *dap_out, int64_t *stats, void *ws, size_t ws_bytes,
                          void *stream) {
    const int rc = orient_impl(g, eps, validate, out, rank, round_out, dap_out, stats, ws, ws_bytes,
                               as_stream(stream), nullptr);
    set_error(rc);
    return rc;
}

extern "C" int arb_orient_method(const arb_csr *g, int method, double eps, int validate, arb_ocsr *out, int32_t *rank,
                                 int32_t *round_out, int32_t *dap_out, int64_t *stats, void *ws, size_t ws_bytes,
                                 void *stream) {
    const int rc = orient_impl(g, eps, validate, out, rank, round_out, dap_out, stats, ws, ws_bytes,
                               as_stream(stream), nullptr, method);
    set_error(rc);
    return rc;
}

extern "C" int arb_orient_batch(const arb_csr *g, const int64_t *graph_vtx_offsets, int64_t G, int64_t max_graph_n,
                                double eps, int validate, arb_ocsr *out, int32_t *rank, int32_t *round_out,
                                int32_t *dap_out, int64_t *stats, void *ws, size_t ws_bytes, void *stream) {
    const BatchDesc b{graph_vtx_offsets, G, max_graph_n};
    const int rc = orient_impl(g, eps, validate, out, rank, round_out, dap_out, stats, ws, ws_bytes,
                               as_stream(stream), &b);
    set_error(rc);
    return rc;
}
