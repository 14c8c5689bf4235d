// Exact k-clique counting on the GPU: Alg. 1 (arb-count) and its per-vertex variant
// arb-count-v (Sec. 3.2) of Shi, Dhulipala, Shun, with the practical optimisations of
// Sec. 3.4 mapped onto gfx950:
//
//  * work item = a root v (candidate set S = N+(v), k-1 vertices still to choose), or,
//    for a root split by the scheduler, a pair (v, c) with c in N+(v)
//    (S = N+(v) ∩ N+(c), k-2 to choose) -- the paper's node vs edge parallelism;
//  * one team (1..8 waves) per item stages S in LDS, relabelled 0..d-1 in rank order
//    (Sec. 3.4: relabel the induced subgraph to [0, O(alpha))), with an LDS hash from
//    vertex id to local id standing in for the paper's mark array;
//  * the second-level intersections (the first non-trivial ones) read N+(u) for every
//    u in S from HBM with coalesced 64-lane loads and keep the members of S: this builds
//    G[S] as one bit row per local vertex (row x = neighbours of x in S above x; in the
//    per-vertex mode the rows are symmetric and masked on use);
//  * deeper levels never touch HBM: every candidate set is a bitmap over local ids,
//    I' = I AND row(x) (Alg. 1, intersect), and the last level adds popcounts instead of
//    materialising I (base case |I|).  Pairs (x, y) of the induced subgraph are spread
//    over the lanes through per-wave ring buffers; each lane then walks its subtree.
//
// Per-vertex counts: a vertex receives, for each clique it belongs to, one unit.  With
// I the candidate set of a node needing two more vertices, every z in I belongs to
// popcount(I AND adj(z)) of that node's cliques, while the vertices chosen so far belong
// to all popcount-sum/2 of them; this keeps the per-vertex pass proportional to the
// bitmap work instead of to the number of cliques.
#pragma once
#include "common.h"

namespace arb {

// ------------------------------------------------------------------ tiers

// local candidate-set capacity per tier: 32 * W (W 32-bit words per bit row)
template <int W> struct TierCfg;
template <> struct TierCfg<2>  { static constexpr int TW = 1, TPB = 4; };
template <> struct TierCfg<4>  { static constexpr int TW = 1, TPB = 4; };
template <> struct TierCfg<8>  { static constexpr int TW = 4, TPB = 1; };
template <> struct TierCfg<12> { static constexpr int TW = 8, TPB = 1; };
template <> struct TierCfg<16> { static constexpr int TW = 8, TPB = 1; };
template <> struct TierCfg<24> { static constexpr int TW = 8, TPB = 1; };

constexpr int kNumTiers = 6;
constexpr int kTierW[kNumTiers] = {2, 4, 8, 12, 16, 24};
static_assert(32 * 24 == ARB_MAX_LOCAL, "largest tier must match ARB_MAX_LOCAL");

__host__ __device__ inline int tier_of(int64_t bound) {
    if (bound <= 64) return 0;
    if (bound <= 128) return 1;
    if (bound <= 256) return 2;
    if (bound <= 384) return 3;
    if (bound <= 512) return 4;
    if (bound <= 768) return 5;
    return -1;
}

constexpr int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

template <int W, bool PV>
struct TeamLds {
    static constexpr int D = 32 * W;             // capacity of S
    static constexpr int RS = W + 1;             // row stride in words (odd: spreads banks)
    static constexpr int HS = pow2_at_least(2 * D);
    static constexpr int HB = __builtin_ctz(HS);
    static constexpr int TW = TierCfg<W>::TW;
    static constexpr int RING = pow2_at_least(D + 64);
    int32_t S[D];
    uint64_t H[HS];
    uint32_t rows[D * RS];
    uint64_t cnt[PV ? D : 1];
    uint32_t ring[TW][RING];
    unsigned long long red[TW];
    int d;
    int pop;
};

constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint32_t hslot(uint32_t key, int hb) {
    return (key * 2654435761u) >> (32 - hb);
}

template <class L>
__device__ __forceinline__ void hash_insert(L *T, uint32_t key, uint32_t val) {
    uint32_t s = hslot(key, L::HB);
    const uint64_t e = ((uint64_t)val << 32) | key;
    while (true) {
        unsigned long long old = atomicCAS((unsigned long long *)&T->H[s], (unsigned long long)kEmpty,
                                           (unsigned long long)e);
        if (old == kEmpty) return;
        s = (s + 1) & (L::HS - 1);
    }
}

template <class L>
__device__ __forceinline__ int hash_find(const L *T, uint32_t key) {
    uint32_t s = hslot(key, L::HB);
    while (true) {
        uint64_t e = T->H[s];
        if (e == kEmpty) return -1;
        if ((uint32_t)e == key) return (int)(e >> 32);
        s = (s + 1) & (L::HS - 1);
    }
}

// bits of word w that stand for local ids greater than z
__device__ __forceinline__ uint32_t gtmask(int z, int w) {
    int zw = z >> 5, zb = z & 31;
    uint32_t hi = zb == 31 ? 0u : (~0u << (zb + 1));
    return w < zw ? 0u : (w > zw ? ~0u : hi);
}

template <int TW, int TPB>
__device__ __forceinline__ void team_sync() {
    if constexpr (TPB == 1) {
        __syncthreads();
    } else {
        static_assert(TW == 1, "multi-team blocks use single-wave teams");
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
}

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Sum of x over the team (every thread of the team must call it).
template <int TW, int TPB, class Lds>
__device__ __forceinline__ unsigned long long team_sum(Lds *T, unsigned long long x, int wv, int lane) {
    const unsigned long long s = wave_sum(x);
    team_sync<TW, TPB>();
    if (lane == 0) T->red[wv] = s;
    team_sync<TW, TPB>();
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < TW; ++w) t += T->red[w];
    return t;
}

struct CountArgs {
    const int64_t *off;
    const int32_t *idx;
    int64_t n;
    int k;
    const int32_t *item_root;
    const int32_t *item_child;
    const int64_t *seg;            // [begin, end) of this tier in the item arrays
    int *head;                     // queue head (persistent)
    unsigned long long *total;
    unsigned long long *pv;        // nullable
    unsigned long long *work;      // nullable
    int32_t *err;
    int chunk;
    int persistent;
    int one_item_per_team;         // non-persistent launch: team g takes item begin + g
};

// ------------------------------------------------------------------ subtree walk

// Lowest set bit of the W-word set R, removed from R; -1 when R is empty.
template <int W>
__device__ __forceinline__ int pop_lowest(uint32_t (&R)[W]) {
    int z = -1;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        if (z < 0 && R[w]) {
            z = w * 32 + __ffs(R[w]) - 1;
            R[w] &= R[w] - 1;
        }
    }
    return z;
}

// Number of L-cliques (L >= 2) inside the candidate set J.  Per-vertex mode: rows are
// symmetric adjacency, members gain their share through cnt; instrumented mode adds the
// search-tree nodes under J to *nodes.
template <int W, bool PV, bool INSTR, int L, class Lds>
__device__ unsigned long long dfs(Lds *T, const uint32_t (&J)[W], unsigned long long *nodes) {
    uint32_t R[W];
    unsigned long long total = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) R[w] = J[w];
    if constexpr (INSTR) {
        unsigned c = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) c += __popc(J[w]);
        *nodes += c;
    }
    while (true) {
        int z = pop_lowest<W>(R);
        if (z < 0) break;
        const uint32_t *rz = &T->rows[z * Lds::RS];
        if constexpr (L == 2) {
            if constexpr (PV) {
                unsigned a = 0, c = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    uint32_t t = J[w] & rz[w];
                    a += __popc(t);
                    c += __popc(t & gtmask(z, w));
                }
                if (a) atomicAdd((unsigned long long *)&T->cnt[z], (unsigned long long)a);
                total += c;
            } else {
                unsigned c = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) c += __popc(J[w] & rz[w]);
                total += c;
            }
        } else {
            uint32_t K[W];
#pragma unroll
            for (int w = 0; w < W; ++w) K[w] = PV ? (J[w] & rz[w] & gtmask(z, w)) : (J[w] & rz[w]);
            unsigned long long c = dfs<W, PV, INSTR, L - 1, Lds>(T, K, nodes);
            if constexpr (PV) {
                if (c) atomicAdd((unsigned long long *)&T->cnt[z], c);
            }
            total += c;
        }
    }
    return total;
}

template <int W, int LMAX, bool PV, bool INSTR, class Lds>
__device__ __forceinline__ unsigned long long dfs_dispatch(Lds *T, const uint32_t (&J)[W], int L,
                                                           unsigned long long *nodes) {
    if constexpr (LMAX >= 2) if (L == 2) return dfs<W, PV, INSTR, 2, Lds>(T, J, nodes);
    if constexpr (LMAX >= 3) if (L == 3) return dfs<W, PV, INSTR, 3, Lds>(T, J, nodes);
    if constexpr (LMAX >= 4) if (L == 4) return dfs<W, PV, INSTR, 4, Lds>(T, J, nodes);
    if constexpr (LMAX >= 5) if (L == 5) return dfs<W, PV, INSTR, 5, Lds>(T, J, nodes);
    if constexpr (LMAX >= 6) if (L == 6) return dfs<W, PV, INSTR, 6, Lds>(T, J, nodes);
    if constexpr (LMAX >= 7) if (L == 7) return dfs<W, PV, INSTR, 7, Lds>(T, J, nodes);
    if constexpr (LMAX >= 8) if (L == 8) return dfs<W, PV, INSTR, 8, Lds>(T, J, nodes);
    if constexpr (LMAX >= 9) if (L == 9) return dfs<W, PV, INSTR, 9, Lds>(T, J, nodes);
    return 0;
}
static_assert(ARB_MAX_K - 3 <= 9, "dfs_dispatch covers L up to ARB_MAX_K - 3");
constexpr int kMaxDepth = ARB_MAX_K - 3;

// One pair (x, y) of the induced subgraph, x < y, both chosen: count the cliques that
// extend it with `need` more vertices from S (need >= 1).
template <int W, int LMAX, bool PV, bool INSTR, class Lds>
__device__ unsigned long long do_pair(Lds *T, uint32_t p, int need, unsigned long long *nodes) {
    const int x = (int)(p >> 16), y = (int)(p & 0xffffu);
    const uint32_t *rx = &T->rows[x * Lds::RS];
    const uint32_t *ry = &T->rows[y * Lds::RS];
    if constexpr (INSTR) *nodes += 1;
    uint32_t J[W];
    if (need == 1 || LMAX < 2) {
        if constexpr (PV) {
            unsigned a = 0, c = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                uint32_t t = rx[w] & ry[w];
                a += __popc(t & gtmask(x, w));
                c += __popc(t & gtmask(y, w));
            }
            if (a) atomicAdd((unsigned long long *)&T->cnt[y], (unsigned long long)a);
            if (c) atomicAdd((unsigned long long *)&T->cnt[x], (unsigned long long)c);
            return c;
        } else {
            unsigned c = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) c += __popc(rx[w] & ry[w]);
            return c;
        }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) J[w] = PV ? (rx[w] & ry[w] & gtmask(y, w)) : (rx[w] & ry[w]);
    unsigned long long c = dfs_dispatch<W, LMAX, PV, INSTR, Lds>(T, J, need, nodes);
    if constexpr (PV) {
        if (c) {
            atomicAdd((unsigned long long *)&T->cnt[x], c);
            atomicAdd((unsigned long long *)&T->cnt[y], c);
        }
    }
    return c;
}

// ------------------------------------------------------------------ one work item

template <int W, int LMAX, bool PV, bool INSTR>
__device__ void process_item(TeamLds<W, PV> *T, const CountArgs &a, int32_t root, int32_t child,
                             int tlid, unsigned long long *acc) {
    using Lds = TeamLds<W, PV>;
    constexpr int TW = TierCfg<W>::TW, TPB = TierCfg<W>::TPB;
    constexpr int TT = 64 * TW;
    const int lane = tlid & 63, wv = tlid >> 6;
    const uint64_t below = lanes_below_mask();

    team_sync<TW, TPB>();            // previous item finished with the LDS
    int need;
    if (child < 0) {
        const int64_t s0 = a.off[root];
        const int64_t d = a.off[root + 1] - s0;
        if (d > Lds::D) {
            if (tlid == 0) atomicOr(a.err, 1);
            return;
        }
        for (int i = tlid; i < d; i += TT) T->S[i] = a.idx[s0 + i];
        if (tlid == 0) T->d = (int)d;
        need = a.k - 1;
    } else {
        // S = N+(root) ∩ N+(child): wave 0 walks N+(child) and binary-searches N+(root)
        if (wv == 0) {
            const int64_t rs = a.off[root], re = a.off[root + 1];
            const int64_t cs = a.off[child], ce = a.off[child + 1];
            int cntS = 0;
            for (int64_t b = cs; b < ce; b += 64) {
                int64_t p = b + lane;
                bool hit = false;
                int32_t w = 0;
                if (p < ce) {
                    w = a.idx[p];
                    int64_t lo = rs, hi = re;
                    while (lo < hi) {
                        int64_t mid = lo + ((hi - lo) >> 1);
                        if (a.idx[mid] < w) lo = mid + 1; else hi = mid;
                    }
                    hit = lo < re && a.idx[lo] == w;
                }
                uint64_t m = __ballot(hit);
                int pos = cntS + __popcll(m & below);
                if (hit && pos < Lds::D) T->S[pos] = w;
                cntS += __popcll(m);
            }
            if (cntS > Lds::D) {
                if (lane == 0) atomicOr(a.err, 1);
                cntS = 0;
            }
            if (lane == 0) T->d = cntS;
        }
        need = a.k - 2;
    }
    team_sync<TW, TPB>();
    const int d = T->d;
    if (d < need || d == 0) return;     // no clique fits (need >= 1 here)

    for (int i = tlid; i < Lds::HS; i += TT) T->H[i] = kEmpty;
    if (need >= 3)
        for (int i = tlid; i < d * Lds::RS; i += TT) T->rows[i] = 0u;
    if constexpr (PV)
        for (int i = tlid; i < d; i += TT) T->cnt[i] = 0ull;
    team_sync<TW, TPB>();
    for (int i = tlid; i < d; i += TT) hash_insert(T, (uint32_t)T->S[i], (uint32_t)i);
    team_sync<TW, TPB>();

    unsigned long long mine = 0;      // this lane's share of the item's clique count
    unsigned long long nodes = 0;     // instrumented: search-tree nodes (depth <= k-2)
    unsigned long long gather = 0;    // instrumented: words of N+(u) lists

    if (need == 1) {
        if (tlid == 0) mine = (unsigned long long)d;
        if constexpr (PV)
            for (int i = tlid; i < d; i += TT) T->cnt[i] = 1ull;
    } else {
        const int32_t maxS = T->S[d - 1];
        for (int i = wv; i < d; i += TW) {
            const int32_t u = T->S[i];
            const int64_t s = a.off[u], e = a.off[u + 1];
            if constexpr (INSTR) {
                if (lane == 0) gather += (unsigned long long)(e - s);
            }
            unsigned rowcnt = 0;
            for (int64_t b = s; b < e; b += 64) {
                const int64_t p = b + lane;
                const int32_t w = p < e ? a.idx[p] : 0x7fffffff;
                if (__shfl(w, 0, 64) > maxS) break;       // rows ascend: nothing further matches
                const int j = w <= maxS ? hash_find(T, (uint32_t)w) : -1;
                const bool hit = j >= 0;
                if (need == 2) {
                    uint64_t m = __ballot(hit);
                    if (hit) mine += 1;
                    rowcnt += (unsigned)__popcll(m);
                    if constexpr (PV) {
                        if (hit) atomicAdd((unsigned long long *)&T->cnt[j], 1ull);
                    }
                } else if (hit) {
                    atomicOr(&T->rows[i * Lds::RS + (j >> 5)], 1u << (j & 31));
                    if constexpr (PV) atomicOr(&T->rows[j * Lds::RS + (i >> 5)], 1u << (i & 31));
                }
            }
            if constexpr (PV) {
                if (need == 2 && lane == 0 && rowcnt)
                    atomicAdd((unsigned long long *)&T->cnt[i], (unsigned long long)rowcnt);
            }
        }
        if constexpr (INSTR) {
            if (tlid == 0) nodes += (unsigned long long)d;     // depth-1 nodes
        }
        if (need >= 3) {
            team_sync<TW, TPB>();
            // pairs (x, y), y > x adjacent, spread over the lanes through the wave's ring
            uint32_t *ring = T->ring[wv];
            unsigned head = 0, tail = 0;
            const int pneed = need - 2;
            for (int x = wv; x < d; x += TW) {
                uint32_t bits = 0;
                if (lane < W) {
                    bits = T->rows[x * Lds::RS + lane];
                    if constexpr (PV) bits &= gtmask(x, lane);
                }
                unsigned c = __popc(bits);
                unsigned pre = c;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    unsigned y = __shfl_up(pre, o, 64);
                    if (lane >= o) pre += y;
                }
                unsigned tot = __shfl(pre, 63, 64);
                pre -= c;
                unsigned pos = tail + pre;
                while (bits) {
                    int b = __ffs(bits) - 1;
                    bits &= bits - 1;
                    ring[pos & (Lds::RING - 1)] = ((uint32_t)x << 16) | (uint32_t)(lane * 32 + b);
                    ++pos;
                }
                tail += tot;
                wave_fence();
                while (tail - head >= 64) {
                    uint32_t p = ring[(head + lane) & (Lds::RING - 1)];
                    mine += do_pair<W, LMAX, PV, INSTR, Lds>(T, p, pneed, &nodes);
                    head += 64;
                }
                wave_fence();
            }
            if (tail != head) {
                if (lane < (int)(tail - head)) {
                    uint32_t p = ring[(head + lane) & (Lds::RING - 1)];
                    mine += do_pair<W, LMAX, PV, INSTR, Lds>(T, p, pneed, &nodes);
                }
            }
        }
    }

    *acc += mine;
    if constexpr (PV || INSTR) {
        const unsigned long long item = team_sum<TW, TPB>(T, mine, wv, lane);
        if constexpr (PV) {
            for (int i = tlid; i < d; i += TT) {
                unsigned long long c = T->cnt[i];
                if (c) atomicAdd(&a.pv[T->S[i]], c);
            }
            if (tlid == 0 && item) {
                atomicAdd(&a.pv[root], item);
                if (child >= 0) atomicAdd(&a.pv[child], item);
            }
        }
        if constexpr (INSTR) {
            const unsigned long long tn = team_sum<TW, TPB>(T, nodes, wv, lane);
            const unsigned long long tg = team_sum<TW, TPB>(T, gather, wv, lane);
            if (tlid == 0 && child < 0) a.work[root] = tg + (unsigned long long)((d + 31) / 32) * tn;
        }
    }
}

template <int W, int LMAX, bool PV, bool INSTR>
__global__ void __launch_bounds__(64 * TierCfg<W>::TW * TierCfg<W>::TPB)
k_count(CountArgs a) {
    using Lds = TeamLds<W, PV>;
    constexpr int TW = TierCfg<W>::TW, TPB = TierCfg<W>::TPB;
    extern __shared__ __align__(16) unsigned char smem[];
    const int team = threadIdx.x / (64 * TW);
    const int tlid = threadIdx.x % (64 * TW);
    Lds *T = reinterpret_cast<Lds *>(smem + (size_t)team * ((sizeof(Lds) + 15) & ~size_t(15)));
    const int64_t beg = a.seg[0], end = a.seg[1];
    unsigned long long acc = 0;
    const int64_t gteam = (int64_t)blockIdx.x * TPB + team;
    if (a.one_item_per_team) {
        int64_t it = beg + gteam;
        if (it < end) process_item<W, LMAX, PV, INSTR>(T, a, a.item_root[it], a.item_child[it], tlid, &acc);
    } else if (!a.persistent) {
        const int64_t nteams = (int64_t)gridDim.x * TPB;
        for (int64_t it = beg + gteam; it < end; it += nteams)
            process_item<W, LMAX, PV, INSTR>(T, a, a.item_root[it], a.item_child[it], tlid, &acc);
    } else {
        while (true) {
            team_sync<TW, TPB>();
            if (tlid == 0) T->pop = atomicAdd(a.head, a.chunk);
            team_sync<TW, TPB>();
            const int64_t first = beg + (int64_t)T->pop;
            if (first >= end) break;
            const int64_t last = min(first + (int64_t)a.chunk, end);
            for (int64_t it = first; it < last; ++it)
                process_item<W, LMAX, PV, INSTR>(T, a, a.item_root[it], a.item_child[it], tlid, &acc);
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(a.total, acc);
}

template <int W, bool PV>
constexpr size_t team_bytes() {
    return (sizeof(TeamLds<W, PV>) + 15) & ~size_t(15);
}

template <int W, int LMAX, bool PV, bool INSTR>
static int launch_tier(const CountArgs &a, unsigned grid, hipStream_t s) {
    constexpr int TW = TierCfg<W>::TW, TPB = TierCfg<W>::TPB;
    const size_t lds = team_bytes<W, PV>() * TPB;
    static bool configured = false;
    if (!configured) {
        if (hipFuncSetAttribute((const void *)k_count<W, LMAX, PV, INSTR>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return ARB_EHIP;
        configured = true;
    }
    k_count<W, LMAX, PV, INSTR><<<grid, 64 * TW * TPB, lds, s>>>(a);
    ARB_CHECK_LAUNCH();
    return ARB_OK;
}

template <int LMAX, bool PV, bool INSTR>
static int launch_tier_rt(int tier, const CountArgs &a, unsigned grid, hipStream_t s) {
    switch (tier) {
        case 0: return launch_tier<2, LMAX, PV, INSTR>(a, grid, s);
        case 1: return launch_tier<4, LMAX, PV, INSTR>(a, grid, s);
        case 2: return launch_tier<8, LMAX, PV, INSTR>(a, grid, s);
        case 3: return launch_tier<12, LMAX, PV, INSTR>(a, grid, s);
        case 4: return launch_tier<16, LMAX, PV, INSTR>(a, grid, s);
        case 5: return launch_tier<24, LMAX, PV, INSTR>(a, grid, s);
    }
    return ARB_EINVAL;
}

// Instantiates the tier launchers of one recursion depth (one translation unit each).
#define ARB_COUNT_DEPTH_UNIT(LM)                                                            \
    int launch_count_depth##LM(int tier, bool pv, bool instr, const CountArgs &a,          \
                               unsigned grid, hipStream_t s) {                             \
        if (pv) return launch_tier_rt<LM, true, false>(tier, a, grid, s);                  \
        if (instr) return launch_tier_rt<LM, false, true>(tier, a, grid, s);               \
        return launch_tier_rt<LM, false, false>(tier, a, grid, s);                         \
    }

inline int tier_teams_per_block(int tier) {
    switch (tier) {
        case 0: return TierCfg<2>::TPB;
        case 1: return TierCfg<4>::TPB;
        case 2: return TierCfg<8>::TPB;
        case 3: return TierCfg<12>::TPB;
        case 4: return TierCfg<16>::TPB;
        default: return TierCfg<24>::TPB;
    }
}

inline size_t tier_block_lds(int tier, bool pv) {
    switch (tier) {
        case 0: return (pv ? team_bytes<2, true>() : team_bytes<2, false>()) * TierCfg<2>::TPB;
        case 1: return (pv ? team_bytes<4, true>() : team_bytes<4, false>()) * TierCfg<4>::TPB;
        case 2: return pv ? team_bytes<8, true>() : team_bytes<8, false>();
        case 3: return pv ? team_bytes<12, true>() : team_bytes<12, false>();
        case 4: return pv ? team_bytes<16, true>() : team_bytes<16, false>();
        default: return pv ? team_bytes<24, true>() : team_bytes<24, false>();
    }
}


#define ARB_DECLARE_DEPTH(LM) \
    int launch_count_depth##LM(int tier, bool pv, bool instr, const CountArgs &a, unsigned grid, hipStream_t s);
ARB_DECLARE_DEPTH(1)
ARB_DECLARE_DEPTH(2)
ARB_DECLARE_DEPTH(3)
ARB_DECLARE_DEPTH(4)
ARB_DECLARE_DEPTH(5)
ARB_DECLARE_DEPTH(6)
ARB_DECLARE_DEPTH(7)
ARB_DECLARE_DEPTH(8)
ARB_DECLARE_DEPTH(9)
#undef ARB_DECLARE_DEPTH

}  // namespace arb
