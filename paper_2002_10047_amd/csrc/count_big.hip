// Counting for roots whose out-neighbourhood exceeds the largest LDS tier (k = 3, 4):
// Alg. 1 at the root as in the tiers (Sec. 3.2, 3.4), with G[N+(v)] as upper-triangular
// bit rows in a per-team slice of global scratch instead of LDS.  One 16-wave team per
// root; S = N+(v) and an LDS hash from id to local id serve the second level (the
// gathered N+(u) lists set bits with global atomics); at k = 4 the pairs (x, y) of G[S]
// go through per-wave rings to the lanes, each adding popcount(row x AND row y) over the
// words at or above y's word.  Per-vertex counts as in the tiers: a pair's common upper
// neighbours z each gain 1 and x, y gain their number.
#include "count_kernels.h"

namespace arb {

constexpr int kBigGatherUnroll = 8;   // independent 4-byte list loads in flight per lane

template <bool PV>
struct BigLds {
    static constexpr int TW = 16;
    static constexpr int HS = 2 * kBigMax;
    static constexpr int HB = 13;
    static constexpr int SPAN = 0;          // membership always through the hash
    static constexpr int RING = 128;        // per-wave pair ring, rows written in windows
    int32_t S[kBigMax];
    unsigned long long H[HS];
    unsigned long long cnt[PV ? kBigMax : 1];
    union {
        uint32_t ring[TW][RING];
        ListEnt lt[TW][64];
    } q;
    unsigned long long red[TW];
    int d;
    int pop;
    int next;
};
static_assert((1 << BigLds<true>::HB) == BigLds<true>::HS, "hash size");
static_assert(sizeof(BigLds<true>) <= 160 * 1024, "big-root LDS");

// second level of a big root: lists N+(S[i]) for i = wv, wv + 16, ... as one stream per wave
template <bool PV, class Lds>
__device__ void big_gather(AS3<Lds> *T, const CountArgs &a, int d, int need, int32_t first, int32_t last, int wv,
                           int lane, uint32_t *grow, int W, unsigned long long &mine, unsigned long long &words) {
    AS3<ListEnt> *lt = T->q.lt[wv];
    const int nl = wv < d ? (d - wv + Lds::TW - 1) / Lds::TW : 0;
    for (int gb = 0; gb < nl; gb += 64) {
        const int t = gb + lane;
        int64_t s = 0, e = 0;
        int row = 0;
        if (t < nl) {
            row = wv + Lds::TW * t;
            const int32_t u = T->S[row];
            s = a.off[u];
            e = a.off[u + 1];
        }
        const int64_t len = e - s;
        words += (unsigned long long)len;
        int64_t end = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(end, o, 64);
            if (lane >= o) end += y;
        }
        const int64_t total = __shfl(end, 63, 64);
        lt[lane].delta = s - (end - len);
        lt[lane].end = end;
        lt[lane].row = row;
        wave_fence();
        int c = 0;
        int64_t c_end = lt[0].end;
        int64_t c_delta = lt[0].delta;
        int c_row = lt[0].row;
        for (int64_t base = 0; base < total; base += 64 * kBigGatherUnroll) {
            int32_t w[kBigGatherUnroll];
            int r[kBigGatherUnroll];
#pragma unroll
            for (int q = 0; q < kBigGatherUnroll; ++q) {
                const int64_t pos = base + 64 * q + lane;
                w[q] = 0x7fffffff;
                r[q] = 0;
                if (pos < total) {
                    while (pos >= c_end) {
                        ++c;
                        c_end = lt[c].end;
                        c_delta = lt[c].delta;
                        c_row = lt[c].row;
                    }
                    w[q] = a.idx[pos + c_delta];
                    r[q] = c_row;
                }
            }
#pragma unroll
            for (int q = 0; q < kBigGatherUnroll; ++q) {
                const int j = member_find(T, w[q], first, last, false);
                if (j < 0) continue;
                const int i = r[q];
                if (need == 2) {
                    mine += 1;
                    if constexpr (PV) {
                        lds_add(&T->cnt[j], 1ull);
                        lds_add(&T->cnt[i], 1ull);
                    }
                } else {
                    atomicOr(&grow[(int64_t)i * W + (j >> 5)], 1u << (j & 31));
                }
            }
        }
        wave_fence();
    }
}

// popcount(row x AND row y) over the words at or above y's word; per-vertex: each common
// upper neighbour z gains 1
template <bool PV, class Lds>
__device__ __forceinline__ unsigned big_pair(AS3<Lds> *T, const uint32_t *grow, int W, int x, int y) {
    const uint32_t *rx = grow + (int64_t)x * W;
    const uint32_t *ry = grow + (int64_t)y * W;
    unsigned c = 0;
    for (int w = y >> 5; w < W; ++w) {
        uint32_t t = rx[w] & ry[w];
        c += __popc(t);
        if constexpr (PV) {
            while (t) {
                const int b = __ffs(t) - 1;
                t &= t - 1;
                lds_add(&T->cnt[w * 32 + b], 1ull);
            }
        }
    }
    if constexpr (PV) {
        if (c) {
            lds_add(&T->cnt[x], (unsigned long long)c);
            lds_add(&T->cnt[y], (unsigned long long)c);
        }
    }
    return c;
}

template <bool PV, bool INSTR>
__global__ void __launch_bounds__(1024) k_count_big(CountArgs a, BigArgs b) {
    using Lds = BigLds<PV>;
    constexpr int TW = Lds::TW, TT = 64 * TW;
    extern __shared__ __align__(16) unsigned char smem[];
    AS3<Lds> *T = (AS3<Lds> *)smem;
    const int tlid = threadIdx.x, lane = tlid & 63, wv = tlid >> 6;
    uint32_t *grow = b.rows + (int64_t)blockIdx.x * b.team_words;
    const int64_t beg = a.seg[0], end = a.seg[1];
    unsigned long long acc = 0;
    while (true) {
        __syncthreads();
        if (tlid == 0) T->pop = atomicAdd(a.head, 1);
        __syncthreads();
        const int64_t it = beg + (int64_t)T->pop;
        if (it >= end) break;
        const int32_t root = a.item_root[it];
        const int64_t s0 = a.roff[root];
        const int64_t d64 = a.roff[root + 1] - s0;
        if (d64 > b.dbig || d64 > kBigMax || a.item_child[it] != -1) {
            if (tlid == 0) atomicOr(a.err, 1);
            continue;
        }
        const int d = (int)d64, W = (d + 31) / 32;
        const int need = a.k - 1;                       // 2 or 3
        for (int i = tlid; i < d; i += TT) T->S[i] = a.ridx[s0 + i];
        for (int i = tlid; i < Lds::HS; i += TT) T->H[i] = kEmpty;
        if constexpr (PV)
            for (int i = tlid; i < d; i += TT) T->cnt[i] = 0ull;
        if (need == 3)
            for (int64_t i = tlid; i < (int64_t)d * W; i += TT) grow[i] = 0u;
        if (tlid == 0) T->next = TW;
        // the zeroed rows must reach L2 before any wave's atomics
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        for (int i = tlid; i < d; i += TT) hash_insert(T, (uint32_t)T->S[i], (uint32_t)i);
        __syncthreads();
        const int32_t first = T->S[0], last = T->S[d - 1];
        unsigned long long mine = 0, words = 0, nodes = 0;
        big_gather<PV, Lds>(T, a, d, need, first, last, wv, lane, grow, W, mine, words);
        if (need == 3) {
            // the rows were set by global atomics of all waves: complete them, then read
            // them past this CU's L1
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            AS3<uint32_t> *ring = T->q.ring[wv];
            unsigned head = 0, tail = 0;
            int x = wv;
            while (x < d) {
                const uint32_t *rx = grow + (int64_t)x * W;
                for (int cw = 0; cw < W; cw += 64) {
                    uint32_t bits = cw + lane < W ? rx[cw + lane] : 0u;
                    const unsigned c = __popc(bits);
                    unsigned pre = c;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const unsigned y = __shfl_up(pre, o, 64);
                        if (lane >= o) pre += y;
                    }
                    const unsigned stop_all = tail + __shfl(pre, 63, 64);
                    unsigned pos = tail + pre - c;
                    while (true) {
                        while (bits && pos - head < (unsigned)Lds::RING) {
                            const int bb = __ffs(bits) - 1;
                            bits &= bits - 1;
                            ring[pos & (Lds::RING - 1)] = ((uint32_t)x << 16) | (uint32_t)((cw + lane) * 32 + bb);
                            ++pos;
                        }
                        wave_fence();
                        const bool all = stop_all - head <= (unsigned)Lds::RING;
                        const unsigned stop = all ? stop_all : head + Lds::RING;
                        while (stop - head >= 64) {
                            const uint32_t p = ring[(head + lane) & (Lds::RING - 1)];
                            mine += big_pair<PV, Lds>(T, grow, W, (int)(p >> 16), (int)(p & 0xffffu));
                            if constexpr (INSTR) nodes += 1;
                            head += 64;
                        }
                        wave_fence();
                        if (all) break;
                    }
                    tail = stop_all;
                }
                int nx = 0;
                if (lane == 0) nx = __hip_atomic_fetch_add(&T->next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                x = __shfl(nx, 0, 64);
            }
            if (tail != head && lane < (int)(tail - head)) {
                const uint32_t p = ring[(head + lane) & (Lds::RING - 1)];
                mine += big_pair<PV, Lds>(T, grow, W, (int)(p >> 16), (int)(p & 0xffffu));
                if constexpr (INSTR) nodes += 1;
            }
        }
        const unsigned long long item = team_sum<TW, 1>(T, mine, wv, lane);
        if (a.per_root != nullptr && tlid == 0 && item) atomicAdd(&a.per_root[root], item);
        if constexpr (PV) {
            for (int i = tlid; i < d; i += TT) {
                const unsigned long long c = T->cnt[i];
                if (c) atomicAdd(&a.pv[T->S[i]], c);
            }
            if (tlid == 0 && item) atomicAdd(&a.pv[root], item);
        }
        if constexpr (INSTR) {
            // work label: gathered words + ceil(d/32) per search-tree node (d at depth 1,
            // the pairs at depth 2 when k = 4)
            const unsigned long long tn = team_sum<TW, 1>(T, nodes, wv, lane);
            const unsigned long long tg = team_sum<TW, 1>(T, words, wv, lane);
            if (tlid == 0) a.work[root] = tg + (unsigned long long)W * ((unsigned long long)d + tn);
        }
        acc += mine;
        // the next item clears and rewrites this team's rows
        __syncthreads();
    }
    acc = wave_sum(acc);
    if (lane == 0 && acc) atomicAdd(a.total, acc);
}

template <bool PV, bool INSTR>
static int launch_big(const CountArgs &a, const BigArgs &b, unsigned grid, hipStream_t s) {
    const size_t lds = (sizeof(BigLds<PV>) + 15) & ~size_t(15);
    static bool configured = false;
    if (!configured) {
        if (hipFuncSetAttribute((const void *)k_count_big<PV, INSTR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return ARB_EHIP;
        configured = true;
    }
    k_count_big<PV, INSTR><<<grid, 1024, lds, s>>>(a, b);
    ARB_CHECK_LAUNCH();
    return ARB_OK;
}

int launch_count_big(bool pv, bool instr, const CountArgs &a, const BigArgs &b, unsigned grid, hipStream_t s) {
    if (pv) return launch_big<true, false>(a, b, grid, s);
    if (instr) return launch_big<false, true>(a, b, grid, s);
    return launch_big<false, false>(a, b, grid, s);
}

}  // namespace arb
