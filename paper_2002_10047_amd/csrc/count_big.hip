// Counting for work items whose candidate set exceeds the largest LDS tier: Alg. 1 at the
// item as in the tiers (Sec. 3.2, 3.4), with G[S] as bit rows in a per-team slice of
// global scratch (L2 / Infinity Cache resident) instead of LDS.  Items are whole roots
// with ARB_MAX_LOCAL < d+ <= dbig (from the schedule), and (root, child) pair items whose
// set N+(root) ∩ N+(child) overflowed the largest LDS tier (appended to an overflow list
// by the tier kernels, which run before this kernel).  One 16-wave team per item:
//   * S and an LDS hash from id to local id serve the second level; the gathered N+(u)
//     lists set row bits with global atomics (upper rows: row x = x's neighbours above x;
//     symmetric rows in the per-vertex mode);
//   * k - 1 = 3 (k = 4 roots, k = 5 pairs): the pairs (x, y) go through per-wave rings
//     to the lanes, each adding popcount(row x AND row y) over the words from y's on;
//   * deeper: the pair phase is wave-cooperative: a wave claims a row x and holds it
//     across its lanes (lane l: words l and l + 64, rows of up to 4096 bits), then for each
//     member y of the row it reads row y with one coalesced load per lane and walks
//     J = row x AND row y above y, every set held across the lanes the same way (members
//     taken in ascending order with a ballot; frames of a private stack for the levels
//     above the last two), each node costing one coalesced row read.
// Per-vertex counts as in the tiers: at a node needing two more vertices with set I, each
// z in I gains popcount(I AND adj(z)), the chosen vertices gain the node's cliques.
#include "count_kernels.h"

namespace arb {

constexpr int kBigGatherUnroll = 8;   // independent 4-byte list loads in flight per lane
constexpr int kWaveFrames = ARB_MAX_K - 4;

__device__ __forceinline__ uint32_t big_filter_hash(int32_t w) { return ((uint32_t)w * 2246822519u) >> 18; }

// The team's bit rows in global scratch.  Symmetric rows (per-vertex mode) are full rows
// of RS words (RS: ceil(d / 32) rounded up to a multiple of 4, so that rows are 16-byte
// aligned).  Upper rows hold no bit below their own vertex, so they are stored from the
// 16-byte vector holding their own word on: row x keeps vectors x / 128 .. RS / 4 - 1, and
// the rows are packed one after another (half the scratch of full rows, which keeps more
// of a team's rows in the L2).
template <bool FULL>
struct BigRows {
    uint32_t *g;
    int RS;
    // words before row x: 4 * sum_{i < x} (RS / 4 - i / 128)
    __device__ __forceinline__ int64_t start(int x) const {
        if constexpr (FULL) {
            return (int64_t)x * RS;
        } else {
            const int64_t q = x >> 7, r = x & 127;
            return 4 * ((int64_t)x * (RS >> 2) - (64 * q * (q - 1) + r * q));
        }
    }
    // first stored word of row x
    __device__ __forceinline__ int lo(int x) const { return FULL ? 0 : 4 * (x >> 7); }
    // row x as an array indexed by word (only words lo(x) .. RS - 1 are stored)
    __device__ __forceinline__ uint32_t *row(int x) const { return g + start(x) - lo(x); }
    __device__ __forceinline__ int64_t words(int d) const { return start(d); }
};

template <bool PV>
struct BigLds {
    static constexpr int TW = 16;
    static constexpr int HS = 2 * kBigMax;
    static constexpr int HB = 13;
    static constexpr int SPAN = 0;          // membership always through the hash
    static constexpr int RING = 128;        // per-wave pair ring, rows written in windows
    int32_t S[kBigMax];
    unsigned long long H[HS];
    // 16384-bit filter of S (bit big_filter_hash(s) per member s): most second-level
    // entries are no members, and a clear bit rejects one with a single LDS read instead
    // of a hash probe sequence
    static constexpr int FW = 512;
    uint32_t flt[FW];
    unsigned long long cnt[PV ? kBigMax : 1];
    union {
        uint32_t ring[TW][RING];    // pair phase at k - 1 = 3: (x << 16 | y) per pair
        ListEnt lt[TW][64];         // second level
    } q;
    // upper rows are built in LDS a window of rows at a time (row i's bits all come from
    // the list N+(S[i]), so a window needs only its own lists) and then copied out
    static constexpr int WINW = PV ? 1 : 12288;
    uint32_t win[WINW];
    unsigned long long red[TW];
    int d;
    int pop;
    int next;
};
static_assert((1 << BigLds<true>::HB) == BigLds<true>::HS, "hash size");
static_assert(sizeof(BigLds<true>) <= 160 * 1024 && sizeof(BigLds<false>) <= 160 * 1024, "big-item LDS");

// second level: lists N+(S[i]) for i = rbeg + wv, rbeg + wv + 16, ... < rend as one stream
// per wave; with WIN the found bits go to the LDS window of rows rbeg .. rend - 1, else
// to the global rows with atomics
template <bool PV, bool SYM, bool WIN, class Lds>
__device__ void big_gather(AS3<Lds> *T, const CountArgs &a, int rbeg, int rend, int need, int32_t first,
                           int32_t last, int wv, int lane, const BigRows<PV> &rows, unsigned long long &mine,
                           unsigned long long &words) {
    AS3<ListEnt> *lt = T->q.lt[wv];
    const int nl = rbeg + wv < rend ? (rend - rbeg - wv + Lds::TW - 1) / Lds::TW : 0;
    for (int gb = 0; gb < nl; gb += 64) {
        const int t = gb + lane;
        int64_t s = 0, e = 0;
        int row = 0;
        if (t < nl) {
            row = rbeg + wv + Lds::TW * t;
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
                const uint32_t h = big_filter_hash(w[q]);
                if (!((T->flt[h >> 5] >> (h & 31u)) & 1u)) continue;
                const int j = member_find(T, w[q], first, last, false);
                if (j < 0) continue;
                const int i = r[q];
                if (need == 2) {
                    mine += 1;
                    if constexpr (PV) {
                        lds_add(&T->cnt[j], 1ull);
                        lds_add(&T->cnt[i], 1ull);
                    }
                } else if constexpr (WIN) {
                    lds_or(&T->win[(i - rbeg) * rows.RS + (j >> 5)], 1u << (j & 31));
                } else {
                    atomicOr(&rows.row(i)[j >> 5], 1u << (j & 31));          // j > i
                    if constexpr (SYM) atomicOr(&rows.row(j)[i >> 5], 1u << (i & 31));
                }
            }
        }
        wave_fence();
    }
}

// One pair (x, y), x < y, at k - 1 = 3: popcount(row x AND row y) over the members above y
// (the words at or above y's word; rows may be symmetric), read as 16-byte vectors from the
// one holding y's word (words past ceil(d / 32) are zero); per-vertex: each
// common member z above y gains 1, x and y gain the pair's count
template <bool PV, class Lds>
__device__ __forceinline__ unsigned pair_words(AS3<Lds> *T, int w0, uint32_t t0, uint32_t t1, uint32_t t2,
                                               uint32_t t3) {
    uint32_t t[4] = {t0, t1, t2, t3};
    unsigned c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        c += __popc(t[q]);
        if constexpr (PV) {
            while (t[q]) {
                lds_add(&T->cnt[(w0 + q) * 32 + __ffs(t[q]) - 1], 1ull);
                t[q] &= t[q] - 1;
            }
        }
    }
    return c;
}

template <bool PV, class Lds>
__device__ __forceinline__ unsigned big_pair(AS3<Lds> *T, const BigRows<PV> &rows, int x, int y) {
    const uint4 *rx = reinterpret_cast<const uint4 *>(rows.row(x));
    const uint4 *ry = reinterpret_cast<const uint4 *>(rows.row(y));
    const int v0 = y >> 7, vn = rows.RS >> 2;
    // the vector holding y's word: only the members above y; the ones after it whole, two
    // vectors of each row in flight at a time
    uint4 ax = rx[v0], ay = ry[v0];
    unsigned c = pair_words<PV, Lds>(T, 4 * v0, ax.x & ay.x & gtmask(y, 4 * v0), ax.y & ay.y & gtmask(y, 4 * v0 + 1),
                                     ax.z & ay.z & gtmask(y, 4 * v0 + 2), ax.w & ay.w & gtmask(y, 4 * v0 + 3));
    for (int v = v0 + 1; v < vn; v += 2) {
        const uint4 a0 = rx[v], b0 = ry[v];
        uint4 a1 = make_uint4(0u, 0u, 0u, 0u), b1 = a1;
        if (v + 1 < vn) {
            a1 = rx[v + 1];
            b1 = ry[v + 1];
        }
        c += pair_words<PV, Lds>(T, 4 * v, a0.x & b0.x, a0.y & b0.y, a0.z & b0.z, a0.w & b0.w);
        c += pair_words<PV, Lds>(T, 4 * v + 4, a1.x & b1.x, a1.y & b1.y, a1.z & b1.z, a1.w & b1.w);
    }
    if constexpr (PV) {
        if (c) {
            lds_add(&T->cnt[x], (unsigned long long)c);
            lds_add(&T->cnt[y], (unsigned long long)c);
        }
    }
    return c;
}

// A set of local ids held across the wave: lane l keeps words l (h0) and l + 64 (h1).
struct WSet {
    uint32_t h0, h1;
};

// words lo .. W - 1 of a row (the words below lo are zero)
__device__ __forceinline__ WSet wload(const uint32_t *row, int lo, int W, int lane) {
    WSet r;
    r.h0 = lane < W && lane >= lo ? row[lane] : 0u;
    r.h1 = lane + 64 < W && lane + 64 >= lo ? row[lane + 64] : 0u;
    return r;
}

__device__ __forceinline__ WSet wand(WSet a, WSet b) { return WSet{a.h0 & b.h0, a.h1 & b.h1}; }

// members above z (bits of the lane's words that stand for ids > z)
__device__ __forceinline__ WSet wabove(WSet a, int z, int lane) {
    return WSet{a.h0 & gtmask(z, lane), a.h1 & gtmask(z, lane + 64)};
}

__device__ __forceinline__ unsigned wpopc(WSet a) { return (unsigned)(__popc(a.h0) + __popc(a.h1)); }

// lowest member of the wave's set, removed from it; -1 when empty (wave-uniform)
__device__ __forceinline__ int wpop(WSet &a, int lane) {
    uint64_t m = __ballot(a.h0 != 0u);
    int base = 0;
    uint32_t word;
    int src;
    if (m) {
        src = __ffsll((unsigned long long)m) - 1;
        word = __shfl(a.h0, src, 64);
    } else {
        m = __ballot(a.h1 != 0u);
        if (!m) return -1;
        src = __ffsll((unsigned long long)m) - 1;
        word = __shfl(a.h1, src, 64);
        base = 64;
    }
    const int z = (base + src) * 32 + __ffs(word) - 1;
    if (lane == src) {
        if (base == 0) a.h0 &= a.h0 - 1;
        else a.h1 &= a.h1 - 1;
    }
    return z;
}

__device__ __forceinline__ bool wempty(WSet a) { return __ballot((a.h0 | a.h1) != 0u) == 0; }

// per-vertex credit at a node needing two more vertices with set I: each z in I gains its
// neighbours in I (symmetric rows); returns the lane's share of the node's cliques
template <bool PV, bool INSTR, class Lds>
__device__ __forceinline__ unsigned long long wleaf(AS3<Lds> *T, const BigRows<PV> &rows, int W, WSet I, int lane,
                                                    unsigned long long &nodes) {
    if constexpr (INSTR) nodes += wpopc(I);
    unsigned long long c = 0;
    WSet R = I;
    while (true) {
        const int z = wpop(R, lane);
        if (z < 0) break;
        const WSet rz = wload(rows.row(z), rows.lo(z), W, lane);
        c += wpopc(wand(R, rz));                          // R: I's members above z
        if constexpr (PV) {
            const unsigned long long az = wave_sum((unsigned long long)wpopc(wand(I, rz)));
            if (lane == 0 && az) lds_add(&T->cnt[z], az);
        }
    }
    return c;
}

// L-cliques (L >= 2) inside the wave's set J: frames of a private stack hold the untaken
// members of every level above the last two; returns the lane's share
template <bool PV, bool INSTR, class Lds>
__device__ __attribute__((noinline)) unsigned long long wdfs(AS3<Lds> *T, const BigRows<PV> rows, int W, WSet J,
                                                              int L, int lane, unsigned long long *nodes_out) {
    unsigned long long nodes = 0;
    if (L == 2) {
        const unsigned long long c = wleaf<PV, INSTR, Lds>(T, rows, W, J, lane, nodes);
        if constexpr (INSTR) *nodes_out += nodes;
        return c;
    }
    WSet R[kWaveFrames];
    int Z[kWaveFrames];
    unsigned long long C[kWaveFrames];
    int f = 0;
    R[0] = J;
    C[0] = 0;
    if constexpr (INSTR) nodes += wpopc(J);
    while (true) {
        const int z = wpop(R[f], lane);
        if (z < 0) {
            if (f == 0) break;
            const unsigned long long c = C[f];
            --f;
            if constexpr (PV) {
                const unsigned long long t = wave_sum(c);
                if (lane == 0 && t) lds_add(&T->cnt[Z[f]], t);
            }
            C[f] += c;
            continue;
        }
        const WSet K = wand(R[f], wload(rows.row(z), rows.lo(z), W, lane));  // R: members above z
        const int lvl = L - f;                  // vertices to choose in frame f, z included
        if (wempty(K)) continue;
        if (lvl == 3) {
            const unsigned long long c = wleaf<PV, INSTR, Lds>(T, rows, W, K, lane, nodes);
            if constexpr (PV) {
                const unsigned long long t = wave_sum(c);
                if (lane == 0 && t) lds_add(&T->cnt[z], t);
            }
            C[f] += c;
        } else {
            if constexpr (INSTR) nodes += wpopc(K);
            Z[f] = z;
            ++f;
            R[f] = K;
            C[f] = 0;
        }
    }
    if constexpr (INSTR) *nodes_out += nodes;
    return C[0];
}

template <bool PV, bool INSTR>
__global__ void __launch_bounds__(1024) k_count_big(CountArgs a, BigArgs b) {
    using Lds = BigLds<PV>;
    constexpr int TW = Lds::TW, TT = 64 * TW;
    extern __shared__ __align__(16) unsigned char smem[];
    AS3<Lds> *T = (AS3<Lds> *)smem;
    const int tlid = threadIdx.x, lane = tlid & 63, wv = tlid >> 6;
    const uint64_t below = lanes_below_mask();
    uint32_t *grow = b.rows + (int64_t)blockIdx.x * b.team_words;
    const int64_t beg = a.seg[0], end = a.seg[1];
    const int64_t nseg = b.parts & kBigSegment ? end - beg : 0;
    unsigned long long acc = 0;
    while (true) {
        __syncthreads();
        if (tlid == 0) T->pop = atomicAdd(a.head, 1);
        __syncthreads();
        // schedule items first, then the overflowed pair items of the tier kernels
        const int64_t q = (int64_t)T->pop;
        int64_t it;
        if (q < nseg) {
            it = beg + q;
        } else {
            if (!(b.parts & kBigOverflow)) break;
            const int64_t o = q - nseg;
            const int64_t novf = (int64_t)*a.ovf_count;
            if (o >= (novf < a.ovf_cap ? novf : a.ovf_cap)) break;
            it = a.ovf_items[o];
        }
        const int32_t root = a.item_root[it];
        const int32_t child = a.item_child[it];
        const unsigned long long t_start = INSTR ? (unsigned long long)clock64() : 0ull;
        int need;
        if (child == -1) {
            const int64_t s0 = a.roff[root];
            const int64_t d64 = a.roff[root + 1] - s0;
            if (d64 > b.dbig) {
                if (tlid == 0) atomicOr(a.err, 1);
                continue;
            }
            for (int i = tlid; i < (int)d64; i += TT) T->S[i] = a.ridx[s0 + i];
            if (tlid == 0) T->d = (int)d64;
            need = a.k - 1;
        } else if (child >= 0) {
            // S = N+(root) ∩ N+(child): wave 0 walks N+(child), binary-searching N+(root)
            if (wv == 0) {
                const int64_t rs = a.roff[root], re = a.roff[root + 1];
                const int64_t cs = a.off[child], ce = a.off[child + 1];
                int cntS = 0;
                for (int64_t p0 = cs; p0 < ce; p0 += 64) {
                    const int64_t p = p0 + lane;
                    bool hit = false;
                    int32_t w = 0;
                    if (p < ce) {
                        w = a.idx[p];
                        int64_t lo = rs, hi = re;
                        while (lo < hi) {
                            const int64_t mid = lo + ((hi - lo) >> 1);
                            if (a.ridx[mid] < w) lo = mid + 1; else hi = mid;
                        }
                        hit = lo < re && a.ridx[lo] == w;
                    }
                    const uint64_t m = __ballot(hit);
                    const int pos = cntS + __popcll(m & below);
                    if (hit && pos < b.dbig) T->S[pos] = w;
                    cntS += __popcll(m);
                }
                if (cntS > b.dbig) {
                    if (lane == 0) atomicOr(a.err, 1);
                    cntS = 0;
                }
                if (lane == 0) T->d = cntS;
            }
            need = a.k - 2;
        } else {
            if (tlid == 0) atomicOr(a.err, 1);     // split parts never come here
            continue;
        }
        __syncthreads();
        const int d = T->d;
        if (d < need || d == 0) continue;          // no clique fits
        const int W = (d + 31) / 32;
        const BigRows<PV> rows{grow, (W + 3) & ~3};
        for (int i = tlid; i < Lds::HS; i += TT) T->H[i] = kEmpty;
        for (int i = tlid; i < Lds::FW; i += TT) T->flt[i] = 0u;
        if constexpr (PV)
            for (int i = tlid; i < d; i += TT) T->cnt[i] = 0ull;
        if (PV && need >= 3)
            for (int64_t i = tlid; i < rows.words(d); i += TT) grow[i] = 0u;
        if (tlid == 0) T->next = TW;
        // the zeroed rows must reach L2 before any wave's atomics
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        for (int i = tlid; i < d; i += TT) {
            hash_insert(T, (uint32_t)T->S[i], (uint32_t)i);
            const uint32_t h = big_filter_hash(T->S[i]);
            lds_or(&T->flt[h >> 5], 1u << (h & 31u));
        }
        __syncthreads();
        const int32_t first = T->S[0], last = T->S[d - 1];
        unsigned long long mine = 0, words = 0, nodes = 0;
        if (need == 1) {
            if (tlid == 0) mine = (unsigned long long)d;
            if constexpr (PV)
                for (int i = tlid; i < d; i += TT) T->cnt[i] = 1ull;
        } else if (PV || need == 2) {
            big_gather<PV, PV, false, Lds>(T, a, 0, d, need, first, last, wv, lane, rows, mine, words);
        } else {
            // upper rows, a window of rows at a time: built in LDS, then copied to the
            // team's packed rows (a wave per row, the row's stored words)
            const int RS = rows.RS;
            const int Rw = Lds::WINW / RS;              // RS <= 128: at least 96 rows
            for (int r0 = 0; r0 < d; r0 += Rw) {
                const int r1 = r0 + Rw < d ? r0 + Rw : d;
                for (int i = tlid; i < (r1 - r0) * RS; i += TT) T->win[i] = 0u;
                __syncthreads();
                big_gather<PV, false, true, Lds>(T, a, r0, r1, need, first, last, wv, lane, rows, mine, words);
                __syncthreads();
                for (int i = r0 + wv; i < r1; i += TW) {
                    uint32_t *gr = rows.row(i);
                    const AS3<uint32_t> *wr = &T->win[(i - r0) * RS];
                    for (int w = rows.lo(i) + lane; w < RS; w += 64) gr[w] = wr[w];
                }
                __syncthreads();
            }
        }
        if (need >= 3) {
            // the rows were written by all waves (global atomics, or stores of the LDS
            // windows): complete them, then read them past this CU's L1
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int pneed = need - 2;
            if (pneed == 1) {
                // k - 1 = 3: pairs through per-wave rings to the lanes, a lane per pair (the
                // lanes' rows are read from L2, word by word from y's word on)
                AS3<uint32_t> *ring = T->q.ring[wv];
                unsigned head = 0, tail = 0;
                int x = wv;
                while (x < d) {
                    const uint32_t *rx = rows.row(x);
                    const int xlo = rows.lo(x);
                    for (int cw = 0; cw < W; cw += 64) {
                        uint32_t bits = cw + lane < W && cw + lane >= xlo ? rx[cw + lane] : 0u;
                        if constexpr (PV) bits &= gtmask(x, cw + lane);      // symmetric rows
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
                                mine += big_pair<PV, Lds>(T, rows, (int)(p >> 16), (int)(p & 0xffffu));
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
                    mine += big_pair<PV, Lds>(T, rows, (int)(p >> 16), (int)(p & 0xffffu));
                    if constexpr (INSTR) nodes += 1;
                }
            } else {
                // deeper: a wave per row x, J = row x AND row y held across the lanes, walked
                // by the wave
                int x = wv;
                while (x < d) {
                    WSet rx = wload(rows.row(x), rows.lo(x), W, lane);
                    if constexpr (PV) rx = wabove(rx, x, lane);       // symmetric rows: members above x
                    WSet Y = rx;
                    unsigned long long cx = 0;                         // per-vertex: cliques through x
                    while (true) {
                        const int y = wpop(Y, lane);
                        if (y < 0) break;
                        if constexpr (INSTR) nodes += lane == 0 ? 1ull : 0ull;
                        WSet ry = wload(rows.row(y), rows.lo(y), W, lane);
                        const WSet J = PV ? wabove(wand(rx, ry), y, lane) : wand(rx, ry);
                        const unsigned long long c = wdfs<PV, INSTR, Lds>(T, rows, W, J, pneed, lane, &nodes);
                        mine += c;
                        if constexpr (PV) {
                            const unsigned long long t = wave_sum(c);
                            if (lane == 0 && t) lds_add(&T->cnt[y], t);
                            cx += t;
                        }
                    }
                    if constexpr (PV) {
                        if (lane == 0 && cx) lds_add(&T->cnt[x], cx);
                    }
                    int nx = 0;
                    if (lane == 0) nx = __hip_atomic_fetch_add(&T->next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    x = __shfl(nx, 0, 64);
                }
            }
        }
        const unsigned long long item = team_sum<TW, 1>(T, mine, wv, lane);
        const int32_t rv = a.root_ids ? a.root_ids[root] : root;     // the root vertex
        if (a.per_root != nullptr && tlid == 0 && item) atomicAdd(&a.per_root[rv], item);
        if constexpr (PV) {
            for (int i = tlid; i < d; i += TT) {
                const unsigned long long c = T->cnt[i];
                if (c) atomicAdd(&a.pv[T->S[i]], c);
            }
            if (tlid == 0 && item) {
                atomicAdd(&a.pv[rv], item);
                if (child >= 0) atomicAdd(&a.pv[child], item);
            }
        }
        if constexpr (INSTR) {
            // work label: gathered words + ceil(d/32) per search-tree node (d at depth 1)
            const unsigned long long tn = team_sum<TW, 1>(T, nodes, wv, lane);
            const unsigned long long tg = team_sum<TW, 1>(T, words, wv, lane);
            if (tlid == 0 && child < 0) a.work[rv] = tg + (unsigned long long)W * ((unsigned long long)d + tn);
            if (tlid == 0 && a.cycles) atomicAdd(&a.cycles[rv], (unsigned long long)clock64() - t_start);
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
