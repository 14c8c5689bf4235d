// Exact k-clique counting on the GPU: Alg. 1 (arb-count) and its per-vertex variant
// arb-count-v (Sec. 3.2) of Shi, Dhulipala, Shun, with the practical optimisations of
// Sec. 3.4 mapped onto gfx950:
//
//  * work item = a root v (candidate set S = N+(v), k-1 vertices still to choose), or,
//    for a root split by the scheduler, a pair (v, c) with c in N+(v)
//    (S = N+(v) ∩ N+(c), k-2 to choose) -- the paper's node vs edge parallelism;
//  * one team (1..16 waves) per item stages S in LDS, relabelled 0..d-1 in rank order
//    (Sec. 3.4: relabel the induced subgraph to [0, O(alpha))), with an LDS hash from
//    vertex id to local id standing in for the paper's mark array;
//  * the second-level intersections (the first non-trivial ones) read N+(u) for every
//    u in S from HBM with coalesced 64-lane loads and keep the members of S: this builds
//    G[S] as one bit row per local vertex (row x = neighbours of x in S above x for
//    totals at k = 4; symmetric rows, masked on use, when subtrees follow the pairs or in
//    the per-vertex mode);
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

#include <type_traits>

namespace arb {

// ------------------------------------------------------------------ tiers

// local candidate-set capacity per tier: 32 * W (W 32-bit words per bit row)
// TW waves per team, TPB teams per block, SPAN: id-range bitmap capacity (bits) used for
// the membership test when the members' ids span fewer than SPAN values (else a hash).
// The two largest tiers run 16-wave teams when counting totals at recursion depth <= 2
// (one 1024-lane block per CU keeps four waves on every SIMD within 128 VGPRs); deeper
// walks and the per-vertex variants need more registers per lane and keep 8-wave teams.
template <int W, bool PV, int LMAX> struct TierCfg {
    static_assert(W <= 32 && W % 2 == 0, "the pair phase spreads a row over 64 lanes, W / 2 < 32 bits each");
    static constexpr bool wide = !PV && LMAX <= 2;
    static constexpr int TW = W == 2 ? 1 : (W <= 8 ? 4 : (wide && W >= 16 ? 16 : 8));
    static constexpr int TPB = W == 2 ? 4 : 1;
    static constexpr int SPAN = W == 2 ? 0 : (W == 4 ? 1 << 16 : (W <= 16 ? 1 << 15 : 1 << 14));
};

template <int W, bool PV, int LMAX>
constexpr int tier_threads() {
    return 64 * TierCfg<W, PV, LMAX>::TW * TierCfg<W, PV, LMAX>::TPB;
}

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

// One list of the second level as a span of the wave's concatenated element stream:
// stream positions [end - len, end) map to idx[q + delta]; row = local id of its vertex.
struct ListEnt {
    int64_t delta;
    int64_t end;
    int32_t row;
    int32_t pad;
};

// Per-vertex counters of the 64-tier up to k = 10 fit 32 bits: a member lies in at most
// C(63, 8) < 2^32 of a root's cliques.  32-bit LDS atomics need no high word.
template <int W, int LMAX> constexpr bool cnt32() { return W == 2 && LMAX <= 7; }

template <int W, bool PV, int TW_, bool C32 = false>
struct TeamLds {
    static constexpr int D = 32 * W;             // capacity of S
    // bit rows are read with Q-word loads: 128-bit loads in the two largest tiers, 32-bit
    // loads below (measured faster there); the row stride RS is a multiple of Q with RS / Q
    // odd, so rows start 4Q-byte aligned and the rows read by 64 lanes spread over all
    // Q-bank groups of the LDS
    static constexpr int Q = W >= 16 ? 4 : 1;
    static constexpr int RS = (W / Q) % 2 == 1 ? W : W + Q;
    static constexpr int HS = pow2_at_least(D <= 128 ? 4 * D : 2 * D);
    static constexpr int HB = __builtin_ctz(HS);
    static constexpr int TW = TW_;
    // per-wave pair ring (power of two): holds a whole row on top of a partial chunk.  An
    // entry is (row << 16 | member), or in the 768-tier (slot << 10 | member) with the row
    // kept in a 64-slot table of the wave's recent non-empty rows: fewer than 64 entries
    // are ever left over from earlier rows, so a slot is reused only after its entries
    // were taken
    static constexpr int RING = pow2_at_least(D + 64);
    static constexpr bool CR = W == 24;
    using RingT = typename std::conditional<CR, uint16_t, uint32_t>::type;
    static constexpr int SPAN = TierCfg<W, PV, 1>::SPAN;
    static constexpr int SW = SPAN > 0 ? SPAN / 32 : 1;
    // in hash mode (always in the 64-tier) the second-level entries are screened with a
    // member filter before the hash probe; the id-range bitmap is as cheap as the filter
    int32_t S[D];
    unsigned long long H[HS];
    uint32_t bm[SW];        // member bitmap over ids first .. first + SPAN - 1
    uint16_t pre[SW];       // local id of the first member in each bitmap word
    uint32_t flt[64];       // 2048-bit filter of S (bit filter_hash(s) per member s)
    alignas(16) uint32_t rows[D * RS];
    using CntT = typename std::conditional<C32, uint32_t, unsigned long long>::type;
    CntT cnt[PV ? D : 1];
    union {
        RingT ring[TW][RING];       // pair phase
        ListEnt lt[TW][64];         // second level: the wave's current 64 lists
    } q;
    uint16_t xs[CR ? TW : 1][64];   // compact ring: row of each slot
    unsigned long long red[TW];
    int d;
    int pop;
    int next;               // next row to claim in the pair phase
};

// Every LDS access goes through pointers in the LDS address space, so that helpers the
// compiler keeps out of line still use DS instructions (never generic/FLAT accesses).
template <class L> using AS3 = __attribute__((address_space(3))) L;

__device__ __forceinline__ void lds_add(AS3<unsigned long long> *p, unsigned long long v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(AS3<uint32_t> *p, unsigned long long v) {
    __hip_atomic_fetch_add(p, (uint32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_or(AS3<uint32_t> *p, uint32_t v) {
    __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ unsigned long long lds_cas(AS3<unsigned long long> *p, unsigned long long expect,
                                                      unsigned long long desired) {
    __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return expect;
}

template <int W> struct Bits { uint32_t w[W]; };
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
struct Acc { unsigned long long c, nodes; };

// Words [FROM rounded down to a multiple of Q, W) of bit row z, as Q-word LDS loads; the
// words below are left unset.
template <int W, int FROM, class Lds>
__device__ __forceinline__ void load_row(const AS3<Lds> *T, int z, uint32_t (&r)[W]) {
    constexpr int Q = Lds::Q;
    static_assert(W % Q == 0 && Lds::RS % Q == 0, "rows are whole Q-word vectors");
    const AS3<uint32_t> *p = &T->rows[z * Lds::RS];
#pragma unroll
    for (int q = FROM / Q; q < W / Q; ++q) {
        if constexpr (Q == 4) {
            const u32x4 v = *reinterpret_cast<const AS3<u32x4> *>(p + 4 * q);
            r[4 * q] = v.x;
            r[4 * q + 1] = v.y;
            r[4 * q + 2] = v.z;
            r[4 * q + 3] = v.w;
        } else if constexpr (Q == 2) {
            const u32x2 v = *reinterpret_cast<const AS3<u32x2> *>(p + 2 * q);
            r[2 * q] = v.x;
            r[2 * q + 1] = v.y;
        } else {
            r[q] = p[q];
        }
    }
}

// r[w] &= word w of bit row z, for every w < W, as Q-word LDS loads
template <int W, class Lds>
__device__ __forceinline__ void and_row(const AS3<Lds> *T, int z, uint32_t (&r)[W]) {
    constexpr int Q = Lds::Q;
    const AS3<uint32_t> *p = &T->rows[z * Lds::RS];
#pragma unroll
    for (int q = 0; q < W / Q; ++q) {
        if constexpr (Q == 4) {
            const u32x4 v = *reinterpret_cast<const AS3<u32x4> *>(p + 4 * q);
            r[4 * q] &= v.x;
            r[4 * q + 1] &= v.y;
            r[4 * q + 2] &= v.z;
            r[4 * q + 3] &= v.w;
        } else {
            r[q] &= p[q];
        }
    }
}

constexpr uint64_t kEmpty = ~0ull;

__device__ __forceinline__ uint32_t hslot(uint32_t key, int hb) {
    return (key * 2654435761u) >> (32 - hb);
}

template <class L>
__device__ __forceinline__ void hash_insert(AS3<L> *T, uint32_t key, uint32_t val) {
    uint32_t s = hslot(key, L::HB);
    const uint64_t e = ((uint64_t)val << 32) | key;
    while (true) {
        unsigned long long old = lds_cas(&T->H[s], (unsigned long long)kEmpty, (unsigned long long)e);
        if (old == kEmpty) return;
        s = (s + 1) & (L::HS - 1);
    }
}

template <class L>
__device__ __forceinline__ int hash_find(const AS3<L> *T, uint32_t key) {
    uint32_t s = hslot(key, L::HB);
    while (true) {
        unsigned long long e = T->H[s];
        if (e == kEmpty) return -1;
        if ((uint32_t)e == key) return (int)(e >> 32);
        s = (s + 1) & (L::HS - 1);
    }
}

// Local id of vertex w in S, or -1: an id-range bitmap when the members span fewer
// than SPAN ids (bit test, then the first-member-in-word index plus a popcount),
// otherwise the hash.
template <class L>
__device__ __forceinline__ int member_find(const AS3<L> *T, int32_t w, int32_t first, int32_t last, bool bmode) {
    if ((uint32_t)(w - first) > (uint32_t)(last - first)) return -1;
    if constexpr (L::SPAN > 0) {
        if (bmode) {
            const uint32_t o = (uint32_t)(w - first);
            const uint32_t word = T->bm[o >> 5];
            const uint32_t bit = o & 31u;
            if (!((word >> bit) & 1u)) return -1;
            return (int)T->pre[o >> 5] + __popc(word & ((1u << bit) - 1u));
        }
    }
    return hash_find(T, (uint32_t)w);
}

// Bit of vertex id w in the 2048-bit member filter: most second-level list entries are
// not in S (on R-MAT 20, 99% in the 64-tier), and a set bit is needed for a member, so a
// clear bit rejects an entry without a hash probe.  The filter's 64 words sit one per
// lane and are read with a lane shuffle, which has no bank conflicts.
__device__ __forceinline__ uint32_t filter_hash(int32_t w) { return ((uint32_t)w * 2246822519u) >> 21; }

// bits of word w that stand for local ids greater than z
__device__ __forceinline__ uint32_t gtmask(int z, int w) {
    int zw = z >> 5, zb = z & 31;
    uint32_t hi = zb == 31 ? 0u : (~0u << (zb + 1));
    return w < zw ? 0u : (w > zw ? ~0u : hi);
}

// bits of word w that stand for local ids less than z
__device__ __forceinline__ uint32_t ltmask(int z, int w) {
    int zw = z >> 5, zb = z & 31;
    return w > zw ? 0u : (w < zw ? ~0u : ((1u << zb) - 1u));
}

// Bit rows of the induced subgraph: with subtrees below the pairs (LMAX >= 2) or per-vertex
// counts, row x holds all of x's neighbours in S (symmetric), and the pairs (x, y), x < y,
// are dealt grouped by their larger end y (column order: y's row below y).  Pairs sharing
// y draw their candidate sets from the same row, so the 64 lanes that take a step's pairs
// get subtrees of similar size.  Otherwise (k = 4 without per-vertex counts) row x holds
// only x's neighbours above x and the pairs are dealt by rows.
template <bool PV, int LMAX> constexpr bool sym_rows() { return PV || LMAX >= 2; }

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
__device__ __forceinline__ unsigned long long team_sum(AS3<Lds> *T, unsigned long long x, int wv, int lane) {
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
    const int64_t *off;            // directed CSR (rank space)
    const int32_t *idx;
    const int64_t *roff;           // root candidate sets: N+(v) (= off/idx), or any sorted subset
    const int32_t *ridx;           //   of the graph's vertices per root (peeling updates)
    int64_t n;
    int64_t m;
    int k;
    const int32_t *item_root;
    const int32_t *item_child;
    const int64_t *seg;            // [begin, end) of this tier in the item arrays
    int *head;                     // queue head (persistent)
    unsigned long long *total;
    unsigned long long *pv;        // nullable
    unsigned long long *per_root;  // nullable: cliques whose lowest-ranked vertex is the root
    unsigned long long *work;      // nullable
    unsigned long long *cycles;    // nullable (instrumented): shader clock cycles per root
    const int32_t *root_ids;       // nullable: item roots are positions in this list of vertices
    int32_t *err;
    int chunk;
    int span_max;                  // id-range bitmap used when the span is below this
    int persistent;
    int one_item_per_team;         // non-persistent launch: team g takes item begin + g
    // pair items whose set overflows the largest LDS tier are listed here for the
    // global-scratch kernel (null: no such kernel, the overflow is an error)
    int64_t *ovf_items;
    unsigned long long *ovf_count;
    int64_t ovf_cap;
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

// Number of L-cliques (L >= 2) inside the candidate set J (.c); in instrumented mode
// also the search-tree nodes under J (.nodes).  Per-vertex mode: rows are symmetric
// adjacency and members gain their share through cnt.  Levels L >= 4 stay out of line
// to bound code size.
template <int W, bool PV, bool INSTR, int L, class Lds>
__device__ Acc dfs_body(AS3<Lds> *T, Bits<W> J);

template <int W, bool PV, bool INSTR, int L, class Lds>
__device__ __forceinline__ Acc dfs(AS3<Lds> *T, Bits<W> J) {
    return dfs_body<W, PV, INSTR, L, Lds>(T, J);
}

// The 64-tier (W = 2: local ids < 64) walks its sets as 64-bit words: one find-first-set
// per member, one 8-byte row read, and the leaf takes two members per step so that their
// row reads are in flight together.
template <class Lds>
__device__ __forceinline__ uint64_t row64(const AS3<Lds> *T, int z) {
    const AS3<uint32_t> *p = &T->rows[z * Lds::RS];
    return (uint64_t)p[0] | ((uint64_t)p[1] << 32);
}

template <bool PV, bool INSTR, int L, class Lds>
__device__ __forceinline__ Acc dfs64(AS3<Lds> *T, uint64_t J);

template <bool PV, bool INSTR, int L, class Lds>
__device__ __attribute__((noinline)) Acc dfs64_body(AS3<Lds> *T, uint64_t J) {
    return dfs64<PV, INSTR, L, Lds>(T, J);
}

template <bool PV, bool INSTR, int L, class Lds>
__device__ __forceinline__ Acc dfs64(AS3<Lds> *T, uint64_t J) {
    Acc out{0ull, 0ull};
    if constexpr (INSTR) out.nodes += (unsigned long long)__popcll(J);
    uint64_t R = J;                         // members not taken yet: those above the last one
    if constexpr (L == 2) {
        unsigned leaf = 0;
        while (R) {
            const int z1 = __builtin_ctzll(R);
            R &= R - 1;
            const uint64_t above1 = R;
            const bool two = R != 0;
            const int z2 = two ? __builtin_ctzll(R) : z1;
            R &= R - 1;
            const uint64_t r1 = row64(T, z1), r2 = row64(T, z2);
            if constexpr (PV) {
                // each member belongs to as many of the node's cliques as it has neighbours
                // in J (the rows are symmetric), and the node's cliques, the edges of J, are
                // half the sum of those: no separate count of the neighbours above
                const unsigned a1 = (unsigned)__popcll(J & r1);
                if (a1) lds_add(&T->cnt[z1], (unsigned long long)a1);
                const unsigned a2 = two ? (unsigned)__popcll(J & r2) : 0u;
                if (a2) lds_add(&T->cnt[z2], (unsigned long long)a2);
                leaf += a1 + a2;
                (void)above1;
            } else {
                leaf += (unsigned)__popcll(above1 & r1) + (unsigned)__popcll(R & r2);   // R = 0 unless two
            }
        }
        out.c += PV ? leaf >> 1 : leaf;
    } else {
        while (R) {
            const int z = __builtin_ctzll(R);
            R &= R - 1;
            const uint64_t K = R & row64(T, z);
            Acc sub;
            if constexpr (L - 1 <= 3) sub = dfs64<PV, INSTR, L - 1, Lds>(T, K);
            else sub = dfs64_body<PV, INSTR, L - 1, Lds>(T, K);
            if constexpr (PV) {
                if (sub.c) lds_add(&T->cnt[z], sub.c);
            }
            out.c += sub.c;
            out.nodes += sub.nodes;
        }
    }
    return out;
}

template <int W, bool PV, bool INSTR, int L, class Lds>
__device__ __attribute__((always_inline)) inline Acc dfs_inline(AS3<Lds> *T, const Bits<W> &J) {
    if constexpr (W == 2) return dfs64<PV, INSTR, L, Lds>(T, (uint64_t)J.w[0] | ((uint64_t)J.w[1] << 32));
    Acc out{0ull, 0ull};
    if constexpr (INSTR) {
        unsigned c = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) c += __popc(J.w[w]);
        out.nodes += c;
    }
    if constexpr (L == 2 && !PV) {
        // leaf level: member z of J adds the edges from z to the members of J above z.
        // Members are taken in ascending order, so the bits of z's word still to be taken
        // are J's members above z in that word; the AND covers that word and the words
        // above it (the vectors below z's are never loaded).  The leaf's sum is below
        // 768 * 768 / 2, so it is kept in 32 bits
        unsigned leaf = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            uint32_t bits = J.w[w];
            if constexpr (Lds::TW >= 16) {
                // 16-wave teams: 128 VGPRs, one member per step
                while (bits) {
                    const int z = w * 32 + __ffs(bits) - 1;
                    bits &= bits - 1;
                    uint32_t r[W];
                    load_row<W, 0, Lds>(T, z, r);
                    leaf += __popc(bits & r[w]);
#pragma unroll
                    for (int v = w + 1; v < W; ++v) leaf += __popc(J.w[v] & r[v]);
                }
            } else {
                while (bits) {
                    // two members per step, so that the second row's loads overlap the first's
                    const int z1 = w * 32 + __ffs(bits) - 1;
                    bits &= bits - 1;
                    const uint32_t above1 = bits;
                    const bool two = bits != 0;
                    const int z2 = two ? w * 32 + __ffs(bits) - 1 : z1;
                    bits &= bits - 1;
                    uint32_t r1[W], r2[W];
                    load_row<W, 0, Lds>(T, z1, r1);
                    load_row<W, 0, Lds>(T, z2, r2);
                    unsigned c2 = __popc(bits & r2[w]);
                    leaf += __popc(above1 & r1[w]);
#pragma unroll
                    for (int v = w + 1; v < W; ++v) {
                        leaf += __popc(J.w[v] & r1[v]);
                        c2 += __popc(J.w[v] & r2[v]);
                    }
                    leaf += two ? c2 : 0u;
                }
            }
        }
        out.c += leaf;
        return out;
    }
    uint32_t R[W];
#pragma unroll
    for (int w = 0; w < W; ++w) R[w] = J.w[w];
    while (true) {
        int z = pop_lowest<W>(R);
        if (z < 0) break;
        uint32_t rz[W];
        load_row<W, 0, Lds>(T, z, rz);
        if constexpr (L == 2) {
            // per-vertex leaf level (symmetric rows): z's neighbours in J are its credit, and
            // the node's count, the edges of J, is half the sum of the credits
            unsigned a = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) a += __popc(J.w[w] & rz[w]);
            if (a) lds_add(&T->cnt[z], (unsigned long long)a);
            out.c += a;
        } else {
            Bits<W> K;
#pragma unroll
            for (int w = 0; w < W; ++w) K.w[w] = R[w] & rz[w];   // R: J's members above z
            Acc sub;
            if constexpr (L - 1 <= 3) sub = dfs_inline<W, PV, INSTR, L - 1, Lds>(T, K);
            else sub = dfs_body<W, PV, INSTR, L - 1, Lds>(T, K);
            if constexpr (PV) {
                if (sub.c) lds_add(&T->cnt[z], sub.c);
            }
            out.c += sub.c;
            out.nodes += sub.nodes;
        }
    }
    if constexpr (L == 2) out.c >>= 1;      // every edge of J was counted from both ends
    return out;
}

template <int W, bool PV, bool INSTR, int L, class Lds>
__device__ __attribute__((noinline)) Acc dfs_body(AS3<Lds> *T, Bits<W> J) {
    return dfs_inline<W, PV, INSTR, L, Lds>(T, J);
}

// Walks with more than 7 vertices still to choose (k > 10): the levels down to the fourth
// keep their untaken candidates in a stack of frames in private memory instead of in the
// registers of nested calls, so that one function serves every depth up to ARB_MAX_K - 3;
// the last three levels run inline.  Frame f holds the set from which L - f vertices are
// still to be chosen.  Without instrumentation a frame whose set has fewer members than
// vertices to choose is not entered (it holds no clique).
constexpr int kDeepFrames = ARB_MAX_K - 6;
constexpr int kDeepMin = 8;

template <int W, bool PV, bool INSTR, class Lds>
__device__ __attribute__((noinline)) Acc dfs_deep(AS3<Lds> *T, Bits<W> J, int L) {
    uint32_t R[kDeepFrames][W];
    int Z[kDeepFrames];
    unsigned long long C[kDeepFrames], N[kDeepFrames];
    int f = 0;
    unsigned pc0 = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        R[0][w] = J.w[w];
        pc0 += __popc(J.w[w]);
    }
    C[0] = 0;
    N[0] = INSTR ? pc0 : 0;
    while (true) {
        int z = -1;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (z < 0 && R[f][w]) {
                z = w * 32 + __ffs(R[f][w]) - 1;
                R[f][w] &= R[f][w] - 1;
            }
        }
        if (z < 0) {                       // frame f done: credit the parent's chosen vertex
            if (f == 0) return Acc{C[0], N[0]};
            const unsigned long long c = C[f], nn = N[f];
            --f;
            if constexpr (PV) {
                if (c) lds_add(&T->cnt[Z[f]], c);
            }
            C[f] += c;
            N[f] += nn;
            continue;
        }
        uint32_t rz[W];
        load_row<W, 0, Lds>(T, z, rz);
        Bits<W> K;
        unsigned pc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            K.w[w] = R[f][w] & rz[w];      // R: the frame's members above z
            pc += __popc(K.w[w]);
        }
        const int lvl = L - f;             // vertices to choose in frame f, z included
        if (lvl == 4) {
            const Acc sub = dfs_inline<W, PV, INSTR, 3, Lds>(T, K);
            if constexpr (PV) {
                if (sub.c) lds_add(&T->cnt[z], sub.c);
            }
            C[f] += sub.c;
            N[f] += sub.nodes;
        } else {
            if (!INSTR && pc < (unsigned)(lvl - 1)) continue;
            Z[f] = z;
            ++f;
#pragma unroll
            for (int w = 0; w < W; ++w) R[f][w] = K.w[w];
            C[f] = 0;
            N[f] = INSTR ? pc : 0;
        }
    }
}

template <int W, int LMAX, bool PV, bool INSTR, class Lds>
__device__ __forceinline__ Acc dfs_dispatch(AS3<Lds> *T, const Bits<W> &J, int L) {
    if constexpr (LMAX >= 2) if (L == 2) return dfs_inline<W, PV, INSTR, 2, Lds>(T, J);
    if constexpr (LMAX >= 3) if (L == 3) return dfs_inline<W, PV, INSTR, 3, Lds>(T, J);
    if constexpr (LMAX >= 4) if (L == 4) return dfs_body<W, PV, INSTR, 4, Lds>(T, J);
    if constexpr (LMAX >= 5) if (L == 5) return dfs_body<W, PV, INSTR, 5, Lds>(T, J);
    if constexpr (LMAX >= 6) if (L == 6) return dfs_body<W, PV, INSTR, 6, Lds>(T, J);
    if constexpr (LMAX >= 7) if (L == 7) return dfs_body<W, PV, INSTR, 7, Lds>(T, J);
    if constexpr (LMAX >= kDeepMin) if (L >= kDeepMin) return dfs_deep<W, PV, INSTR, Lds>(T, J, L);
    return Acc{0ull, 0ull};
}
static_assert(ARB_MAX_K - 3 - kDeepMin + 4 <= kDeepFrames, "dfs_deep's frames cover L up to ARB_MAX_K - 3");

// One pair (x, y) of the induced subgraph, x < y, both chosen: count the cliques that
// extend it with `need` more vertices from S (need >= 1); .nodes as in dfs.
template <int W, int LMAX, bool PV, bool INSTR, class Lds>
__device__ __forceinline__ Acc do_pair(AS3<Lds> *T, int x, int y, int need) {
    constexpr bool SYM = sym_rows<PV, LMAX>();
    Acc out{0ull, INSTR ? 1ull : 0ull};
    if (LMAX >= 2 && need >= 2) {
        // J = row x AND row y (above y), ANDed in place one Q-word vector at a time so
        // that the two rows are never held in registers together
        Bits<W> J;
        load_row<W, 0, Lds>(T, x, J.w);
        and_row<W, Lds>(T, y, J.w);
        if constexpr (SYM) {
#pragma unroll
            for (int w = 0; w < W; ++w) J.w[w] &= gtmask(y, w);
        }
        const Acc sub = dfs_dispatch<W, LMAX, PV, INSTR, Lds>(T, J, need);
        if constexpr (PV) {
            if (sub.c) {
                lds_add(&T->cnt[x], sub.c);
                lds_add(&T->cnt[y], sub.c);
            }
        }
        out.c = sub.c;
        out.nodes += sub.nodes;
        return out;
    }
    uint32_t rx[W], ry[W];
    load_row<W, 0, Lds>(T, x, rx);
    load_row<W, 0, Lds>(T, y, ry);
    {
        if constexpr (PV) {
            unsigned a = 0, c = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                uint32_t t = rx[w] & ry[w];
                a += __popc(t & gtmask(x, w));
                c += __popc(t & gtmask(y, w));
            }
            if (a) lds_add(&T->cnt[y], (unsigned long long)a);
            if (c) lds_add(&T->cnt[x], (unsigned long long)c);
            out.c = c;
        } else {
            unsigned c = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) c += __popc(rx[w] & ry[w] & (SYM ? gtmask(y, w) : ~0u));
            out.c = c;
        }
        return out;
    }
}

// ------------------------------------------------------------------ second level

// independent 4-byte loads in flight per lane: 8, or 4 in the 128-tier, whose kernels
// then fit 5 waves per SIMD (measured faster there)
template <int W> constexpr int gather_unroll() { return W == 4 ? 4 : 8; }

// Second level of the recursion: for the lists N+(S[i]), i = g0, g0 + gstep, ... < d,
// keep the entries that are members of S.  A wave takes 64 lists at a time, concatenates
// them into one element stream and consumes it 64 * gather_unroll entries per step, each
// lane walking its own cursor through the list table in LDS, so that short and long
// lists alike keep gather_unroll loads per lane in flight.
template <int W, bool PV, bool SYM, class Lds>
__device__ __forceinline__ void gather_lists(AS3<Lds> *T, const CountArgs &a, int d, int need, int g0, int gstep,
                                             int32_t first, int32_t last, bool bmode, int wv, int lane,
                                             unsigned long long &mine, unsigned long long &words) {
    AS3<ListEnt> *lt = T->q.lt[wv];
    const uint32_t fw = bmode ? 0u : T->flt[lane];          // this lane's word of the member filter
    const int nl = g0 < d ? (d - g0 + gstep - 1) / gstep : 0;
    for (int gb = 0; gb < nl; gb += 64) {
        const int t = gb + lane;
        int64_t s = 0, e = 0;
        int row = 0;
        if (t < nl) {
            row = g0 + gstep * t;
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
        int c = 0;                                  // this lane's cursor into the table
        int64_t c_end = lt[0].end;
        int64_t c_delta = lt[0].delta;
        int c_row = lt[0].row;
        constexpr int GU = gather_unroll<W>();
        for (int64_t base = 0; base < total; base += 64 * GU) {
            int32_t w[GU];
            int r[GU];
#pragma unroll
            for (int q = 0; q < GU; ++q) {
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
            bool maybe[GU];
            if (bmode) {
#pragma unroll
                for (int q = 0; q < GU; ++q) maybe[q] = true;
            } else {
#pragma unroll
                for (int q = 0; q < GU; ++q) {
                    const uint32_t h = filter_hash(w[q]);
                    maybe[q] = (__shfl(fw, (int)(h >> 5), 64) >> (h & 31u)) & 1u;
                }
            }
#pragma unroll
            for (int q = 0; q < GU; ++q) {
                if (!maybe[q]) continue;
                const int j = member_find(T, w[q], first, last, bmode);
                if (j < 0) continue;
                const int i = r[q];
                if (need == 2) {
                    mine += 1;
                    if constexpr (PV) {
                        lds_add(&T->cnt[j], 1ull);
                        lds_add(&T->cnt[i], 1ull);
                    }
                } else {
                    lds_or(&T->rows[i * Lds::RS + (j >> 5)], 1u << (j & 31));
                    if constexpr (SYM) lds_or(&T->rows[j * Lds::RS + (i >> 5)], 1u << (i & 31));
                }
            }
        }
        wave_fence();                               // table reused by the next 64 lists
    }
}

// ------------------------------------------------------------------ one work item

template <int W, int LMAX, bool PV, bool INSTR>
__device__ __forceinline__ unsigned long long process_item(AS3<TeamLds<W, PV, TierCfg<W, PV, LMAX>::TW, cnt32<W, LMAX>()>> *T,
                                                             const CountArgs a, int64_t it, int32_t root,
                                                             int32_t child, int tlid) {
    using Cfg = TierCfg<W, PV, LMAX>;
    constexpr int TW = Cfg::TW, TPB = Cfg::TPB;
    using Lds = TeamLds<W, PV, TW, cnt32<W, LMAX>()>;
    constexpr int TT = 64 * TW;
    const int lane = tlid & 63, wv = tlid >> 6;
    const uint64_t below = lanes_below_mask();

    team_sync<TW, TPB>();            // previous item finished with the LDS
    const unsigned long long t_start = INSTR ? (unsigned long long)clock64() : 0ull;
    // child >= 0: the pair item (root, child); child == -1: the whole root; child <= -2:
    // part `part` of P of a split root, which takes every P-th row of the root's work
    int P = 1, part = 0;
    if (child < -1) {
        const int q = -child - 2;
        P = q & 127;
        part = q >> 7;
    }
    int need;
    if (child < 0) {
        const int64_t s0 = a.roff[root];
        const int64_t d = a.roff[root + 1] - s0;
        if (d > Lds::D) {
            if (tlid == 0) atomicOr(a.err, 1);
            return 0;
        }
        for (int i = tlid; i < d; i += TT) T->S[i] = a.ridx[s0 + i];
        if (tlid == 0) T->d = (int)d;
        need = a.k - 1;
    } else {
        // S = N+(root) ∩ N+(child): wave 0 walks N+(child) and binary-searches N+(root)
        if (wv == 0) {
            const int64_t rs = a.roff[root], re = a.roff[root + 1];
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
                        if (a.ridx[mid] < w) lo = mid + 1; else hi = mid;
                    }
                    hit = lo < re && a.ridx[lo] == w;
                }
                uint64_t m = __ballot(hit);
                int pos = cntS + __popcll(m & below);
                if (hit && pos < Lds::D) T->S[pos] = w;
                cntS += __popcll(m);
            }
            if (cntS > Lds::D) {
                // too large for LDS: the global-scratch kernel (run after the tiers) takes it
                if (lane == 0) {
                    const unsigned long long o = a.ovf_items ? atomicAdd(a.ovf_count, 1ull) : ~0ull;
                    if (o < (unsigned long long)a.ovf_cap) a.ovf_items[o] = it;
                    else atomicOr(a.err, 1);
                }
                cntS = 0;
            }
            if (lane == 0) T->d = cntS;
        }
        need = a.k - 2;
    }
    team_sync<TW, TPB>();
    const int d = T->d;
    if (d < need || d == 0) return 0;   // no clique fits (need >= 1 here)

    const int32_t first = T->S[0], last = T->S[d - 1];
    bool bmode = false;
    if constexpr (Lds::SPAN > 0)
        bmode = (int64_t)last - (int64_t)first < (int64_t)min(Lds::SPAN, a.span_max);
    if (bmode) {
        const int nw = ((last - first) >> 5) + 1;
        for (int i = tlid; i < nw; i += TT) T->bm[i] = 0u;
    } else {
        for (int i = tlid; i < Lds::HS; i += TT) T->H[i] = kEmpty;
    }
    if (!bmode)
        for (int i = tlid; i < 64; i += TT) T->flt[i] = 0u;
    if (need >= 3)
        for (int i = tlid; i < d * Lds::RS; i += TT) T->rows[i] = 0u;
    if (tlid == 0) T->next = TW;
    if constexpr (PV)
        for (int i = tlid; i < d; i += TT) T->cnt[i] = 0ull;
    team_sync<TW, TPB>();
    if (bmode) {
        for (int i = tlid; i < d; i += TT) {
            const uint32_t o = (uint32_t)(T->S[i] - first);
            lds_or(&T->bm[o >> 5], 1u << (o & 31u));
            if (i == 0 || ((uint32_t)(T->S[i - 1] - first) >> 5) != (o >> 5)) T->pre[o >> 5] = (uint16_t)i;
        }
    } else {
        for (int i = tlid; i < d; i += TT) {
            hash_insert(T, (uint32_t)T->S[i], (uint32_t)i);
            const uint32_t h = filter_hash(T->S[i]);
            lds_or(&T->flt[h >> 5], 1u << (h & 31u));
        }
    }
    team_sync<TW, TPB>();

    unsigned long long mine = 0;      // this lane's share of the item's clique count
    unsigned long long nodes = 0;     // instrumented: search-tree nodes (depth <= k-2)
    unsigned long long gather = 0;    // instrumented: words of N+(u) lists

    if (need == 1) {
        if (tlid == 0) mine = (unsigned long long)d;
        if constexpr (PV)
            for (int i = tlid; i < d; i += TT) T->cnt[i] = 1ull;
    } else {
        // second level; with k-1 = 2 (no bit rows) the gather is the whole work, so parts
        // split its lists
        const int g0 = need == 2 ? part + P * wv : wv, gstep = need == 2 ? P * TW : TW;
        unsigned long long words = 0;
        gather_lists<W, PV, sym_rows<PV, LMAX>(), Lds>(T, a, d, need, g0, gstep, first, last, bmode, wv, lane, mine, words);
        if constexpr (INSTR) gather += words;
        if constexpr (INSTR) {
            if (tlid == 0) nodes += (unsigned long long)d;     // depth-1 nodes
        }
        if (need >= 3) {
            team_sync<TW, TPB>();
            // pairs (x, y), x < y adjacent, spread over the lanes through the wave's ring,
            // a row r at a time: r = x with its members above x (upper rows), or r = y with
            // its members below y (symmetric rows).  When subtrees lie below the pairs
            // (pneed >= 2) the waves of a team claim rows in ascending order from a team
            // counter, one claim ahead; otherwise rows are dealt round-robin
            constexpr bool SYM = sym_rows<PV, LMAX>();
            using RingT = typename Lds::RingT;
            AS3<RingT> *ring = T->q.ring[wv];
            unsigned head = 0, tail = 0;          // ring positions [head, tail) not yet taken
            const int pneed = need - 2;
            unsigned slot = 0;
            // 64-tier, at least four vertices below each pair (k >= 7): the lanes deal
            // triples (x, y, z), z a member of the pair's common set above both, through a
            // second ring in the (now unused) hash table, so that the subtrees the lanes
            // walk side by side are one level smaller and vary less than whole pair
            // subtrees.  With three vertices below (k = 6) the extra pass costs more than
            // the better balance gains
            constexpr bool TRIPLES = W == 2 && !INSTR && LMAX >= 4;
            const bool triples = TRIPLES && pneed >= 4;
            AS3<uint32_t> *ring3 = reinterpret_cast<AS3<uint32_t> *>(&T->H[0]);
            constexpr unsigned RING3 = 2 * Lds::HS;          // 512 entries of x | y << 6 | z << 12
            unsigned head3 = 0, tail3 = 0;
            auto take3 = [&](uint32_t e) {
                const int x = (int)(e & 63u), y = (int)((e >> 6) & 63u), z = (int)(e >> 12);
                const uint64_t K = row64(T, x) & row64(T, y) & row64(T, z) & ~((2ull << z) - 1ull);
                Bits<W> KB;
                KB.w[0] = (uint32_t)K;
                KB.w[1] = (uint32_t)(K >> 32);
                const Acc sub = dfs_dispatch<W, LMAX, PV, INSTR, Lds>(T, KB, pneed - 1);
                if constexpr (PV) {
                    if (sub.c) {
                        lds_add(&T->cnt[x], sub.c);
                        lds_add(&T->cnt[y], sub.c);
                        lds_add(&T->cnt[z], sub.c);
                    }
                }
                mine += sub.c;
            };
            // every lane of the wave: its pair (valid or not) goes into the triple ring; the
            // pair is (row << 16 | member) of either row kind, and both kinds give the same
            // set above the larger of the two
            auto deal3 = [&](uint32_t p, bool valid) {
                const int py = (int)(p >> 16), px = (int)(p & 0xffffu);
                const int hi = py > px ? py : px;
                uint64_t R = valid ? row64(T, px) & row64(T, py) & ~((2ull << hi) - 1ull) : 0ull;
                const uint32_t base = (uint32_t)px | ((uint32_t)py << 6);
                while (true) {
                    const unsigned c = (unsigned)__popcll(R);
                    unsigned pre = c;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const unsigned t = __shfl_up(pre, o, 64);
                        if (lane >= o) pre += t;
                    }
                    const unsigned total = __shfl(pre, 63, 64);
                    if (total == 0) break;
                    const unsigned space = RING3 - (tail3 - head3);
                    const unsigned start = pre - c;
                    unsigned cnt = start >= space ? 0u : (c < space - start ? c : space - start);
                    unsigned pos = tail3 + start;
                    while (cnt) {
                        const int z = __builtin_ctzll(R);
                        R &= R - 1;
                        ring3[pos & (RING3 - 1)] = base | ((uint32_t)z << 12);
                        ++pos;
                        --cnt;
                    }
                    tail3 += total < space ? total : space;
                    wave_fence();
                    while (tail3 - head3 >= 64) {
                        take3(ring3[(head3 + lane) & (RING3 - 1)]);
                        head3 += 64;
                    }
                    wave_fence();
                }
            };
            auto take = [&](uint32_t p) {
                int pr, pm;          // the entry's row and member
                if constexpr (Lds::CR) {
                    pr = T->xs[wv][p >> 10];
                    pm = (int)(p & 1023u);
                } else {
                    pr = (int)(p >> 16);
                    pm = (int)(p & 0xffffu);
                }
                const int px = SYM ? pm : pr, py = SYM ? pr : pm;
                const Acc r = do_pair<W, LMAX, PV, INSTR, Lds>(T, px, py, pneed);
                mine += r.c;
                nodes += r.nodes;
            };
            const bool dyn = TW > 1 && pneed >= 2;
            int xi = wv, claim = 0;
            if (dyn && lane == 0)
                claim = __hip_atomic_fetch_add(&T->next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            while (true) {
                const int row = part + P * xi;
                if (row >= d) break;
                // lane l expands bits [l B, l B + B) of the row, B = W / 2, so that a dense
                // row costs at most B steps
                constexpr int B = W / 2;
                const int g = lane * B;
                uint32_t bits;
                {
                    const AS3<uint32_t> *rw = &T->rows[row * Lds::RS + (g >> 5)];
                    const int sh = g & 31;
                    uint64_t win = rw[0];
                    if (sh + B > 32) win |= (uint64_t)rw[1] << 32;
                    bits = (uint32_t)(win >> sh) & (uint32_t)((1ull << B) - 1);
                    if constexpr (SYM) {
                        const int lim = row - g;     // members below the row's own id
                        bits &= lim >= B ? ~0u : (lim <= 0 ? 0u : ((1u << lim) - 1u));
                    }
                }
                const unsigned c = __popc(bits);
                unsigned pre = c;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const unsigned y = __shfl_up(pre, o, 64);
                    if (lane >= o) pre += y;
                }
                const unsigned end = tail + __shfl(pre, 63, 64);
                unsigned pos = tail + pre - c;
                uint32_t tag;
                if constexpr (Lds::CR) {
                    if (end != tail) {
                        slot = (slot + 1) & 63u;
                        if (lane == 0) T->xs[wv][slot] = (uint16_t)row;
                    }
                    tag = slot << 10;
                } else {
                    tag = (uint32_t)row << 16;
                }
                while (bits) {
                    const int b = __ffs(bits) - 1;
                    bits &= bits - 1;
                    ring[pos & (Lds::RING - 1)] = (RingT)(tag | (uint32_t)(g + b));
                    ++pos;
                }
                wave_fence();
                while (end - head >= 64) {
                    if (triples) deal3(ring[(head + lane) & (Lds::RING - 1)], true);
                    else take(ring[(head + lane) & (Lds::RING - 1)]);
                    head += 64;
                }
                wave_fence();
                tail = end;
                if (dyn) {
                    xi = __shfl(claim, 0, 64);
                    if (lane == 0 && part + P * xi < d)
                        claim = __hip_atomic_fetch_add(&T->next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    xi += TW;
                }
            }
            if (triples) {
                if (tail != head) deal3(ring[(head + lane) & (Lds::RING - 1)], lane < (int)(tail - head));
                if (tail3 != head3 && lane < (int)(tail3 - head3)) take3(ring3[(head3 + lane) & (RING3 - 1)]);
            } else if (tail != head && lane < (int)(tail - head)) {
                take(ring[(head + lane) & (Lds::RING - 1)]);
            }
        }
    }

    unsigned long long item = 0;
    const int32_t rv = a.root_ids ? a.root_ids[root] : root;     // the root vertex
    if (PV || a.per_root != nullptr) item = team_sum<TW, TPB>(T, mine, wv, lane);
    if (a.per_root != nullptr && tlid == 0 && item) atomicAdd(&a.per_root[rv], item);
    if constexpr (PV || INSTR) {
        if constexpr (PV) {
            for (int i = tlid; i < d; i += TT) {
                unsigned long long c = T->cnt[i];
                if (c) atomicAdd(&a.pv[T->S[i]], c);
            }
            if (tlid == 0 && item) {
                atomicAdd(&a.pv[rv], item);
                if (child >= 0) atomicAdd(&a.pv[child], item);
            }
        }
        if constexpr (INSTR) {
            const unsigned long long tn = team_sum<TW, TPB>(T, nodes, wv, lane);
            const unsigned long long tg = team_sum<TW, TPB>(T, gather, wv, lane);
            if (tlid == 0 && child < 0) a.work[rv] = tg + (unsigned long long)((d + 31) / 32) * tn;
            if (tlid == 0 && a.cycles) atomicAdd(&a.cycles[rv], (unsigned long long)clock64() - t_start);
        }
    }
    return mine;
}

// Waves per SIMD the register allocation must allow: in the two smallest tiers the
// latency of the list reads and of the LDS row reads of the walk dominates, and more
// resident waves hide more of it (measured: 5 beats the 3-4 that their register use would
// give, at every depth, for totals and per-vertex counts alike; 6 is slower)
template <int W, bool PV, int LMAX> constexpr int tier_min_waves() {
    return W == 2 || W == 4 ? 5 : 1;
}

template <int W, int LMAX, bool PV, bool INSTR>
__global__ void __launch_bounds__((tier_threads<W, PV, LMAX>()))
__attribute__((amdgpu_waves_per_eu(tier_min_waves<W, PV, LMAX>())))
k_count(CountArgs a) {
    using Cfg = TierCfg<W, PV, LMAX>;
    constexpr int TW = Cfg::TW, TPB = Cfg::TPB;
    using Lds = TeamLds<W, PV, TW, cnt32<W, LMAX>()>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int team = threadIdx.x / (64 * TW);
    const int tlid = threadIdx.x % (64 * TW);
    AS3<Lds> *T = (AS3<Lds> *)(smem + (size_t)team * ((sizeof(Lds) + 15) & ~size_t(15)));
    const int64_t beg = a.seg[0], end = a.seg[1];
    unsigned long long acc = 0;
    const int64_t gteam = (int64_t)blockIdx.x * TPB + team;
    if (a.one_item_per_team) {
        int64_t it = beg + gteam;
        if (it < end) acc += process_item<W, LMAX, PV, INSTR>(T, a, it, a.item_root[it], a.item_child[it], tlid);
    } else if (!a.persistent) {
        const int64_t nteams = (int64_t)gridDim.x * TPB;
        for (int64_t it = beg + gteam; it < end; it += nteams)
            acc += process_item<W, LMAX, PV, INSTR>(T, a, it, a.item_root[it], a.item_child[it], tlid);
    } else {
        while (true) {
            team_sync<TW, TPB>();
            if (tlid == 0) T->pop = atomicAdd(a.head, a.chunk);
            team_sync<TW, TPB>();
            const int64_t first = beg + (int64_t)T->pop;
            if (first >= end) break;
            const int64_t last = min(first + (int64_t)a.chunk, end);
            for (int64_t it = first; it < last; ++it)
                acc += process_item<W, LMAX, PV, INSTR>(T, a, it, a.item_root[it], a.item_child[it], tlid);
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(a.total, acc);
}

template <int W, bool PV, int LMAX>
constexpr size_t block_lds() {
    using Cfg = TierCfg<W, PV, LMAX>;
    return ((sizeof(TeamLds<W, PV, Cfg::TW, cnt32<W, LMAX>()>) + 15) & ~size_t(15)) * Cfg::TPB;
}

template <int W>
constexpr bool tier_fits_lds() {
    return block_lds<W, true, 1>() <= 160 * 1024 && block_lds<W, false, 1>() <= 160 * 1024 &&
           block_lds<W, true, kDeepMin>() <= 160 * 1024 && block_lds<W, false, kDeepMin>() <= 160 * 1024;
}
static_assert(tier_fits_lds<2>() && tier_fits_lds<4>() && tier_fits_lds<8>() && tier_fits_lds<12>() &&
                  tier_fits_lds<16>() && tier_fits_lds<24>(), "a tier's block exceeds the CU's LDS");

template <int W, int LMAX, bool PV, bool INSTR>
static int launch_tier(const CountArgs &a, unsigned grid, hipStream_t s) {
    constexpr int TW = TierCfg<W, PV, LMAX>::TW, TPB = TierCfg<W, PV, LMAX>::TPB;
    const size_t lds = block_lds<W, PV, LMAX>();
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

inline int tier_teams_per_block(int tier) { return tier == 0 ? TierCfg<2, false, 1>::TPB : 1; }

template <int W>
constexpr size_t tier_lds_of(bool pv, int lmax) {
    return pv ? (lmax <= 2 ? block_lds<W, true, 1>() : block_lds<W, true, 3>())
              : (lmax <= 2 ? block_lds<W, false, 1>() : block_lds<W, false, 3>());
}

// LDS bytes of one block of the tier's kernel at recursion depth lmax
inline size_t tier_block_lds(int tier, bool pv, int lmax) {
    switch (tier) {
        case 0: return tier_lds_of<2>(pv, lmax);
        case 1: return tier_lds_of<4>(pv, lmax);
        case 2: return tier_lds_of<8>(pv, lmax);
        case 3: return tier_lds_of<12>(pv, lmax);
        case 4: return tier_lds_of<16>(pv, lmax);
        default: return tier_lds_of<24>(pv, lmax);
    }
}

// Items whose candidate set exceeds ARB_MAX_LOCAL (count_big.hip): one 16-wave team per
// item, S and its hash in LDS, the bit rows of G[S] in a per-team slice of global scratch
// (L2 / Infinity Cache resident), up to kBigMax vertices.
constexpr int kBigMax = 4096;
constexpr int kBigSegment = 1;     // a launch takes the schedule's items of the big tier
constexpr int kBigOverflow = 2;    // ... and / or the pair items the tier kernels overflowed
struct BigArgs {
    uint32_t *rows;        // scratch: teams x team_words words
    int64_t team_words;
    int dbig;              // roots with ARB_MAX_LOCAL < d+ <= dbig and overflowed pair
                           // sets up to dbig take this path
    int parts;             // kBigSegment | kBigOverflow
};

// Largest out-degree the peel can produce on m edges: d(d+1) <= 2(2+eps)m, so at eps = 1
// d < sqrt(6m) (larger eps: such roots fall back to per-out-neighbour items).
inline int big_dmax(int64_t m) {
    double r = 1.0;
    while (r * r < 6.0 * (double)m && r < kBigMax) r += 1.0;
    const int d = (int)r;
    return d > ARB_MAX_LOCAL ? (d < kBigMax ? d : kBigMax) : 0;
}
// at most m / (ARB_MAX_LOCAL + 1) roots can be that large
inline int64_t big_teams(int64_t m) {
    const int64_t t = m / (ARB_MAX_LOCAL + 1);
    return big_dmax(m) == 0 ? 0 : (t < 1 ? 1 : (t > 256 ? 256 : t));
}
// rows of ceil(dbig / 32) words padded to a multiple of 4 (16-byte rows)
inline int64_t big_team_words(int dbig) { return (int64_t)dbig * ((((dbig + 31) / 32) + 3) & ~3); }

int launch_count_big(bool pv, bool instr, const CountArgs &a, const BigArgs &b, unsigned grid, hipStream_t s);

// count.hip: the counting driver with optional per-root candidate sets (see there)
int count_with_roots(const arb_ocsr *dg, int k, uint64_t *total_dev, uint64_t *per_vertex, uint64_t *per_root_out,
                     uint64_t *work_out, const arb_count_opts *opts_in, void *ws, size_t ws_bytes, hipStream_t s,
                     const int64_t *roff, const int32_t *ridx, int64_t rnnz, uint64_t *cycles_out = nullptr,
                     const int32_t *root_ids = nullptr, int64_t nroots = 0, bool pv_zeroed = false);

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
#undef ARB_DECLARE_DEPTH

}  // namespace arb
