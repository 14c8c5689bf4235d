// arb-peel (Alg. 2, Sec. 4.1): k-clique vertex peeling, a 1/k-approximation of the
// k-clique densest subgraph.  Starting from the per-vertex k-clique counts C (arb-count-v),
// each round removes every present vertex whose count equals the least present count
// (the set A, taken from a bucket structure of the counts, below), and Update lowers the
// counts of the vertices that shared k-cliques with A:
// for each v in A, the (k-1)-cliques of G[I_v], I_v = {u in N(v) : u present and (u not
// in A, or u in A ranked above v)}, are counted per vertex with the counting kernels (the
// candidate set of root v is I_v instead of N+(v)); every removed k-clique is counted once
// (by its lowest-ranked vertex of A).  A round's work is proportional to A, its update
// sets and the vertices whose counts changed, not to n: the counting driver takes A as a
// list of roots.  The largest density cliques(S) / |S| over the rounds is reported.  Everything is in rank space; the undirected rows are built once
// from the directed graph (in-neighbours, then out-neighbours, both ascending).
#include "count_kernels.h"

namespace arb {

// undirected rank-space rows: in-degree count per target
__global__ void k_indeg(int64_t m, const int32_t *idx, unsigned long long *indeg) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&indeg[idx[p]], 1ull);
}

// arc keys for the stable transpose: key = target, value = source
__global__ void k_arc_pairs(int64_t n, const int64_t *off, const int32_t *idx, uint32_t *key, int32_t *val) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves)
        for (int64_t p = off[v] + lane; p < off[v + 1]; p += 64) {
            key[p] = (uint32_t)idx[p];
            val[p] = (int32_t)v;
        }
}

__global__ void k_undirected_deg(int64_t n, const int64_t *off, const unsigned long long *indeg, int64_t *deg) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        deg[v] = (int64_t)indeg[v] + (off[v + 1] - off[v]);
}

// row v = its in-neighbours (sources of the sorted transpose, ascending) then N+(v)
__global__ void k_undirected_fill(int64_t n, const int64_t *off, const int32_t *idx, const int64_t *uoff,
                                  const int64_t *toff, const int32_t *tsrc, int32_t *uidx) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves) {
        const int64_t nin = toff[v + 1] - toff[v];
        for (int64_t i = lane; i < nin; i += 64) uidx[uoff[v] + i] = tsrc[toff[v] + i];
        for (int64_t i = lane; i < off[v + 1] - off[v]; i += 64) uidx[uoff[v] + nin + i] = idx[off[v] + i];
    }
}

// ------------------------------------------------------------------ buckets of counts
//
// The least present count is found without a pass over all vertices: L lists the present
// vertices sorted by (count, id) as of its last rebuild, and U lists the vertices whose
// counts dropped since (their L entries are stale).  Every present vertex is either a
// valid L entry (present, not in U: its count is its sort key) at or after L's head, or
// in U.  So the least count is min(count of the first valid L entry, least count in U),
// and A is the run of valid L entries with that count plus the U entries with it.  L's
// head only moves past entries that stay invalid (removed, or stale until the rebuild);
// L is rebuilt, and U emptied, when U outgrows a share of L.

// advance L's head to its first valid entry; sc[1] = min(sc[1], its count)
__global__ void k_l_head(const int32_t *L, int64_t llen, int64_t *head, const int32_t *present, const int32_t *inU,
                        const unsigned long long *C, unsigned long long *mn) {
    const int lane = threadIdx.x & 63;
    if (threadIdx.x >= 64) return;
    int64_t h = *head;
    while (h < llen) {
        const int64_t p = h + lane;
        const bool ok = p < llen && present[L[p]] && !inU[L[p]];
        const uint64_t m = __ballot(ok);
        if (m) {
            h += __ffsll((unsigned long long)m) - 1;
            break;
        }
        h += 64;
    }
    if (h > llen) h = llen;
    if (lane == 0) {
        *head = h;
        if (h < llen) atomicMin(mn, C[L[h]]);
    }
}

// sc[1] = min(sc[1], least count of present U entries)
__global__ void k_u_min(const int32_t *U, const unsigned long long *ucnt, const int32_t *present,
                        const unsigned long long *C, unsigned long long *mn) {
    const int64_t nu = (int64_t)*ucnt;
    unsigned long long x = ~0ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nu; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = U[i];
        if (present[u] && C[u] < x) x = C[u];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    if ((threadIdx.x & 63) == 0 && x != ~0ull) atomicMin(mn, x);
}

__device__ __forceinline__ void join_A(int32_t v, int r, int32_t *inA, int32_t *round, int32_t *A,
                                       unsigned long long *na) {
    inA[v] = 1;
    round[v] = r;
    A[atomicAdd(na, 1ull)] = v;
}

// A from L: the valid entries from the head on whose count is the least (one wave)
__global__ void k_l_collect(const int32_t *L, int64_t llen, const int64_t *head, const int32_t *present,
                            const int32_t *inU, const unsigned long long *C, const unsigned long long *mn, int r,
                            int32_t *inA, int32_t *round, int32_t *A, unsigned long long *na) {
    const int lane = threadIdx.x & 63;
    if (threadIdx.x >= 64) return;
    const unsigned long long m = *mn;
    for (int64_t h = *head; h < llen; h += 64) {
        const int64_t p = h + lane;
        bool ok = false, past = false;
        int32_t v = 0;
        if (p < llen) {
            v = L[p];
            if (present[v] && !inU[v]) {
                ok = C[v] == m;
                past = C[v] > m;
            }
        }
        if (ok) join_A(v, r, inA, round, A, na);
        if (__ballot(past)) break;          // sorted: no valid entry further on has count m
    }
}

// A from U: present entries whose count is the least
__global__ void k_u_collect(const int32_t *U, const unsigned long long *ucnt, const int32_t *present,
                            const unsigned long long *C, const unsigned long long *mn, int r, int32_t *inA,
                            int32_t *round, int32_t *A, unsigned long long *na) {
    const int64_t nu = (int64_t)*ucnt;
    const unsigned long long m = *mn;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nu; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = U[i];
        if (present[u] && C[u] == m) join_A(u, r, inA, round, A, na);
    }
}

// |I_v| for the p-th vertex v of A: present neighbours not in A, or in A and ranked above v
__global__ void k_update_count(const int32_t *A, int64_t na, const int64_t *uoff, const int32_t *uidx,
                               const int32_t *present, const int32_t *inA, int64_t *cnt) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = wave; q < na; q += nwaves) {
        const int32_t v = A[q];
        int64_t c = 0;
        for (int64_t p = uoff[v] + lane; p < uoff[v + 1]; p += 64) {
            const int32_t u = uidx[p];
            c += present[u] && (!inA[u] || u > v);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) cnt[q] = c;
    }
}

__global__ void k_update_fill(const int32_t *A, int64_t na, const int64_t *uoff, const int32_t *uidx,
                              const int32_t *present, const int32_t *inA, const int64_t *roff, int32_t *ridx) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = lanes_below_mask();
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = wave; q < na; q += nwaves) {
        const int32_t v = A[q];
        int64_t at = roff[q];
        for (int64_t b = uoff[v]; b < uoff[v + 1]; b += 64) {
            const int64_t p = b + lane;
            int32_t u = 0;
            bool keep = false;
            if (p < uoff[v + 1]) {
                u = uidx[p];
                keep = present[u] && (!inA[u] || u > v);
            }
            const uint64_t m = __ballot(keep);
            if (keep) ridx[at + __popcll(m & below)] = u;
            at += __popcll(m);
        }
    }
}

// A leaves the present set (its decrements are dropped)
__global__ void k_remove_A(const int32_t *A, int64_t na, int32_t *present, int32_t *inA, unsigned long long *dec) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < na; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = A[q];
        present[v] = 0;
        inA[v] = 0;
        dec[v] = 0;
    }
}

// the vertices that lost cliques (entries of the update sets): count -= decrement, once
// each (the decrement is taken with an exchange), and into U
__global__ void k_apply_dec(const int32_t *ridx, const int64_t *rend, const int32_t *present,
                            unsigned long long *C, unsigned long long *dec, int32_t *inU, int32_t *U,
                            unsigned long long *ucnt) {
    const int64_t ne = *rend;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < ne; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = ridx[p];
        const unsigned long long d = atomicExch(&dec[u], 0ull);
        if (d && present[u]) {
            C[u] -= d;
            if (atomicExch(&inU[u], 1) == 0) U[atomicAdd(ucnt, 1ull)] = u;
        }
    }
}

// rebuild of L: flags of present vertices, then keys of the listed ones
__global__ void k_present_flag(int64_t n, const int32_t *present, int64_t *flag) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        flag[v] = present[v] ? 1 : 0;
}

__global__ void k_present_list(int64_t n, const int32_t *present, const int64_t *pos, int32_t *L) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (present[v]) L[pos[v]] = (int32_t)v;
}

__global__ void k_count_key(const int32_t *L, int64_t len, const unsigned long long *C, int hi, uint32_t *key) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long c = C[L[i]];
        key[i] = hi ? (uint32_t)(c >> 32) : (uint32_t)c;
    }
}

__global__ void k_clear_u(const int32_t *U, const unsigned long long *ucnt, int32_t *inU) {
    const int64_t nu = (int64_t)*ucnt;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nu; i += (int64_t)gridDim.x * blockDim.x)
        inU[U[i]] = 0;
}

struct PeelExactWs {
    int64_t *uoff, *toff, *roff, *cnt, *head;
    int32_t *uidx, *ridx, *tsrc, *present, *inA, *inU, *L, *U, *A;
    uint32_t *key, *key_alt;
    int32_t *val_alt;
    unsigned long long *indeg, *C, *dec, *sc;
    void *scan_ws, *radix_ws, *count_ws;
    size_t count_bytes;
};

static size_t carve_peel_exact(Carver &c, int64_t n, int64_t m, int k, PeelExactWs *w) {
    const int64_t nn = n > 0 ? n : 1, mm = m > 0 ? m : 1;
    const int64_t nk = nn > mm ? nn : mm;          // radix keys: arcs (transpose) or vertices (L)
    w->uoff = c.take<int64_t>(nn + 1);
    w->toff = c.take<int64_t>(nn + 1);
    w->roff = c.take<int64_t>(nn + 1);
    w->cnt = c.take<int64_t>(nn + 1);
    w->head = c.take<int64_t>(1);
    w->uidx = c.take<int32_t>(2 * mm);
    w->ridx = c.take<int32_t>(2 * mm);
    w->tsrc = c.take<int32_t>(mm);
    w->present = c.take<int32_t>(nn);
    w->inA = c.take<int32_t>(nn);
    w->inU = c.take<int32_t>(nn);
    w->L = c.take<int32_t>(nn);
    w->U = c.take<int32_t>(nn);
    w->A = c.take<int32_t>(nn);
    w->key = c.take<uint32_t>(nk);
    w->key_alt = c.take<uint32_t>(nk);
    w->val_alt = c.take<int32_t>(nk);
    w->indeg = c.take<unsigned long long>(nn);
    w->C = c.take<unsigned long long>(nn);
    w->dec = c.take<unsigned long long>(nn);
    w->sc = c.take<unsigned long long>(8);
    w->scan_ws = c.take<char>(scan_workspace(nn + 1));
    w->radix_ws = c.take<char>(radix_workspace(nk));
    w->count_bytes = arb_count_workspace(n, 2 * mm, k);
    w->count_ws = c.take<char>(w->count_bytes);
    return c.used;
}

__global__ void k_u64_fill_span(unsigned long long *p, unsigned long long v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_u64_to_i64(int64_t n, const unsigned long long *in, int64_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int64_t)in[i];
}

__global__ void k_u64_set(unsigned long long *p, unsigned long long v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

}  // namespace arb

using namespace arb;

extern "C" size_t arb_peel_workspace(int64_t n, int64_t m, int k) {
    Carver c(nullptr);
    PeelExactWs w;
    return carve_peel_exact(c, n, m, k, &w) + 256;
}

extern "C" int arb_peel(const arb_ocsr *dg, int k, double *best_density, int64_t *rounds, int32_t *round_out,
                        void *ws, size_t ws_bytes, void *stream) {
    hipStream_t s = as_stream(stream);
    auto fail = [](int rc) { set_error(rc); return rc; };
    if (!dg || !best_density || !ws || dg->n < 0 || dg->m < 0 || !dg->offsets || (dg->m > 0 && !dg->indices))
        return fail(ARB_EINVAL);
    if (k < 3 || k > ARB_MAX_K || (dg->n > 0 && !round_out)) return fail(ARB_EINVAL);
    const int64_t n = dg->n, m = dg->m;
    if (ws_bytes < arb_peel_workspace(n, m, k)) return fail(ARB_EWORKSPACE);
    *best_density = 0.0;
    if (rounds) *rounds = 0;
    if (n == 0) return fail(ARB_OK);
    Carver cv(ws);
    PeelExactWs w;
    carve_peel_exact(cv, n, m, k, &w);
    int rc;
    const unsigned gb = grid_for(n, 256, 4096), gw = grid_for(n * 64, 256, 8192);
    arb_count_opts opts;
    arb_count_default_opts(&opts);
    // undirected rows in rank space: stable transpose of the arcs, then in- and out-lists
    if (m > 0) {
        k_u64_fill_span<<<gb, 256, 0, s>>>(w.indeg, 0ull, n);
        k_indeg<<<grid_for(m, 256, 4096), 256, 0, s>>>(m, dg->indices, w.indeg);
        k_arc_pairs<<<gw, 256, 0, s>>>(n, dg->offsets, dg->indices, w.key, w.tsrc);
        if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
        int bits = 1;
        while ((int64_t(1) << bits) < n) ++bits;
        if ((rc = radix_sort_u32(w.key, w.tsrc, w.key_alt, w.val_alt, m, bits, w.radix_ws, s))) return fail(rc);
    } else {
        k_u64_fill_span<<<gb, 256, 0, s>>>(w.indeg, 0ull, n);
    }
    // toff: scan of in-degrees; uoff: scan of in + out degrees
    k_undirected_deg<<<gb, 256, 0, s>>>(n, dg->offsets, w.indeg, w.cnt);
    if ((rc = exclusive_scan_i64(w.cnt, w.uoff, n, w.scan_ws, s))) return fail(rc);
    k_u64_to_i64<<<gb, 256, 0, s>>>(n, w.indeg, w.cnt);
    if ((rc = exclusive_scan_i64(w.cnt, w.toff, n, w.scan_ws, s))) return fail(rc);
    k_undirected_fill<<<gw, 256, 0, s>>>(n, dg->offsets, dg->indices, w.uoff, w.toff, w.tsrc, w.uidx);
    if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
    // initial per-vertex counts
    if ((rc = count_with_roots(dg, k, reinterpret_cast<uint64_t *>(w.sc), reinterpret_cast<uint64_t *>(w.C), nullptr,
                               nullptr, &opts, w.count_ws, w.count_bytes, s, nullptr, nullptr, 0)))
        return fail(rc);
    if ((rc = fill_i32(w.present, 1, n, s)) || (rc = fill_i32(round_out, -1, n, s)) || (rc = fill_i32(w.inA, 0, n, s)) ||
        (rc = fill_i32(w.inU, 0, n, s)))
        return fail(rc);
    k_u64_fill_span<<<gb, 256, 0, s>>>(w.dec, 0ull, n);
    k_u64_set<<<1, 64, 0, s>>>(w.sc + 4, 0ull);
    if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
    uint64_t T = 0;
    ARB_HIP(hipMemcpyAsync(&T, w.sc, sizeof(T), hipMemcpyDeviceToHost, s));
    ARB_HIP(hipStreamSynchronize(s));
    double best = (double)T / (double)n;
    int64_t left = n, r = 0, llen = 0;
    uint64_t ucnt = 0;
    // L = present vertices sorted by (count, id): two stable passes over the 32-bit halves
    auto rebuild = [&]() -> int {
        k_present_flag<<<gb, 256, 0, s>>>(n, w.present, w.cnt);
        if (hipGetLastError() != hipSuccess) return ARB_EHIP;
        int e = exclusive_scan_i64(w.cnt, w.toff, n, w.scan_ws, s);
        if (e) return e;
        k_present_list<<<gb, 256, 0, s>>>(n, w.present, w.toff, w.L);
        k_clear_u<<<grid_for((int64_t)ucnt, 256, 4096), 256, 0, s>>>(w.U, w.sc + 4, w.inU);
        k_u64_set<<<1, 64, 0, s>>>(w.sc + 4, 0ull);
        if (hipGetLastError() != hipSuccess) return ARB_EHIP;
        if (hipMemcpyAsync(&llen, w.toff + n, sizeof(llen), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return ARB_EHIP;
        for (int hi = 0; hi < 2; ++hi) {
            k_count_key<<<grid_for(llen, 256, 4096), 256, 0, s>>>(w.L, llen, w.C, hi, w.key);
            if (hipGetLastError() != hipSuccess) return ARB_EHIP;
            if ((e = radix_sort_u32(w.key, w.L, w.key_alt, w.val_alt, llen, 32, w.radix_ws, s))) return e;
        }
        ucnt = 0;
        return fill_i64(w.head, 0, 1, s);
    };
    if ((rc = rebuild())) return fail(rc);
    while (left > 0) {
        // A = the present vertices of least count, from the head of L and from U
        k_u64_set<<<1, 64, 0, s>>>(w.sc + 1, ~0ull);
        k_u64_set<<<1, 64, 0, s>>>(w.sc + 2, 0ull);
        k_l_head<<<1, 64, 0, s>>>(w.L, llen, w.head, w.present, w.inU, w.C, w.sc + 1);
        const unsigned gu = grid_for((int64_t)ucnt, 256, 4096);
        k_u_min<<<gu, 256, 0, s>>>(w.U, w.sc + 4, w.present, w.C, w.sc + 1);
        k_l_collect<<<1, 64, 0, s>>>(w.L, llen, w.head, w.present, w.inU, w.C, w.sc + 1, (int)r, w.inA, round_out,
                                     w.A, w.sc + 2);
        k_u_collect<<<gu, 256, 0, s>>>(w.U, w.sc + 4, w.present, w.C, w.sc + 1, (int)r, w.inA, round_out, w.A,
                                       w.sc + 2);
        if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
        uint64_t na = 0;
        ARB_HIP(hipMemcpyAsync(&na, w.sc + 2, sizeof(na), hipMemcpyDeviceToHost, s));
        ARB_HIP(hipStreamSynchronize(s));
        if (na == 0) return fail(ARB_ELIMIT);           // cannot happen while vertices are present
        // Update: per-vertex (k-1)-cliques of G[I_v] for the roots v of A
        const int64_t nA = (int64_t)na;
        const unsigned ga = grid_for(nA * 64, 256, 8192);
        k_update_count<<<ga, 256, 0, s>>>(w.A, nA, w.uoff, w.uidx, w.present, w.inA, w.cnt);
        if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
        if ((rc = exclusive_scan_i64(w.cnt, w.roff, nA, w.scan_ws, s))) return fail(rc);
        k_update_fill<<<ga, 256, 0, s>>>(w.A, nA, w.uoff, w.uidx, w.present, w.inA, w.roff, w.ridx);
        if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
        if ((rc = count_with_roots(dg, k, reinterpret_cast<uint64_t *>(w.sc + 3), reinterpret_cast<uint64_t *>(w.dec),
                                   nullptr, nullptr, &opts, w.count_ws, w.count_bytes, s, w.roff, w.ridx, 2 * m,
                                   nullptr, w.A, nA, true)))
            return fail(rc);
        k_remove_A<<<grid_for(nA, 256, 4096), 256, 0, s>>>(w.A, nA, w.present, w.inA, w.dec);
        k_apply_dec<<<gb, 256, 0, s>>>(w.ridx, w.roff + nA, w.present, w.C, w.dec, w.inU, w.U, w.sc + 4);
        if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
        uint64_t rs[2] = {0, 0};
        ARB_HIP(hipMemcpyAsync(rs, w.sc + 3, sizeof(rs), hipMemcpyDeviceToHost, s));
        ARB_HIP(hipStreamSynchronize(s));
        T -= rs[0];
        ucnt = rs[1];
        left -= nA;
        ++r;
        if (left > 0) {
            const double dens = (double)T / (double)left;
            if (dens > best) best = dens;
            if ((int64_t)ucnt > (llen / 8 > 4096 ? llen / 8 : 4096) && (rc = rebuild())) return fail(rc);
        }
    }
    *best_density = best;
    if (rounds) *rounds = r;
    return fail(ARB_OK);
}
