// arb-peel (Alg. 2, Sec. 4.1): k-clique vertex peeling, a 1/k-approximation of the
// k-clique densest subgraph.  Starting from the per-vertex k-clique counts C (arb-count-v),
// each round removes every present vertex whose count equals the least present count
// (the set A), and Update lowers the counts of the vertices that shared k-cliques with A:
// for each v in A, the (k-1)-cliques of G[I_v], I_v = {u in N(v) : u present and (u not
// in A, or u in A ranked above v)}, are counted per vertex with the counting kernels (the
// candidate set of root v is I_v instead of N+(v)); every removed k-clique is counted once
// (by its lowest-ranked vertex of A).  The largest density cliques(S) / |S| over the
// rounds is reported.  Everything is in rank space; the undirected rows are built once
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

// least count among present vertices
__global__ void k_min_present(int64_t n, const int32_t *present, const unsigned long long *C,
                              unsigned long long *mn) {
    unsigned long long x = ~0ull;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (present[v] && C[v] < x) x = C[v];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    if ((threadIdx.x & 63) == 0 && x != ~0ull) atomicMin(mn, x);
}

// A = present vertices with the least count; round[v] = r for them; na[0] = |A|
__global__ void k_mark_min(int64_t n, const int32_t *present, const unsigned long long *C, const unsigned long long *mn,
                           int32_t *inA, int32_t *round, int r, unsigned long long *na) {
    unsigned long long c = 0;
    const unsigned long long m = mn[0];
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const bool a = present[v] && C[v] == m;
        inA[v] = a ? 1 : 0;
        if (a) {
            round[v] = r;
            c += 1;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(na, c);
}

// |I_v| for v in A (0 otherwise)
__global__ void k_update_count(int64_t n, const int64_t *uoff, const int32_t *uidx, const int32_t *present,
                               const int32_t *inA, int64_t *cnt) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves) {
        int64_t c = 0;
        if (inA[v])
            for (int64_t p = uoff[v] + lane; p < uoff[v + 1]; p += 64) {
                const int32_t u = uidx[p];
                c += present[u] && (!inA[u] || u > v);
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) cnt[v] = c;
    }
}

__global__ void k_update_fill(int64_t n, const int64_t *uoff, const int32_t *uidx, const int32_t *present,
                              const int32_t *inA, const int64_t *roff, int32_t *ridx) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = lanes_below_mask();
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves) {
        if (!inA[v]) continue;
        int64_t at = roff[v];
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

// C -= the removed cliques of each vertex; A leaves the present set
__global__ void k_apply_update(int64_t n, int32_t *present, const int32_t *inA, unsigned long long *C,
                               const unsigned long long *dec) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (inA[v]) {
            present[v] = 0;
        } else if (present[v]) {
            C[v] -= dec[v];
        }
    }
}

struct PeelExactWs {
    int64_t *uoff, *toff, *roff, *cnt;
    int32_t *uidx, *ridx, *tsrc, *present, *inA;
    uint32_t *key, *key_alt;
    int32_t *val_alt;
    unsigned long long *indeg, *C, *dec, *sc;
    void *scan_ws, *radix_ws, *count_ws;
    size_t count_bytes;
};

static size_t carve_peel_exact(Carver &c, int64_t n, int64_t m, int k, PeelExactWs *w) {
    const int64_t nn = n > 0 ? n : 1, mm = m > 0 ? m : 1;
    w->uoff = c.take<int64_t>(nn + 1);
    w->toff = c.take<int64_t>(nn + 1);
    w->roff = c.take<int64_t>(nn + 1);
    w->cnt = c.take<int64_t>(nn + 1);
    w->uidx = c.take<int32_t>(2 * mm);
    w->ridx = c.take<int32_t>(2 * mm);
    w->tsrc = c.take<int32_t>(mm);
    w->present = c.take<int32_t>(nn);
    w->inA = c.take<int32_t>(nn);
    w->key = c.take<uint32_t>(mm);
    w->key_alt = c.take<uint32_t>(mm);
    w->val_alt = c.take<int32_t>(mm);
    w->indeg = c.take<unsigned long long>(nn);
    w->C = c.take<unsigned long long>(nn);
    w->dec = c.take<unsigned long long>(nn);
    w->sc = c.take<unsigned long long>(8);
    w->scan_ws = c.take<char>(scan_workspace(nn + 1));
    w->radix_ws = c.take<char>(radix_workspace(mm));
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
    if ((rc = fill_i32(w.present, 1, n, s))) return fail(rc);
    if ((rc = fill_i32(round_out, -1, n, s))) return fail(rc);
    uint64_t T = 0;
    ARB_HIP(hipMemcpyAsync(&T, w.sc, sizeof(T), hipMemcpyDeviceToHost, s));
    ARB_HIP(hipStreamSynchronize(s));
    double best = (double)T / (double)n;
    int64_t left = n, r = 0;
    while (left > 0) {
        k_u64_set<<<1, 64, 0, s>>>(w.sc + 1, ~0ull);
        k_u64_set<<<1, 64, 0, s>>>(w.sc + 2, 0ull);
        k_min_present<<<gb, 256, 0, s>>>(n, w.present, w.C, w.sc + 1);
        k_mark_min<<<gb, 256, 0, s>>>(n, w.present, w.C, w.sc + 1, w.inA, round_out, (int)r, w.sc + 2);
        k_update_count<<<gw, 256, 0, s>>>(n, w.uoff, w.uidx, w.present, w.inA, w.cnt);
        if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
        if ((rc = exclusive_scan_i64(w.cnt, w.roff, n, w.scan_ws, s))) return fail(rc);
        k_update_fill<<<gw, 256, 0, s>>>(n, w.uoff, w.uidx, w.present, w.inA, w.roff, w.ridx);
        int64_t rn = 0;
        uint64_t na = 0;
        ARB_HIP(hipMemcpyAsync(&rn, w.roff + n, sizeof(rn), hipMemcpyDeviceToHost, s));
        ARB_HIP(hipMemcpyAsync(&na, w.sc + 2, sizeof(na), hipMemcpyDeviceToHost, s));
        ARB_HIP(hipStreamSynchronize(s));
        if (na == 0) return fail(ARB_ELIMIT);           // cannot happen while vertices are present
        // removed k-cliques (w.sc[3]) and per-vertex decrements (w.dec)
        if ((rc = count_with_roots(dg, k, reinterpret_cast<uint64_t *>(w.sc + 3), reinterpret_cast<uint64_t *>(w.dec),
                                   nullptr, nullptr, &opts, w.count_ws, w.count_bytes, s, w.roff, w.ridx, rn)))
            return fail(rc);
        k_apply_update<<<gb, 256, 0, s>>>(n, w.present, w.inA, w.C, w.dec);
        uint64_t removed = 0;
        ARB_HIP(hipMemcpyAsync(&removed, w.sc + 3, sizeof(removed), hipMemcpyDeviceToHost, s));
        ARB_HIP(hipStreamSynchronize(s));
        T -= removed;
        left -= (int64_t)na;
        ++r;
        if (left > 0) {
            const double dens = (double)T / (double)left;
            if (dens > best) best = dens;
        }
    }
    *best_density = best;
    if (rounds) *rounds = r;
    return fail(ARB_OK);
}
