// arb-approx-peel (Sec. 4.2): a 1/(k(1+eps))-approximation of the k-clique densest
// subgraph.  Round after round, on the subgraph S of vertices still present: count the
// k-cliques of G[S] per vertex (arb-count-v on the directed graph restricted to S -- an
// ordering restricted to a subgraph is still a low out-degree orientation of it), record
// the density |cliques(S)| / |S|, and remove every present vertex with at most
// k(1+eps) times that density k-cliques.  The average per-vertex count is k times the
// density, so every round removes vertices; the densest S seen is the answer.
#include "common.h"

namespace arb {

// kept arcs of each row: both ends present
__global__ void k_alive_count(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *alive, int64_t *cnt) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves) {
        int64_t c = 0;
        if (alive[v])
            for (int64_t p = off[v] + lane; p < off[v + 1]; p += 64) c += alive[idx[p]] != 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) cnt[v] = c;
    }
}

__global__ void k_alive_fill(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *alive,
                             const int64_t *out_off, int32_t *out_idx) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = lanes_below_mask();
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves) {
        if (!alive[v]) continue;
        int64_t at = out_off[v];
        for (int64_t b = off[v]; b < off[v + 1]; b += 64) {
            const int64_t p = b + lane;
            int32_t u = 0;
            bool keep = false;
            if (p < off[v + 1]) {
                u = idx[p];
                keep = alive[u] != 0;
            }
            const uint64_t m = __ballot(keep);
            if (keep) out_idx[at + __popcll(m & below)] = u;
            at += __popcll(m);
        }
    }
}

// remove present vertices with count <= t; left[0] counts the vertices still present
__global__ void k_approx_remove(int64_t n, int32_t *alive, const unsigned long long *pv, double t,
                                unsigned long long *left) {
    unsigned long long c = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (!alive[v]) continue;
        if ((double)pv[v] <= t) alive[v] = 0;
        else c += 1;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(left, c);
}

__global__ void k_copy_i32(int64_t n, const int32_t *src, int32_t *dst) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        dst[v] = src[v];
}

struct PeelWs {
    int64_t *foff;
    int32_t *fidx;
    unsigned long long *pv, *tot, *left;
    int32_t *alive;
    void *scan_ws, *count_ws;
    size_t count_bytes;
};

static size_t carve_peel(Carver &c, int64_t n, int64_t m, int k, PeelWs *w) {
    const int64_t nn = n > 0 ? n : 1;
    w->foff = c.take<int64_t>(nn + 1);
    w->fidx = c.take<int32_t>(m > 0 ? m : 1);
    w->pv = c.take<unsigned long long>(nn);
    w->tot = c.take<unsigned long long>(4);
    w->left = c.take<unsigned long long>(4);
    w->alive = c.take<int32_t>(nn);
    w->scan_ws = c.take<char>(scan_workspace(nn + 1));
    w->count_bytes = arb_count_workspace(n, m, k);
    w->count_ws = c.take<char>(w->count_bytes);
    return c.used;
}

}  // namespace arb

using namespace arb;

extern "C" size_t arb_approx_peel_workspace(int64_t n, int64_t m, int k) {
    Carver c(nullptr);
    PeelWs w;
    return carve_peel(c, n, m, k, &w) + 256;
}

extern "C" int arb_approx_peel(const arb_ocsr *dg, int k, double eps, const arb_count_opts *opts,
                               double *best_density, int64_t *rounds, int32_t *best_mask, void *ws, size_t ws_bytes,
                               void *stream) {
    hipStream_t s = as_stream(stream);
    auto fail = [](int rc) { set_error(rc); return rc; };
    if (!dg || !best_density || !ws || dg->n < 0 || dg->m < 0 || !dg->offsets || (dg->m > 0 && !dg->indices))
        return fail(ARB_EINVAL);
    if (k < 1 || k > ARB_MAX_K || !(eps > 0.0 && eps <= 64.0)) return fail(ARB_EINVAL);
    const int64_t n = dg->n, m = dg->m;
    if (ws_bytes < arb_approx_peel_workspace(n, m, k)) return fail(ARB_EWORKSPACE);
    Carver cv(ws);
    PeelWs w;
    carve_peel(cv, n, m, k, &w);
    *best_density = 0.0;
    int64_t r = 0;
    int rc;
    if (n > 0) {
        if ((rc = fill_i32(w.alive, 1, n, s))) return fail(rc);
        if (best_mask && (rc = fill_i32(best_mask, 1, n, s))) return fail(rc);
    }
    const unsigned gb = grid_for(n, 256, 4096), gw = grid_for(n * 64, 256, 8192);
    int64_t present = n;
    double best = -1.0;
    while (present > 0) {
        // G[S]: the directed graph restricted to present vertices
        k_alive_count<<<gw, 256, 0, s>>>(n, dg->offsets, dg->indices, w.alive, w.foff);
        if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
        if ((rc = exclusive_scan_i64(w.foff, w.foff, n, w.scan_ws, s))) return fail(rc);
        k_alive_fill<<<gw, 256, 0, s>>>(n, dg->offsets, dg->indices, w.alive, w.foff, w.fidx);
        if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
        int64_t fm = 0;
        ARB_HIP(hipMemcpyAsync(&fm, w.foff + n, sizeof(fm), hipMemcpyDeviceToHost, s));
        ARB_HIP(hipStreamSynchronize(s));
        const arb_ocsr f{n, fm, w.foff, w.fidx};
        if ((rc = arb_count_async(&f, k, reinterpret_cast<uint64_t *>(w.tot), reinterpret_cast<uint64_t *>(w.pv),
                                  nullptr, nullptr, opts, w.count_ws, w.count_bytes, stream)))
            return rc;
        uint64_t C = 0;
        ARB_HIP(hipMemcpyAsync(&C, w.tot, sizeof(C), hipMemcpyDeviceToHost, s));
        ARB_HIP(hipStreamSynchronize(s));
        const double density = (double)C / (double)present;
        if (density > best) {
            best = density;
            if (best_mask) k_copy_i32<<<gb, 256, 0, s>>>(n, w.alive, best_mask);
        }
        // remove every present vertex with at most k (1 + eps) density k-cliques
        const double t = ((double)k * (1.0 + eps) * (double)C) / (double)present;
        if ((rc = fill_i64(reinterpret_cast<int64_t *>(w.left), 0, 1, s))) return fail(rc);
        k_approx_remove<<<gb, 256, 0, s>>>(n, w.alive, w.pv, t, w.left);
        if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
        uint64_t left = 0;
        ARB_HIP(hipMemcpyAsync(&left, w.left, sizeof(left), hipMemcpyDeviceToHost, s));
        ARB_HIP(hipStreamSynchronize(s));
        if ((int64_t)left >= present) return fail(ARB_ELIMIT);   // cannot happen: the average is <= t
        present = (int64_t)left;
        ++r;
    }
    *best_density = best < 0 ? 0.0 : best;
    if (rounds) *rounds = r;
    return fail(ARB_OK);
}
