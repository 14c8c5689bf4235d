// Colorful sparsification (Sec. 3.3 and its proofs in the appendix): every vertex has a
// colour out of c; the sparsified graph keeps exactly the edges whose two endpoints share
// a colour, so a k-clique survives iff it is monochromatic (probability p^(k-1), p = 1/c)
// and C * c^(k-1) estimates the k-clique count without bias.  The colours are an input
// (drawn by the caller), so the filter itself is deterministic.
#include "common.h"

namespace arb {

// kept[v] = neighbours of v with v's colour (one wave per row)
__global__ void k_keep_count(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *color, int64_t *kept) {
    const int lane = threadIdx.x & 63;
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves) {
        const int32_t cv = color[v];
        int64_t c = 0;
        for (int64_t p = off[v] + lane; p < off[v + 1]; p += 64) c += color[idx[p]] == cv;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) kept[v] = c;
    }
}

// the kept neighbours of each row, in their original (ascending) order
__global__ void k_keep_fill(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *color,
                            const int64_t *out_off, int32_t *out_idx) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = lanes_below_mask();
    int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = wave; v < n; v += nwaves) {
        const int32_t cv = color[v];
        int64_t at = out_off[v];
        for (int64_t b = off[v]; b < off[v + 1]; b += 64) {
            const int64_t p = b + lane;
            int32_t u = 0;
            bool keep = false;
            if (p < off[v + 1]) {
                u = idx[p];
                keep = color[u] == cv;
            }
            const uint64_t m = __ballot(keep);
            if (keep) out_idx[at + __popcll(m & below)] = u;
            at += __popcll(m);
        }
    }
}

}  // namespace arb

using namespace arb;

extern "C" size_t arb_sparsify_workspace(int64_t n, int64_t nnz) {
    (void)nnz;
    const int64_t nn = n > 0 ? n : 1;
    return (size_t)(nn + 1) * sizeof(int64_t) + scan_workspace(nn + 1) + 512;
}

extern "C" int arb_sparsify(const arb_csr *g, const int32_t *colors, int64_t *out_offsets, int32_t *out_indices,
                            int64_t *out_nnz, void *ws, size_t ws_bytes, void *stream) {
    hipStream_t s = as_stream(stream);
    auto fail = [](int rc) { set_error(rc); return rc; };
    if (!g || !out_offsets || !out_nnz || !ws || g->n < 0 || g->nnz < 0 || (g->n > 0 && (!g->offsets || !colors)) ||
        (g->nnz > 0 && (!g->indices || !out_indices)))
        return fail(ARB_EINVAL);
    if (ws_bytes < arb_sparsify_workspace(g->n, g->nnz)) return fail(ARB_EWORKSPACE);
    const int64_t n = g->n;
    if (n == 0) {
        if (fill_i64(out_offsets, 0, 1, s)) return fail(ARB_EHIP);
        *out_nnz = 0;
        return fail(ARB_OK);
    }
    Carver cv(ws);
    int64_t *kept = cv.take<int64_t>(n + 1);
    void *scan_ws = cv.take<char>(scan_workspace(n + 1));
    const unsigned grid = grid_for(n * 64, 256, 8192);
    k_keep_count<<<grid, 256, 0, s>>>(n, g->offsets, g->indices, colors, kept);
    if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
    int rc = exclusive_scan_i64(kept, out_offsets, n, scan_ws, s);
    if (rc) return fail(rc);
    k_keep_fill<<<grid, 256, 0, s>>>(n, g->offsets, g->indices, colors, out_offsets, out_indices);
    if (hipGetLastError() != hipSuccess) return fail(ARB_EHIP);
    int64_t h = 0;
    if (hipMemcpyAsync(&h, out_offsets + n, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(ARB_EHIP);
    *out_nnz = h;
    return fail(ARB_OK);
}

extern "C" double arb_colorful_estimate(uint64_t count, int colors, int k) {
    if (colors < 1 || k < 1) {
        set_error(ARB_EINVAL);
        return 0.0;
    }
    set_error(ARB_OK);
    double scale = 1.0;
    for (int i = 0; i < k - 1; ++i) scale *= (double)colors;
    return (double)count * scale;
}
