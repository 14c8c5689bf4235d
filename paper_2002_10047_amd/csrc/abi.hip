// Small C-ABI entry points: id-space mapping and error reporting.
#include "common.h"

namespace arb {

__global__ void k_permute_u64(const int32_t *rank, const uint64_t *in, uint64_t *out, int64_t n) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        out[v] = in[rank[v]];
}

// One block per segment, 64-bit sums reduced in a fixed order.
__global__ void k_segment_sum(const unsigned long long *in, const int64_t *off, int64_t G, unsigned long long *out) {
    __shared__ unsigned long long red[256];
    for (int64_t g = blockIdx.x; g < G; g += gridDim.x) {
        unsigned long long s = 0;
        for (int64_t i = off[g] + threadIdx.x; i < off[g + 1]; i += blockDim.x) s += in[i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[g] = red[0];
        __syncthreads();
    }
}

}  // namespace arb

using namespace arb;

extern "C" int arb_segment_sum_u64(const uint64_t *in, const int64_t *offsets, int64_t G, uint64_t *out, void *stream) {
    if (G < 0 || (G > 0 && (!in || !offsets || !out))) {
        set_error(ARB_EINVAL);
        return ARB_EINVAL;
    }
    if (G > 0) {
        k_segment_sum<<<grid_for(G, 1, 4096), 256, 0, as_stream(stream)>>>(
            reinterpret_cast<const unsigned long long *>(in), offsets, G, reinterpret_cast<unsigned long long *>(out));
        if (hipGetLastError() != hipSuccess) {
            set_error(ARB_EHIP);
            return ARB_EHIP;
        }
    }
    set_error(ARB_OK);
    return ARB_OK;
}

// Batch counting: per-root counts of the union, then per-graph sums over the rank ranges
// (contiguous per graph after arb_orient_batch).  Workspace: the count's, then the
// per-root counts and the grand total.
static size_t batch_extra(int64_t n) { return ((size_t)(n > 0 ? n : 1) + 1) * sizeof(uint64_t) + 256; }

extern "C" size_t arb_count_batch_workspace(int64_t n, int64_t m, int k, int64_t G) {
    (void)G;
    return ((arb_count_workspace(n, m, k) + 255) & ~size_t(255)) + batch_extra(n);
}

extern "C" int arb_count_batch_async(const arb_ocsr *dg, const int64_t *graph_vtx_offsets, int64_t G, int k,
                                     uint64_t *per_vertex, uint64_t *totals_dev, uint64_t *total_dev,
                                     const arb_count_opts *opts, void *ws, size_t ws_bytes, void *stream) {
    if (!dg || !graph_vtx_offsets || !totals_dev || !ws || G < 1 || dg->n < 0 || G > dg->n + 1) {
        set_error(ARB_EINVAL);
        return ARB_EINVAL;
    }
    const int64_t n = dg->n;
    const size_t cws = (arb_count_workspace(n, dg->m, k) + 255) & ~size_t(255);
    if (ws_bytes < cws + batch_extra(n)) {
        set_error(ARB_EWORKSPACE);
        return ARB_EWORKSPACE;
    }
    uint64_t *per_root = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + cws);
    uint64_t *total = total_dev ? total_dev : per_root + (n > 0 ? n : 1);
    int rc = arb_count_async(dg, k, total, per_vertex, per_root, nullptr, opts, ws, cws, stream);
    if (rc) return rc;
    return arb_segment_sum_u64(per_root, graph_vtx_offsets, G, totals_dev, stream);
}

extern "C" int arb_permute_u64(const int32_t *rank, const uint64_t *in, uint64_t *out, int64_t n, void *stream) {
    if (n < 0 || (n > 0 && (!rank || !in || !out)) || in == out) {
        set_error(ARB_EINVAL);
        return ARB_EINVAL;
    }
    if (n > 0) {
        k_permute_u64<<<grid_for(n, 256, 4096), 256, 0, as_stream(stream)>>>(rank, in, out, n);
        if (hipGetLastError() != hipSuccess) {
            set_error(ARB_EHIP);
            return ARB_EHIP;
        }
    }
    set_error(ARB_OK);
    return ARB_OK;
}

extern "C" int arb_last_error(void) { return last_error(); }

extern "C" const char *arb_error_string(int code) {
    switch (code) {
        case ARB_OK: return "ok";
        case ARB_EINVAL: return "invalid argument";
        case ARB_EGRAPH: return "graph violates the required CSR layout";
        case ARB_EWORKSPACE: return "workspace too small";
        case ARB_EHIP: return "HIP runtime error";
        case ARB_ELIMIT: return "implementation limit exceeded";
        case ARB_EMISMATCH: return "schedules disagree on the total";
        default: return "unknown error";
    }
}
