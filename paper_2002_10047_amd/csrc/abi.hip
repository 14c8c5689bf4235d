// Small C-ABI entry points: id-space mapping and error reporting.
#include "common.h"

namespace arb {

__global__ void k_permute_u64(const int32_t *rank, const uint64_t *in, uint64_t *out, int64_t n) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        out[v] = in[rank[v]];
}

}  // namespace arb

using namespace arb;

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
        default: return "unknown error";
    }
}
