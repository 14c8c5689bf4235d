// Measurement probes for the roofline peaks: LDS read bandwidth and device-memory copy
// bandwidth on the current GPU.  They are not part of the counting path; bench.py runs
// them next to the timed steps and takes the larger of the published and the measured
// peak.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/arb_probe.h"

namespace {

constexpr int kLdsWords = 16384;   // 64 KiB per block

// Every lane reads 16-byte vectors at conflict-free addresses (a wave covers 1 KiB of
// consecutive words), rotating through the block's buffer; the xor keeps the loads live.
__global__ void __launch_bounds__(1024) k_lds_read(uint32_t *out, int iters) {
    __shared__ __align__(16) uint32_t buf[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += blockDim.x) buf[i] = (uint32_t)i * 2654435761u;
    __syncthreads();
    uint32_t acc = 0;
    const int lane = threadIdx.x & 63;
    int base = ((threadIdx.x >> 6) * 256) & (kLdsWords - 1);
#pragma unroll 8
    for (int it = 0; it < iters; ++it) {
        const int a = (base + lane * 4) & (kLdsWords - 1);
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        const u4 v = *reinterpret_cast<const u4 *>(&buf[a]);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
        base = (base + 256) & (kLdsWords - 1);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ void k_copy16(const uint4 *src, uint4 *dst, int64_t n16) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

extern "C" int arb_probe_lds_read(uint32_t *scratch, int64_t scratch_words, int blocks_per_cu, double *bytes_per_s,
                                  void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    if (!scratch || !bytes_per_s || blocks_per_cu < 1 || blocks_per_cu > 2) return 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 4;
    const int blocks = cus * blocks_per_cu, threads = 1024, iters = 20000;
    if (scratch_words < (int64_t)blocks * threads) return 3;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 4;
    k_lds_read<<<blocks, threads, 0, s>>>(scratch, 64);   // warm-up
    hipEventRecord(a, s);
    k_lds_read<<<blocks, threads, 0, s>>>(scratch, iters);
    hipEventRecord(b, s);
    float ms = 0.f;
    const bool ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess;
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (!ok || hipGetLastError() != hipSuccess || ms <= 0.f) return 4;
    *bytes_per_s = (double)blocks * threads * iters * 16.0 / (ms * 1e-3);
    return 0;
}

extern "C" int arb_probe_copy(const void *src, void *dst, int64_t bytes, int reps, double *bytes_per_s,
                              void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!src || !dst || bytes < 16 || reps < 1 || !bytes_per_s || (bytes & 15)) return 1;
    const int64_t n16 = bytes / 16;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 4;
    const unsigned grid = (unsigned)cus * 8;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 4;
    k_copy16<<<grid, 256, 0, s>>>(static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
    hipEventRecord(a, s);
    for (int r = 0; r < reps; ++r)
        k_copy16<<<grid, 256, 0, s>>>(static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
    hipEventRecord(b, s);
    float ms = 0.f;
    const bool ok = hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess;
    hipEventDestroy(a);
    hipEventDestroy(b);
    if (!ok || hipGetLastError() != hipSuccess || ms <= 0.f) return 4;
    *bytes_per_s = 2.0 * (double)bytes * reps / (ms * 1e-3);
    return 0;
}
