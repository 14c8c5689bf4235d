// Internal declarations shared by the HIP sources of libarb.so (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/arb.h"

namespace arb {

constexpr int kWave = 64;

// ------------------------------------------------------------------ errors

void set_error(int code);
int last_error();

#define ARB_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return ARB_EHIP;          \
    } while (0)

#define ARB_CHECK_LAUNCH() ARB_HIP(hipGetLastError())

// ------------------------------------------------------------------ workspace

// Carves 256-byte aligned pieces out of a caller workspace (or only measures when
// base is null).
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T) + 0;
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
};

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline unsigned grid_for(int64_t work, int block, unsigned cap = 1u << 20) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (int64_t)cap) g = cap;
    return (unsigned)g;
}

// ------------------------------------------------------------------ device helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below_mask() {
    int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// ------------------------------------------------------------------ primitives (prims.hip)

// Fill kernels used instead of hipMemsetAsync so that work stays capture-safe.
int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
int fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
int fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);

// Exclusive prefix sum of n int64 values: out[i] = sum_{j<i} in[j] for i <= n (out has
// n+1 entries; in and out may alias).  Workspace from scan_workspace(n).
size_t scan_workspace(int64_t n);
int exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, void *ws, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the bits [0, key_bits) of key.
// Results end in keys/vals; alt buffers are scratch of the same size.
size_t radix_workspace(int64_t n);
int radix_sort_u32(uint32_t *keys, int32_t *vals, uint32_t *keys_alt, int32_t *vals_alt,
                   int64_t n, int key_bits, void *ws, hipStream_t s);

}  // namespace arb
