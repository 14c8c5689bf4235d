// Device-wide primitives: fills, exclusive scan, stable LSD radix sort (gfx950, wave64).
//
// The paper's orientation and directing steps use prefix sum, filter and integer sort
// (Sec. 2, parallel primitives); these are the project's own versions of them.
#include "common.h"

namespace arb {

// ------------------------------------------------------------------ errors

static thread_local int g_last_error = ARB_OK;
void set_error(int code) { g_last_error = code; }
int last_error() { return g_last_error; }

// ------------------------------------------------------------------ fills

template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
static int fill(T *p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return ARB_OK;
    k_fill<T><<<grid_for(n, 256, 4096), 256, 0, s>>>(p, v, n);
    ARB_CHECK_LAUNCH();
    return ARB_OK;
}
int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
int fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
int fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }

// ------------------------------------------------------------------ block scan

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

// Exclusive scan of one value per thread across a 256-thread block; *total gets the sum.
__device__ int64_t block_exclusive_scan(int64_t x, int64_t *lds_wave, int64_t *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t v = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int64_t y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
    }
    if (lane == 63) lds_wave[wid] = v;
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        int64_t t = lds_wave[w];
        if (w < wid) base += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + v - x;
}

__global__ void k_scan_reduce(const int64_t *in, int64_t n, int64_t *partial) {
    __shared__ int64_t lw[kScanBlock / 64];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t j = base + (int64_t)i * kScanBlock + threadIdx.x;
        if (j < n) s += in[j];
    }
    int64_t tot;
    block_exclusive_scan(s, lw, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One block scans all tile partials (exclusive, in place) and writes the grand total.
__global__ void k_scan_partials(int64_t *partial, int64_t ntiles, int64_t *total_out) {
    __shared__ int64_t lw[1024 / 64];
    int64_t carry = 0;
    for (int64_t b = 0; b < ntiles; b += blockDim.x) {
        int64_t j = b + threadIdx.x;
        int64_t x = j < ntiles ? partial[j] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan(x, lw, &tot);
        if (j < ntiles) partial[j] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_apply(const int64_t *in, int64_t *out, int64_t n, const int64_t *partial) {
    __shared__ int64_t lw[kScanBlock / 64];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t j = base + i;
        v[i] = j < n ? in[j] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan(s, lw, &tot) + partial[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t j = base + i;
        if (j < n) out[j] = ex;
        ex += v[i];
    }
}

// n <= one tile: the whole exclusive scan and the total (out[n]) in one block
__global__ void k_scan_single(const int64_t *in, int64_t *out, int64_t n) {
    __shared__ int64_t lw[kScanBlock / 64];
    const int64_t base = (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t j = base + i;
        v[i] = j < n ? in[j] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan(s, lw, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t j = base + i;
        if (j < n) out[j] = ex;
        ex += v[i];
    }
    if (threadIdx.x == 0) out[n] = tot;
}

size_t scan_workspace(int64_t n) {
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    return (size_t)(ntiles + 1) * sizeof(int64_t) + 256;
}

int exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, void *ws, hipStream_t s) {
    int64_t *partial = static_cast<int64_t *>(ws);
    if (n <= 0) {
        k_fill<int64_t><<<1, 64, 0, s>>>(out, 0, 1);
        ARB_CHECK_LAUNCH();
        return ARB_OK;
    }
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles == 1) {
        k_scan_single<<<1, kScanBlock, 0, s>>>(in, out, n);
        ARB_CHECK_LAUNCH();
        return ARB_OK;
    }
    // Blocked layout inside k_scan_apply (thread-contiguous runs) differs from the
    // strided one in k_scan_reduce, but both cover exactly one tile per block.
    k_scan_reduce<<<(unsigned)ntiles, kScanBlock, 0, s>>>(in, n, partial);
    ARB_CHECK_LAUNCH();
    k_scan_partials<<<1, 1024, 0, s>>>(partial, ntiles, out + n);
    ARB_CHECK_LAUNCH();
    k_scan_apply<<<(unsigned)ntiles, kScanBlock, 0, s>>>(in, out, n, partial);
    ARB_CHECK_LAUNCH();
    return ARB_OK;
}

// ------------------------------------------------------------------ radix sort

constexpr int kRsBlock = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsBlock * kRsItems;

// Digit histogram of each tile, stored digit-major: hist[d * ntiles + tile].
__global__ void k_rs_hist(const uint32_t *keys, int64_t n, int shift, int64_t ntiles, int64_t *hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int i = 0; i < kRsItems; ++i) {
        int64_t j = base + (int64_t)i * kRsBlock + threadIdx.x;
        if (j < n) atomicAdd(&h[(keys[j] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: inside a tile, elements keep their order among equal digits.  The tile
// is walked in 256-element chunks; inside a chunk, wave w's elements come before wave
// w+1's, and inside a wave, lower lanes first.
__global__ void k_rs_scatter(const uint32_t *keys, const int32_t *vals, uint32_t *okeys, int32_t *ovals,
                             int64_t n, int shift, int64_t ntiles, const int64_t *hist) {
    __shared__ int64_t tile_base[256];
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[kRsBlock / 64][256];
    __shared__ uint32_t wpre[kRsBlock / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    tile_base[tid] = hist[(int64_t)tid * ntiles + blockIdx.x];
    running[tid] = 0;
    const uint64_t below = lanes_below_mask();
    int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int c = 0; c < kRsItems; ++c) {
        int64_t j = base + (int64_t)c * kRsBlock + tid;
        bool valid = j < n;
        uint32_t key = valid ? keys[j] : 0u;
        int32_t val = valid ? vals[j] : 0;
        uint32_t dg = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (dg >> b) & 1u;
            uint64_t bb = __ballot(valid && bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t rank_w = (uint32_t)__popcll(peers & below);
        uint32_t cnt_w = (uint32_t)__popcll(peers);
#pragma unroll
        for (int w = 0; w < kRsBlock / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        if (valid && rank_w == 0) wcnt[wid][dg] = cnt_w;
        __syncthreads();
        {
            uint32_t run = running[tid];
#pragma unroll
            for (int w = 0; w < kRsBlock / 64; ++w) {
                wpre[w][tid] = run;
                run += wcnt[w][tid];
            }
            running[tid] = run;
        }
        __syncthreads();
        if (valid) {
            int64_t pos = tile_base[dg] + wpre[wid][dg] + rank_w;
            okeys[pos] = key;
            ovals[pos] = val;
        }
        (void)lane;
    }
}

template <class T>
__global__ void k_copy(const T *src, T *dst, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

size_t radix_workspace(int64_t n) {
    int64_t ntiles = (n + kRsTile - 1) / kRsTile;
    int64_t h = 256 * ntiles;
    return (size_t)(h + 1) * sizeof(int64_t) + scan_workspace(h) + 512;
}

int radix_sort_u32(uint32_t *keys, int32_t *vals, uint32_t *keys_alt, int32_t *vals_alt,
                   int64_t n, int key_bits, void *ws, hipStream_t s) {
    if (n <= 1) return ARB_OK;
    int64_t ntiles = (n + kRsTile - 1) / kRsTile;
    int64_t h = 256 * ntiles;
    Carver cv(ws);
    int64_t *hist = cv.take<int64_t>(h + 1);
    void *scan_ws = cv.take<char>(scan_workspace(h));
    uint32_t *ka = keys, *kb = keys_alt;
    int32_t *va = vals, *vb = vals_alt;
    int passes = 0;
    for (int shift = 0; shift < key_bits; shift += 8, ++passes) {
        k_rs_hist<<<(unsigned)ntiles, kRsBlock, 0, s>>>(ka, n, shift, ntiles, hist);
        ARB_CHECK_LAUNCH();
        int rc = exclusive_scan_i64(hist, hist, h, scan_ws, s);
        if (rc) return rc;
        k_rs_scatter<<<(unsigned)ntiles, kRsBlock, 0, s>>>(ka, va, kb, vb, n, shift, ntiles, hist);
        ARB_CHECK_LAUNCH();
        uint32_t *tk = ka; ka = kb; kb = tk;
        int32_t *tv = va; va = vb; vb = tv;
    }
    if (passes & 1) {
        k_copy<uint32_t><<<grid_for(n, 256, 4096), 256, 0, s>>>(ka, keys, n);
        ARB_CHECK_LAUNCH();
        k_copy<int32_t><<<grid_for(n, 256, 4096), 256, 0, s>>>(va, vals, n);
        ARB_CHECK_LAUNCH();
    }
    return ARB_OK;
}

}  // namespace arb
