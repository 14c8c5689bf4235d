// Learned cost model for scheduling: per-root features, an MLP 3 -> 64 -> 64 -> 64 -> 1
// with ReLU (bfloat16 weights, float32 arithmetic), its backward pass, the loss gradient
// and Adam.  The model predicts log2(1 + work) of a root, where work is the measure the
// counting kernels report (gathered words plus bitmap words of the search tree, the
// quantity whose total Sec. 3.2 bounds by O(m alpha^(k-2))), so that heavy roots are
// scheduled and split first.  Degree order is the fallback schedule.
#include "common.h"

namespace arb {

constexpr int H = 64;
constexpr int oW1 = 0, oB1 = oW1 + H * 3, oW2 = oB1 + H, oB2 = oW2 + H * H, oW3 = oB2 + H,
              oB3 = oW3 + H * H, oW4 = oB3 + H, oB4 = oW4 + H, NP = oB4 + 1;
static_assert(NP == ARB_MLP_PARAMS, "parameter layout");

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);       // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void load_weights(const uint16_t *wb, float *W) {
    for (int i = threadIdx.x; i < NP; i += blockDim.x) W[i] = bf16_to_f32(wb[i]);
    __syncthreads();
}

// ------------------------------------------------------------------ features

// A group of 16 lanes per row (four per wave); rows with more than 64 out-neighbours are
// summed by the whole wave after its groups' rows, four loads in flight per lane.
// Rows with fewer than dmin entries are skipped (their features are left as they were).
__global__ void k_feat_rows(int64_t n, const int64_t *off, const int32_t *idx, float *feat, int64_t dmin) {
    const int lane = threadIdx.x & 63, sl = lane & 15;
    int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) >> 4;
    for (; r - (lane >> 4) < n; r += ngrp) {          // while the wave's first group has a row
        int64_t s = 0, e = 0;
        bool on = false;
        if (r < n) {
            s = off[r];
            e = off[r + 1];
            on = e - s >= dmin;
            if (!on) e = s;
        }
        const bool big = e - s > 64;
        int64_t sum = 0;
        if (!big && e > s) {           // up to four entries per lane, their loads side by side
            int32_t u[4];
            int64_t lo[4], hi[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) u[q] = idx[s + sl + 16 * q < e ? s + sl + 16 * q : s];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lo[q] = off[u[q]];
                hi[q] = off[u[q] + 1];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (s + sl + 16 * q < e) sum += hi[q] - lo[q];
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 16);
        uint64_t m = __ballot(big && sl == 0);
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const int64_t ss = __shfl(s, src, 64), ee = __shfl(e, src, 64);
            int64_t part = 0;
            for (int64_t p0 = ss + lane; p0 < ee; p0 += 256) {
                int32_t u[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = p0 + 64 * q < ee ? idx[p0 + 64 * q] : -1;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (u[q] >= 0) part += off[u[q] + 1] - off[u[q]];
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
            if ((lane >> 4) == (src >> 4)) sum = part;
        }
        if (on && sl == 0) {
            feat[3 * r + 0] = log2f(1.0f + (float)(e - s));
            feat[3 * r + 1] = log2f(1.0f + (float)sum);
        }
    }
}

__global__ void k_feat_round(int64_t n, const int32_t *round_orig, const int32_t *rank, float *feat,
                             const int64_t *off, int64_t dmin) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rv = rank[v];
        if (dmin > 0 && off[rv + 1] - off[rv] < dmin) continue;
        feat[3 * rv + 2] = round_orig ? (float)round_orig[v] : 0.f;
    }
}

// ------------------------------------------------------------------ forward

// One row per thread; weights converted once per block into LDS and read as broadcasts.
__global__ void __launch_bounds__(256) k_mlp_fwd(const uint16_t *wb, const float *x, int64_t rows, float *y,
                                                  float *act) {
    __shared__ float W[NP];
    load_weights(wb, W);
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        const float x0 = x[3 * r], x1 = x[3 * r + 1], x2 = x[3 * r + 2];
        float h1[H], h2[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float z = W[oB1 + j];
            z = fmaf(W[oW1 + 3 * j + 0], x0, z);
            z = fmaf(W[oW1 + 3 * j + 1], x1, z);
            z = fmaf(W[oW1 + 3 * j + 2], x2, z);
            if (act) act[r * 192 + j] = z;
            h1[j] = fmaxf(z, 0.f);
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float z = W[oB2 + j];
#pragma unroll
            for (int i = 0; i < H; ++i) z = fmaf(W[oW2 + H * j + i], h1[i], z);
            if (act) act[r * 192 + 64 + j] = z;
            h2[j] = fmaxf(z, 0.f);
        }
        float out = W[oB4];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float z = W[oB3 + j];
#pragma unroll
            for (int i = 0; i < H; ++i) z = fmaf(W[oW3 + H * j + i], h2[i], z);
            if (act) act[r * 192 + 128 + j] = z;
            out = fmaf(W[oW4 + j], fmaxf(z, 0.f), out);
        }
        y[r] = out;
    }
}

// Inference on the matrix cores: each wave takes 16 rows at a time and computes the hidden
// layers transposed, H'^T = W H^T, with v_mfma_f32_16x16x16_bf16 (bf16 inputs, fp32
// accumulation).  The weights are bf16 already; each fp32 activation enters as the sum of
// two bf16 terms (hi = rne(h), lo = rne(h - hi)), so the products keep about 16 bits of
// the activation and the result agrees with the fp32 kernel to ~1e-5 relative.
// Operand layout of the 16x16x16 instruction (lane l, element e in 0..3):
//   A[i][k]: i = l % 16, k = 4 (l / 16) + e;  B[k][j]: k = 4 (l / 16) + e, j = l % 16;
//   D[i][j]: i = 4 (l / 16) + e, j = l % 16.
// With A = a 16x16 block of W (output unit x input unit) and B = a block of H^T (input
// unit x row), lane l holds the row r = l % 16 in both B and D, and D's 16x16 block nb of
// H'^T is exactly the B operand of block kb = nb for the next layer.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16v4 __attribute__((ext_vector_type(4)));

// hi = rne(h), lo = rne(h - hi) with the packed hardware conversion
__device__ __forceinline__ void split_bf16(const f32x4 h, bf16x4 &hi, bf16x4 &lo) {
    const bf16v4 a = __builtin_convertvector(h, bf16v4);
    const bf16v4 b = __builtin_convertvector(h - __builtin_convertvector(a, f32x4), bf16v4);
    hi = __builtin_bit_cast(bf16x4, a);
    lo = __builtin_bit_cast(bf16x4, b);
}

// With off != nullptr (the schedule's use), tiles whose 16 roots all have fewer than
// dmin out-neighbours (roots whose cost the schedule does not read) are skipped; their y
// stays unset.
__global__ void __launch_bounds__(256) k_mlp_fwd_mfma(const uint16_t *wb, const float *x, int64_t rows, float *y,
                                                       const int64_t *off, int64_t dmin) {
    __shared__ float W[NP];
    load_weights(wb, W);
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, q = lane >> 4;
    // A operands of layers 2 and 3: W[nb*16 + r16][kb*16 + 4q .. +3]
    // (from the block's float copy: exact, the weights are bf16 values)
    bf16x4 A2[4][4], A3[4][4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = (nb * 16 + r16) * H + kb * 16 + 4 * q + e;
                A2[nb][kb][e] = (short)f32_to_bf16(W[oW2 + o]);
                A3[nb][kb][e] = (short)f32_to_bf16(W[oW3 + o]);
            }
    const int64_t tiles = (rows + 15) / 16;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t t = wave; t < tiles; t += nwaves) {
        const int64_t r = t * 16 + r16;
        const bool live = r < rows;
        if (off && !__any(live && off[r + 1] - off[r] >= dmin)) continue;
        const float x0 = live ? x[3 * r] : 0.f, x1 = live ? x[3 * r + 1] : 0.f, x2 = live ? x[3 * r + 2] : 0.f;
        // layer 1 (VALU) straight into B layout: units kb*16 + 4q + e of row r
        bf16x4 Bhi[4], Blo[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            f32x4 h;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = kb * 16 + 4 * q + e;
                float z = W[oB1 + j];
                z = fmaf(W[oW1 + 3 * j + 0], x0, z);
                z = fmaf(W[oW1 + 3 * j + 1], x1, z);
                z = fmaf(W[oW1 + 3 * j + 2], x2, z);
                h[e] = fmaxf(z, 0.f);
            }
            split_bf16(h, Bhi[kb], Blo[kb]);
        }
        // layers 2 and 3 on the matrix cores
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            const int ob = layer == 0 ? oB2 : oB3;
            f32x4 D[4];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
                for (int e = 0; e < 4; ++e) D[nb][e] = W[ob + nb * 16 + 4 * q + e];
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    const bf16x4 a = layer == 0 ? A2[nb][kb] : A3[nb][kb];
                    D[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, Bhi[kb], D[nb], 0, 0, 0);
                    D[nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, Blo[kb], D[nb], 0, 0, 0);
                }
            }
            if (layer == 0) {
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    f32x4 h;
#pragma unroll
                    for (int e = 0; e < 4; ++e) h[e] = fmaxf(D[nb][e], 0.f);
                    split_bf16(h, Bhi[nb], Blo[nb]);
                }
            } else {
                // layer 4: this lane's 16 units of row r, then the four lanes of the row
                float out = 0.f;
#pragma unroll
                for (int nb = 0; nb < 4; ++nb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) out = fmaf(W[oW4 + nb * 16 + 4 * q + e], fmaxf(D[nb][e], 0.f), out);
                out += __shfl_xor(out, 16, 64);
                out += __shfl_xor(out, 32, 64);
                if (q == 0 && live) y[r] = out + W[oB4];
            }
        }
    }
}

// ------------------------------------------------------------------ backward

// Per row: deltas of the three hidden layers (pre-activation gradients) from dy.
__global__ void __launch_bounds__(256) k_mlp_deltas(const uint16_t *wb, const float *act, const float *dy,
                                                     int64_t rows, float *delta) {
    __shared__ float W[NP];
    load_weights(wb, W);
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        const float g = dy[r];
        float d3[H], d2[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            d3[j] = act[r * 192 + 128 + j] > 0.f ? g * W[oW4 + j] : 0.f;
            delta[r * 192 + 128 + j] = d3[j];
        }
#pragma unroll
        for (int i = 0; i < H; ++i) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < H; ++j) s = fmaf(W[oW3 + H * j + i], d3[j], s);
            d2[i] = act[r * 192 + 64 + i] > 0.f ? s : 0.f;
            delta[r * 192 + 64 + i] = d2[i];
        }
#pragma unroll
        for (int i = 0; i < H; ++i) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < H; ++j) s = fmaf(W[oW2 + H * j + i], d2[j], s);
            delta[r * 192 + i] = act[r * 192 + i] > 0.f ? s : 0.f;
        }
    }
}

constexpr int kGradRows = 256;   // rows per partial-gradient block
constexpr int kGradTile = 16;    // rows staged in LDS at a time

// Partial gradients of one block of rows: part[blockIdx][p] for all parameters.
__global__ void __launch_bounds__(256) k_mlp_grad_part(const float *x, const float *act, const float *delta,
                                                        const float *dy, int64_t rows, float *part) {
    __shared__ float sx[kGradTile][3], sdy[kGradTile];
    __shared__ float sh[kGradTile][192];   // relu(z): h1, h2, h3
    __shared__ float sd[kGradTile][192];   // deltas d1, d2, d3
    const int t = threadIdx.x;
    // parameter ownership: thread t owns W2/W3 entries t + 256 q (q < 16), plus the small ones
    float aw2[16], aw3[16];
    float a_small[2] = {0.f, 0.f};   // entries t and t+256 of [W1 (192) | b1 b2 b3 (192) | W4 (64) | b4 (1)] = 449
#pragma unroll
    for (int q = 0; q < 16; ++q) { aw2[q] = 0.f; aw3[q] = 0.f; }
    const int64_t r0 = (int64_t)blockIdx.x * kGradRows;
    const int64_t r1 = min(r0 + kGradRows, rows);
    for (int64_t rb = r0; rb < r1; rb += kGradTile) {
        const int nr = (int)min<int64_t>(kGradTile, r1 - rb);
        __syncthreads();
        for (int i = t; i < kGradTile * 192; i += 256) {
            const int rr = i / 192, c = i % 192;
            float z = rr < nr ? act[(rb + rr) * 192 + c] : 0.f;
            sh[rr][c] = fmaxf(z, 0.f);
            sd[rr][c] = rr < nr ? delta[(rb + rr) * 192 + c] : 0.f;
        }
        if (t < kGradTile * 3) {
            const int rr = t / 3, c = t % 3;
            sx[rr][c] = rr < nr ? x[(rb + rr) * 3 + c] : 0.f;
        }
        if (t < kGradTile) sdy[t] = t < nr ? dy[rb + t] : 0.f;
        __syncthreads();
        for (int rr = 0; rr < nr; ++rr) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int e = t + 256 * q;           // entry e of a 64x64 matrix: row j = e/64, col i = e%64
                const int j = e >> 6, i = e & 63;
                aw2[q] = fmaf(sd[rr][64 + j], sh[rr][i], aw2[q]);        // dW2[j][i] = d2[j] h1[i]
                aw3[q] = fmaf(sd[rr][128 + j], sh[rr][64 + i], aw3[q]);  // dW3[j][i] = d3[j] h2[i]
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int e = t + 256 * q;
                float v = 0.f;
                if (e < 192) v = sd[rr][e / 3] * sx[rr][e % 3];            // dW1[j][c] = d1[j] x[c]
                else if (e < 384) v = sd[rr][e - 192];                      // db1, db2, db3
                else if (e < 448) v = sdy[rr] * sh[rr][128 + (e - 384)];    // dW4[j] = dy h3[j]
                else if (e == 448) v = sdy[rr];                             // db4
                a_small[q] += v;
            }
        }
    }
    float *out = part + (int64_t)blockIdx.x * NP;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = t + 256 * q;
        out[oW2 + e] = aw2[q];
        out[oW3 + e] = aw3[q];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = t + 256 * q;
        if (e < 192) out[oW1 + e] = a_small[q];
        else if (e < 256) out[oB1 + (e - 192)] = a_small[q];
        else if (e < 320) out[oB2 + (e - 256)] = a_small[q];
        else if (e < 384) out[oB3 + (e - 320)] = a_small[q];
        else if (e < 448) out[oW4 + (e - 384)] = a_small[q];
        else if (e == 448) out[oB4] = a_small[q];
    }
}

// grad[p] = sum over blocks of part[b][p], in block order (deterministic).
__global__ void k_mlp_grad_sum(const float *part, int nblocks, float *grad) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NP; p += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * NP + p];
        grad[p] = s;
    }
}

// dy = (y - t) / N; loss = sum (y - t)^2 / (2N) (one block, fixed order).
__global__ void k_mse(const float *y, const float *tgt, int64_t rows, float *dy, float *loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
        const float e = y[r] - tgt[r];
        dy[r] = e / (float)rows;
        s += (double)e * (double)e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = (float)(red[0] / (2.0 * (double)rows));
}

__global__ void k_adam(float *w, uint16_t *wb, const float *g, float *m, float *v, float lr, float c1, float c2) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < NP; p += gridDim.x * blockDim.x) {
        const float gp = g[p];
        const float mp = b1 * m[p] + (1.f - b1) * gp;
        const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
        m[p] = mp;
        v[p] = vp;
        const float mh = mp / c1, vh = vp / c2;
        const float wp = w[p] - lr * mh / (sqrtf(vh) + eps);
        w[p] = wp;
        wb[p] = f32_to_bf16(wp);
    }
}

__global__ void k_to_bf16(const float *w, uint16_t *wb, int64_t n) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        wb[p] = f32_to_bf16(w[p]);
}

int learned_cost(const arb_ocsr *dg, int k, const uint16_t *w, const float *feat, float *cost, hipStream_t s) {
    if (dg->n == 0) return ARB_OK;
    // the schedule reads the cost of roots above the 64-tier only
    const int64_t dmin = k - 1 > 65 ? k - 1 : 65;
    k_mlp_fwd_mfma<<<grid_for((dg->n + 15) / 16 * 64, 256, 512), 256, 0, s>>>(w, feat, dg->n, cost, dg->offsets, dmin);
    ARB_CHECK_LAUNCH();
    return ARB_OK;
}

}  // namespace arb

using namespace arb;

extern "C" int arb_features_min_degree(const arb_ocsr *dg, const int32_t *round_orig, const int32_t *rank,
                                       int64_t min_degree, float *feat, void *stream) {
    hipStream_t s = as_stream(stream);
    if (!dg || !feat || dg->n < 0 || !dg->offsets || (dg->m > 0 && !dg->indices) || (round_orig && !rank) ||
        min_degree < 0) {
        set_error(ARB_EINVAL);
        return ARB_EINVAL;
    }
    const int64_t n = dg->n;
    if (n > 0) {
        k_feat_rows<<<grid_for(n * 16, 256, 8192), 256, 0, s>>>(n, dg->offsets, dg->indices, feat, min_degree);
        if (rank)
            k_feat_round<<<grid_for(n, 256, 4096), 256, 0, s>>>(n, round_orig, rank, feat, dg->offsets, min_degree);
        else
            k_feat_round<<<1, 64, 0, s>>>(0, nullptr, nullptr, feat, nullptr, 0);
        if (hipGetLastError() != hipSuccess) { set_error(ARB_EHIP); return ARB_EHIP; }
    }
    set_error(ARB_OK);
    return ARB_OK;
}

extern "C" int arb_features(const arb_ocsr *dg, const int32_t *round_orig, const int32_t *rank, float *feat,
                            void *stream) {
    return arb_features_min_degree(dg, round_orig, rank, 0, feat, stream);
}

extern "C" int arb_mlp_forward(const uint16_t *w_bf16, const float *x, int64_t rows, float *y, float *act,
                               void *stream) {
    if (!w_bf16 || (rows > 0 && (!x || !y)) || rows < 0) { set_error(ARB_EINVAL); return ARB_EINVAL; }
    if (rows > 0) {
        if (act)
            k_mlp_fwd<<<grid_for(rows, 256, 4096), 256, 0, as_stream(stream)>>>(w_bf16, x, rows, y, act);
        else
            k_mlp_fwd_mfma<<<grid_for((rows + 15) / 16 * 64, 256, 512), 256, 0, as_stream(stream)>>>(w_bf16, x, rows,
                                                                                                    y, nullptr, 0);
        if (hipGetLastError() != hipSuccess) { set_error(ARB_EHIP); return ARB_EHIP; }
    }
    set_error(ARB_OK);
    return ARB_OK;
}

extern "C" size_t arb_mlp_workspace(int64_t rows) {
    const int64_t nb = (rows + kGradRows - 1) / kGradRows;
    return (size_t)(rows * 192 + (nb > 0 ? nb : 1) * NP) * sizeof(float) + 512;
}

extern "C" int arb_mlp_backward(const uint16_t *w_bf16, const float *x, const float *act, const float *dy,
                                int64_t rows, float *grad, void *ws, size_t ws_bytes, void *stream) {
    hipStream_t s = as_stream(stream);
    if (!w_bf16 || !grad || rows < 1 || !x || !act || !dy || !ws) { set_error(ARB_EINVAL); return ARB_EINVAL; }
    if (ws_bytes < arb_mlp_workspace(rows)) { set_error(ARB_EWORKSPACE); return ARB_EWORKSPACE; }
    Carver cv(ws);
    float *delta = cv.take<float>(rows * 192);
    const int nb = (int)((rows + kGradRows - 1) / kGradRows);
    float *part = cv.take<float>((size_t)nb * NP);
    k_mlp_deltas<<<grid_for(rows, 256, 4096), 256, 0, s>>>(w_bf16, act, dy, rows, delta);
    k_mlp_grad_part<<<nb, 256, 0, s>>>(x, act, delta, dy, rows, part);
    k_mlp_grad_sum<<<grid_for(NP, 256), 256, 0, s>>>(part, nb, grad);
    if (hipGetLastError() != hipSuccess) { set_error(ARB_EHIP); return ARB_EHIP; }
    set_error(ARB_OK);
    return ARB_OK;
}

extern "C" int arb_mse_grad(const float *y, const float *target, int64_t rows, float *dy, float *loss, void *stream) {
    if (!y || !target || !dy || rows < 1) { set_error(ARB_EINVAL); return ARB_EINVAL; }
    k_mse<<<1, 256, 0, as_stream(stream)>>>(y, target, rows, dy, loss);
    if (hipGetLastError() != hipSuccess) { set_error(ARB_EHIP); return ARB_EHIP; }
    set_error(ARB_OK);
    return ARB_OK;
}

extern "C" int arb_adam_step(float *w, uint16_t *w_bf16, const float *grad, float *m, float *v, float lr, int step,
                             void *stream) {
    if (!w || !w_bf16 || !grad || !m || !v || step < 1 || !(lr > 0.f)) { set_error(ARB_EINVAL); return ARB_EINVAL; }
    const float c1 = 1.f - powf(0.9f, (float)step), c2 = 1.f - powf(0.999f, (float)step);
    k_adam<<<grid_for(NP, 256), 256, 0, as_stream(stream)>>>(w, w_bf16, grad, m, v, lr, c1, c2);
    if (hipGetLastError() != hipSuccess) { set_error(ARB_EHIP); return ARB_EHIP; }
    set_error(ARB_OK);
    return ARB_OK;
}

extern "C" int arb_to_bf16(const float *w, uint16_t *w_bf16, int64_t count, void *stream) {
    if (!w || !w_bf16 || count < 0) { set_error(ARB_EINVAL); return ARB_EINVAL; }
    if (count > 0) {
        k_to_bf16<<<grid_for(count, 256, 4096), 256, 0, as_stream(stream)>>>(w, w_bf16, count);
        if (hipGetLastError() != hipSuccess) { set_error(ARB_EHIP); return ARB_EHIP; }
    }
    set_error(ARB_OK);
    return ARB_OK;
}
