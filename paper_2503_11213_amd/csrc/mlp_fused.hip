// Fused inference of the PSF surrogate MLP (Sec. 3.2, Supplement S1.4):
// Fourier encoding, every hidden layer and the softmax output layer in one
// kernel, so activations never leave LDS and logits never leave registers.
//
// A workgroup of four waves owns 64 rows.  Hidden layers: the bf16
// activations [64][256] live in LDS (double buffer); wave w computes output
// columns [64 w, 64 w + 64) with v_mfma_f32_16x16x32_bf16, its weight
// fragments read straight from L2 (the whole bf16 network is 1.8 MB) one
// k-step ahead of use.  Output layer (2 ks^2 columns, tiles of 64): pass 1
// computes each tile's logits and keeps a running (max, sum of exp) per row
// and lane; the lanes of a row and then the four waves merge them; pass 2
// recomputes the tiles and writes softmax probabilities (bf16 or float32).
// The recomputation doubles the output layer's matrix work but removes the
// float32 logit round trip through HBM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/sdirt.h"

namespace sdirt {

typedef uint16_t bf16_t;
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

constexpr int kFRows = 64;             // rows per workgroup
constexpr int kFWidth = 256;           // hidden width (fixed)
constexpr int kFStride = kFWidth + 8;  // LDS row stride in bf16 (bank spread)
constexpr int kFThreads = 256;

struct FusedArgs {
    long long n_rows;
    int n_hidden, n_out, n_freq, feat_pad;
    float x_half, y_half, iv_lo, iv_hi, lam_lo, lam_hi;
    const float* x;                 // [n_rows][4]
    const float* params;            // float32 master (biases)
    long long b_off[17];            // bias offsets per layer
    const bf16_t* W[17];            // bf16 weights [out][in_pad]
    void* out;                      // [n_rows][n_out]
    int out_bf16;
};

__device__ inline bf16_t f2bf_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

__device__ inline bf16x8_t load_b8(const bf16_t* p) {
    return *reinterpret_cast<const bf16x8_t*>(p);
}

__device__ inline void merge_ms(float& m, float& s, float m2, float s2) {
    const float mn = fmaxf(m, m2);
    s = (m == -INFINITY ? 0.f : s * __expf(m - mn)) + (m2 == -INFINITY ? 0.f : s2 * __expf(m2 - mn));
    m = mn;
}

// acc[i][j] = H[rows 16 i ..][0..K) x W[cols 16 j ..][0..K)^T for this wave's
// column block; B fragments prefetched one k-step ahead.
__device__ inline void layer_mma(const bf16_t* H, const bf16_t* W, int ldw, int K, int col0,
                                 int n_valid, floatx4_t acc[4][4]) {
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, kg = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    bf16x8_t b[4], bn[4];
    const bf16x8_t zero = {};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = col0 + 16 * j + r16;
        b[j] = n < n_valid ? load_b8(W + (size_t)n * ldw + kg) : zero;
    }
    for (int k0 = 0; k0 < K; k0 += 32) {
        if (k0 + 32 < K) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n = col0 + 16 * j + r16;
                bn[j] = n < n_valid ? load_b8(W + (size_t)n * ldw + k0 + 32 + kg) : zero;
            }
        }
        bf16x8_t a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a[i] = *reinterpret_cast<const bf16x8_t*>(H + (16 * i + r16) * kFStride + k0 + kg);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (k0 + 32 < K) {
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = bn[j];
        }
    }
}

__global__ __launch_bounds__(kFThreads) void mlp_fused_fwd_kernel(const FusedArgs A) {
    __shared__ bf16_t H[2][kFRows * kFStride];
    __shared__ float stat_m[4][kFRows], stat_s[4][kFRows];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g4 = (lane >> 4) * 4;
    const long long row0 = (long long)blockIdx.x * kFRows;
    // ---- encoding: 64 rows x feat_pad features, 4 threads per row ----------
    {
        const int row = tid >> 2, part = tid & 3;     // input `part` of the row
        const long long gr = row0 + row;
        float v = 0.f;
        if (gr < A.n_rows) {
            const float xv = A.x[gr * 4 + part];
            if (part == 0) v = xv / A.x_half;
            else if (part == 1) v = xv / A.y_half;
            else if (part == 2) v = 2.f * (xv - A.iv_lo) / (A.iv_hi - A.iv_lo) - 1.f;
            else v = 2.f * (xv - A.lam_lo) / (A.lam_hi - A.lam_lo) - 1.f;
        }
        bf16_t* h = H[0] + row * kFStride + part * 2 * A.n_freq;
        float sc = 1.f;
        for (int k = 0; k < A.n_freq; ++k) {
            float s, c;
            sincospif(sc * v, &s, &c);
            h[2 * k] = f2bf_rne(s);
            h[2 * k + 1] = f2bf_rne(c);
            sc *= 2.f;
        }
        for (int f = 8 * A.n_freq + part; f < A.feat_pad; f += 4) H[0][row * kFStride + f] = 0;
    }
    __syncthreads();
    // ---- hidden layers ------------------------------------------------------
    int cur = 0;
    floatx4_t acc[4][4];
    for (int l = 0; l < A.n_hidden; ++l) {
        const int K = l == 0 ? A.feat_pad : kFWidth;
        const int col0 = wave * 64;
        layer_mma(H[cur], A.W[l], K, K, col0, kFWidth, acc);
        const float* bias = A.params + A.b_off[l];
        bf16_t* Ho = H[1 - cur];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = col0 + 16 * j + r16;
            const float bn = bias[n];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Ho[(16 * i + g4 + r) * kFStride + n] = f2bf_rne(fmaxf(acc[i][j][r] + bn, 0.f));
        }
        __syncthreads();
        cur = 1 - cur;
    }
    // ---- output layer: pass 1, running max / sum per row ---------------------
    const int Lo = A.n_hidden;
    const bf16_t* Wo = A.W[Lo];
    const float* bo = A.params + A.b_off[Lo];
    const int ntile = (A.n_out + 63) / 64;
    float m[16], s[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) { m[k] = -INFINITY; s[k] = 0.f; }
    for (int t = wave; t < ntile; t += 4) {
        layer_mma(H[cur], Wo, kFWidth, kFWidth, 64 * t, A.n_out, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float tm = -INFINITY;
                float z[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int n = 64 * t + 16 * j + r16;
                    z[j] = n < A.n_out ? acc[i][j][r] + bo[n] : -INFINITY;
                    tm = fmaxf(tm, z[j]);
                }
                float ts = 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) ts += z[j] == -INFINITY ? 0.f : __expf(z[j] - tm);
                merge_ms(m[4 * i + r], s[4 * i + r], tm, ts);
            }
    }
    // merge over the 16 lanes holding the same rows, then over the 4 waves
#pragma unroll
    for (int k = 0; k < 16; ++k) {
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const float m2 = __shfl_xor(m[k], o, 64);
            const float s2 = __shfl_xor(s[k], o, 64);
            merge_ms(m[k], s[k], m2, s2);
        }
    }
    if (r16 == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                stat_m[wave][16 * i + g4 + r] = m[4 * i + r];
                stat_s[wave][16 * i + g4 + r] = s[4 * i + r];
            }
    }
    __syncthreads();
    float inv_s[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * i + g4 + r;
            float mm = stat_m[0][row], ss = stat_s[0][row];
            for (int w = 1; w < 4; ++w) merge_ms(mm, ss, stat_m[w][row], stat_s[w][row]);
            m[4 * i + r] = mm;
            inv_s[4 * i + r] = ss > 0.f ? 1.f / ss : 0.f;
        }
    // ---- pass 2: recompute and write probabilities ---------------------------
    for (int t = wave; t < ntile; t += 4) {
        layer_mma(H[cur], Wo, kFWidth, kFWidth, 64 * t, A.n_out, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = 64 * t + 16 * j + r16;
            if (n >= A.n_out) continue;
            const float bn = bo[n];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const long long gr = row0 + 16 * i + g4 + r;
                    if (gr >= A.n_rows) continue;
                    const float p = __expf(acc[i][j][r] + bn - m[4 * i + r]) * inv_s[4 * i + r];
                    if (A.out_bf16) reinterpret_cast<bf16_t*>(A.out)[gr * A.n_out + n] = f2bf_rne(p);
                    else reinterpret_cast<float*>(A.out)[gr * A.n_out + n] = p;
                }
        }
    }
}

int launch_mlp_fused(const FusedArgs& A, hipStream_t st) {
    if (A.n_rows <= 0) return SDIRT_OK;
    const long long blocks = (A.n_rows + kFRows - 1) / kFRows;
    if (blocks > 0x7fffffffLL) return SDIRT_EUNSUPPORTED;
    hipLaunchKernelGGL(mlp_fused_fwd_kernel, dim3((unsigned)blocks), dim3(kFThreads), 0, st, A);
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

}  // namespace sdirt
