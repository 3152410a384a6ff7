// DP-PSF surrogate MLP (Sec. 3.2, Supplement S1.4) on gfx950 matrix cores.
//
// Network: Fourier encoding of (h_x, h_y, 1/d, lambda) to 64 features, five
// ReLU layers of width 256, a linear layer to 2 x ks x ks logits and a joint
// softmax (the sum-normalised left/right PSF).  Training loss: the squared
// error of each output scaled by the largest value of its target PSF
// (max-normalised targets), averaged over the batch; Adam.
//
// Every matrix product runs in one bf16 "NT" GEMM kernel, C = A B^T with A
// [M][K] and B [N][K] both K-contiguous, on v_mfma_f32_16x16x32_bf16 with
// float32 accumulation: 128 x 128 output tiles, four waves of 64 x 64, K in
// steps of 64 through padded LDS tiles.  Epilogues fuse bias, ReLU, the ReLU
// derivative mask, column sums (bias gradients), bf16 conversion and a
// transposed bf16 copy (the operand layout of the weight-gradient GEMMs).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/sdirt.h"
#include "mlp_fused.hpp"

namespace sdirt {

int launch_fill_zero(void* p, size_t bytes, hipStream_t stream);

typedef uint16_t bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __host__ inline bf16_t f2bf(float f) {
    // round to nearest even
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40);   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

__device__ inline float bf2f(bf16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

constexpr int kGB = 256;               // threads per GEMM block
constexpr int kBM = 128, kBN = 128, kBK = 64;
constexpr int kLdsStride = kBK + 8;    // bf16 elements per LDS row (padding)

struct GemmArgs {
    const bf16_t* A; int lda;     // [M][K]
    const bf16_t* B; int ldb;     // [N][K]
    int M, N, K;                  // K % kBK == 0, operands zero-padded in K
    const float* bias;            // [N] or null
    int relu;
    const bf16_t* mask; int ldm;  // multiply by (mask[m][n] > 0) or null
    float* Cf; int ldcf;          // float32 result or null
    bf16_t* Cb; int ldcb;         // bf16 result or null
    bf16_t* CbT; int ldcbt;       // bf16 transposed result [N][M] or null
    float* colpart;               // partial column sums of the result or null:
                                  // row 2 (m / 128) + (m % 128) / 64 of
                                  // [2 ceil(M / 128)][N], each written once
};

__global__ __launch_bounds__(kGB) void gemm_nt_kernel(const GemmArgs g) {
    __shared__ bf16_t sA[kBM * kLdsStride];
    __shared__ bf16_t sB[kBN * kLdsStride];
    const int tiles_n = (g.N + kBN - 1) / kBN;
    const int bm = blockIdx.x / tiles_n, bn = blockIdx.x % tiles_n;
    const int m0 = bm * kBM, n0 = bn * kBN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int r16 = lane & 15, kg = (lane >> 4) * 8;
    // global -> register staging of one 128 x 64 tile of A and of B: each
    // thread moves 4 x 16 B of each; the next tile's loads are in flight
    // while the current tile feeds the matrix cores.
    uint4 ra[4], rb[4];
    auto load_tile = [&](int k0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int e = tid + t * kGB;
            const int row = e >> 3, seg = (e & 7) * 8;
            ra[t] = uint4{0u, 0u, 0u, 0u};
            rb[t] = uint4{0u, 0u, 0u, 0u};
            if (m0 + row < g.M)
                ra[t] = *reinterpret_cast<const uint4*>(g.A + (size_t)(m0 + row) * g.lda + k0 + seg);
            if (n0 + row < g.N)
                rb[t] = *reinterpret_cast<const uint4*>(g.B + (size_t)(n0 + row) * g.ldb + k0 + seg);
        }
    };
    load_tile(0);
    for (int k0 = 0; k0 < g.K; k0 += kBK) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int e = tid + t * kGB;
            const int row = e >> 3, seg = (e & 7) * 8;
            *reinterpret_cast<uint4*>(&sA[row * kLdsStride + seg]) = ra[t];
            *reinterpret_cast<uint4*>(&sB[row * kLdsStride + seg]) = rb[t];
        }
        __syncthreads();
        if (k0 + kBK < g.K) load_tile(k0 + kBK);
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 32) {
            bf16x8 af[4], bfr[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                af[i] = *reinterpret_cast<const bf16x8*>(&sA[(wm + i * 16 + r16) * kLdsStride + kk + kg]);
                bfr[i] = *reinterpret_cast<const bf16x8*>(&sB[(wn + i * 16 + r16) * kLdsStride + kk + kg]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // epilogue: lane holds C[wm + 16 i + 4 (lane / 16) + r][wn + 16 j + lane % 16]
    const int rbase = (lane >> 4) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = n0 + wn + j * 16 + r16;
        const bool nok = n < g.N;
        const float b = (g.bias && nok) ? g.bias[n] : 0.f;
        float csum = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + rbase + r;
                if (!nok || m >= g.M) continue;
                float v = acc[i][j][r] + b;
                if (g.relu) v = fmaxf(v, 0.f);
                if (g.mask && !(bf2f(g.mask[(size_t)m * g.ldm + n]) > 0.f)) v = 0.f;
                csum += v;
                if (g.Cf) g.Cf[(size_t)m * g.ldcf + n] = v;
                const bf16_t vb = f2bf(v);
                if (g.Cb) g.Cb[(size_t)m * g.ldcb + n] = vb;
                if (g.CbT) g.CbT[(size_t)n * g.ldcbt + m] = vb;
            }
        }
        if (g.colpart) {
            // lanes l, l+16, l+32, l+48 share the column: the wave's 64 rows
            // of it, stored (not accumulated) so that the final sum over
            // the parts has a fixed order
            csum += __shfl_xor(csum, 16, 64);
            csum += __shfl_xor(csum, 32, 64);
            if (nok && lane < 16) g.colpart[(size_t)(2 * bm + (wave >> 1)) * g.N + n] = csum;
        }
    }
}

// ---- network pieces -------------------------------------------------------

struct MlpDims {
    int n_hidden, width, n_out, n_freq, n_feat, n_out_pad, loss;
    int L;                              // number of linear layers
    int in_of(int l) const { return l == 0 ? n_feat : width; }
    int out_of(int l) const { return l == L - 1 ? n_out : width; }
    size_t w_off(int l) const {         // offset of W_l in the parameter vector
        size_t o = 0;
        for (int q = 0; q < l; ++q) o += (size_t)out_of(q) * in_of(q) + out_of(q);
        return o;
    }
    size_t b_off(int l) const { return w_off(l) + (size_t)out_of(l) * in_of(l); }
    size_t n_params() const { return w_off(L); }
    int ld_out(int l) const { return l == L - 1 ? n_out_pad : width; }
};

static int dims_of(const sdirt_mlp_desc* d, MlpDims* m) {
    if (!d) return SDIRT_EINVAL;
    if (d->n_hidden < 1 || d->n_hidden > 16 || d->width < 64 || d->width % 64 ||
        d->width > 4096 || d->n_out < 1 || d->n_out > 65536 || d->n_freq < 1 || d->n_freq > 16)
        return SDIRT_EINVAL;
    if (!(d->x_half > 0) || !(d->y_half > 0) || !(d->iv_hi > d->iv_lo) || !(d->lam_hi > d->lam_lo))
        return SDIRT_EINVAL;
    if (d->loss != SDIRT_LOSS_L2MAX && d->loss != SDIRT_LOSS_KL) return SDIRT_EINVAL;
    m->loss = d->loss;
    m->n_hidden = d->n_hidden;
    m->width = d->width;
    m->n_out = d->n_out;
    m->n_freq = d->n_freq;
    m->n_feat = 2 * d->n_freq * 4;
    m->n_out_pad = ((d->n_out + kBK - 1) / kBK) * kBK;
    m->L = d->n_hidden + 1;
    return SDIRT_OK;
}

static int feat_pad(const MlpDims& m) { return ((m.n_feat + kBK - 1) / kBK) * kBK; }

// Workspace carve-up for a batch of B rows (B % 64 == 0).
struct MlpWs {
    bf16_t* W[17];   // [out][in_pad]
    bf16_t* WT[17];  // [in][out_pad]
    bf16_t* WF[17];  // fragment-major copy for the fused inference kernels
    bf16_t* H[17];   // H[0] features [B][feat_pad]; H[l] [B][width]
    bf16_t* HT[17];  // transposed [width or feat_pad][B]
    float* logits;   // [B][n_out]
    float* dz;       // [B][n_out]
    bf16_t* dzb;     // [B][n_out_pad]
    bf16_t* dzT;     // [n_out_pad][B]
    bf16_t* dA[2];   // ping-pong [B][width]
    bf16_t* dAT[2];  // [width][B]
    float* grads;    // [n_params]
    float* part;     // [2 ceil(B / 128)][width] partial bias-gradient sums
    float* target;   // [B][n_out] (training gather)
    float* xb;       // [B][4]
    float* loss;     // [1]
    size_t bytes;
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static MlpWs carve(const MlpDims& m, int B, char* base) {
    MlpWs w;
    std::memset(&w, 0, sizeof(w));
    size_t off = 0;
    auto take = [&](size_t bytes) { char* p = base ? base + off : nullptr; off += align256(bytes); return p; };
    const int fp = feat_pad(m);
    for (int l = 0; l < m.L; ++l) {
        const int in_pad = l == 0 ? fp : m.width;
        const int out = m.out_of(l);
        const int out_pad = l == m.L - 1 ? m.n_out_pad : m.width;
        w.W[l] = (bf16_t*)take((size_t)out * in_pad * 2);
        w.WT[l] = (bf16_t*)take((size_t)in_pad * out_pad * 2);
        w.WF[l] = (bf16_t*)take((size_t)((out + 63) / 64) * 64 * in_pad * 2);
    }
    w.H[0] = (bf16_t*)take((size_t)B * fp * 2);
    w.HT[0] = (bf16_t*)take((size_t)fp * B * 2);
    for (int l = 1; l < m.L; ++l) {
        w.H[l] = (bf16_t*)take((size_t)B * m.width * 2);
        w.HT[l] = (bf16_t*)take((size_t)m.width * B * 2);
    }
    w.logits = (float*)take((size_t)B * m.n_out * 4);
    w.dz = (float*)take((size_t)B * m.n_out * 4);
    w.dzb = (bf16_t*)take((size_t)B * m.n_out_pad * 2);
    w.dzT = (bf16_t*)take((size_t)m.n_out_pad * B * 2);
    for (int k = 0; k < 2; ++k) {
        w.dA[k] = (bf16_t*)take((size_t)B * m.width * 2);
        w.dAT[k] = (bf16_t*)take((size_t)m.width * B * 2);
    }
    w.grads = (float*)take(m.n_params() * 4);
    w.part = (float*)take((size_t)2 * ((B + 127) / 128) * m.width * 4);
    w.target = (float*)take((size_t)B * m.n_out * 4);
    w.xb = (float*)take((size_t)B * 4 * 4);
    w.loss = (float*)take(256);
    w.bytes = off;
    return w;
}

// float32 master parameters -> bf16 W [out][in_pad] and W^T [in][out_pad]
__global__ void cast_weights_kernel(const float* W, int out, int in, int in_pad, int out_pad,
                                    bf16_t* Wb, bf16_t* WTb) {
    const size_t n = (size_t)out_pad * in_pad;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const int o = (int)(e / in_pad), i = (int)(e % in_pad);
        const float v = (o < out && i < in) ? W[(size_t)o * in + i] : 0.f;
        const bf16_t b = f2bf(v);
        if (o < out) Wb[(size_t)o * in_pad + i] = b;
        WTb[(size_t)i * out_pad + o] = b;
    }
}

// float32 master parameters -> bf16 in matrix-core fragment order for the
// fused inference kernels: WF[((nb * KS + ks) * 64 + lane) * 8 + e] holds
// W[16 nb + lane % 16][32 ks + 8 (lane / 16) + e] (KS = in_pad / 32), zero
// past `out` (rows padded to a multiple of 64) and past `in`, so that one
// B fragment of v_mfma_f32_16x16x32_bf16 is 1 KB of contiguous memory.
__global__ void frag_weights_kernel(const float* W, int out, int in, int in_pad, int out_pad64,
                                    bf16_t* WF) {
    const size_t n = (size_t)out_pad64 * in_pad;
    const int KS = in_pad / 32;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const int el = (int)(e & 7);
        const int ln = (int)((e >> 3) & 63);
        const size_t blk = e >> 9;                      // nb * KS + ks
        const int ks = (int)(blk % KS), nb = (int)(blk / KS);
        const int o = 16 * nb + (ln & 15), i = 32 * ks + 8 * (ln >> 4) + el;
        WF[e] = f2bf((o < out && i < in) ? W[(size_t)o * in + i] : 0.f);
    }
}

struct EncArgs {
    int B, n_freq, feat_pad;
    float x_half, y_half, iv_lo, iv_hi, lam_lo, lam_hi;
    const float* x;
    bf16_t* H;
    bf16_t* HT;
};

// Fourier features [sin(2^k pi v), cos(2^k pi v)] per input, (input, k, sin/cos)
__global__ void encode_kernel(const EncArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const float* x = a.x + 4 * (size_t)b;
    float v[4];
    v[0] = x[0] / a.x_half;
    v[1] = x[1] / a.y_half;
    v[2] = 2.f * (x[2] - a.iv_lo) / (a.iv_hi - a.iv_lo) - 1.f;
    v[3] = 2.f * (x[3] - a.lam_lo) / (a.lam_hi - a.lam_lo) - 1.f;
    bf16_t* h = a.H + (size_t)b * a.feat_pad;
    int f = 0;
    for (int i = 0; i < 4; ++i) {
        float sc = 1.f;
        for (int k = 0; k < a.n_freq; ++k) {
            float s, c;
            sincospif(sc * v[i], &s, &c);
            const bf16_t bs = f2bf(s), bc = f2bf(c);
            h[f] = bs;
            a.HT[(size_t)f * a.B + b] = bs;
            h[f + 1] = bc;
            a.HT[(size_t)(f + 1) * a.B + b] = bc;
            f += 2;
            sc *= 2.f;
        }
    }
    for (; f < a.feat_pad; ++f) {
        h[f] = 0;
        a.HT[(size_t)f * a.B + b] = 0;
    }
}

struct SoftArgs {
    int B, n_out, n_out_pad;
    float inv_batch;
    int kl;                  // Kullback-Leibler loss instead of max-scaled L2
    int vjp;                 // target is an upstream gradient dL/dp (no loss)
    const float* logits;
    const float* target;     // null: inference
    void* out;               // inference output [B][n_out] (f32 or bf16) or null
    int out_bf16;
    float* dz;               // training: float32 dz [B][n_out]
    bf16_t* dzb;             // bf16 [B][n_out_pad]
    bf16_t* dzT;             // bf16 [n_out_pad][B]
    float* loss;
};

__device__ inline float block_reduce(float v, float* red, bool is_max) {
    for (int o = 32; o > 0; o >>= 1) {
        const float w = __shfl_xor(v, o, 64);
        v = is_max ? fmaxf(v, w) : v + w;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = red[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = is_max ? fmaxf(r, red[k]) : r + red[k];
    __syncthreads();
    return r;
}

// Joint softmax of one row; with a target: loss and its gradient.
__global__ __launch_bounds__(256) void softmax_loss_kernel(const SoftArgs a) {
    __shared__ float red[4];
    const int b = blockIdx.x;
    const float* z = a.logits + (size_t)b * a.n_out;
    float mx = -INFINITY;
    for (int i = threadIdx.x; i < a.n_out; i += blockDim.x) mx = fmaxf(mx, z[i]);
    mx = block_reduce(mx, red, true);
    float sum = 0.f;
    for (int i = threadIdx.x; i < a.n_out; i += blockDim.x) sum += __expf(z[i] - mx);
    sum = block_reduce(sum, red, false);
    const float inv = 1.f / sum;
    if (!a.target) {
        for (int i = threadIdx.x; i < a.n_out; i += blockDim.x) {
            const float p = __expf(z[i] - mx) * inv;
            if (a.out_bf16) reinterpret_cast<bf16_t*>(a.out)[(size_t)b * a.n_out + i] = f2bf(p);
            else reinterpret_cast<float*>(a.out)[(size_t)b * a.n_out + i] = p;
        }
        return;
    }
    const float* t = a.target + (size_t)b * a.n_out;
    if (a.vjp) {
        // upstream gradient t = dL/dp through the softmax:
        // dz_i = p_i (t_i - sum_j p_j t_j); the row's value sum_i p_i t_i
        float pg = 0.f;
        for (int i = threadIdx.x; i < a.n_out; i += blockDim.x)
            pg += __expf(z[i] - mx) * inv * t[i];
        pg = block_reduce(pg, red, false);
        if (threadIdx.x == 0) atomicAdd(a.loss, pg);
        for (int i = threadIdx.x; i < a.n_out_pad; i += blockDim.x) {
            float g = 0.f;
            if (i < a.n_out) {
                const float p = __expf(z[i] - mx) * inv;
                g = p * (t[i] - pg);
                a.dz[(size_t)b * a.n_out + i] = g;
            }
            const bf16_t gb = f2bf(g);
            a.dzb[(size_t)b * a.n_out_pad + i] = gb;
            a.dzT[(size_t)i * a.B + b] = gb;
        }
        return;
    }
    if (a.kl) {
        // KL(t || p) = sum_i t_i (log t_i - log p_i); d/dz_i = p_i sum(t) - t_i
        const float lse = mx + __logf(sum);
        float lsum = 0.f, ts = 0.f;
        for (int i = threadIdx.x; i < a.n_out; i += blockDim.x) {
            const float ti = t[i];
            ts += ti;
            if (ti > 0.f) lsum += ti * (__logf(ti) - (z[i] - lse));
        }
        lsum = block_reduce(lsum, red, false);
        ts = block_reduce(ts, red, false);
        if (threadIdx.x == 0) atomicAdd(a.loss, lsum * a.inv_batch);
        for (int i = threadIdx.x; i < a.n_out_pad; i += blockDim.x) {
            float g = 0.f;
            if (i < a.n_out) {
                const float p = __expf(z[i] - mx) * inv;
                g = (p * ts - t[i]) * a.inv_batch;
                a.dz[(size_t)b * a.n_out + i] = g;
            }
            const bf16_t gb = f2bf(g);
            a.dzb[(size_t)b * a.n_out_pad + i] = gb;
            a.dzT[(size_t)i * a.B + b] = gb;
        }
        return;
    }
    float tm = 0.f;
    for (int i = threadIdx.x; i < a.n_out; i += blockDim.x) tm = fmaxf(tm, t[i]);
    tm = block_reduce(tm, red, true);
    const float it2 = tm > 0.f ? 1.f / (tm * tm) : 0.f;
    float lsum = 0.f, pg = 0.f;
    for (int i = threadIdx.x; i < a.n_out; i += blockDim.x) {
        const float p = __expf(z[i] - mx) * inv;
        const float d = p - t[i];
        lsum += d * d * it2;
        pg += p * (2.f * d * it2 * a.inv_batch);
    }
    lsum = block_reduce(lsum, red, false);
    pg = block_reduce(pg, red, false);
    if (threadIdx.x == 0) atomicAdd(a.loss, lsum * a.inv_batch);
    for (int i = threadIdx.x; i < a.n_out_pad; i += blockDim.x) {
        float g = 0.f;
        if (i < a.n_out) {
            const float p = __expf(z[i] - mx) * inv;
            const float gp = 2.f * (p - t[i]) * it2 * a.inv_batch;
            g = p * (gp - pg);
            a.dz[(size_t)b * a.n_out + i] = g;
        }
        const bf16_t gb = f2bf(g);
        a.dzb[(size_t)b * a.n_out_pad + i] = gb;
        a.dzT[(size_t)i * a.B + b] = gb;
    }
}

// y += x (float32, n elements)
__global__ void accumulate_kernel(float* y, const float* x, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        y[i] += x[i];
}

// column sums of a float32 [B][N] matrix (bias gradient)
__global__ void colsum_kernel(const float* X, int B, int N, float* out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += X[(size_t)b * N + n];
    out[n] = s;
}

__global__ void adam_kernel(float* p, float* m, float* v, const float* g, size_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

// gather a training batch: sample index from a counter hash of (seed, step, b)
__device__ inline uint32_t mix32(uint32_t h) {
    h ^= h >> 16; h *= 0x85EBCA6Bu; h ^= h >> 13; h *= 0xC2B2AE35u; h ^= h >> 16;
    return h;
}

__global__ void gather_kernel(const float* x_all, const float* t_all, int n_samples, int n_out,
                              uint32_t seed, uint32_t step, int B, float* xb, float* tb) {
    const int b = blockIdx.x;
    const uint32_t h = mix32(mix32(mix32(seed ^ 0x9E3779B9u) ^ step) ^ (uint32_t)b);
    const size_t idx = (size_t)(((uint64_t)h * (uint64_t)n_samples) >> 32);
    if (threadIdx.x < 4) xb[(size_t)b * 4 + threadIdx.x] = x_all[idx * 4 + threadIdx.x];
    for (int i = threadIdx.x; i < n_out; i += blockDim.x)
        tb[(size_t)b * n_out + i] = t_all[idx * n_out + i];
}

// ---- host orchestration ---------------------------------------------------

static void gemm(const GemmArgs& g, hipStream_t st) {
    const int tiles = ((g.M + kBM - 1) / kBM) * ((g.N + kBN - 1) / kBN);
    hipLaunchKernelGGL(gemm_nt_kernel, dim3(tiles), dim3(kGB), 0, st, g);
}

static GemmArgs gargs() {
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    return g;
}

static void cast_all(const MlpDims& m, const MlpWs& w, const float* params, hipStream_t st) {
    const int fp = feat_pad(m);
    for (int l = 0; l < m.L; ++l) {
        const int in = m.in_of(l), out = m.out_of(l);
        const int in_pad = l == 0 ? fp : m.width;
        const int out_pad = l == m.L - 1 ? m.n_out_pad : m.width;
        const size_t n = (size_t)out_pad * in_pad;
        const int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
        hipLaunchKernelGGL(cast_weights_kernel, dim3(blocks), dim3(256), 0, st,
                           params + m.w_off(l), out, in, in_pad, out_pad, w.W[l], w.WT[l]);
    }
}

static void frag_all(const MlpDims& m, const MlpWs& w, const float* params, hipStream_t st) {
    const int fp = feat_pad(m);
    for (int l = 0; l < m.L; ++l) {
        const int in = m.in_of(l), out = m.out_of(l);
        const int in_pad = l == 0 ? fp : m.width;
        const int out_pad64 = (out + 63) / 64 * 64;
        const size_t n = (size_t)out_pad64 * in_pad;
        const int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
        hipLaunchKernelGGL(frag_weights_kernel, dim3(blocks), dim3(256), 0, st,
                           params + m.w_off(l), out, in, in_pad, out_pad64, w.WF[l]);
    }
}

// forward of B rows whose inputs are x; logits left in w.logits
static void forward_rows(const MlpDims& m, const sdirt_mlp_desc* d, const MlpWs& w,
                         const float* params, int B, const float* x, hipStream_t st,
                         bool keep_transposed) {
    EncArgs e;
    e.B = B; e.n_freq = m.n_freq; e.feat_pad = feat_pad(m);
    e.x_half = (float)d->x_half; e.y_half = (float)d->y_half;
    e.iv_lo = (float)d->iv_lo; e.iv_hi = (float)d->iv_hi;
    e.lam_lo = (float)d->lam_lo; e.lam_hi = (float)d->lam_hi;
    e.x = x; e.H = w.H[0]; e.HT = w.HT[0];
    hipLaunchKernelGGL(encode_kernel, dim3((B + 255) / 256), dim3(256), 0, st, e);
    for (int l = 0; l < m.L; ++l) {
        GemmArgs g = gargs();
        g.A = w.H[l]; g.lda = l == 0 ? feat_pad(m) : m.width;
        g.B = w.W[l]; g.ldb = g.lda;
        g.M = B; g.N = m.out_of(l); g.K = g.lda;
        g.bias = params + m.b_off(l);
        if (l < m.L - 1) {
            g.relu = 1;
            g.Cb = w.H[l + 1]; g.ldcb = m.width;
            if (keep_transposed) { g.CbT = w.HT[l + 1]; g.ldcbt = B; }
        } else {
            g.Cf = w.logits; g.ldcf = m.n_out;
        }
        gemm(g, st);
    }
}

// loss gradient for the batch already in w.H / w.logits; grads into w.grads
static void backward_rows(const MlpDims& m, const MlpWs& w, const float* params, int B,
                          const float* target, hipStream_t st, bool vjp = false) {
    SoftArgs s;
    std::memset(&s, 0, sizeof(s));
    s.B = B; s.n_out = m.n_out; s.n_out_pad = m.n_out_pad;
    s.inv_batch = vjp ? 1.f : 1.f / B;
    s.vjp = vjp;
    s.kl = !vjp && m.loss == SDIRT_LOSS_KL;
    s.logits = w.logits; s.target = target; s.dz = w.dz; s.dzb = w.dzb; s.dzT = w.dzT;
    s.loss = w.loss;
    hipLaunchKernelGGL(softmax_loss_kernel, dim3(B), dim3(256), 0, st, s);
    const int Lh = m.L - 1;
    const int nparts = 2 * ((B + 127) / 128);   // partial bias sums per column
    // last layer: db = colsum(dz), dW = dz^T H, dH = dz W (masked by H > 0);
    // every bias gradient is a fixed-order sum (no atomics), so training is
    // bitwise reproducible
    hipLaunchKernelGGL(colsum_kernel, dim3((m.n_out + 255) / 256), dim3(256), 0, st,
                       w.dz, B, m.n_out, w.grads + m.b_off(Lh));
    {
        GemmArgs g = gargs();
        g.A = w.dzT; g.lda = B; g.B = w.HT[Lh]; g.ldb = B;
        g.M = m.n_out; g.N = m.width; g.K = B;
        g.Cf = w.grads + m.w_off(Lh); g.ldcf = m.width;
        gemm(g, st);
    }
    int cur = 0;
    {
        GemmArgs g = gargs();
        g.A = w.dzb; g.lda = m.n_out_pad; g.B = w.WT[Lh]; g.ldb = m.n_out_pad;
        g.M = B; g.N = m.width; g.K = m.n_out_pad;
        g.mask = w.H[Lh]; g.ldm = m.width;
        g.Cb = w.dA[cur]; g.ldcb = m.width; g.CbT = w.dAT[cur]; g.ldcbt = B;
        g.colpart = w.part;
        gemm(g, st);
        hipLaunchKernelGGL(colsum_kernel, dim3((m.width + 255) / 256), dim3(256), 0, st,
                           (const float*)w.part, nparts, m.width, w.grads + m.b_off(Lh - 1));
    }
    for (int l = Lh - 1; l >= 0; --l) {
        const int in_pad = l == 0 ? feat_pad(m) : m.width;
        {   // dW_l = dA_l^T H_l
            GemmArgs g = gargs();
            g.A = w.dAT[cur]; g.lda = B; g.B = w.HT[l]; g.ldb = B;
            g.M = m.width; g.N = m.in_of(l); g.K = B;
            g.Cf = w.grads + m.w_off(l); g.ldcf = m.in_of(l);
            gemm(g, st);
        }
        if (l > 0) {   // dA_{l-1} = (dA_l W_l) * [H_l > 0], bias grad of layer l-1
            GemmArgs g = gargs();
            g.A = w.dA[cur]; g.lda = m.width; g.B = w.WT[l]; g.ldb = m.width;
            g.M = B; g.N = m.width; g.K = m.width;
            g.mask = w.H[l]; g.ldm = m.width;
            g.Cb = w.dA[1 - cur]; g.ldcb = m.width; g.CbT = w.dAT[1 - cur]; g.ldcbt = B;
            g.colpart = w.part;
            gemm(g, st);
            hipLaunchKernelGGL(colsum_kernel, dim3((m.width + 255) / 256), dim3(256), 0, st,
                               (const float*)w.part, nparts, m.width, w.grads + m.b_off(l - 1));
            cur = 1 - cur;
        }
        (void)in_pad;
    }
}


int mlp_n_params(const sdirt_mlp_desc* d, long long* out) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    *out = (long long)m.n_params();
    return SDIRT_OK;
}

int mlp_workspace_size(const sdirt_mlp_desc* d, int batch, size_t* out) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (batch < 64 || batch % 64) return SDIRT_EINVAL;
    *out = carve(m, batch, nullptr).bytes;
    return SDIRT_OK;
}

// Fused inference of a width-256 network (every layer and the softmax in one
// pass over the rows): fragment-ordered weights into w.WF, then chunks of
// `chunk` rows whose last hidden activations pass through hbuf.
static int forward_fused(const MlpDims& m, const sdirt_mlp_desc* d, const MlpWs& w,
                         bf16_t* hbuf, long long chunk, const float* params, long long n_rows,
                         const float* x, void* out, int out_dtype, hipStream_t st,
                         bool convert_weights = true) {
    if (convert_weights) frag_all(m, w, params, st);
    FusedArgs f;
    std::memset(&f, 0, sizeof(f));
    f.n_rows = n_rows;
    f.n_hidden = m.n_hidden; f.n_out = m.n_out; f.n_freq = m.n_freq;
    f.feat_pad = feat_pad(m);
    f.x_half = (float)d->x_half; f.y_half = (float)d->y_half;
    f.iv_lo = (float)d->iv_lo; f.iv_hi = (float)d->iv_hi;
    f.lam_lo = (float)d->lam_lo; f.lam_hi = (float)d->lam_hi;
    f.x = x; f.params = params;
    for (int l = 0; l < m.L; ++l) { f.b_off[l] = (long long)m.b_off(l); f.W[l] = w.WF[l]; }
    f.out = out; f.out_bf16 = out_dtype == SDIRT_BF16;
    return launch_mlp_fused(f, hbuf, chunk, st);
}

int mlp_forward(const sdirt_mlp_desc* d, const float* params, long long n_rows, const float* x,
                void* out, int out_dtype, void* workspace, int ws_batch, hipStream_t st) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (!params || !x || !out || !workspace || n_rows < 0) return SDIRT_EINVAL;
    if (ws_batch < 64 || ws_batch % 64) return SDIRT_EINVAL;
    if (out_dtype != SDIRT_F32 && out_dtype != SDIRT_BF16) return SDIRT_EUNSUPPORTED;
    const MlpWs w = carve(m, ws_batch, (char*)workspace);
    if (m.width == 256) {
        // The fused path needs only the fragment-ordered weights and one
        // chunk of last hidden activations (512 B per row): the workspace
        // from the first activation buffer to its end holds the largest
        // chunk that fits, in whole 256-row workgroups of the output layer.
        const size_t avail = w.bytes - (size_t)((char*)w.H[0] - (char*)workspace);
        const long long chunk = (long long)(avail / (m.width * sizeof(bf16_t))) / 256 * 256;
        return forward_fused(m, d, w, w.H[0], chunk, params, n_rows, x, out, out_dtype, st);
    }
    cast_all(m, w, params, st);
    const size_t esz = out_dtype == SDIRT_BF16 ? 2 : 4;
    for (long long r0 = 0; r0 < n_rows; r0 += ws_batch) {
        const int B = (int)std::min<long long>(ws_batch, n_rows - r0);
        forward_rows(m, d, w, params, B, x + 4 * r0, st, false);
        SoftArgs s;
        std::memset(&s, 0, sizeof(s));
        s.B = B; s.n_out = m.n_out; s.n_out_pad = m.n_out_pad;
        s.logits = w.logits;
        s.out = (char*)out + (size_t)r0 * m.n_out * esz;
        s.out_bf16 = out_dtype == SDIRT_BF16;
        hipLaunchKernelGGL(softmax_loss_kernel, dim3(B), dim3(256), 0, st, s);
    }
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

// ---- allocation-free inference ----------------------------------------------
// The fused inference above with its working memory (the fragment-ordered
// weights and one chunk of last hidden activations) in a static device array
// instead of a caller workspace, for callers that cannot allocate device
// memory.  Each device holds its own copy of the array for the life of the
// process; its device address is looked up once per device, with that device
// current, and only that address is handed to kernels.  Nothing in it needs
// clearing: every call rewrites the weights (padding included) and each
// chunk's activations before reading them.  Calls that overlap on one
// device (other streams, other host threads) share the array and race.
constexpr size_t kNoAllocBytes = (size_t)SDIRT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

static int scratch_address(void** addr) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SDIRT_ENODEVICE;
    if (dev < 0 || dev >= kMaxDevices) return SDIRT_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return SDIRT_ELAUNCH;
        g_scratch_addr[dev] = p;
    }
    *addr = g_scratch_addr[dev];
    return SDIRT_OK;
}

int mlp_forward_noalloc(const sdirt_mlp_desc* d, const float* params, long long n_rows,
                        const float* x, void* out, int out_dtype, hipStream_t st) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (!params || !x || !out || n_rows < 0) return SDIRT_EINVAL;
    if (out_dtype != SDIRT_F32 && out_dtype != SDIRT_BF16) return SDIRT_EUNSUPPORTED;
    if (m.width != 256) return SDIRT_EUNSUPPORTED;
    // layout: the layers' fragment-ordered weights, then the chunk buffer
    const int fp = feat_pad(m);
    size_t wf_off[17], off = 0;
    for (int l = 0; l < m.L; ++l) {
        const int in_pad = l == 0 ? fp : m.width;
        wf_off[l] = off;
        off += align256((size_t)((m.out_of(l) + 63) / 64) * 64 * in_pad * 2);
    }
    const size_t row_bytes = (size_t)m.width * sizeof(bf16_t);   // one row of hbuf
    if (off + 64 * row_bytes > kNoAllocBytes) return SDIRT_ESCRATCH;
    const long long chunk =
        std::min<long long>(65536, (long long)((kNoAllocBytes - off) / row_bytes) / 64 * 64);
    void* base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    MlpWs w;
    std::memset(&w, 0, sizeof(w));
    for (int l = 0; l < m.L; ++l) w.WF[l] = (bf16_t*)((char*)base + wf_off[l]);
    bf16_t* hbuf = (bf16_t*)((char*)base + off);
    return forward_fused(m, d, w, hbuf, chunk, params, n_rows, x, out, out_dtype, st);
}

// ---- network with the tracer as fallback --------------------------------
// Per point of a list-mode query: the band of its inverse depth among the
// caller's band edges; points whose band's network error exceeds the bar (or
// that fall outside every band) are traced, the others take the network's
// PSF.  The routing kernel also forms the network inputs of a chunk.
constexpr int kMaxBands = 64;

struct RouteArgs {
    const double* points;            // [P][4] h_x, h_y, depth, slot
    long long r0;
    int n;                           // points in this chunk
    int n_bands;
    double edges[kMaxBands + 1];
    int traced_band[kMaxBands];      // 1 where the band's error exceeds the bar
    float lambda[SDIRT_MAX_LAMBDAS];
    int n_lambda;
    float* x;                        // [n][4] network inputs of the chunk
    int* source;                     // [P] 0 network, 1 traced
};

__global__ void hybrid_route_kernel(const RouteArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n) return;
    const long long q = a.r0 + t;
    const double* p = a.points + 4 * q;
    const double iv = 1.0 / p[2];
    int traced = 1;
    if (iv >= a.edges[0] && iv <= a.edges[a.n_bands]) {
        int b = 0;
        for (int k = 1; k < a.n_bands; ++k) b += iv >= a.edges[k];
        traced = a.traced_band[b];
    }
    const int slot = (int)p[3];
    a.source[q] = traced;
    float* x = a.x + 4 * (size_t)t;
    x[0] = (float)p[0];
    x[1] = (float)p[1];
    x[2] = (float)iv;
    x[3] = (slot >= 0 && slot < a.n_lambda) ? a.lambda[slot] : 0.f;
}

int trace_dp_psf_impl(const sdirt_lens*, const sdirt_sensor*, const sdirt_psf_query*, void*,
                      double*, hipStream_t, int, const int*);

int psf_hybrid(const sdirt_mlp_desc* d, const float* params, const sdirt_lens* lens,
               const sdirt_sensor* sensor, const sdirt_psf_query* query, int n_bands,
               const double* band_edges, const double* band_error, double max_error,
               float* psf_out, int* source_out, void* workspace, int ws_batch,
               hipStream_t st) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (!params || !lens || !sensor || !query || !band_edges || !band_error || !psf_out ||
        !source_out || !workspace)
        return SDIRT_EINVAL;
    if (!query->points || query->n_points < 1 || !query->wavelengths) return SDIRT_EINVAL;
    if (ws_batch < 64 || ws_batch % 64) return SDIRT_EINVAL;
    if (n_bands < 1 || n_bands > kMaxBands || !std::isfinite(max_error) || max_error < 0)
        return SDIRT_EINVAL;
    for (int k = 0; k <= n_bands; ++k)
        if (!std::isfinite(band_edges[k]) || (k > 0 && !(band_edges[k] > band_edges[k - 1])))
            return SDIRT_EINVAL;
    for (int k = 0; k < n_bands; ++k)
        if (!std::isfinite(band_error[k])) return SDIRT_EINVAL;
    if (query->n_wavelengths < 1 || query->n_wavelengths > SDIRT_MAX_LAMBDAS) return SDIRT_EINVAL;
    // the two sources must agree on what a PSF is: a jointly sum-normalised
    // float32 [2][ks][ks] block, the network's width-256 fused kernels
    if (query->normalize != SDIRT_NORM_SUM || query->out_dtype != SDIRT_F32) return SDIRT_EUNSUPPORTED;
    if (2 * query->ks * query->ks != m.n_out) return SDIRT_EINVAL;
    if (m.width != 256) return SDIRT_EUNSUPPORTED;
    RouteArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.points = query->points;
    ra.n_bands = n_bands;
    for (int k = 0; k <= n_bands; ++k) ra.edges[k] = band_edges[k];
    for (int k = 0; k < n_bands; ++k) ra.traced_band[k] = band_error[k] > max_error ? 1 : 0;
    ra.n_lambda = query->n_wavelengths;
    for (int l = 0; l < ra.n_lambda; ++l) ra.lambda[l] = (float)query->wavelengths[l];
    ra.source = source_out;
    const MlpWs w = carve(m, ws_batch, (char*)workspace);
    ra.x = w.xb;
    const long long P = query->n_points;
    // 1. routing and the network's PSF for every point (traced points are
    //    overwritten below), chunk by chunk through the workspace
    for (long long r0 = 0; r0 < P; r0 += ws_batch) {
        const int nb = (int)std::min<long long>(ws_batch, P - r0);
        ra.r0 = r0;
        ra.n = nb;
        hipLaunchKernelGGL(hybrid_route_kernel, dim3((nb + 255) / 256), dim3(256), 0, st, ra);
        if ((rc = forward_fused(m, d, w, w.H[m.n_hidden], ws_batch, params, nb, w.xb,
                                psf_out + r0 * m.n_out, SDIRT_F32, st, r0 == 0)))
            return rc;
    }
    // 2. the tracer for the points routed to it (masked list-mode trace)
    return trace_dp_psf_impl(lens, sensor, query, psf_out, nullptr, st, 0, source_out);
}

int mlp_render(const sdirt_mlp_desc* d, const float* params, const sdirt_mlp_render_desc* rd,
               const float* img, const float* depth, float* out, void* workspace, int ws_batch,
               hipStream_t st) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (!params || !rd || !img || !depth || !out || !workspace) return SDIRT_EINVAL;
    if (ws_batch < 64 || ws_batch % 64) return SDIRT_EINVAL;
    if (rd->N < 1 || rd->C < 1 || rd->H < 1 || rd->W < 1) return SDIRT_EINVAL;
    if (rd->C > 4) return SDIRT_EUNSUPPORTED;
    if (rd->ks < 1 || rd->ks % 2 == 0 || 2 * rd->ks * rd->ks != m.n_out) return SDIRT_EINVAL;
    if (m.width != 256 || rd->ks > 65) return SDIRT_EUNSUPPORTED;
    if (!std::isfinite(rd->pitch) || !(rd->pitch > 0)) return SDIRT_EINVAL;
    for (int c = 0; c < rd->C; ++c)
        if (!std::isfinite(rd->wavelength[c]) || !(rd->wavelength[c] > 0)) return SDIRT_EINVAL;
    if ((long long)rd->H * rd->W > (1LL << 30)) return SDIRT_EUNSUPPORTED;
    const MlpWs w = carve(m, ws_batch, (char*)workspace);
    frag_all(m, w, params, st);
    FusedArgs f;
    std::memset(&f, 0, sizeof(f));
    f.n_hidden = m.n_hidden; f.n_out = m.n_out; f.n_freq = m.n_freq;
    f.feat_pad = feat_pad(m);
    f.x_half = (float)d->x_half; f.y_half = (float)d->y_half;
    f.iv_lo = (float)d->iv_lo; f.iv_hi = (float)d->iv_hi;
    f.lam_lo = (float)d->lam_lo; f.lam_hi = (float)d->lam_hi;
    f.params = params;
    for (int l = 0; l < m.L; ++l) { f.b_off[l] = (long long)m.b_off(l); f.W[l] = w.WF[l]; }
    f.depth = depth; f.img = img; f.rout = out;
    f.img_n = rd->N; f.img_c = rd->C; f.img_h = rd->H; f.img_w = rd->W; f.ks = rd->ks;
    f.tiles_x = (rd->W + 7) / 8; f.tiles_y = (rd->H + 7) / 8;
    f.pitch = (float)rd->pitch;
    for (int c = 0; c < rd->C; ++c) f.lam[c] = (float)rd->wavelength[c];
    f.n_rows = (long long)rd->N * rd->C * f.tiles_x * f.tiles_y * 64;
    // as in the fused inference: one chunk of last hidden activations, as
    // large as the workspace past the weights holds, in 256-row workgroups
    const size_t avail = w.bytes - (size_t)((char*)w.H[0] - (char*)workspace);
    const long long chunk = (long long)(avail / (m.width * sizeof(bf16_t))) / 256 * 256;
    return launch_mlp_render(f, w.H[0], chunk, st);
}

int mlp_backward(const sdirt_mlp_desc* d, const float* params, int batch, const float* x,
                 const float* target, float* grads_out, float* loss_out, void* workspace,
                 hipStream_t st) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (!params || !x || !target || !workspace) return SDIRT_EINVAL;
    if (batch < 64 || batch % 64) return SDIRT_EINVAL;
    const MlpWs w = carve(m, batch, (char*)workspace);
    cast_all(m, w, params, st);
    if ((rc = launch_fill_zero(w.loss, 4, st))) return rc;
    forward_rows(m, d, w, params, batch, x, st, true);
    backward_rows(m, w, params, batch, target, st);
    if (grads_out)
        (void)hipMemcpyAsync(grads_out, w.grads, m.n_params() * 4, hipMemcpyDeviceToDevice, st);
    if (loss_out)
        (void)hipMemcpyAsync(loss_out, w.loss, 4, hipMemcpyDeviceToDevice, st);
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

int mlp_vjp(const sdirt_mlp_desc* d, const float* params, long long n_rows, const float* x,
            const float* grad_psf, float* grads_out, float* value_out, void* workspace,
            int ws_batch, hipStream_t st) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (!params || !grads_out || !workspace || n_rows < 0) return SDIRT_EINVAL;
    if (n_rows > 0 && (!x || !grad_psf)) return SDIRT_EINVAL;
    if (ws_batch < 64 || ws_batch % 64) return SDIRT_EINVAL;
    const MlpWs w = carve(m, ws_batch, (char*)workspace);
    const size_t np = m.n_params();
    if ((rc = launch_fill_zero(grads_out, np * 4, st))) return rc;
    if (value_out && (rc = launch_fill_zero(value_out, 4, st))) return rc;
    if (n_rows == 0) return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
    cast_all(m, w, params, st);
    const int gblocks = (int)std::min<size_t>((np + 255) / 256, 2048);
    for (long long r0 = 0; r0 < n_rows; r0 += ws_batch) {
        const long long nb = std::min<long long>(ws_batch, n_rows - r0);
        const int B = (int)((nb + 63) / 64 * 64);
        const float* xb = x + r0 * 4;
        const float* gb = grad_psf + r0 * m.n_out;
        if (nb < B) {
            // ragged tail: rows padded with zero inputs and zero gradients,
            // which add nothing
            if ((rc = launch_fill_zero(w.xb, (size_t)B * 16, st))) return rc;
            if ((rc = launch_fill_zero(w.target, (size_t)B * m.n_out * 4, st))) return rc;
            (void)hipMemcpyAsync(w.xb, xb, (size_t)nb * 16, hipMemcpyDeviceToDevice, st);
            (void)hipMemcpyAsync(w.target, gb, (size_t)nb * m.n_out * 4, hipMemcpyDeviceToDevice, st);
            xb = w.xb;
            gb = w.target;
        }
        if ((rc = launch_fill_zero(w.loss, 4, st))) return rc;
        forward_rows(m, d, w, params, B, xb, st, true);
        backward_rows(m, w, params, B, gb, st, true);
        hipLaunchKernelGGL(accumulate_kernel, dim3(gblocks), dim3(256), 0, st, grads_out,
                           (const float*)w.grads, np);
        if (value_out)
            hipLaunchKernelGGL(accumulate_kernel, dim3(1), dim3(64), 0, st, value_out,
                               (const float*)w.loss, (size_t)1);
    }
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

static void adam_launch(size_t n, float* p, float* mm, float* vv, const float* g, int step,
                        float lr, hipStream_t st) {
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, step)));
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, st, p, mm, vv, g, n, lr,
                       (float)b1, (float)b2, 1e-8f, c1, c2);
}

int mlp_adam(const sdirt_mlp_desc* d, float* params, float* m1, float* m2, const float* grads,
             int step, float lr, hipStream_t st) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (!params || !m1 || !m2 || !grads || step < 1 || !std::isfinite(lr)) return SDIRT_EINVAL;
    adam_launch(m.n_params(), params, m1, m2, grads, step, lr, st);
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

int mlp_train_step(const sdirt_mlp_desc* d, float* params, float* m1, float* m2, int step,
                   float lr, int batch, const float* x, const float* target, float* loss_out,
                   void* workspace, hipStream_t st) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (!params || !m1 || !m2 || !x || !target || !workspace) return SDIRT_EINVAL;
    if (batch < 64 || batch % 64 || step < 1 || !std::isfinite(lr)) return SDIRT_EINVAL;
    const MlpWs w = carve(m, batch, (char*)workspace);
    cast_all(m, w, params, st);
    if ((rc = launch_fill_zero(w.loss, 4, st))) return rc;
    forward_rows(m, d, w, params, batch, x, st, true);
    backward_rows(m, w, params, batch, target, st);
    adam_launch(m.n_params(), params, m1, m2, w.grads, step, lr, st);
    if (loss_out)
        (void)hipMemcpyAsync(loss_out, w.loss, 4, hipMemcpyDeviceToDevice, st);
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

int mlp_train(const sdirt_mlp_desc* d, float* params, float* m1, float* m2, int step0,
              int n_steps, float lr0, float lr_min, int total_steps, int batch,
              long long n_samples, const float* x_all, const float* t_all, uint32_t seed,
              float* loss_trace, void* workspace, hipStream_t st) {
    MlpDims m;
    int rc = dims_of(d, &m);
    if (rc) return rc;
    if (!params || !m1 || !m2 || !x_all || !t_all || !workspace) return SDIRT_EINVAL;
    if (batch < 64 || batch % 64 || n_steps < 0 || step0 < 0 || total_steps < 1 ||
        n_samples < 1 || n_samples > 0x7fffffffLL)
        return SDIRT_EINVAL;
    const MlpWs w = carve(m, batch, (char*)workspace);
    for (int k = 0; k < n_steps; ++k) {
        const int step = step0 + k;
        const double frac = std::min(1.0, (double)step / total_steps);
        const float lr = (float)(lr_min + 0.5 * (lr0 - lr_min) * (1.0 + std::cos(M_PI * frac)));
        hipLaunchKernelGGL(gather_kernel, dim3(batch), dim3(256), 0, st, x_all, t_all,
                           (int)n_samples, m.n_out, seed, (uint32_t)step, batch, w.xb, w.target);
        cast_all(m, w, params, st);
        launch_fill_zero(w.loss, 4, st);
        forward_rows(m, d, w, params, batch, w.xb, st, true);
        backward_rows(m, w, params, batch, w.target, st);
        adam_launch(m.n_params(), params, m1, m2, w.grads, step + 1, lr, st);
        if (loss_trace)
            (void)hipMemcpyAsync(loss_trace + k, w.loss, 4, hipMemcpyDeviceToDevice, st);
    }
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

}  // namespace sdirt
