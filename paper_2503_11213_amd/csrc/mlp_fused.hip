// Inference of the PSF surrogate MLP (Sec. 3.2, Supplement S1.4) in two
// kernels per chunk of rows, with every matrix product on
// v_mfma_f32_16x16x32_bf16 (float32 accumulation).
//
// Trunk: a workgroup of four waves owns 64 rows; the Fourier encoding and
// every hidden layer run with the bf16 activations [64][256] in LDS (double
// buffer), wave w computing output columns [64 w, 64 w + 64); the last
// activations go to a chunk buffer in HBM (512 B per row).
// Head: the softmax output layer (2 ks^2 columns, tiles of 64) of 256 rows,
// each wave holding its 64 rows' activations in registers while the weight
// tiles stream through LDS, two workgroups per compute unit.  Pass 1
// computes each tile's logits and keeps a running (max, sum of 2^z) per row
// and lane; the lanes of a row merge them; pass 2 recomputes the tiles and
// writes 2^(z - max - log2 sum) (bf16 or float32).  Recomputing doubles the
// output layer's matrix work but keeps the float32 logits out of HBM.
// Weights are read in matrix-core fragment order (one 1 KB contiguous piece
// per fragment).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "../../include/sdirt.h"
#include "mlp_fused.hpp"

namespace sdirt {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

constexpr int kFRows = 64;             // rows per workgroup
constexpr int kFWidth = 256;           // hidden width (fixed)
constexpr int kFStride = kFWidth + 8;  // LDS row stride in bf16 (bank spread)
constexpr int kFThreads = 256;


// float -> bf16, round to nearest even (v_cvt_pk_bf16_f32)
__device__ inline bf16_t f2bf_rne(float f) {
    const __bf16 h = (__bf16)f;
    return __builtin_bit_cast(bf16_t, h);
}

__device__ inline bf16x8_t load_b8(const bf16_t* p) {
    return *reinterpret_cast<const bf16x8_t*>(p);
}

// Weights arrive in matrix-core fragment order (see frag_weights_kernel):
// the B fragment of column block nb (16 outputs) and k-step ks of a layer
// with KS k-steps is the 1 KB at WF + (nb * KS + ks) * 512 elements, lane l
// reading its 16 bytes at offset 8 l.  One load instruction of a wave then
// covers 8 contiguous cache lines instead of 64 scattered ones.
__device__ inline bf16x8_t load_frag(const bf16_t* WF, int KS, int nb, int ks, int lane) {
    return load_b8(WF + ((size_t)(nb * KS + ks) * 64 + lane) * 8);
}

// acc[i][j] = H[rows 16 i ..][0..K) x W[cols col0 + 16 j ..][0..K)^T, K = 32 KS,
// with B fragments two k-steps ahead in static even/odd buffers and the
// first products starting from zero.
__device__ inline void frag_mma(const bf16_t* H, const bf16_t* WF, int KS, int col0,
                                floatx4_t acc[4][4]) {
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, kg = (lane >> 4) * 8;
    const int nb0 = col0 / 16;
    const bf16_t* hp[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) hp[i] = H + (16 * i + r16) * kFStride + kg;
    bf16x8_t be[4], bo[4], a[4];
    const bf16x8_t zero = {};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        be[j] = load_frag(WF, KS, nb0 + j, 0, lane);
        bo[j] = KS > 1 ? load_frag(WF, KS, nb0 + j, 1, lane) : zero;
    }
#pragma unroll 1
    for (int ks = 0; ks < KS; ks += 2) {
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const bf16x8_t*>(hp[i] + 32 * ks);
        if (ks == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        a[i], be[j], floatx4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], be[j], acc[i][j], 0, 0, 0);
        }
        if (ks + 2 < KS) {
#pragma unroll
            for (int j = 0; j < 4; ++j) be[j] = load_frag(WF, KS, nb0 + j, ks + 2, lane);
        }
        if (ks + 1 < KS) {
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const bf16x8_t*>(hp[i] + 32 * ks + 32);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bo[j], acc[i][j], 0, 0, 0);
            if (ks + 3 < KS) {
#pragma unroll
                for (int j = 0; j < 4; ++j) bo[j] = load_frag(WF, KS, nb0 + j, ks + 3, lane);
            }
        }
    }
}

// Decoding of a pixel row (see FusedArgs): the image, channel and pixel; the
// pixel is clamped into the image for the padding rows of edge tiles.
struct PixelRow {
    int n, c, x0, y0, x, y;
};
__device__ inline PixelRow pixel_row(const FusedArgs& A, long long gr) {
    const long long T = (long long)A.tiles_x * A.tiles_y;
    const long long blk = gr >> 6;
    const int p = (int)(gr & 63);
    const long long ic = blk / T;
    const int tile = (int)(blk - ic * T);
    PixelRow r;
    r.n = (int)(ic / A.img_c);
    r.c = (int)(ic - (long long)r.n * A.img_c);
    const int ty = tile / A.tiles_x, tx = tile - ty * A.tiles_x;
    r.y0 = 8 * ty;
    r.x0 = 8 * tx;
    r.y = min(r.y0 + (p >> 3), A.img_h - 1);
    r.x = min(r.x0 + (p & 7), A.img_w - 1);
    return r;
}

// Input `part` of a pixel row, in float32: h_x = (x - (W - 1) / 2) pitch,
// h_y likewise, 1 / depth, the channel's wavelength.
__device__ inline float pixel_input(const FusedArgs& A, long long gr, int part) {
    const PixelRow r = pixel_row(A, gr);
    if (part == 0) return ((float)r.x - 0.5f * (float)(A.img_w - 1)) * A.pitch;
    if (part == 1) return ((float)r.y - 0.5f * (float)(A.img_h - 1)) * A.pitch;
    if (part == 2) return 1.0f / A.depth[((size_t)r.n * A.img_h + r.y) * A.img_w + r.x];
    return A.lam[r.c];
}

// Trunk: encoding and hidden layers of 64 rows of the chunk [r_begin, r_end);
// the last hidden activations go to hout ([rows of the chunk][256] bf16).
__global__ __launch_bounds__(kFThreads, 2) void mlp_trunk_kernel(const FusedArgs A, long long r_begin,
                                                            long long r_end, bf16_t* hout) {
    __shared__ bf16_t H[2][kFRows * kFStride];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g4 = (lane >> 4) * 4;
    const long long row0 = r_begin + (long long)blockIdx.x * kFRows;
    // ---- encoding: 64 rows x feat_pad features, 4 threads per row ----------
    {
        const int row = tid >> 2, part = tid & 3;     // input `part` of the row
        const long long gr = row0 + row;
        float v = 0.f;
        if (gr < r_end) {
            const float xv = A.depth ? pixel_input(A, gr, part) : A.x[gr * 4 + part];
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
        frag_mma(H[cur], A.W[l], K / 32, col0, acc);
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
    // ---- last hidden activations to the chunk buffer (16-byte pieces) ------
    for (int e = tid; e < kFRows * (kFWidth / 8); e += kFThreads) {
        const int row = e / (kFWidth / 8), c8 = e % (kFWidth / 8);
        if (row0 + row < r_end)
            *reinterpret_cast<bf16x8_t*>(hout + (size_t)(row0 - r_begin + row) * kFWidth + 8 * c8) =
                *reinterpret_cast<const bf16x8_t*>(H[cur] + row * kFStride + 8 * c8);
    }
}

// ---- head ---------------------------------------------------------------------
// The softmax output layer (n_out = 2 ks^2 columns, tiles of 64) of 256 rows
// per workgroup; wave w owns rows [64 w, 64 w + 64) and holds their hidden
// activations in registers, as matrix-core B operands, for the whole kernel.
// The weight tiles (32 KB each, fragment order) stream through a two-slot
// LDS ring: each is copied once per workgroup by direct global-to-LDS loads
// (a quarter per wave) while the waves work on the other slot, and read by
// all four waves, so that a weight byte fetched from L2 serves 256 rows per
// pass.  (Read by each wave from L2 for its own 64 rows, the weights kept
// the vector-memory unit 71 % busy and the matrix cores 31 %.)  Tile t's 64
// biases come along into a small LDS slot.  A tile is taken in two halves of
// 32 columns, which keeps the accumulators at 32 registers beside the 128 of
// the hidden rows, within the 256 of a wave at two workgroups per compute
// unit.
// Transposed products (weights as the A operand): acc[i][j] holds
// C[column 16 j + 4 (l / 16) + r][row 16 i + l % 16] of a half, so lane l
// owns rows 16 i + l % 16 and, in each column block j, four consecutive
// columns; the softmax statistics take 4 registers per quantity and the
// four lanes of a row merge theirs with two exchanges (no cross-wave step).
// Pass 1 keeps a running (reference, sum of 2^z) per row and lane; pass 2
// recomputes each tile and writes 2^(z - M - log2 S).  Two workgroups per
// compute unit: one's softmax runs while the other's products keep the
// matrix cores busy.
constexpr int kHRows = 256;                     // rows per workgroup
constexpr int kHJ = 2;                          // 16-column blocks per half tile
constexpr int kHCols = 32 * kHJ;                // columns per tile (two halves)
constexpr int kHTile = kHCols * kFWidth;        // bf16 elements per weight tile (32 KB)

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(3))) const float lds_cfloat_t;

template <bool BF16>
__global__ __launch_bounds__(kFThreads, 2) void mlp_head_kernel(const FusedArgs A, long long r_begin,
                                                              long long r_end, const bf16_t* hin) {
    // the two ring slots are separate arrays, so that the compiler can see
    // that a copy into one slot does not feed reads of the other
    __shared__ __align__(16) bf16_t wt0[kHTile], wt1[kHTile];
    __shared__ __align__(16) float bt0[kHCols], bt1[kHCols];
    constexpr int KS = kFWidth / 32;
    constexpr float kL2E = 1.4426950408889634f;
    constexpr float kNone = -1e30f;
    constexpr float kSlack = 32.f;
    typedef typename std::conditional<BF16, __bf16, float>::type OutT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g4 = (lane >> 4) * 4, kg = (lane >> 4) * 8;
    const long long row0 = r_begin + (long long)blockIdx.x * kHRows + 64 * wave;
    const int Lo = A.n_hidden;
    const bf16_t* Wo = A.W[Lo];
    const float* bo = A.params + A.b_off[Lo];
    const int n_out = A.n_out;
    const int ntile = (n_out + kHCols - 1) / kHCols;
    OutT* outp = reinterpret_cast<OutT*>(A.out);
    // whole 4-byte words per four columns: bf16 pairs need an even row pitch
    const bool words = !BF16 || (n_out & 1) == 0;

    // copy of tile t into a ring slot: wave w takes fragments w, w + 4, ...
    // (each 64 lanes x 16 B); wave 0 also the tile's biases, the lanes past
    // the last column reading the last bias (their logits are masked)
    auto fetch = [&](int t, bf16_t* w, float* b) __attribute__((always_inline)) {
        const bf16_t* src = Wo + (size_t)t * kHTile + lane * 8;
#pragma unroll
        for (int f = wave; f < 2 * kHJ * KS; f += 4)
            __builtin_amdgcn_global_load_lds(src + f * 512, (lds_ptr_t)(w + f * 512), 16, 0, 0);
        if (wave == 0)
            __builtin_amdgcn_global_load_lds(bo + min(kHCols * t + lane, n_out - 1), (lds_ptr_t)b, 4, 0, 0);
    };
    fetch(0, wt0, bt0);
    bf16x8_t h[4][KS];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const long long gr = row0 + 16 * i + r16;
        const bf16_t* hp = hin + (size_t)(gr - r_begin) * kFWidth + kg;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) h[i][ks] = gr < r_end ? load_b8(hp + 32 * ks) : bf16x8_t{};
    }
    floatx4_t acc[4][kHJ];
    // products of half `half` of the tile in slot w
    auto products = [&](const bf16_t* w, int half) __attribute__((always_inline)) {
        const bf16_t* wb = w + lane * 8 + half * kHJ * KS * 512;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            // one k-step's fragments at a time (the scheduler would
            // otherwise hoist all the reads)
            __builtin_amdgcn_sched_barrier(0);
            bf16x8_t a[kHJ];
#pragma unroll
            for (int j = 0; j < kHJ; ++j) a[j] = *reinterpret_cast<const bf16x8_t*>(wb + (j * KS + ks) * 512);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < kHJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        a[j], h[i][ks], ks == 0 ? floatx4_t{0.f, 0.f, 0.f, 0.f} : acc[i][j], 0, 0, 0);
        }
    };
    // biases of this lane's four columns in block j of a half, times log2 e;
    // `none` past n_out
    auto biases = [&](const float* b, int col0, int j, float none) __attribute__((always_inline)) {
        const floatx4_t v = *reinterpret_cast<const floatx4_t*>(b + (col0 % kHCols) + 16 * j + g4);
        floatx4_t bl;
#pragma unroll
        for (int r = 0; r < 4; ++r) bl[r] = col0 + 16 * j + g4 + r < n_out ? v[r] * kL2E : none;
        return bl;
    };
    // Pass 1.  Logits are carried in base 2 (z log2 e) so that every
    // exponential is one v_exp_f32; -1e30 stands for "no column yet"
    // (finite, so no special cases: its exponentials vanish).  m[i], the
    // reference of row 16 i + l % 16's running sum s[i] = sum 2^(z - m[i]),
    // is kept at or above every logit of the row seen so far and raised (to
    // kSlack above the new maximum) only when a logit passes it, so that
    // between raises a half costs one exponential per logit and no
    // rescaling; the terms stay in (0, 1] and far from underflow.
    float m[4], s[4], mls[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) { m[i] = kNone; s[i] = 0.f; mls[i] = 1e30f; }
    auto stats = [&](const float* b, int col0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < kHJ; ++j) {
            const floatx4_t bl = biases(b, col0, j, kNone);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[i][j][r] = fmaf(acc[i][j][r], kL2E, bl[r]);
        }
        // each row's largest logit of the half, compared once with its
        // reference
        float zm[4];
        bool raise = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            zm[i] = kNone;
#pragma unroll
            for (int j = 0; j < kHJ; ++j)
                zm[i] = fmaxf(zm[i], fmaxf(fmaxf(acc[i][j][0], acc[i][j][1]), fmaxf(acc[i][j][2], acc[i][j][3])));
            raise |= zm[i] > m[i];
        }
        if (__ballot(raise)) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float mn = fmaxf(m[i], zm[i] + kSlack);
                s[i] *= __builtin_amdgcn_exp2f(m[i] - mn);
                m[i] = mn;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float a = 0.f;
#pragma unroll
            for (int j = 0; j < kHJ; ++j)
                a += (__builtin_amdgcn_exp2f(acc[i][j][0] - m[i]) + __builtin_amdgcn_exp2f(acc[i][j][1] - m[i])) +
                     (__builtin_amdgcn_exp2f(acc[i][j][2] - m[i]) + __builtin_amdgcn_exp2f(acc[i][j][3] - m[i]));
            s[i] += a;
        }
    };
    // merge over the 4 lanes holding the same rows; per row M + log2(S), so
    // that p = 2^(z - M - log2 S)
    auto merge = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int o = 16; o < 64; o <<= 1) {
                const float m2 = __shfl_xor(m[i], o, 64);
                const float s2 = __shfl_xor(s[i], o, 64);
                const float mn = fmaxf(m[i], m2);
                s[i] = s[i] * __builtin_amdgcn_exp2f(m[i] - mn) + s2 * __builtin_amdgcn_exp2f(m2 - mn);
                m[i] = mn;
            }
            mls[i] = s[i] > 0.f ? m[i] + __builtin_amdgcn_logf(s[i]) : 1e30f;
        }
    };
    // Pass 2: the probabilities of a half as output words (bf16 pairs or
    // float bits), then their stores (each lane writes four consecutive
    // columns per block)
    uint32_t pw[4][kHJ][4];
    auto probs = [&](const float* b, int col0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < kHJ; ++j) {
            const floatx4_t bl = biases(b, col0, j, 0.f);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float p[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    p[r] = __builtin_amdgcn_exp2f(fmaf(acc[i][j][r], kL2E, bl[r]) - mls[i]);
                if (BF16) {
                    pw[i][j][0] = (uint32_t)f2bf_rne(p[0]) | ((uint32_t)f2bf_rne(p[1]) << 16);
                    pw[i][j][1] = (uint32_t)f2bf_rne(p[2]) | ((uint32_t)f2bf_rne(p[3]) << 16);
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) pw[i][j][r] = __builtin_bit_cast(uint32_t, p[r]);
                }
            }
        }
    };
    auto store = [&](int col0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < kHJ; ++j) {
            const int n0 = col0 + 16 * j + g4;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long gr = row0 + 16 * i + r16;
                if (gr >= r_end) continue;
                OutT* q = outp + gr * n_out + n0;
                if (words && n0 + 3 < n_out) {
                    uint32_t* w = reinterpret_cast<uint32_t*>(q);
#pragma unroll
                    for (int e = 0; e < (BF16 ? 2 : 4); ++e) w[e] = pw[i][j][e];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (n0 + r >= n_out) continue;
                        if constexpr (BF16)
                            reinterpret_cast<uint16_t*>(q)[r] = (uint16_t)(pw[i][j][r >> 1] >> (16 * (r & 1)));
                        else
                            reinterpret_cast<uint32_t*>(q)[r] = pw[i][j][r];
                    }
                }
            }
        }
    };
    // Step k of the 2 ntile steps (pass 1 over the tiles, then pass 2)
    // reads slot k & 1.  It starts when this wave's copies are done
    // (vector-memory count 0, which also covers earlier output stores) and
    // all waves are past step k - 1; it then starts the copy of step k + 1's
    // tile into the other slot (which step k - 1 read) and takes the two
    // halves of its own tile.  The slot is a compile-time choice, so that
    // the reads of one slot need not wait for the copy into the other.
    auto step = [&](int k, auto slot) __attribute__((always_inline)) {
        constexpr int SL = decltype(slot)::value;
        const bf16_t* w = SL ? wt1 : wt0;
        const float* b = SL ? bt1 : bt0;
        __builtin_amdgcn_s_waitcnt(0x0f70);          // vmcnt(0)
        __syncthreads();
        if (k + 1 < 2 * ntile) fetch((k + 1) % ntile, SL ? wt0 : wt1, SL ? bt0 : bt1);
        const bool pass1 = k < ntile;
        const int t = pass1 ? k : k - ntile;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int col0 = kHCols * t + 32 * half;
            products(w, half);
            if (pass1) {
                stats(b, col0);
            } else {
                probs(b, col0);
                store(col0);
            }
        }
        if (k == ntile - 1) merge();
    };
    for (int k = 0; k < 2 * ntile; k += 2) {
        step(k, std::integral_constant<int, 0>());
        step(k + 1, std::integral_constant<int, 1>());
    }
}

int launch_mlp_fused(const FusedArgs& A, bf16_t* hbuf, long long chunk, hipStream_t st) {
    if (A.n_rows <= 0) return SDIRT_OK;
    if (chunk < kFRows) return SDIRT_EINVAL;
    for (long long r0 = 0; r0 < A.n_rows; r0 += chunk) {
        const long long r1 = std::min(A.n_rows, r0 + chunk);
        const long long blocks = (r1 - r0 + kFRows - 1) / kFRows;
        const long long hblocks = (r1 - r0 + kHRows - 1) / kHRows;
        if (blocks > 0x7fffffffLL) return SDIRT_EUNSUPPORTED;
        hipLaunchKernelGGL(mlp_trunk_kernel, dim3((unsigned)blocks), dim3(kFThreads), 0, st, A, r0, r1, hbuf);
        if (A.out_bf16)
            hipLaunchKernelGGL(mlp_head_kernel<true>, dim3((unsigned)hblocks), dim3(kFThreads), 0, st, A, r0,
                               r1, (const bf16_t*)hbuf);
        else
            hipLaunchKernelGGL(mlp_head_kernel<false>, dim3((unsigned)hblocks), dim3(kFThreads), 0, st, A, r0,
                               r1, (const bf16_t*)hbuf);
    }
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

// Fused surrogate render: the softmax layer of the pixel rows, reduced
// against each pixel's image window in the same pass instead of being
// written out.  With the column k of a row taken as (side s, tap (i, j)) and
// w_k the image value under that tap (clamped image), the row's outputs are
//     out_s = sum_{k in side s} 2^(z_k - M) w_k / sum_k 2^(z_k - M),
// so one pass keeps per row a running reference M, the sum S and the two
// weighted sums (all rescaled together when M rises).  A workgroup takes 256
// rows, wave w one 8 x 8 pixel tile of one channel (rows [64 w, 64 w + 64)),
// with the tile's clamped (8 + ks - 1)^2 image halo in LDS and its hidden
// activations in registers; the weight tiles of 32 columns (16 KB) stream
// through a two-slot LDS ring as in the inference head, each copied once per
// workgroup and read by all four waves.  Transposed products: lane l holds
// rows 16 i + l % 16 and, per column block j, four consecutive columns, so
// the running state takes 4 registers per quantity and the four lanes of a
// row merge theirs at the end.
constexpr int kRHCols = 32;                      // columns per render-head weight tile
constexpr int kRHTile = kRHCols * kFWidth;       // bf16 elements per tile (16 KB)

__global__ __launch_bounds__(kFThreads, 2) void mlp_render_head_kernel(const FusedArgs A,
                                                                     long long r_begin,
                                                                     long long r_end,
                                                                     const bf16_t* hin) {
    __shared__ __align__(16) bf16_t wt0[kRHTile], wt1[kRHTile];
    __shared__ __align__(16) float bt0[64], bt1[64];
    extern __shared__ float halos[];                     // [4 waves][(8 + ks - 1)^2]
    constexpr int KS = kFWidth / 32;
    constexpr float kL2E = 1.4426950408889634f;
    constexpr float kNone = -1e30f;
    constexpr float kSlack = 32.f;
    // wave-uniform values in scalar registers
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r16 = lane & 15, g4 = (lane >> 4) * 4, kg = (lane >> 4) * 8;
    const long long row0 = r_begin + (long long)blockIdx.x * kHRows + 64 * wave;
    const bool active = row0 < r_end;                    // the wave has a tile
    const int ks = A.ks, kk = ks * ks, pad = (ks - 1) / 2, hh = 8 + ks - 1;
    const float inv_ks = 1.f / (float)ks;
    const int Lo = A.n_hidden;
    const bf16_t* Wo = A.W[Lo];
    const float* bo = A.params + A.b_off[Lo];
    const int n_out = A.n_out;
    const int ntile = (n_out + kRHCols - 1) / kRHCols;
    auto fetch = [&](int t, bf16_t* w, float* b) __attribute__((always_inline)) {
        const bf16_t* src = Wo + (size_t)t * kRHTile + lane * 8;
#pragma unroll
        for (int f = wave; f < 2 * KS; f += 4)
            __builtin_amdgcn_global_load_lds(src + f * 512, (lds_ptr_t)(w + f * 512), 16, 0, 0);
        if (wave == 0)
            __builtin_amdgcn_global_load_lds(bo + min(kRHCols * t + lane, n_out - 1), (lds_ptr_t)b, 4,
                                             0, 0);
    };
    fetch(0, wt0, bt0);
    const PixelRow pr = pixel_row(A, active ? row0 : r_begin);   // the wave's tile
    float* halo = halos + wave * hh * hh;
    if (active) {
        const float* im = A.img + ((size_t)pr.n * A.img_c + pr.c) * A.img_h * A.img_w;
        for (int e = lane; e < hh * hh; e += 64) {
            const int r = e / hh, q = e - r * hh;
            const int yy = min(max(pr.y0 - pad + r, 0), A.img_h - 1);
            const int xx = min(max(pr.x0 - pad + q, 0), A.img_w - 1);
            halo[e] = im[(size_t)yy * A.img_w + xx];
        }
    }
    bf16x8_t h[4][KS];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const long long gr = row0 + 16 * i + r16;
        const bf16_t* hp = hin + (size_t)(gr - r_begin) * kFWidth + kg;
#pragma unroll
        for (int ks8 = 0; ks8 < KS; ++ks8) h[i][ks8] = gr < r_end ? load_b8(hp + 32 * ks8) : bf16x8_t{};
    }
    // the lane's row 16 i + l % 16 is pixel (row / 8, row % 8) of the tile;
    // tap (ti, tj) of that pixel reads halo[py + 2 pad - ti][px + 2 pad - tj],
    // i.e. hb[i] - (ti hh + tj) = hb[i] - (tap + 7 ti), as hh - ks = 7
    // (as LDS byte addresses, so that a read's address is one subtraction:
    // hb4[i] - coff4)
    const unsigned hbase = (unsigned)(size_t)(lds_cfloat_t*)halos;
    unsigned hb4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = 16 * i + r16;
        hb4[i] = hbase + 4u * (wave * hh * hh + ((row >> 3) + 2 * pad) * hh + (row & 7) + 2 * pad);
    }
    auto halo_at = [&](int i, int cb) __attribute__((always_inline)) {
        return *(lds_cfloat_t*)(size_t)(hb4[i] - (unsigned)cb);
    };
    floatx4_t acc[4][2];
    auto products = [&](const bf16_t* w) __attribute__((always_inline)) {
        const bf16_t* wb = w + lane * 8;
#pragma unroll
        for (int k8 = 0; k8 < KS; ++k8) {
            __builtin_amdgcn_sched_barrier(0);
            bf16x8_t a[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) a[j] = *reinterpret_cast<const bf16x8_t*>(wb + (j * KS + k8) * 512);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        a[j], h[i][k8], k8 == 0 ? floatx4_t{0.f, 0.f, 0.f, 0.f} : acc[i][j], 0, 0, 0);
        }
    };
    float m[4], s[4], al[4], ar[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) { m[i] = kNone; s[i] = 0.f; al[i] = 0.f; ar[i] = 0.f; }
    // one tile: logits in base 2 with the bias, the lazily raised reference
    // (as in the inference head), then the terms 2^(z - M) into S and, times
    // the image value under the column's tap, into the side's sum
    auto reduce = [&](const float* b, int t) __attribute__((always_inline)) {
        int coff4[2][4];                 // byte offsets of the columns' taps
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const floatx4_t v = *reinterpret_cast<const floatx4_t*>(b + 16 * j + g4);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = kRHCols * t + 16 * j + g4 + r;
                const bool valid = n < n_out;
                const float bl = valid ? v[r] * kL2E : kNone;
                const int tap = valid ? n - (n >= kk ? kk : 0) : 0;
                const int ti = (int)(((float)tap + 0.5f) * inv_ks);
                coff4[j][r] = 4 * (tap + 7 * ti);
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i][j][r] = fmaf(acc[i][j][r], kL2E, bl);
            }
        }
        // each row's largest logit of the tile, compared once with its
        // reference
        float zm[4];
        bool raise = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            zm[i] = fmaxf(fmaxf(fmaxf(acc[i][0][0], acc[i][0][1]), fmaxf(acc[i][0][2], acc[i][0][3])),
                          fmaxf(fmaxf(acc[i][1][0], acc[i][1][1]), fmaxf(acc[i][1][2], acc[i][1][3])));
            raise |= zm[i] > m[i];
        }
        if (__ballot(raise)) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float mn = fmaxf(m[i], zm[i] + kSlack);
                const float sc = __builtin_amdgcn_exp2f(m[i] - mn);
                s[i] *= sc; al[i] *= sc; ar[i] *= sc;
                m[i] = mn;
            }
        }
        // outputs [0, ks^2) are the left kernel's taps, [ks^2, 2 ks^2) the
        // right's: a tile wholly inside one of them (all but the one that
        // holds columns ks^2 - 1 and ks^2) adds its weighted terms to that
        // side's sum; that one tile also sums its right columns apart
        const int c0 = kRHCols * t;
        float ews[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float es = 0.f;
            ews[i] = 0.f;
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float e = __builtin_amdgcn_exp2f(acc[i][j][r] - m[i]);
                    es += e;
                    ews[i] = fmaf(e, halo_at(i, coff4[j][r]), ews[i]);
                }
            s[i] += es;
        }
        // the right side's part of each row's weighted sum: all of it, none,
        // or (the one straddling tile) its right columns summed apart; the
        // updates are arithmetic selects, so both sums stay in registers
        const bool straddle = c0 < kk && c0 + kRHCols > kk;
        float er[4] = {0.f, 0.f, 0.f, 0.f};
        if (straddle) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float e = __builtin_amdgcn_exp2f(acc[i][j][r] - m[i]);
                        er[i] = fmaf(c0 + 16 * j + g4 + r >= kk ? e : 0.f, halo_at(i, coff4[j][r]), er[i]);
                    }
        }
        const bool rs = c0 >= kk;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float rp = straddle ? er[i] : (rs ? ews[i] : 0.f);
            ar[i] += rp;
            al[i] += ews[i] - rp;
        }
    };

    // tile steps as in the inference head: wait for this wave's copies and
    // the other waves, start the next tile's copy into the other slot, then
    // the products and the reduction of this one
    auto step = [&](int t, auto slot) __attribute__((always_inline)) {
        constexpr int SL = decltype(slot)::value;
        __builtin_amdgcn_s_waitcnt(0x0f70);          // vmcnt(0)
        __syncthreads();
        if (t + 1 < ntile) fetch(t + 1, SL ? wt0 : wt1, SL ? bt0 : bt1);
        if (active) {
            products(SL ? wt1 : wt0);
            reduce(SL ? bt1 : bt0, t);
        }
    };
    int t = 0;
    for (; t + 1 < ntile; t += 2) {
        step(t, std::integral_constant<int, 0>());
        step(t + 1, std::integral_constant<int, 1>());
    }
    if (t < ntile) step(t, std::integral_constant<int, 0>());
    if (!active) return;
    // merge over the 4 lanes holding the same rows
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int o = 16; o < 64; o <<= 1) {
            const float m2 = __shfl_xor(m[i], o, 64);
            const float s2 = __shfl_xor(s[i], o, 64);
            const float l2 = __shfl_xor(al[i], o, 64);
            const float q2 = __shfl_xor(ar[i], o, 64);
            const float mn = fmaxf(m[i], m2);
            const float f1 = __builtin_amdgcn_exp2f(m[i] - mn), f2 = __builtin_amdgcn_exp2f(m2 - mn);
            s[i] = s[i] * f1 + s2 * f2;
            al[i] = al[i] * f1 + l2 * f2;
            ar[i] = ar[i] * f1 + q2 * f2;
            m[i] = mn;
        }
    }
    if (lane < 16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * i + r16;
            const int y = pr.y0 + (row >> 3), x = pr.x0 + (row & 7);
            if (row0 + row < r_end && y < A.img_h && x < A.img_w) {
                const float inv = 1.f / s[i];
                const size_t plane = (size_t)A.img_h * A.img_w;
                float* o = A.rout + ((size_t)pr.n * 2 * A.img_c + pr.c) * plane + (size_t)y * A.img_w + x;
                o[0] = al[i] * inv;
                o[(size_t)A.img_c * plane] = ar[i] * inv;
            }
        }
    }
}

int launch_mlp_render(const FusedArgs& A, bf16_t* hbuf, long long chunk, hipStream_t st) {
    if (A.n_rows <= 0) return SDIRT_OK;
    if (chunk < kFRows || chunk % kFRows) return SDIRT_EINVAL;
    const int hh = 8 + A.ks - 1;
    const size_t shm = (size_t)4 * hh * hh * sizeof(float);
    if (shm + 2 * (kRHTile * sizeof(bf16_t) + 64 * sizeof(float)) > 160 * 1024) return SDIRT_EUNSUPPORTED;
    (void)hipFuncSetAttribute((const void*)mlp_render_head_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
    for (long long r0 = 0; r0 < A.n_rows; r0 += chunk) {
        const long long r1 = std::min(A.n_rows, r0 + chunk);
        const long long blocks = (r1 - r0 + kFRows - 1) / kFRows;
        const long long hblocks = (r1 - r0 + kHRows - 1) / kHRows;
        if (blocks > 0x7fffffffLL) return SDIRT_EUNSUPPORTED;
        hipLaunchKernelGGL(mlp_trunk_kernel, dim3((unsigned)blocks), dim3(kFThreads), 0, st, A, r0, r1, hbuf);
        hipLaunchKernelGGL(mlp_render_head_kernel, dim3((unsigned)hblocks), dim3(kFThreads), shm, st, A, r0,
                           r1, (const bf16_t*)hbuf);
    }
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

}  // namespace sdirt
