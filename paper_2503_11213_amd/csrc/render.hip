// Pixel-wise DP rendering (Sec. 3.2, Supplement S1.3) for gfx950.
//
// out[n, s*C + c, y, x] = sum_{i,j} K[n,y,x,c',s][i][j]
//                         * img[n, c, clamp(y+pad-i), clamp(x+pad-j)]
//
// A workgroup owns a TH x TW tile of output pixels and stages the clamped
// (TH+ks-1) x (TW+ks-1) image halo of all C channels in LDS.  One wave
// renders one pixel at a time: its 64 lanes stride over the ks*ks taps, so
// every PSF row segment is read from HBM (dense source) or L2/MALL (bank
// source) by contiguous lanes, each PSF value exactly once; the 2C partial
// sums are reduced across the wave at the end.  The image adjoint gathers
// per halo position instead (see render_bwd_kernel).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/sdirt.h"

namespace sdirt {

int launch_fill_zero(void* p, size_t bytes, hipStream_t stream);

constexpr int kRBlock = 256;
constexpr int kWaves = kRBlock / 64;
constexpr int kTH = 8, kTW = 8;

struct RenderArgs {
    int N, C, H, W, ks, pad;
    int source, Cp, bf16;
    int F, D, L;
    long long t_r[SDIRT_MAX_BANK_F];   // squared-radius thresholds (half px)
    float t_z[SDIRT_MAX_BANK_D];       // depth thresholds (rounded up)
    int lam_of_c[4];
    int tiles_x, tiles_y;
    int use_fast;        // bank source: register-blocked kernel when ks allows
    const float* img;
    const void* psf;
    const float* depth;
    float* out;          // forward output
    const float* gout;   // backward input
    float* gimg;         // backward output
};

__device__ inline float wsum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Generic-path variants: dense kernels shared by all channels (Cp = 1),
// dense per-channel kernels, traced bank (nearest entry, mirrored).
enum RenderMode { kModeShared = 0, kModeDense = 1, kModeBank = 2 };

template <bool BF16> struct PsfT { typedef float type; };
template <> struct PsfT<true> { typedef uint16_t type; };

template <bool BF16>
__device__ inline float psf_at(const typename PsfT<BF16>::type* p, int idx) {
    if constexpr (BF16) return __uint_as_float(((uint32_t)p[idx]) << 16);
    else return p[idx];
}

// Kernels of one output pixel: a pointer per channel c and side s (wave
// uniform), and the bank mirrors (the side swap folded into the pointers).
template <int NC, bool BF16>
struct PixelKernel {
    const typename PsfT<BF16>::type* ptr[NC][2];
    int flip_x, flip_y;
};

template <int NC, int MODE, bool BF16>
__device__ inline void pixel_kernel(const RenderArgs& A, int n, int y, int x,
                                    PixelKernel<NC, BF16>* pk) {
    typedef typename PsfT<BF16>::type T;
    const T* psf = reinterpret_cast<const T*>(A.psf);
    const int kk = A.ks * A.ks;
    if (MODE != kModeBank) {
        const size_t pix = ((size_t)n * A.H + y) * A.W + x;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int cp = MODE == kModeShared ? 0 : c;
#pragma unroll
            for (int s = 0; s < 2; ++s)
                pk->ptr[c][s] = psf + ((pix * A.Cp + cp) * 2 + s) * kk;
        }
        pk->flip_x = 0;
        pk->flip_y = 0;
    } else {
        const long long X2 = 2LL * x - (A.W - 1);
        const long long Y2 = 2LL * y - (A.H - 1);
        const long long R2 = X2 * X2 + Y2 * Y2;
        int fi = 0;
        for (int k = 0; k < A.F - 1; ++k) fi += R2 > A.t_r[k];
        const float z = A.depth[((size_t)n * A.H + y) * A.W + x];
        int di = 0;
        for (int k = 0; k < A.D - 1; ++k) di += z < A.t_z[k];
        pk->flip_x = X2 < 0;
        pk->flip_y = Y2 < 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const size_t e = ((size_t)fi * A.D + di) * A.L + A.lam_of_c[c];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int ss = pk->flip_x ? 1 - s : s;
                pk->ptr[c][s] = psf + (e * 2 + ss) * kk;
            }
        }
    }
}

__device__ inline void stage_halo(const RenderArgs& A, int n, int y0, int x0,
                                  float* halo, int hh, int hw) {
    for (int c = 0; c < A.C; ++c) {
        const float* im = A.img + ((size_t)n * A.C + c) * A.H * A.W;
        for (int e = threadIdx.x; e < hh * hw; e += kRBlock) {
            const int r = e / hw, q = e - r * hw;
            const int yy = min(max(y0 - A.pad + r, 0), A.H - 1);
            const int xx = min(max(x0 - A.pad + q, 0), A.W - 1);
            halo[(c * hh + r) * hw + q] = im[(size_t)yy * A.W + xx];
        }
    }
}

template <int NC, int MODE, bool BF16>
__global__ __launch_bounds__(kRBlock) void render_fwd_kernel(const RenderArgs A) {
    extern __shared__ float halo[];
    const int ks = A.ks, kk = ks * ks;
    const int hh = kTH + ks - 1, hw = kTW + ks - 1;
    const int tile = blockIdx.x;
    const int n = tile / (A.tiles_x * A.tiles_y);
    const int rem = tile - n * A.tiles_x * A.tiles_y;
    const int y0 = (rem / A.tiles_x) * kTH, x0 = (rem % A.tiles_x) * kTW;
    stage_halo(A, n, y0, x0, halo, hh, hw);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int di = 64 / ks, dj = 64 % ks;
    for (int p = wave; p < kTH * kTW; p += kWaves) {
        const int y = y0 + p / kTW, x = x0 + p % kTW;
        if (y >= A.H || x >= A.W) continue;
        PixelKernel<NC, BF16> pk;
        pixel_kernel<NC, MODE, BF16>(A, n, y, x, &pk);
        float acc[2][NC];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[s][c] = 0.f;
        const int ly = y - y0 + ks - 1, lx = x - x0 + ks - 1;
        int i = lane / ks, j = lane % ks;
#pragma unroll 4
        for (int t = lane; t < kk; t += 64) {
            const int si = (MODE == kModeBank && pk.flip_y) ? ks - 1 - i : i;
            const int sj = (MODE == kModeBank && pk.flip_x) ? ks - 1 - j : j;
            const int st = si * ks + sj;
            const int hoff = (ly - i) * hw + (lx - j);
            if (MODE == kModeShared) {
                const float kl = psf_at<BF16>(pk.ptr[0][0], st);
                const float kr = psf_at<BF16>(pk.ptr[0][1], st);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const float v = halo[c * hh * hw + hoff];
                    acc[0][c] = fmaf(kl, v, acc[0][c]);
                    acc[1][c] = fmaf(kr, v, acc[1][c]);
                }
            } else {
                float kl[NC], kr[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    kl[c] = psf_at<BF16>(pk.ptr[c][0], st);
                    kr[c] = psf_at<BF16>(pk.ptr[c][1], st);
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const float v = halo[c * hh * hw + hoff];
                    acc[0][c] = fmaf(kl[c], v, acc[0][c]);
                    acc[1][c] = fmaf(kr[c], v, acc[1][c]);
                }
            }
            i += di;
            j += dj;
            if (j >= ks) { j -= ks; ++i; }
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const float v = wsum(acc[s][c]);
                if (lane == 0)
                    A.out[(((size_t)n * 2 * NC + s * NC + c) * A.H + y) * A.W + x] = v;
            }
    }
}

// Image adjoint as a gather: a thread owns halo positions of the tile (the
// clamped image pixels its 8 x 8 output pixels read) and, looping over those
// output pixels, accumulates K[tap] * grad for the one tap of each pixel that
// lands on its position.  Every kernel value is read once, by contiguous
// lanes along kernel rows, with no LDS traffic and no LDS atomics; the
// accumulated halo is folded onto the clamped image pixels with global
// atomics (neighbouring tiles overlap there).
constexpr int kGPer = 10;  // halo positions per thread per pass

template <int NC, int MODE, bool BF16>
__global__ __launch_bounds__(kRBlock) void render_bwd_kernel(const RenderArgs A) {
    const int ks = A.ks;
    const int hh = kTH + ks - 1, hw = kTW + ks - 1, nh = hh * hw;
    const int tile = blockIdx.x;
    const int n = tile / (A.tiles_x * A.tiles_y);
    const int rem = tile - n * A.tiles_x * A.tiles_y;
    const int y0 = (rem / A.tiles_x) * kTH, x0 = (rem % A.tiles_x) * kTW;
    const int tid = threadIdx.x;
    for (int base = 0; base < nh; base += kRBlock * kGPer) {
        int rr[kGPer], qq[kGPer];
        float acc[kGPer][NC];
#pragma unroll
        for (int k = 0; k < kGPer; ++k) {
            const int e = base + k * kRBlock + tid;
            rr[k] = e < nh ? e / hw : -(1 << 20);    // out of range: no tap matches
            qq[k] = e < nh ? e - rr[k] * hw : 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[k][c] = 0.f;
        }
        for (int p = 0; p < kTH * kTW; ++p) {
            const int y = y0 + p / kTW, x = x0 + p % kTW;
            if (y >= A.H || x >= A.W) continue;
            PixelKernel<NC, BF16> pk;
            pixel_kernel<NC, MODE, BF16>(A, n, y, x, &pk);
            float g[2][NC];
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    g[s][c] = A.gout[(((size_t)n * 2 * NC + s * NC + c) * A.H + y) * A.W + x];
            const int ly = y - y0 + ks - 1, lx = x - x0 + ks - 1;
#pragma unroll
            for (int k = 0; k < kGPer; ++k) {
                // positions outside this pixel's taps load tap 0 and add
                // nothing: the loads stay unconditional so that all of them
                // are in flight together
                const int i = ly - rr[k], j = lx - qq[k];
                const bool hit = (unsigned)i < (unsigned)ks && (unsigned)j < (unsigned)ks;
                const int si = (MODE == kModeBank && pk.flip_y) ? ks - 1 - i : i;
                const int sj = (MODE == kModeBank && pk.flip_x) ? ks - 1 - j : j;
                const int st = hit ? si * ks + sj : 0;
                if (MODE == kModeShared) {
                    float kl = psf_at<BF16>(pk.ptr[0][0], st);
                    float kr = psf_at<BF16>(pk.ptr[0][1], st);
                    kl = hit ? kl : 0.f;
                    kr = hit ? kr : 0.f;
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        acc[k][c] = fmaf(kl, g[0][c], fmaf(kr, g[1][c], acc[k][c]));
                } else {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        float kl = psf_at<BF16>(pk.ptr[c][0], st);
                        float kr = psf_at<BF16>(pk.ptr[c][1], st);
                        kl = hit ? kl : 0.f;
                        kr = hit ? kr : 0.f;
                        acc[k][c] = fmaf(kl, g[0][c], fmaf(kr, g[1][c], acc[k][c]));
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kGPer; ++k) {
            if (rr[k] < 0) continue;
            const int yy = min(max(y0 - A.pad + rr[k], 0), A.H - 1);
            const int xx = min(max(x0 - A.pad + qq[k], 0), A.W - 1);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (acc[k][c] != 0.f)
                    atomicAdd(&A.gimg[(((size_t)n * NC + c) * A.H + yy) * A.W + xx], acc[k][c]);
        }
    }
}

// ---- bank source, register-blocked path ----------------------------------
//
// Neighbouring pixels mostly share one bank entry, so the bank render is a
// sum over entries of ordinary shift-invariant convolutions restricted to the
// pixels that use them.  A thread owns a strip of 8 horizontally adjacent
// output pixels, a wave an 8 x 64 block, a workgroup a 32 x 64 tile whose
// clamped image halo (one channel at a time) sits in LDS.  The wave loops
// over the distinct entries of its block (wave-uniform); for each it runs a
// direct convolution with the entry's kernel read through the scalar cache
// (wave-uniform addresses), a 70-wide register window of the halo row and
// 16 accumulators, and keeps the result for the strip pixels that use the
// entry.  The adjoint scatters each kernel row's 1-D correlation with the
// strip's gradients into the LDS halo (one LDS atomic per halo column, not
// per tap) and folds the halo back with clamped global atomics.
constexpr int kFW = 64, kFH = 32, kStrip = 8;

template <int KS, bool BWD = false>
struct FastGeom {
    // Forward: rows padded to a multiple of 4 floats (+4) for float4 window
    // reads.  Adjoint: an odd row stride (1 mod 32) so the 8 rows x 8 strips
    // of a wave hit distinct LDS banks (at most 2 lanes per bank) in the
    // scatter's atomic adds.
    static constexpr int HWF = ((kFW + KS - 1 + 3) / 4) * 4 + 4;
    static constexpr int HWB = ((kFW + KS - 1 + 30) / 32) * 32 + 1;
    static constexpr int HW = BWD ? HWB : HWF;
    static constexpr int HH = kFH + KS - 1;
    static constexpr int WIN = ((KS + kStrip - 1 + 3) / 4) * 4;   // window, float4s
};

__device__ inline int wave_min_int(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// Bank key of pixel (y, x): ((fi * D + di) * 2 + flip_x) * 2 + flip_y.
__device__ inline int bank_key(const RenderArgs& A, int n, int y, int x) {
    const long long X2 = 2LL * x - (A.W - 1);
    const long long Y2 = 2LL * y - (A.H - 1);
    const long long R2 = X2 * X2 + Y2 * Y2;
    int fi = 0;
    for (int k = 0; k < A.F - 1; ++k) fi += R2 > A.t_r[k];
    const float z = A.depth[((size_t)n * A.H + y) * A.W + x];
    int di = 0;
    for (int k = 0; k < A.D - 1; ++k) di += z < A.t_z[k];
    return ((fi * A.D + di) * 2 + (X2 < 0 ? 1 : 0)) * 2 + (Y2 < 0 ? 1 : 0);
}

template <int KS>
__device__ inline void stage_fast_halo(const RenderArgs& A, int n, int c, int y0, int x0,
                                       float* halo) {
    using G = FastGeom<KS>;
    const int pad = (KS - 1) / 2;
    const float* im = A.img + ((size_t)n * A.C + c) * A.H * A.W;
    for (int e = threadIdx.x; e < G::HH * G::HW; e += kRBlock) {
        const int r = e / G::HW, q = e - r * G::HW;
        const int yy = min(max(y0 - pad + r, 0), A.H - 1);
        const int xx = min(max(x0 - pad + q, 0), A.W - 1);
        halo[e] = im[(size_t)yy * A.W + xx];
    }
}

template <int KS, bool FX>
__device__ inline void conv_strip(const float* __restrict__ kl, const float* __restrict__ kr,
                                  bool fy, const float* halo, int ly, int hc,
                                  float accL[kStrip], float accR[kStrip]) {
    using G = FastGeom<KS>;
#pragma unroll
    for (int q = 0; q < kStrip; ++q) { accL[q] = 0.f; accR[q] = 0.f; }
    for (int i = 0; i < KS; ++i) {
        const int si = fy ? KS - 1 - i : i;
        const float* rl = kl + si * KS;
        const float* rr = kr + si * KS;
        float win[G::WIN];
        const float4* src = reinterpret_cast<const float4*>(halo + (ly - i) * G::HW + hc);
#pragma unroll
        for (int m = 0; m < G::WIN / 4; ++m) {
            const float4 v = src[m];
            win[4 * m] = v.x; win[4 * m + 1] = v.y; win[4 * m + 2] = v.z; win[4 * m + 3] = v.w;
        }
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int sj = FX ? KS - 1 - j : j;
            const float a = rl[sj], b = rr[sj];
#pragma unroll
            for (int q = 0; q < kStrip; ++q) {
                accL[q] = fmaf(a, win[q - j + KS - 1], accL[q]);
                accR[q] = fmaf(b, win[q - j + KS - 1], accR[q]);
            }
        }
    }
}

template <int KS, bool FX>
__device__ inline void conv_strip_bwd(const float* __restrict__ kl, const float* __restrict__ kr,
                                      bool fy, float* hgrad, int ly, int hc,
                                      const float gL[kStrip], const float gR[kStrip]) {
    using G = FastGeom<KS, true>;
    for (int i = 0; i < KS; ++i) {
        const int si = fy ? KS - 1 - i : i;
        const float* rl = kl + si * KS;
        const float* rr = kr + si * KS;
        float acc[KS + kStrip - 1];
#pragma unroll
        for (int m = 0; m < KS + kStrip - 1; ++m) acc[m] = 0.f;
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int sj = FX ? KS - 1 - j : j;
            const float a = rl[sj], b = rr[sj];
#pragma unroll
            for (int q = 0; q < kStrip; ++q)
                acc[q - j + KS - 1] = fmaf(a, gL[q], fmaf(b, gR[q], acc[q - j + KS - 1]));
        }
        float* dst = hgrad + (ly - i) * G::HW + hc;
#pragma unroll
        for (int m = 0; m < KS + kStrip - 1; ++m) atomicAdd(&dst[m], acc[m]);
    }
}

template <int KS, bool BWD>
__global__ __launch_bounds__(kRBlock) void render_bank_fast_kernel(const RenderArgs A,
                                                                 const float* __restrict__ bank) {
    using G = FastGeom<KS, BWD>;
    extern __shared__ float halo[];     // [HH][HW]
    const int pad = (KS - 1) / 2;
    const int kk = KS * KS;
    const int tilesx = (A.W + kFW - 1) / kFW, tilesy = (A.H + kFH - 1) / kFH;
    const int tile = blockIdx.x;
    const int n = tile / (tilesx * tilesy);
    const int rem = tile - n * tilesx * tilesy;
    const int y0 = (rem / tilesx) * kFH, x0 = (rem % tilesx) * kFW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tr = wave * 8 + (lane >> 3);        // row within the tile
    const int tc = lane & 7;                      // strip within the row
    const int y = y0 + tr, xs = x0 + tc * kStrip;
    const int ly = tr + KS - 1;                   // halo row of tap i = 0
    const int hc = tc * kStrip;                   // halo column of the window start
    int key[kStrip];
#pragma unroll
    for (int q = 0; q < kStrip; ++q)
        key[q] = (y < A.H && xs + q < A.W) ? bank_key(A, n, y, xs + q) : 0x7fffffff;
    for (int c = 0; c < A.C; ++c) {
        const int lam = A.lam_of_c[c];
        float gL[kStrip], gR[kStrip], resL[kStrip], resR[kStrip];
        if (BWD) {
            for (int e = threadIdx.x; e < G::HH * G::HW; e += kRBlock) halo[e] = 0.f;
#pragma unroll
            for (int q = 0; q < kStrip; ++q) {
                const bool ok = key[q] != 0x7fffffff;
                const size_t o = ((size_t)n * 2 * A.C * A.H + y) * A.W + xs + q;
                gL[q] = ok ? A.gout[o + (size_t)c * A.H * A.W] : 0.f;
                gR[q] = ok ? A.gout[o + (size_t)(A.C + c) * A.H * A.W] : 0.f;
            }
        } else {
            stage_fast_halo<KS>(A, n, c, y0, x0, halo);
#pragma unroll
            for (int q = 0; q < kStrip; ++q) { resL[q] = 0.f; resR[q] = 0.f; }
        }
        __syncthreads();
        unsigned done = 0;
#pragma unroll
        for (int q = 0; q < kStrip; ++q) if (key[q] == 0x7fffffff) done |= 1u << q;
        while (true) {
            int mine = 0x7fffffff;
#pragma unroll
            for (int q = kStrip - 1; q >= 0; --q) if (!(done & (1u << q))) mine = key[q];
            const int k = __builtin_amdgcn_readfirstlane(wave_min_int(mine));
            if (k == 0x7fffffff) break;
            const int fyb = k & 1, fxb = (k >> 1) & 1, fd = k >> 2;
            const size_t base = ((size_t)fd * A.L + lam) * 2 * kk;
            const float* kl = bank + base + (fxb ? kk : 0);
            const float* kr = bank + base + (fxb ? 0 : kk);
            if (BWD) {
                float mL[kStrip], mR[kStrip];
#pragma unroll
                for (int q = 0; q < kStrip; ++q) {
                    mL[q] = key[q] == k ? gL[q] : 0.f;
                    mR[q] = key[q] == k ? gR[q] : 0.f;
                }
                if (fxb) conv_strip_bwd<KS, true>(kl, kr, fyb, halo, ly, hc, mL, mR);
                else conv_strip_bwd<KS, false>(kl, kr, fyb, halo, ly, hc, mL, mR);
            } else {
                float aL[kStrip], aR[kStrip];
                if (fxb) conv_strip<KS, true>(kl, kr, fyb, halo, ly, hc, aL, aR);
                else conv_strip<KS, false>(kl, kr, fyb, halo, ly, hc, aL, aR);
#pragma unroll
                for (int q = 0; q < kStrip; ++q)
                    if (key[q] == k) { resL[q] = aL[q]; resR[q] = aR[q]; }
            }
#pragma unroll
            for (int q = 0; q < kStrip; ++q) if (key[q] == k) done |= 1u << q;
        }
        if (BWD) {
            __syncthreads();
            float* gi = A.gimg + ((size_t)n * A.C + c) * A.H * A.W;
            for (int e = threadIdx.x; e < G::HH * G::HW; e += kRBlock) {
                const int r = e / G::HW, q = e - r * G::HW;
                if (q >= kFW + KS - 1) continue;
                const float v = halo[e];
                if (v == 0.f) continue;
                const int yy = min(max(y0 - pad + r, 0), A.H - 1);
                const int xx = min(max(x0 - pad + q, 0), A.W - 1);
                atomicAdd(&gi[(size_t)yy * A.W + xx], v);
            }
        } else if (y < A.H) {
#pragma unroll
            for (int q = 0; q < kStrip; ++q) {
                if (xs + q < A.W) {
                    const size_t o = (((size_t)n * 2 * A.C + c) * A.H + y) * A.W + xs + q;
                    A.out[o] = resL[q];
                    A.out[o + (size_t)A.C * A.H * A.W] = resR[q];
                }
            }
        }
        __syncthreads();
    }
}

// Bank-source image adjoint without LDS atomics.  Each wave owns 8 output
// rows x 64 columns and a private LDS halo of (KS + 7) rows; for each kernel
// row the lane computes the 1-D correlation of its strip's gradients with
// the kernel row (KS + 7 partial column sums), the 8 strips of a row trade
// those partial sums through lane shuffles so that every lane owns two
// disjoint groups of 8 halo columns, and the owner adds them with a plain
// read-modify-write.  The four private halos are summed and folded back
// (clamped) with global atomics once per channel.
constexpr int kBwdHW = 129;      // private halo row stride (1 mod 32: 2 lanes per bank)

template <int KS>
struct BwdGeom {
    static constexpr int PR = KS + kStrip - 1;        // private halo rows
    static constexpr int PW = PR * kBwdHW;            // floats per wave
    static constexpr int NKX = (KS + kStrip - 1 + 7) / 8;
};

template <int KS, bool FX>
__device__ inline void scatter_rows(const float* __restrict__ kl, const float* __restrict__ kr,
                                    bool fy, float* priv, int r, int o, int lane,
                                    const float gL[kStrip], const float gR[kStrip]) {
    using G = BwdGeom<KS>;
    const int base_lane = lane & ~7;
    for (int i = 0; i < KS; ++i) {
        const int si = fy ? KS - 1 - i : i;
        const float* rl = kl + si * KS;
        const float* rr = kr + si * KS;
        float acc[8 * G::NKX];
#pragma unroll
        for (int m = 0; m < 8 * G::NKX; ++m) acc[m] = 0.f;
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int sj = FX ? KS - 1 - j : j;
            const float a = rl[sj], b = rr[sj];
#pragma unroll
            for (int q = 0; q < kStrip; ++q)
                acc[q - j + KS - 1] = fmaf(a, gL[q], fmaf(b, gR[q], acc[q - j + KS - 1]));
        }
        // column 8 * o_src + m of strip o_src belongs to group o_src + m / 8
        float gA[8], gB[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) { gA[q] = 0.f; gB[q] = 0.f; }
#pragma unroll
        for (int kx = 0; kx < G::NKX; ++kx) {
            const int src = base_lane | ((o - kx) & 7);
            const bool lowgrp = o - kx >= 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float v = __shfl(acc[8 * kx + q], src, 64);
                if (lowgrp) gA[q] += v; else gB[q] += v;
            }
        }
        float* row = priv + (r + KS - 1 - i) * kBwdHW;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            row[8 * o + q] += gA[q];
            row[64 + 8 * o + q] += gB[q];
        }
    }
}

template <int KS>
__global__ __launch_bounds__(kRBlock) void render_bank_bwd_kernel(const RenderArgs A,
                                                                const float* __restrict__ bank) {
    using G = BwdGeom<KS>;
    extern __shared__ float lds[];      // 4 private halos [PR][kBwdHW]
    const int pad = (KS - 1) / 2;
    const int kk = KS * KS;
    const int tilesx = (A.W + kFW - 1) / kFW, tilesy = (A.H + kFH - 1) / kFH;
    const int tile = blockIdx.x;
    const int n = tile / (tilesx * tilesy);
    const int rem = tile - n * tilesx * tilesy;
    const int y0 = (rem / tilesx) * kFH, x0 = (rem % tilesx) * kFW;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane >> 3, o = lane & 7;
    const int y = y0 + wave * 8 + r, xs = x0 + o * kStrip;
    float* priv = lds + wave * G::PW;
    int key[kStrip];
#pragma unroll
    for (int q = 0; q < kStrip; ++q)
        key[q] = (y < A.H && xs + q < A.W) ? bank_key(A, n, y, xs + q) : 0x7fffffff;
    for (int c = 0; c < A.C; ++c) {
        const int lam = A.lam_of_c[c];
        for (int e = lane; e < G::PW; e += 64) priv[e] = 0.f;
        float gL[kStrip], gR[kStrip];
#pragma unroll
        for (int q = 0; q < kStrip; ++q) {
            const bool ok = key[q] != 0x7fffffff;
            const size_t off = ((size_t)n * 2 * A.C * A.H + y) * A.W + xs + q;
            gL[q] = ok ? A.gout[off + (size_t)c * A.H * A.W] : 0.f;
            gR[q] = ok ? A.gout[off + (size_t)(A.C + c) * A.H * A.W] : 0.f;
        }
        unsigned done = 0;
#pragma unroll
        for (int q = 0; q < kStrip; ++q) if (key[q] == 0x7fffffff) done |= 1u << q;
        while (true) {
            int mine = 0x7fffffff;
#pragma unroll
            for (int q = kStrip - 1; q >= 0; --q) if (!(done & (1u << q))) mine = key[q];
            const int k = __builtin_amdgcn_readfirstlane(wave_min_int(mine));
            if (k == 0x7fffffff) break;
            const int fyb = k & 1, fxb = (k >> 1) & 1, fd = k >> 2;
            const size_t base = ((size_t)fd * A.L + lam) * 2 * kk;
            const float* kl = bank + base + (fxb ? kk : 0);
            const float* kr = bank + base + (fxb ? 0 : kk);
            float mL[kStrip], mR[kStrip];
#pragma unroll
            for (int q = 0; q < kStrip; ++q) {
                mL[q] = key[q] == k ? gL[q] : 0.f;
                mR[q] = key[q] == k ? gR[q] : 0.f;
            }
            if (fxb) scatter_rows<KS, true>(kl, kr, fyb, priv, r, o, lane, mL, mR);
            else scatter_rows<KS, false>(kl, kr, fyb, priv, r, o, lane, mL, mR);
#pragma unroll
            for (int q = 0; q < kStrip; ++q) if (key[q] == k) done |= 1u << q;
        }
        __syncthreads();
        // sum the four private halos (wave w covers tile-halo rows 8w .. 8w + PR)
        float* gi = A.gimg + ((size_t)n * A.C + c) * A.H * A.W;
        const int HH = kFH + KS - 1, HWc = kFW + KS - 1;
        for (int e = threadIdx.x; e < HH * HWc; e += kRBlock) {
            const int R = e / HWc, Cc = e - R * HWc;
            float v = 0.f;
#pragma unroll
            for (int w = 0; w < kRBlock / 64; ++w) {
                const int rr = R - 8 * w;
                if (rr >= 0 && rr < G::PR) v += lds[w * G::PW + rr * kBwdHW + Cc];
            }
            if (v == 0.f) continue;
            const int yy = min(max(y0 - pad + R, 0), A.H - 1);
            const int xx = min(max(x0 - pad + Cc, 0), A.W - 1);
            atomicAdd(&gi[(size_t)yy * A.W + xx], v);
        }
        __syncthreads();
    }
}

template <int KS, bool BWD>
static bool launch_bank_fast(const RenderArgs& A, hipStream_t st) {
    using G = FastGeom<KS, BWD>;
    const size_t shm = BWD ? (size_t)(kRBlock / 64) * BwdGeom<KS>::PW * sizeof(float)
                           : (size_t)G::HH * G::HW * sizeof(float);
    const int tilesx = (A.W + kFW - 1) / kFW, tilesy = (A.H + kFH - 1) / kFH;
    const dim3 grid((unsigned)((long long)A.N * tilesx * tilesy));
    auto k = BWD ? render_bank_bwd_kernel<KS> : render_bank_fast_kernel<KS, false>;
    if (shm > 65536) (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(k, grid, dim3(kRBlock), shm, st, A, reinterpret_cast<const float*>(A.psf));
    return true;
}

template <bool BWD>
static bool try_bank_fast(const RenderArgs& A, hipStream_t st) {
    if (A.source != SDIRT_SRC_BANK) return false;
    if ((long long)A.F * A.D * 4 >= 0x7fffffffLL) return false;
    switch (A.ks) {
        case 21: return launch_bank_fast<21, BWD>(A, st);
        case 31: return launch_bank_fast<31, BWD>(A, st);
        case 33: return launch_bank_fast<33, BWD>(A, st);
        case 41: return launch_bank_fast<41, BWD>(A, st);
        case 63: return launch_bank_fast<63, BWD>(A, st);
        case 65: return launch_bank_fast<65, BWD>(A, st);
        default: return false;
    }
}

// ---- host ----------------------------------------------------------------

static int pack_render(const sdirt_render_desc* d, RenderArgs* A) {
    if (!d) return SDIRT_EINVAL;
    std::memset(A, 0, sizeof(*A));
    if (d->N < 1 || d->C < 1 || d->H < 1 || d->W < 1) return SDIRT_EINVAL;
    if (d->C > 4) return SDIRT_EUNSUPPORTED;
    if (d->ks < 1 || d->ks % 2 == 0) return SDIRT_EINVAL;
    if (d->ks > SDIRT_MAX_KS) return SDIRT_EUNSUPPORTED;
    if ((long long)d->H * d->W > (1LL << 30)) return SDIRT_EUNSUPPORTED;
    A->N = d->N; A->C = d->C; A->H = d->H; A->W = d->W; A->ks = d->ks;
    A->pad = (d->ks - 1) / 2;
    A->source = d->source;
    if (d->source == SDIRT_SRC_DENSE) {
        if (d->psf_channels != 1 && d->psf_channels != d->C) return SDIRT_EINVAL;
        A->Cp = d->psf_channels;
        if (d->psf_dtype == SDIRT_BF16) A->bf16 = 1;
        else if (d->psf_dtype != SDIRT_F32) return SDIRT_EUNSUPPORTED;
    } else if (d->source == SDIRT_SRC_BANK) {
        if (d->psf_dtype != SDIRT_F32) return SDIRT_EUNSUPPORTED;
        A->Cp = d->C;
        A->F = d->bank_fields; A->D = d->bank_depths; A->L = d->bank_lambdas;
        if (A->F < 1 || A->D < 1 || A->L < 1) return SDIRT_EINVAL;
        if (A->F > SDIRT_MAX_BANK_F || A->D > SDIRT_MAX_BANK_D) return SDIRT_EUNSUPPORTED;
        if (!d->field_radii || !d->inv_depths) return SDIRT_EINVAL;
        if (!std::isfinite(d->pitch) || !(d->pitch > 0)) return SDIRT_EINVAL;
        for (int k = 0; k < A->F; ++k) {
            if (!std::isfinite(d->field_radii[k])) return SDIRT_EINVAL;
            if (k && !(d->field_radii[k] > d->field_radii[k - 1])) return SDIRT_EINVAL;
        }
        for (int k = 0; k < A->D; ++k) {
            if (!std::isfinite(d->inv_depths[k]) || !(d->inv_depths[k] > 0)) return SDIRT_EINVAL;
            if (k && !(d->inv_depths[k] > d->inv_depths[k - 1])) return SDIRT_EINVAL;
        }
        // nearest field radius: R2 (exact integer, half-pixel units) against
        // floor((2 * midpoint / pitch)^2)
        for (int k = 0; k + 1 < A->F; ++k) {
            const double mid = 0.5 * (d->field_radii[k] + d->field_radii[k + 1]);
            const double t = std::floor((2.0 * mid / d->pitch) * (2.0 * mid / d->pitch));
            A->t_r[k] = t < 0 ? -1 : (long long)t;
        }
        // nearest inverse depth: depth < 1 / midpoint(1/d), threshold rounded
        // up to float so the float comparison decides exactly as in float64
        for (int k = 0; k + 1 < A->D; ++k) {
            const double mid = 0.5 * (d->inv_depths[k] + d->inv_depths[k + 1]);
            const double tz = 1.0 / mid;
            float f = (float)tz;
            if ((double)f < tz) f = std::nextafter(f, INFINITY);
            A->t_z[k] = f;
        }
        for (int c = 0; c < d->C; ++c) {
            if (d->lambda_of_channel[c] < 0 || d->lambda_of_channel[c] >= A->L) return SDIRT_EINVAL;
            A->lam_of_c[c] = d->lambda_of_channel[c];
        }
    } else {
        return SDIRT_EINVAL;
    }
    A->use_fast = 1;
    A->tiles_x = (d->W + kTW - 1) / kTW;
    A->tiles_y = (d->H + kTH - 1) / kTH;
    return SDIRT_OK;
}

template <int NC, bool BWD, int MODE, bool BF16>
static void launch_render3(const RenderArgs& A, hipStream_t st) {
    const int hh = kTH + A.ks - 1, hw = kTW + A.ks - 1;
    const size_t shm = (size_t)NC * hh * hw * sizeof(float);
    const dim3 grid((unsigned)((long long)A.N * A.tiles_x * A.tiles_y));
    if (BWD) {
        hipLaunchKernelGGL((render_bwd_kernel<NC, MODE, BF16>), grid, dim3(kRBlock), 0, st, A);
    } else {
        if (shm > 65536) (void)hipFuncSetAttribute((const void*)render_fwd_kernel<NC, MODE, BF16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        hipLaunchKernelGGL((render_fwd_kernel<NC, MODE, BF16>), grid, dim3(kRBlock), shm, st, A);
    }
}

template <int NC, bool BWD>
static void launch_render(const RenderArgs& A, hipStream_t st) {
    if (A.source == SDIRT_SRC_BANK) {
        if (A.bf16) launch_render3<NC, BWD, kModeBank, true>(A, st);
        else launch_render3<NC, BWD, kModeBank, false>(A, st);
    } else if (A.Cp == 1) {
        if (A.bf16) launch_render3<NC, BWD, kModeShared, true>(A, st);
        else launch_render3<NC, BWD, kModeShared, false>(A, st);
    } else {
        if (A.bf16) launch_render3<NC, BWD, kModeDense, true>(A, st);
        else launch_render3<NC, BWD, kModeDense, false>(A, st);
    }
}

template <bool BWD>
static int dispatch_render(const RenderArgs& A, hipStream_t st) {
    if (A.use_fast && try_bank_fast<BWD>(A, st))
        return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
    const int hh = kTH + A.ks - 1, hw = kTW + A.ks - 1;
    if (!BWD && (size_t)A.C * hh * hw * sizeof(float) > 160 * 1024) return SDIRT_EUNSUPPORTED;
    switch (A.C) {
        case 1: launch_render<1, BWD>(A, st); break;
        case 2: launch_render<2, BWD>(A, st); break;
        case 3: launch_render<3, BWD>(A, st); break;
        default: launch_render<4, BWD>(A, st); break;
    }
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

int render_impl(const sdirt_render_desc* desc, const float* img, const void* psf,
                const float* depth, float* out, hipStream_t stream) {
    RenderArgs A;
    int rc = pack_render(desc, &A);
    if (rc) return rc;
    if (!img || !psf || !out) return SDIRT_EINVAL;
    if (A.source == SDIRT_SRC_BANK && !depth) return SDIRT_EINVAL;
    A.img = img; A.psf = psf; A.depth = depth; A.out = out;
    return dispatch_render<false>(A, stream);
}

int render_backward_impl(const sdirt_render_desc* desc, const void* psf,
                         const float* depth, const float* gout, float* gimg,
                         hipStream_t stream) {
    RenderArgs A;
    int rc = pack_render(desc, &A);
    if (rc) return rc;
    if (!gout || !psf || !gimg) return SDIRT_EINVAL;
    if (A.source == SDIRT_SRC_BANK && !depth) return SDIRT_EINVAL;
    A.psf = psf; A.depth = depth; A.gout = gout; A.gimg = gimg;
    if ((rc = launch_fill_zero(gimg, (size_t)A.N * A.C * A.H * A.W * sizeof(float), stream)))
        return rc;
    return dispatch_render<true>(A, stream);
}

}  // namespace sdirt
