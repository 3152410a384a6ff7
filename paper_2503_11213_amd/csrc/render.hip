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
    long long t_r[SDIRT_MAX_BANK_F];   // squared-radius thresholds (half px); 2-D bank: |2x - W + 1|
    float t_z[SDIRT_MAX_BANK_D];       // depth thresholds (rounded up)
    int bank2d, Fy;                    // 2-D bank: F = Fx, Fy rows of the field grid
    long long t_y[SDIRT_MAX_BANK_F];   // 2-D bank: |2y - H + 1| thresholds (half px)
    float ivk[SDIRT_MAX_BANK_D];       // 2-D bank: inverse depths (float32)
    int pass;                          // 2-D bank: 0 = plane d0, weight 1 - w; 1 = d0 + 1, w
    int lam_of_c[4];
    int tiles_x, tiles_y;
    int use_fast;        // bank source: grouped kernels when ks allows
    int split;           // bank source: split-bf16 matrix cores (render and image adjoint)
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

// float -> kernel storage (bf16: round to nearest even)
template <bool BF16>
__device__ inline typename PsfT<BF16>::type to_psf(float v) {
    if constexpr (BF16) return __builtin_bit_cast(uint16_t, (__bf16)v);
    else return v;
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

// A workgroup of the forward owns a band of rows of a tile: bands smaller
// than the tile make many more workgroups than the chip holds at once, so
// the last of them leave little of it idle, while each band stages its own
// image halo (from the caches: the image is small next to the kernels).
// Measured best: one row for float32 per-channel kernels, four otherwise.
template <int MODE, bool BF16>
constexpr int fwd_rows() { return (MODE == kModeDense && !BF16) ? 1 : 4; }

template <int NC, int MODE, bool BF16>
__global__ __launch_bounds__(kRBlock) void render_fwd_kernel(const RenderArgs A) {
    constexpr int kFwdRows = fwd_rows<MODE, BF16>();
    extern __shared__ float halo[];
    const int ks = A.ks, kk = ks * ks;
    const int hh = kFwdRows + ks - 1, hw = kTW + ks - 1;
    constexpr int kBands = kTH / kFwdRows;
    const int tile = blockIdx.x / kBands;
    const int band = blockIdx.x - tile * kBands;
    const int n = tile / (A.tiles_x * A.tiles_y);
    const int rem = tile - n * A.tiles_x * A.tiles_y;
    const int y0 = (rem / A.tiles_x) * kTH + band * kFwdRows, x0 = (rem % A.tiles_x) * kTW;
    if (y0 >= A.H) return;
    stage_halo(A, n, y0, x0, halo, hh, hw);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int di = 64 / ks, dj = 64 % ks;
    for (int p = wave; p < kFwdRows * kTW; p += kWaves) {
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
constexpr int kBwdSync = 8;  // output pixels between workgroup barriers

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
            // keep the waves within a few pixels of each other, so that a
            // pixel's kernel lines are still in L2 when the last wave reads
            // them (2.24 -> 2.18 ms on a 512^2 RGB, 41^2 map)
            if (p && p % kBwdSync == 0) __syncthreads();
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

// Gradient with respect to a dense per-pixel kernel map: for each pixel,
// grad_K[c'][s][i][j] = sum over the channels c reading kernel c' of
// grad_out[s C + c] * img[c][clamp(y + pad - i)][clamp(x + pad - j)].  A
// workgroup owns a band of rows of a tile (as the forward does; measured
// best: one row for per-channel kernels, two for shared ones), whose image
// halo is staged in LDS; one wave writes one pixel's 2 Cp ks^2 values with
// contiguous lanes (an HBM-bound stream, like the forward).
template <bool SHARED> constexpr int grad_rows() { return SHARED ? 2 : 1; }

template <int NC, bool SHARED, bool BF16>
__global__ __launch_bounds__(kRBlock) void render_psf_grad_kernel(const RenderArgs A, void* grad) {
    typedef typename PsfT<BF16>::type T;
    constexpr int kGradRows = grad_rows<SHARED>();
    extern __shared__ float halo[];
    const int ks = A.ks, kk = ks * ks;
    const int hh = kGradRows + ks - 1, hw = kTW + ks - 1;
    constexpr int kBands = kTH / kGradRows;
    const int tile = blockIdx.x / kBands;
    const int band = blockIdx.x - tile * kBands;
    const int n = tile / (A.tiles_x * A.tiles_y);
    const int rem = tile - n * A.tiles_x * A.tiles_y;
    const int y0 = (rem / A.tiles_x) * kTH + band * kGradRows, x0 = (rem % A.tiles_x) * kTW;
    if (y0 >= A.H) return;
    stage_halo(A, n, y0, x0, halo, hh, hw);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T* gk = reinterpret_cast<T*>(grad);
    for (int p = wave; p < kGradRows * kTW; p += kWaves) {
        const int y = y0 + p / kTW, x = x0 + p % kTW;
        if (y >= A.H || x >= A.W) continue;
        float g[2][NC];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                g[s][c] = A.gout[(((size_t)n * 2 * NC + s * NC + c) * A.H + y) * A.W + x];
        const size_t pix = ((size_t)n * A.H + y) * A.W + x;
        const int ly = y - y0 + ks - 1, lx = x - x0 + ks - 1;
        for (int t = lane; t < kk; t += 64) {
            const int i = t / ks, j = t - i * ks;
            const int hoff = (ly - i) * hw + (lx - j);
            if (SHARED) {
                float a0 = 0.f, a1 = 0.f;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const float v = halo[c * hh * hw + hoff];
                    a0 = fmaf(g[0][c], v, a0);
                    a1 = fmaf(g[1][c], v, a1);
                }
                T* o = gk + pix * 2 * kk + t;
                o[0] = (T)to_psf<BF16>(a0);
                o[kk] = (T)to_psf<BF16>(a1);
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const float v = halo[c * hh * hw + hoff];
                    T* o = gk + (pix * NC + c) * 2 * kk + t;
                    o[0] = (T)to_psf<BF16>(g[0][c] * v);
                    o[kk] = (T)to_psf<BF16>(g[1][c] * v);
                }
            }
        }
    }
}

// ---- bank source, grouped paths ------------------------------------------
//
// Neighbouring pixels mostly share one bank entry, so the bank render is a
// sum over entries of ordinary shift-invariant convolutions restricted to the
// pixels that use them.  The unit of work is a strip of 8 horizontally
// adjacent output pixels and one entry.
//
// Forward: a workgroup owns one channel of a 64 x 64 pixel tile (512 strips)
// and first lists its (strip, entry, pixel mask) items grouped by entry, in
// chunks of at most 64 items of one entry; its four waves then take chunks
// as they free up (whole chunks first), with the clamped image halo in LDS.
// Grouping by entry over
// the whole tile keeps the matrix-core columns busy where a fixed pixel block
// would straddle several entries.  Channels are separate workgroups (the
// slowest grid index), which evens out the work per workgroup and keeps one
// wavelength's bank entries in the caches at a time.
//
// A chunk runs on the fp32 matrix cores.  For kernel row i the 8 outputs of a
// strip on both sides are the product of a 16 x P Toeplitz matrix made from
// the row (output (side, q) against window column p holds tap q - p + KS - 1,
// zero outside the kernel) with the strip's P-wide image window, so 16 strips
// of one entry are the 16 columns of a chain of v_mfma_f32_16x16x4_f32.  MFMA
// step t of lane group g = lane / 16 covers window column p = TPG g + t: a
// lane reads TPG consecutive window floats (8-byte LDS reads) and TPG
// consecutive taps.  Each wave stages the entry's kernel row pair in its own
// LDS row buffer between zero margins (mirrored when the entry is flipped in
// x), one row ahead of its use, so out-of-kernel taps read zeros.
constexpr int kStrip = 8;
constexpr int kGT = 64;                         // grouped forward: tile side
constexpr int kGStrips = kGT * kGT / kStrip;    // 512 strips per tile
constexpr int kGMaxItems = 1024;                // item list capacity per batch
constexpr int kGMaxChunks = 64;                 // chunk table capacity per batch

typedef float floatx4_t __attribute__((ext_vector_type(4)));

template <int KS>
struct GroupGeom {
    // rows padded to a multiple of 4 floats (+4) for vector window reads
    static constexpr int HW = ((kGT + KS - 1 + 3) / 4) * 4 + 4;
    static constexpr int HH = kGT + KS - 1;
};

template <int KS>
struct MfmaGeom {
    static constexpr int TPG = 2 * ((KS + kStrip - 1 + 7) / 8);   // MFMA steps per kernel row
    static constexpr int P = 4 * TPG;                              // window columns covered
    static constexpr int PADL = P - KS;                            // zero margin before the taps
    static constexpr int ROW = ((P + kStrip - 1 + 3) / 4) * 4;     // staged row length
    static_assert(P >= KS + kStrip - 1, "window covers every tap of 8 outputs");
    static_assert(kGT - kStrip + P <= GroupGeom<KS>::HW, "window inside the halo row");
};

__device__ inline int wave_min_int(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// 2-D bank: the planes bracketing the pixel's inverse depth and the weight
// of the farther one, in float32 (see the BANK2D source).
__device__ inline void depth_bracket(const RenderArgs& A, float z, int* d0, float* w) {
    const float iv = 1.0f / z;
    int d = 0;
    for (int k = 1; k < A.D - 1; ++k) d += iv >= A.ivk[k];
    float t = 0.f;
    if (A.D > 1) t = fminf(fmaxf((iv - A.ivk[d]) / (A.ivk[d + 1] - A.ivk[d]), 0.f), 1.f);
    *d0 = d;
    *w = t;
}

// Weight of pixel (y, x) in the current pass: 1 for the radial bank; 1 - w
// or w for the 2-D bank.
__device__ inline float pass_weight(const RenderArgs& A, int n, int y, int x) {
    if (!A.bank2d) return 1.f;
    int d0;
    float w;
    depth_bracket(A, A.depth[((size_t)n * A.H + y) * A.W + x], &d0, &w);
    return A.pass ? w : 1.f - w;
}

// Bank key of pixel (y, x): ((entry * 2 + flip_x) * 2 + flip_y), the entry
// fi * D + di (radial bank: nearest radius and inverse depth) or
// (fy * Fx + fx) * D + d (2-D bank: nearest grid point, plane d0 + pass);
// 0x7fffffff for a pixel with nothing to add in the 2-D bank's second pass.
__device__ inline int bank_key(const RenderArgs& A, int n, int y, int x) {
    const long long X2 = 2LL * x - (A.W - 1);
    const long long Y2 = 2LL * y - (A.H - 1);
    const float z = A.depth[((size_t)n * A.H + y) * A.W + x];
    int entry;
    if (A.bank2d) {
        const long long ax = X2 < 0 ? -X2 : X2, ay = Y2 < 0 ? -Y2 : Y2;
        int fx = 0, fy = 0;
        for (int k = 0; k < A.F - 1; ++k) fx += ax > A.t_r[k];
        for (int k = 0; k < A.Fy - 1; ++k) fy += ay > A.t_y[k];
        int d0;
        float w;
        depth_bracket(A, z, &d0, &w);
        if (A.pass && !(w > 0.f)) return 0x7fffffff;
        entry = (fy * A.F + fx) * A.D + d0 + A.pass;
    } else {
        const long long R2 = X2 * X2 + Y2 * Y2;
        int fi = 0;
        for (int k = 0; k < A.F - 1; ++k) fi += R2 > A.t_r[k];
        int di = 0;
        for (int k = 0; k < A.D - 1; ++k) di += z < A.t_z[k];
        entry = fi * A.D + di;
    }
    return (entry * 2 + (X2 < 0 ? 1 : 0)) * 2 + (Y2 < 0 ? 1 : 0);
}

// One lane's share of staging a kernel row pair into a row buffer of ROW
// floats per side (taps from PADL on): taps lane + 64 k of the concatenated
// [left row, right row], mirrored in x when fx.
template <int KS, int ROW, int PADL>
struct RowStager {
    static constexpr int NST = (2 * KS + 63) / 64;
    int src[NST], dst[NST];
    float v[NST];
    __device__ void init(int lane, bool fx) {
#pragma unroll
        for (int k = 0; k < NST; ++k) {
            const int e = min(lane + 64 * k, 2 * KS - 1);
            const int side = e >= KS, c = e - side * KS;
            // relative to the left row; the right kernel is the other half of
            // the entry, after it (or before it, when mirrored)
            src[k] = (side ? (fx ? -KS * KS : KS * KS) : 0) + (fx ? KS - 1 - c : c);
            dst[k] = side * ROW + PADL + c;
        }
    }
    __device__ void load(const float* __restrict__ kl, int row_ofs) {
#pragma unroll
        for (int k = 0; k < NST; ++k) v[k] = kl[row_ofs + src[k]];
    }
    __device__ void store(float* buf) const {
#pragma unroll
        for (int k = 0; k < NST; ++k) buf[dst[k]] = v[k];
    }
};

// Rows of one chunk: NG groups of 16 strips, two accumulator chains each.
template <int KS, int NG>
__device__ inline void bank_mfma_rows(const float* __restrict__ kl, int rstep, bool fx, bool fy,
                                      const float* halo, float* arow, int lane,
                                      const int (&bofs)[4], floatx4_t (&out)[4]) {
    using M = MfmaGeom<KS>;
    using G = GroupGeom<KS>;
    const int m = lane & 15, g = lane >> 4;
    // A read index of step t = 0 (taps then run backwards with t)
    const int aofs = (m >> 3) * M::ROW + M::PADL + (m & 7) + KS - 1 - M::TPG * g;
    RowStager<KS, M::ROW, M::PADL> sg;
    sg.init(lane, fx);
    sg.load(kl, (fy ? KS - 1 : 0) * KS);
    sg.store(arow);
    floatx4_t acc[2][4];
#pragma unroll
    for (int u = 0; u < NG; ++u) {
        acc[0][u] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        acc[1][u] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    }
    int row_ofs = (fy ? KS - 1 : 0) * KS;
    for (int i = 0; i < KS; ++i) {
        const bool more = i + 1 < KS;
        row_ofs += rstep;
        if (more) sg.load(kl, row_ofs);
        __builtin_amdgcn_sched_barrier(0);      // next row's taps in flight during this row
        const float* ar = arow + (i & 1) * 2 * M::ROW + aofs;
        float a[M::TPG];
#pragma unroll
        for (int t = 0; t < M::TPG; ++t) a[t] = ar[-t];
        float b[NG][M::TPG];
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            const float2* src = reinterpret_cast<const float2*>(halo + bofs[u] - i * G::HW);
#pragma unroll
            for (int t = 0; t < M::TPG / 2; ++t) {
                const float2 w = src[t];
                b[u][2 * t] = w.x;
                b[u][2 * t + 1] = w.y;
            }
        }
#pragma unroll
        for (int t = 0; t < M::TPG; ++t)
#pragma unroll
            for (int u = 0; u < NG; ++u)
                acc[t & 1][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[u][t], acc[t & 1][u], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        // the other buffer was last read in row i - 1
        if (more) sg.store(arow + ((i + 1) & 1) * 2 * M::ROW);
    }
#pragma unroll
    for (int u = 0; u < NG; ++u) out[u] = acc[0][u] + acc[1][u];
}

// Kernel gradient of one chunk (cnt <= 64 strips of one entry, in 16 k-steps
// of 4 strips): for kernel row i, the Toeplitz-shaped gradient
//     D[(side, q)][p] = sum over the strips of g[side][q] * window_i[p]
// is a matrix product with the strips as the contraction (A: the strips'
// output gradients, fixed over the rows; B: their image windows from the
// LDS halo), in 16-column blocks of p computed as independent chains.  The
// kernel gradient is its diagonal sum, grad_K[side][i][j] =
// sum_q D[(side, q)][q + KS - 1 - j], formed in registers with lane
// shuffles; one lane per diagonal adds it into the bank entry (mirrors
// applied) with a global atomic.
template <int KS>
struct KGradGeom {
    static constexpr int NB = (KS + kStrip - 1 + 15) / 16;    // 16-column blocks of p
    static constexpr int SCR = 4;                              // per-wave scratch (unused)
    static_assert(kGT - kStrip + KS + kStrip - 1 <= GroupGeom<KS>::HW, "window reads stay in the halo row");
};

// Within each row of 16 lanes: the value of lane l + k (row_shl) or l - k
// (row_shr), by DPP; lanes whose source falls outside the row read 0 and
// are not used by the callers.
__device__ inline float row_shl(float v, int k) {
    int r = 0;
    const int x = __builtin_bit_cast(int, v);
    switch (k) {
        case 1: r = __builtin_amdgcn_update_dpp(0, x, 0x101, 0xf, 0xf, false); break;
        case 2: r = __builtin_amdgcn_update_dpp(0, x, 0x102, 0xf, 0xf, false); break;
        case 3: r = __builtin_amdgcn_update_dpp(0, x, 0x103, 0xf, 0xf, false); break;
        default: r = __builtin_amdgcn_update_dpp(0, x, 0x104, 0xf, 0xf, false); break;
    }
    return __builtin_bit_cast(float, r);
}
__device__ inline float row_shr(float v, int k) {
    int r = 0;
    const int x = __builtin_bit_cast(int, v);
    switch (k) {
        case 15: r = __builtin_amdgcn_update_dpp(0, x, 0x11f, 0xf, 0xf, false); break;
        case 14: r = __builtin_amdgcn_update_dpp(0, x, 0x11e, 0xf, 0xf, false); break;
        case 13: r = __builtin_amdgcn_update_dpp(0, x, 0x11d, 0xf, 0xf, false); break;
        default: r = __builtin_amdgcn_update_dpp(0, x, 0x11c, 0xf, 0xf, false); break;
    }
    return __builtin_bit_cast(float, r);
}

template <int KS>
__device__ inline void bank_kgrad_chunk(const RenderArgs& A, int n, int c, int y0, int x0,
                                        const int* items, int cnt, int fxb, int fyb, float* ge,
                                        const float* halo, float* scr, int lane) {
    using G = GroupGeom<KS>;
    using KG = KGradGeom<KS>;
    const int kk = KS * KS;
    const int m = lane & 15, kq = lane >> 4;          // A: row (side, q) = m, k = kq
    const int side = m >> 3, q = m & 7;
    const int nks = (cnt + 3) >> 2;                   // k-steps of 4 strips
    float ga[16];
    int bofs[16];
    const size_t plane = (size_t)A.C * A.H * A.W;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int j = 4 * t + kq;
        const int it = items[min(j, cnt - 1)];
        const int sid = it & 511;
        const unsigned msk = j < cnt ? (unsigned)it >> 9 : 0u;
        const int y = y0 + (sid >> 3), xs = x0 + (sid & 7) * kStrip;
        // B operand of this lane: window column p = 16 b + m of strip j
        bofs[t] = ((sid >> 3) + KS - 1) * G::HW + (sid & 7) * kStrip;
        float g = 0.f;
        if ((msk >> q) & 1u) {
            g = A.gout[(((size_t)n * 2 * A.C + c) * A.H + y) * A.W + xs + q + side * plane];
            if (A.bank2d) g *= pass_weight(A, n, y, xs + q);
        }
        ga[t] = g;
    }
    (void)scr;
    for (int i = 0; i < KS; ++i) {
        // the NB column blocks as independent accumulation chains, k-step
        // by k-step, so that consecutive products do not wait on each other
        floatx4_t dd[KG::NB];
        int pofs[KG::NB];
#pragma unroll
        for (int b = 0; b < KG::NB; ++b) {
            dd[b] = floatx4_t{0.f, 0.f, 0.f, 0.f};
            // columns past the window (p > KS + 6) are never summed: those
            // lanes read the last window column instead
            pofs[b] = min(16 * b + m, KS + kStrip - 2) - i * G::HW;
        }
        for (int t = 0; t < nks; ++t) {
#pragma unroll
            for (int b = 0; b < KG::NB; ++b)
                dd[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[t], halo[bofs[t] + pofs[b]], dd[b], 0, 0, 0);
        }
        // diagonal sums in registers.  Lane (m, kq) holds D[(s, 4 h + r)][16 b + m]
        // (s = kq / 2, h = kq % 2): first u_b[m] = sum_r D[(s, 4 h + r)][16 b + m + r]
        // (diagonal c = 16 b + m - 4 h; columns past 15 from block b + 1), then
        // S[s][16 b + m] = u_b[m] of h = 0 + u_b[m + 4] of h = 1
        float uu[KG::NB];
#pragma unroll
        for (int b = 0; b < KG::NB; ++b) {
            float u = dd[b][0];
#pragma unroll
            for (int r = 1; r < 4; ++r) {
                const float a = row_shl(dd[b][r], r);                    // lane m + r
                float nx = 0.f;
                if (b + 1 < KG::NB) nx = row_shr(dd[b + 1][r], 16 - r);  // lane m + r - 16
                u += m + r < 16 ? a : nx;
            }
            uu[b] = u;
        }
        const int si = fyb ? KS - 1 - i : i;
        const int sd = kq >> 1;
#pragma unroll
        for (int b = 0; b < KG::NB; ++b) {
            const float a = row_shl(uu[b], 4);
            float nx = 0.f;
            if (b + 1 < KG::NB) nx = row_shr(uu[b + 1], 12);
            const float w = __shfl_xor(m + 4 < 16 ? a : nx, 16, 64);   // h = 1's, on h = 0 lanes
            const float v = uu[b] + w;
            // row i of side sd into the entry: tap j = KS - 1 - c, mirrored
            const int cc = 16 * b + m;
            if ((kq & 1) == 0 && cc < KS && v != 0.f) {
                const int j = KS - 1 - cc;
                const int sj = fxb ? KS - 1 - j : j;
                const int ss = fxb ? 1 - sd : sd;
                atomicAdd(&ge[(size_t)ss * kk + si * KS + sj], v);
            }
        }
    }
}

// ---- split-bf16 forward ----------------------------------------------------
//
// The same entry-grouped chunks on the bf16 matrix cores: every float32
// operand x is split into x_hi = bf16(x) and x_lo = bf16(x - x_hi), and a
// product is taken as A_hi B_hi + A_hi B_lo + A_lo B_hi (the dropped
// A_lo B_lo and the residuals of the splits are below 2^-16 of it), summed in
// float32 by v_mfma_f32_16x16x32_bf16.  For one chunk, the contraction runs
// over (kernel row i, window column p): 8 consecutive window columns of one
// row form a k-group, P = the strip window rounded up to 8 columns, so a row
// is G = P / 8 groups and R consecutive rows (R G a multiple of 4) make T =
// R G / 4 k-steps of 32.  Lane (m, kg) of the A operand (m = (side, q) output
// row, kg = k-group) needs the 8 taps of the reversed kernel row starting at
// 8 pg - q.  Each wave stages, per R rows, the reversed rows of both sides
// once, split into bf16 hi and lo rows between zero margins; a lane reads
// the 5 dwords that hold its 8 taps and shifts them into place by the parity
// of q with v_alignbit (the shift is fixed per lane).  The B operand (image
// windows) is read from hi and lo bf16 halos as aligned 16-byte LDS reads.
// Two accumulator chains per group (hi hi, and hi lo + lo hi) halve the
// dependent MFMA sequence.  The halo rows carry no padding, so that the halo
// (64 KB at ks 65) and the wave buffers fit two workgroups per CU.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
// LDS words written as bf16 halves and read as dwords: accesses through
// these types may alias each other
typedef uint32_t __attribute__((may_alias)) u32_alias;
typedef uint16_t __attribute__((may_alias)) u16_alias;

template <int KS>
struct SplitGeom {
    static constexpr int P = ((KS + kStrip - 1 + 7) / 8) * 8;   // window columns per row
    static constexpr int G = P / 8;                              // k-groups per row
    static constexpr int R = (G % 4 == 0) ? 1 : ((G % 2 == 0) ? 2 : 4);   // rows per super-step
    static constexpr int T = R * G / 4;                          // k-steps per super-step
    static constexpr int NSS = (KS + R - 1) / R;                 // super-steps
    static constexpr int MARG = 8;                               // zero margin before the taps
    // staged row: taps at MARG + u; lane reads reach element P + 9
    static constexpr int RWB = ((MARG + P + 2 + 7) / 8) * 8;
    static constexpr int LO = R * 2 * RWB;                       // lo rows after the hi rows (bf16)
    static constexpr int SCRATCH = LO;                           // floats per wave (hi + lo bf16)
    static constexpr int NTAP = R * 2 * KS;                      // kernel taps per super-step
    static constexpr int HW0 = kGT + KS - 1 > kGT - kStrip + P ? kGT + KS - 1 : kGT - kStrip + P;
    // halo rows of 128 bf16 (16 blocks of 8): odd rows keep their two
    // halves swapped (column ^ 64), which puts the two strip rows of a
    // typical group of 16 strips on different LDS banks
    static constexpr int HWB = 128;
    static constexpr int HH = kGT + KS - 1;
    static_assert(HW0 <= HWB, "strip windows inside the halo row");
    static_assert((R * G) % 4 == 0, "whole k-steps per super-step");
    static_assert(RWB % 2 == 0 && LO % 2 == 0 && HWB % 8 == 0, "aligned fragment reads");
    static_assert(MARG >= kStrip - 1 && RWB >= P + 10, "lane reads stay inside the staged row");
};

__device__ inline uint32_t split_bf16_bits(float v) {
    const __bf16 h = (__bf16)v;
    const __bf16 l = (__bf16)(v - (float)h);
    return (uint32_t)__builtin_bit_cast(uint16_t, h) | ((uint32_t)__builtin_bit_cast(uint16_t, l) << 16);
}

// One lane's share of a super-step's taps: element e = lane + 64 k of
// [R rows][2 sides][KS] (reversed-row order u), read from the entry with its
// mirrors applied, and its place in the staged rows.  Offsets are those of
// super-step 0; super-step ss moves R rows down the entry (up, when flipped
// in y), and rows past the kernel read as zero.
template <int KS>
struct SplitTaps {
    using S = SplitGeom<KS>;
    static constexpr int NL = (S::NTAP + 63) / 64;
    int src[NL], dst[NL], row[NL];
    float v[NL];
    __device__ void init(int lane, bool fx, bool fy) {
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = lane + 64 * k;
            const int r = e / (2 * KS), rem = e - r * 2 * KS;
            const int side = rem >= KS, u = rem - side * KS;
            const int ri = fy ? KS - 1 - r : r;
            // output side s reads the stored side s, or 1 - s mirrored in x;
            // reversed row: R_s[u] = K_s[i][KS - 1 - u]
            src[k] = fx ? (1 - side) * KS * KS + ri * KS + u : side * KS * KS + ri * KS + KS - 1 - u;
            dst[k] = (r * 2 + side) * S::RWB + S::MARG + u;
            row[k] = e < S::NTAP ? r : KS;
        }
    }
    __device__ void load(const float* __restrict__ entry, int ss, int rstep) {
        const int lim = KS - ss * S::R;
        const int ofs = ss * S::R * rstep;
#pragma unroll
        for (int k = 0; k < NL; ++k) v[k] = row[k] < lim ? entry[src[k] + ofs] : 0.f;
    }
    __device__ void store(u16_alias* st) const {
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            if (64 * k + 64 <= S::NTAP || row[k] < KS) {            // e < NTAP
                const uint32_t b = split_bf16_bits(v[k]);
                st[dst[k]] = (uint16_t)b;
                st[S::LO + dst[k]] = (uint16_t)(b >> 16);
            }
        }
    }
};

// Rows of one chunk on the split-bf16 path: NG groups of 16 strips.
template <int KS, int NG>
__device__ inline void bank_split_rows(const float* __restrict__ entry, bool fx, bool fy,
                                       const __bf16* hhi, const __bf16* hlo, float* scratch,
                                       int lane, const int (&bofs)[4], floatx4_t (&out)[4]) {
    using S = SplitGeom<KS>;
    u16_alias* st = reinterpret_cast<u16_alias*>(scratch);
    const u32_alias* sw = reinterpret_cast<const u32_alias*>(scratch);
    const int m = lane & 15, kg = lane >> 4;
    const int side = m >> 3, q = m & 7;
    const uint32_t sh = (q & 1) * 16;
    // per k-step: dword index of the lane's first A word, its row in the
    // super-step and window column
    int ad[S::T], irw[S::T], pcol[S::T];
#pragma unroll
    for (int t = 0; t < S::T; ++t) {
        const int g = 4 * t + kg;
        const int ir = g / S::G, pg = g - ir * S::G;
        ad[t] = ((ir * 2 + side) * S::RWB + S::MARG + 8 * pg - q) >> 1;
        irw[t] = ir;
        pcol[t] = 8 * pg;
    }
    floatx4_t acc_h[NG], acc_l[NG];
#pragma unroll
    for (int u = 0; u < NG; ++u) {
        acc_h[u] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        acc_l[u] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    }
    const int rstep = fy ? -KS : KS;
    SplitTaps<KS> taps;
    taps.init(lane, fx, fy);
    taps.load(entry, 0, rstep);
    for (int ss = 0; ss < S::NSS; ++ss) {
        // the previous super-step's reads of the staged rows are issued
        // before these writes (one wave: LDS accesses stay in order)
        __asm__ volatile("" ::: "memory");
        taps.store(st);
        __asm__ volatile("" ::: "memory");
        if (ss + 1 < S::NSS) taps.load(entry, ss + 1, rstep);
#pragma unroll
        for (int t = 0; t < S::T; ++t) {
            uint32_t h[5], l[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                h[j] = sw[ad[t] + j];
                l[j] = sw[S::LO / 2 + ad[t] + j];
            }
            u32x4_t ah, al;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                ah[j] = __builtin_amdgcn_alignbit(h[j + 1], h[j], sh);
                al[j] = __builtin_amdgcn_alignbit(l[j + 1], l[j], sh);
            }
            const bf16x8_t a_hi = __builtin_bit_cast(bf16x8_t, ah);
            const bf16x8_t a_lo = __builtin_bit_cast(bf16x8_t, al);
            // rows past the kernel (the last super-step's padding) carry
            // zero taps; their image rows are clamped into the halo so that
            // the zero products stay finite
            const int brow = -min(ss * S::R + irw[t], KS - 1) * S::HWB + pcol[t];
            bf16x8_t b_hi[NG], b_lo[NG];
#pragma unroll
            for (int u = 0; u < NG; ++u) {
                // bit 7 of the element offset is the halo row's parity
                int o = bofs[u] + brow;
                o ^= (o >> 1) & 64;
                b_hi[u] = *reinterpret_cast<const bf16x8_t*>(hhi + o);
                b_lo[u] = *reinterpret_cast<const bf16x8_t*>(hlo + o);
            }
#pragma unroll
            for (int u = 0; u < NG; ++u) {
                acc_h[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, b_hi[u], acc_h[u], 0, 0, 0);
                acc_l[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, b_lo[u], acc_l[u], 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < NG; ++u)
                acc_l[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo, b_hi[u], acc_l[u], 0, 0, 0);
        }
    }
#pragma unroll
    for (int u = 0; u < NG; ++u) out[u] = acc_h[u] + acc_l[u];
}

// MODE: kBankFwd (fp32 matrix cores), kBankKGrad (gradient with respect to
// the bank entries, see bank_kgrad_chunk; grad is the bank-shaped
// accumulator), kBankSplit (split-bf16 matrix cores).
enum BankMode { kBankFwd = 0, kBankKGrad = 1, kBankSplit = 2 };

template <int KS, int MODE>
__device__ __forceinline__ void render_bank_fast_body(const RenderArgs A, const float* __restrict__ bank,
                                                      float* __restrict__ grad) {
    constexpr bool KGRAD = MODE == kBankKGrad;
    constexpr bool SPLIT = MODE == kBankSplit;
    using G = GroupGeom<KS>;
    using M = MfmaGeom<KS>;
    using S = SplitGeom<KS>;
    // [HH][HW] float32 image halo, or (split) [HH][HWB] bf16 hi then lo
    extern __shared__ __align__(16) float halo[];
    __shared__ int items[kGMaxItems];                    // strip | mask << 9
    __shared__ int chunk_key[kGMaxChunks], chunk_pos[kGMaxChunks];
    __shared__ int red[kRBlock / 64];
    __shared__ int n_items, n_full, n_part, next_chunk;
    // per wave: kernel-row staging (2 buffers x 2 sides), for KGRAD the
    // block and diagonal-sum scratch of bank_kgrad_chunk, for the split path
    // the shifted hi/lo row copies and the float32 reversed rows
    constexpr int kWaveScratch = KGRAD ? KGradGeom<KS>::SCR : SPLIT ? S::SCRATCH : 4 * M::ROW;
    __shared__ __align__(16) float arows[kRBlock / 64][kWaveScratch];
    const int pad = (KS - 1) / 2;
    const int kk = KS * KS;
    const int tilesx = (A.W + kGT - 1) / kGT, tilesy = (A.H + kGT - 1) / kGT;
    const int nt = A.N * tilesx * tilesy;
    const int c = blockIdx.x / nt;                       // channel slowest: one wavelength's entries at a time
    const int tile = blockIdx.x - c * nt;
    const int n = tile / (tilesx * tilesy);
    const int rem = tile - n * tilesx * tilesy;
    const int y0 = (rem / tilesx) * kGT, x0 = (rem % tilesx) * kGT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float* arow = arows[wave];
    for (int e = lane; e < kWaveScratch; e += 64) arow[e] = 0.f;   // margins stay zero
    // keys of the two strips this thread lists (strip sid: row sid / 8, column block sid % 8)
    int key[2][kStrip];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int sid = tid + h * kRBlock;
        const int y = y0 + (sid >> 3), xs = x0 + (sid & 7) * kStrip;
#pragma unroll
        for (int q = 0; q < kStrip; ++q)
            key[h][q] = (y < A.H && xs + q < A.W) ? bank_key(A, n, y, xs + q) : 0x7fffffff;
    }
    unsigned done = 0;                                   // bit 8 h + q: pixel listed
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < kStrip; ++q)
            if (key[h][q] == 0x7fffffff) done |= 1u << (8 * h + q);
    bool more = true;
    while (more) {
        // ---- list a batch of entries, grouped, in chunks of <= 64 items
        // the chunk counter starts at 0 even when the batch lists nothing
        if (tid == 0) { n_items = 0; n_full = 0; n_part = 0; next_chunk = 0; }
        __syncthreads();
        while (true) {
            int mine = 0x7fffffff;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < kStrip; ++q)
                    if (!(done & (1u << (8 * h + q)))) mine = min(mine, key[h][q]);
            const int wm = wave_min_int(mine);
            if (lane == 0) red[wave] = wm;
            __syncthreads();
            int k = red[0];
#pragma unroll
            for (int w = 1; w < kRBlock / 64; ++w) k = min(k, red[w]);
            const int start = n_items;
            // capacity: a batch ends before an entry that might not fit
            const bool fits = start + kGStrips <= kGMaxItems &&
                              n_full + n_part + kGStrips / 64 <= kGMaxChunks;
            __syncthreads();
            if (k == 0x7fffffff) { more = false; break; }
            if (!fits) break;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                unsigned m = 0;
#pragma unroll
                for (int q = 0; q < kStrip; ++q)
                    if (key[h][q] == k) m |= 1u << q;
                if (m) {
                    const int pos = atomicAdd(&n_items, 1);
                    items[pos] = (tid + h * kRBlock) | (int)(m << 9);
                    done |= m << (8 * h);
                }
            }
            __syncthreads();
            if (tid == 0) {
                // full chunks from the front of the table, partial ones from
                // the back: the waves take the full ones first
                for (int s0 = start; s0 < n_items; s0 += 64) {
                    const int cnt = min(64, n_items - s0);
                    const int slot = cnt == 64 ? n_full++ : kGMaxChunks - 1 - n_part++;
                    chunk_key[slot] = k;
                    chunk_pos[slot] = s0 | (cnt << 16);
                }
            }
            __syncthreads();
        }
        const int T = n_full + n_part, nf = n_full;
        // ---- render the batch
        {
            const int lam = A.lam_of_c[c];
            const float* im = A.img + ((size_t)n * A.C + c) * A.H * A.W;
            if constexpr (SPLIT) {
                u32_alias* hhi = reinterpret_cast<u32_alias*>(halo);
                u32_alias* hlo = hhi + S::HH * S::HWB / 2;
                for (int e = tid; e < S::HH * S::HWB / 2; e += kRBlock) {
                    const int r = e / (S::HWB / 2), q = 2 * (e - r * (S::HWB / 2));
                    const int yy = min(max(y0 - pad + r, 0), A.H - 1);
                    const int x0c = min(max(x0 - pad + q, 0), A.W - 1);
                    const int x1c = min(max(x0 - pad + q + 1, 0), A.W - 1);
                    const uint32_t b0 = split_bf16_bits(im[(size_t)yy * A.W + x0c]);
                    const uint32_t b1 = split_bf16_bits(im[(size_t)yy * A.W + x1c]);
                    const int es = r * (S::HWB / 2) + ((q ^ ((r & 1) << 6)) >> 1);
                    hhi[es] = (b0 & 0xffffu) | (b1 << 16);
                    hlo[es] = (b0 >> 16) | (b1 & 0xffff0000u);
                }
            } else {
                for (int e = tid; e < G::HH * G::HW; e += kRBlock) {
                    const int r = e / G::HW, q = e - r * G::HW;
                    const int yy = min(max(y0 - pad + r, 0), A.H - 1);
                    const int xx = min(max(x0 - pad + q, 0), A.W - 1);
                    halo[e] = im[(size_t)yy * A.W + xx];
                }
            }
            __syncthreads();
            while (true) {
                // chunks go to the waves as they free up
                int j = 0;
                if (lane == 0) j = atomicAdd(&next_chunk, 1);
                j = __builtin_amdgcn_readfirstlane(j);
                if (j >= T) break;
                const int ch = j < nf ? j : kGMaxChunks - 1 - (j - nf);
                const int k = __builtin_amdgcn_readfirstlane(chunk_key[ch]);
                const int cp = __builtin_amdgcn_readfirstlane(chunk_pos[ch]);
                const int cnt = cp >> 16, s0 = cp & 0xffff;
                const int fyb = k & 1, fxb = (k >> 1) & 1, fd = k >> 2;
                if (KGRAD) {
                    bank_kgrad_chunk<KS>(A, n, c, y0, x0, items + s0, cnt, fxb, fyb,
                                         grad + ((size_t)fd * A.L + lam) * 2 * kk, halo, arow, lane);
                    continue;
                }
                int its[4], bofs[4];
                const int ng = (cnt + 15) >> 4;
                floatx4_t acc[4];
                if constexpr (SPLIT) {
                    const float* entry = bank + ((size_t)fd * A.L + lam) * 2 * kk;
                    const __bf16* hhi = reinterpret_cast<const __bf16*>(halo);
                    const __bf16* hlo = hhi + S::HH * S::HWB;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        its[u] = items[s0 + min(16 * u + (lane & 15), cnt - 1)];
                        const int sid = its[u] & 511;
                        // B operand of lane (strip, kg): halo row (strip row + KS - 1 - i),
                        // columns 8 (strip column) + 8 pg + [0, 8)
                        bofs[u] = ((sid >> 3) + KS - 1) * S::HWB + (sid & 7) * kStrip;
                    }
                    switch (ng) {
                        case 1: bank_split_rows<KS, 1>(entry, fxb, fyb, hhi, hlo, arow, lane, bofs, acc); break;
                        case 2: bank_split_rows<KS, 2>(entry, fxb, fyb, hhi, hlo, arow, lane, bofs, acc); break;
                        case 3: bank_split_rows<KS, 3>(entry, fxb, fyb, hhi, hlo, arow, lane, bofs, acc); break;
                        default: bank_split_rows<KS, 4>(entry, fxb, fyb, hhi, hlo, arow, lane, bofs, acc); break;
                    }
                } else {
                    // left output side reads the stored right kernel when mirrored
                    const float* kl = bank + ((size_t)fd * A.L + lam) * 2 * kk + (fxb ? kk : 0);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        its[u] = items[s0 + min(16 * u + (lane & 15), cnt - 1)];
                        const int sid = its[u] & 511;
                        bofs[u] = ((sid >> 3) + KS - 1) * G::HW + (sid & 7) * kStrip + M::TPG * (lane >> 4);
                    }
                    const int rstep = fyb ? -KS : KS;
                    switch (ng) {
                        case 1: bank_mfma_rows<KS, 1>(kl, rstep, fxb, fyb, halo, arow, lane, bofs, acc); break;
                        case 2: bank_mfma_rows<KS, 2>(kl, rstep, fxb, fyb, halo, arow, lane, bofs, acc); break;
                        case 3: bank_mfma_rows<KS, 3>(kl, rstep, fxb, fyb, halo, arow, lane, bofs, acc); break;
                        default: bank_mfma_rows<KS, 4>(kl, rstep, fxb, fyb, halo, arow, lane, bofs, acc); break;
                    }
                }
                // lane holds outputs q = 4 (g & 1) + r of side g >> 1 of its strip
                const int g = lane >> 4;
                const size_t side_ofs = (g >> 1) ? (size_t)A.C * A.H * A.W : 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool valid = u < ng && 16 * u + (lane & 15) < cnt;
                    const unsigned msk = valid ? (unsigned)its[u] >> 9 : 0u;
                    const int sid = its[u] & 511;
                    const int y = y0 + (sid >> 3), xs = x0 + (sid & 7) * kStrip + 4 * (g & 1);
                    const size_t o = (((size_t)n * 2 * A.C + c) * A.H + y) * A.W + xs + side_ofs;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (msk & (1u << (4 * (g & 1) + r))) {
                            if (!A.bank2d) {
                                A.out[o + r] = acc[u][r];
                            } else {
                                // 2-D bank: the pass's share of the depth
                                // blend, written by the first pass, added by
                                // the second
                                const float wt = pass_weight(A, n, y, xs + r);
                                A.out[o + r] = A.pass ? fmaf(wt, acc[u][r], A.out[o + r]) : wt * acc[u][r];
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <int KS, int MODE>
__global__ __launch_bounds__(kRBlock) void render_bank_fast_kernel(const RenderArgs A,
                                                                 const float* __restrict__ bank,
                                                                 float* __restrict__ grad) {
    render_bank_fast_body<KS, MODE>(A, bank, grad);
}

// The split-bf16 forward, compiled for two workgroups per CU (its LDS use is
// sized for that).
template <int KS>
__global__ __launch_bounds__(kRBlock, 2) void render_bank_split_kernel(const RenderArgs A,
                                                                     const float* __restrict__ bank) {
    render_bank_fast_body<KS, kBankSplit>(A, bank, nullptr);
}

// Bank-source image adjoint on the matrix cores.  A one-wave workgroup owns
// a 32 x 32 pixel band (4 strip columns of 32 rows) and a private LDS copy of
// the band's image-halo gradient (under 40 KB for ks <= 65, so four such
// waves share a compute unit).  It takes the band's entries one at a time;
// per strip column, an entry's strips (at most 32, all in distinct rows) form
// one or two groups of 16, and up to four groups run together.  For
// kernel row i a group's halo contribution is the transposed Toeplitz matrix
// of the row pair (window column p against output (side, q)) times the
// 16 x 16 matrix of the strips' masked output gradients, in blocks of 16
// window columns (four k-steps of v_mfma_f32_16x16x4_f32 over (side, q)).
// Lane l then holds the block's columns 4 (l / 16) .. + 3 for strip l % 16
// and adds them into the halo with one float4 read-modify-write.  The
// strips of a group lie in distinct rows, so a group's read-modify-writes of
// one kernel row never touch one address twice and go out together,
// interleaved with the group's products of the next row; successive groups
// and rows are ordered by program order (LDS operations of one wave execute
// in order).
// A workgroup handles one channel of its band and finally folds the halo
// onto the clamped image pixels with global atomics.
constexpr int kBR = 32, kBW = 32;                     // band rows, columns
constexpr int kBS = kBW / kStrip;                     // strips per band row
static_assert(kBR * kBS == 128, "two strips per lane");

template <int KS>
struct BandGeom {
    static constexpr int NB = (KS + kStrip - 1 + 15) / 16;         // 16-column blocks of the window
    static constexpr int WP = ((KS + kStrip - 1 + 3) / 4) * 4;     // window columns written
    static constexpr int HH = kBR + KS - 1;
    // written columns, then one float4 column of lane-private slots; an odd
    // number of float4s per row puts 16 consecutive rows in distinct banks
    static constexpr int HW0 = kBW - kStrip + WP + 4;
    static constexpr int HW = (HW0 / 4) % 2 ? HW0 : HW0 + 4;
    static constexpr int SLOT = HW - 4;                            // private slot column
    static constexpr int PADL = 16 * NB - KS;                      // staged row: zero margin
    static constexpr int ROW = ((16 * NB + kStrip - 1 + 3) / 4) * 4;
    static_assert(HW % 4 == 0, "float4 rows");
    static_assert(SLOT >= kBW + KS - 1, "private slots lie outside the folded halo");
};

// All kernel rows of one pass: NG groups of 16 strips of one entry (each
// group from a single strip column).  gb: the lane's B operands (output
// gradients of (side, q) for the four k-steps), hofs: the lane's halo offset
// at i = 0, act: the lane holds a strip.  Lanes with nothing to add at a
// block (no strip, or window columns past the last tap) direct that block's
// read-modify-write to a private float4 in the halo's last column, which is
// never folded, so every read-modify-write runs on all lanes.  Row i's
// products are added in during row i + 1, group by group: a group's reads,
// its products of the next row (covering the read latency), then its sums.
// Groups of different columns may overlap, so each group's writes precede
// the next group's reads.
template <int KS, int NG>
__device__ inline void band_mfma_pass(const float* __restrict__ kl, int rstep, bool fx, bool fy,
                                      float* hgrad, float* arow, int lane,
                                      const float (&gb)[4][4], const int (&hofs)[4],
                                      const bool (&act)[4]) {
    using G = BandGeom<KS>;
    const int prow = lane & 15, g = lane >> 4;
    // A operand of block b, k-step k: tap q + KS - 1 - p of side k >> 1,
    // q = 4 (k & 1) + g, p = 16 b + prow
    const int aofs = G::PADL + g + KS - 1 - prow;
    int taddr[NG][G::NB], tstep[NG][G::NB];
#pragma unroll
    for (int u = 0; u < NG; ++u)
#pragma unroll
        for (int b = 0; b < G::NB; ++b) {
            const bool ok = act[u] && 16 * b + 4 * g < G::WP;
            taddr[u][b] = ok ? hofs[u] + 16 * b : (lane % G::HH) * G::HW + G::SLOT;
            tstep[u][b] = ok ? G::HW : 0;
        }
    RowStager<KS, G::ROW, G::PADL> sg;
    sg.init(lane, fx);
    int row_ofs = (fy ? KS - 1 : 0) * KS;
    sg.load(kl, row_ofs);
    sg.store(arow);
    row_ofs += rstep;
    sg.load(kl, row_ofs);
    sg.store(arow + 2 * G::ROW);
    float a[G::NB][4];
#pragma unroll
    for (int b = 0; b < G::NB; ++b)
#pragma unroll
        for (int k = 0; k < 4; ++k) a[b][k] = arow[(k >> 1) * G::ROW + aofs + 4 * (k & 1) - 16 * b];
    floatx4_t dprev[NG][G::NB];
    for (int i = 0; i <= KS; ++i) {
        const bool prev = i > 0, cur_row = i < KS;
        if (i + 2 < KS) {
            row_ofs += rstep;
            sg.load(kl, row_ofs);                       // row i + 2 in flight
        }
        floatx4_t d[NG][G::NB];
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            float4 cur[G::NB];
            if (prev) {
#pragma unroll
                for (int b = 0; b < G::NB; ++b)
                    cur[b] = *reinterpret_cast<const float4*>(hgrad + taddr[u][b]);
            }
            if (cur_row) {
#pragma unroll
                for (int b = 0; b < G::NB; ++b)
                    d[u][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b][0], gb[u][0],
                                                                   floatx4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
                for (int k = 1; k < 4; ++k)
#pragma unroll
                    for (int b = 0; b < G::NB; ++b)
                        d[u][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[b][k], gb[u][k], d[u][b], 0, 0, 0);
            }
            if (prev) {
#pragma unroll
                for (int b = 0; b < G::NB; ++b) {
                    float4 v = cur[b];
                    v.x += dprev[u][b][0]; v.y += dprev[u][b][1];
                    v.z += dprev[u][b][2]; v.w += dprev[u][b][3];
                    *reinterpret_cast<float4*>(hgrad + taddr[u][b]) = v;
                    taddr[u][b] -= tstep[u][b];
                }
            }
        }
        if (i + 1 < KS) {
            const float* ar = arow + ((i + 1) & 1) * 2 * G::ROW + aofs;
#pragma unroll
            for (int b = 0; b < G::NB; ++b)
#pragma unroll
                for (int k = 0; k < 4; ++k) a[b][k] = ar[(k >> 1) * G::ROW + 4 * (k & 1) - 16 * b];
        }
        // row i's buffer was read one row ago
        if (i + 2 < KS) sg.store(arow + (i & 1) * 2 * G::ROW);
        if (cur_row) {
#pragma unroll
            for (int u = 0; u < NG; ++u)
#pragma unroll
                for (int b = 0; b < G::NB; ++b) dprev[u][b] = d[u][b];
        }
    }
}

// Group j of an entry's strips in a band: groups of 16 taken column by
// column (nc: strips per column).
__device__ inline void band_group(int j, const int (&nc)[kBS], int& col, int& s0, int& cnt) {
    col = -1; s0 = 0; cnt = 0;
#pragma unroll
    for (int c = 0; c < kBS; ++c) {
        const int gc = (nc[c] + 15) >> 4;
        if (col < 0 && j < gc) { col = c; s0 = 16 * j; cnt = min(16, nc[c] - s0); }
        if (col < 0) j -= gc;
    }
}

template <int KS>
__global__ __launch_bounds__(64) void render_bank_bwd_kernel(const RenderArgs A,
                                                           const float* __restrict__ bank) {
    using G = BandGeom<KS>;
    extern __shared__ __align__(16) float hgrad[];       // [HH][HW]
    __shared__ int items[kBS * kBR];                     // per strip column: strip | mask << 9
    __shared__ __align__(16) float arow[4 * G::ROW];     // 2 buffers x 2 sides
    const int pad = (KS - 1) / 2;
    const int kk = KS * KS;
    const int bandsx = (A.W + kBW - 1) / kBW, bandsy = (A.H + kBR - 1) / kBR;
    const int nb = A.N * bandsx * bandsy;
    const int c = blockIdx.x / nb;                       // channel slowest: one wavelength's entries at a time
    const int band = blockIdx.x - c * nb;
    const int n = band / (bandsx * bandsy);
    const int rem = band - n * bandsx * bandsy;
    const int y0 = (rem / bandsx) * kBR, x0 = (rem % bandsx) * kBW;
    const int lane = threadIdx.x;
    // strip lane + 64 h: row (lane + 64 h) / 4, column lane % 4
    int key[2][kStrip];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int sid = lane + 64 * h;
        const int y = y0 + sid / kBS, xs = x0 + (sid % kBS) * kStrip;
#pragma unroll
        for (int q = 0; q < kStrip; ++q)
            key[h][q] = (y < A.H && xs + q < A.W) ? bank_key(A, n, y, xs + q) : 0x7fffffff;
    }
    for (int e = lane; e < G::HH * G::HW; e += 64) hgrad[e] = 0.f;
    for (int e = lane; e < 4 * G::ROW; e += 64) arow[e] = 0.f;   // margins stay zero
    const unsigned long long colmask = 0x1111111111111111ull << (lane & 3);
    const size_t plane = (size_t)A.C * A.H * A.W;
    {
        const int lam = A.lam_of_c[c];
        unsigned done = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < kStrip; ++q)
                if (key[h][q] == 0x7fffffff) done |= 1u << (8 * h + q);
        while (true) {
            int mine = 0x7fffffff;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < kStrip; ++q)
                    if (!(done & (1u << (8 * h + q)))) mine = min(mine, key[h][q]);
            const int k = __builtin_amdgcn_readfirstlane(wave_min_int(mine));
            if (k == 0x7fffffff) break;
            // list the entry's strips per column (at most 32 each)
            int ccount = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                unsigned m = 0;
#pragma unroll
                for (int q = 0; q < kStrip; ++q)
                    if (key[h][q] == k) m |= 1u << q;
                const unsigned long long bal = __ballot(m != 0) & colmask;
                const int pre = __popcll(bal & ((1ull << lane) - 1ull));
                if (m) {
                    items[(lane & 3) * kBR + ccount + pre] = (lane + 64 * h) | (int)(m << 9);
                    done |= m << (8 * h);
                }
                ccount += __popcll(bal);
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            const int fyb = k & 1, fxb = (k >> 1) & 1, fd = k >> 2;
            const float* kl = bank + ((size_t)fd * A.L + lam) * 2 * kk + (fxb ? kk : 0);
            const int rstep = fyb ? -KS : KS;
            const int g = lane >> 4;
            int nc[kBS], ngt = 0;
#pragma unroll
            for (int col = 0; col < kBS; ++col) {
                nc[col] = __builtin_amdgcn_readlane(ccount, col);
                ngt += (nc[col] + 15) >> 4;
            }
            // passes of up to four groups share the staged kernel rows
            for (int p0 = 0; p0 < ngt; p0 += 4) {
                const int np = min(4, ngt - p0);
                float gb[4][4];
                int hofs[4];
                bool act[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int col, s0, cnt;
                    band_group(min(p0 + u, ngt - 1), nc, col, s0, cnt);
                    act[u] = u < np && (lane & 15) < cnt;
                    const int it = items[col * kBR + s0 + min(lane & 15, cnt - 1)];
                    const int sid = it & 127;
                    const unsigned msk = act[u] ? (unsigned)it >> 9 : 0u;
                    const int tr = sid / kBS, tc = sid % kBS;
                    hofs[u] = (tr + KS - 1) * G::HW + tc * kStrip + 4 * g;
                    const int y = min(y0 + tr, A.H - 1);
                    const size_t orow = (((size_t)n * 2 * A.C + c) * A.H + y) * A.W;
#pragma unroll
                    for (int kq = 0; kq < 4; ++kq) {
                        const int q = 4 * (kq & 1) + g;
                        const int xq = min(x0 + tc * kStrip + q, A.W - 1);
                        const size_t o = orow + xq + (kq >> 1) * plane;
                        const float v = A.gout[o];                   // in bounds even if masked
                        const float wt = A.bank2d ? pass_weight(A, n, y, xq) : 1.f;
                        gb[u][kq] = (msk >> q) & 1u ? v * wt : 0.f;
                    }
                }
                switch (np) {
                    case 1: band_mfma_pass<KS, 1>(kl, rstep, fxb, fyb, hgrad, arow, lane, gb, hofs, act); break;
                    case 2: band_mfma_pass<KS, 2>(kl, rstep, fxb, fyb, hgrad, arow, lane, gb, hofs, act); break;
                    case 3: band_mfma_pass<KS, 3>(kl, rstep, fxb, fyb, hgrad, arow, lane, gb, hofs, act); break;
                    default: band_mfma_pass<KS, 4>(kl, rstep, fxb, fyb, hgrad, arow, lane, gb, hofs, act); break;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        // fold the band's halo gradient (clamped)
        __syncthreads();
        float* gi = A.gimg + ((size_t)n * A.C + c) * A.H * A.W;
        for (int e = lane; e < G::HH * G::HW; e += 64) {
            const int R = e / G::HW, Cc = e - R * G::HW;
            const float v = hgrad[e];
            if (v == 0.f || Cc >= kBW + KS - 1) continue;
            const int yy = min(max(y0 - pad + R, 0), A.H - 1);
            const int xx = min(max(x0 - pad + Cc, 0), A.W - 1);
            atomicAdd(&gi[(size_t)yy * A.W + xx], v);
        }
    }
}

// ---- split-bf16 image adjoint ----------------------------------------------
//
// The bank adjoint scatters each output's gradient through its own entry's
// kernel.  A workgroup owns a 64 x 64 pixel tile and an LDS float32 copy of
// its halo gradient; entries are taken in batches, and for an entry the unit
// of work is a segment of 16 consecutive strip rows of one strip column
// (strips or pixels outside the entry carry zero gradient).  For kernel row
// i, strip n of a segment adds D_i[n][p] = sum over (side, q) of
// g[n][(side, q)] * K_side[i][KS - 1 - p + q] at halo row (strip row n +
// KS - 1 - i), column 8 (strip column) + p, for the window columns p < P =
// 16 NB: per block of 16 columns, two v_mfma_f32_16x16x32_bf16 on one tap
// fragment (each tap's hi and lo parts side by side along K): g_hi, repeated
// against both parts, gives g_hi (K_hi + K_lo), and g_lo with zeros against
// the lo parts g_lo K_hi.  The halo row of (n, i) is fixed
// along n - i, so the gradient operand's rows are rotated by one strip per
// kernel row (DPP row_ror): row m holds strip (m + i) mod 16, and
// accumulator row m keeps adding into one halo row until its strip index
// wraps.  The row it finished continues, in the segment below, in that
// segment's accumulator row m (which starts strip 0 at that kernel row), so
// a run of vertically adjacent segments hands each finished row down the
// run, and only the lowest segment adds its finished row (16 lanes of one
// register) into the LDS halo with ds_add_f32; the rows above move down one
// segment and the top one restarts from zero.  All products go through one
// instruction type (an MFMA reading another type's result as its
// accumulator has returned stale rows).  Taps are staged per kernel row in
// natural order between zero margins, one dword per tap (hi | lo << 16), so
// a lane reads its four taps as four whole dwords.  Finally the halo is
// added onto the clamped image pixels with global atomics.
constexpr int kSBSlots = 8;                       // entries per batch
constexpr int kSBGroups = 4;                      // segments per run (a tile column)
constexpr int kSBChunks = kSBSlots * 16;          // runs per batch (<= 2 per column)

template <int KS>
struct SplitBwdGeom {
    static constexpr int NB = (KS + kStrip - 1 + 15) / 16;      // 16-column blocks of the window
    static constexpr int P = 16 * NB;
    static constexpr int PW = KS + kStrip - 1;                   // window columns with taps
    static constexpr int MARG = ((P - KS + 1) / 2) * 2;          // zero margin before the taps
    static constexpr int RW = ((MARG + KS + 9 + 7) / 8) * 8;     // staged row (taps)
    static constexpr int SCRATCH = 2 * RW;                       // dwords per wave (two sides)
    static constexpr int NTAP = 2 * KS;                          // taps of one kernel row
    static constexpr int HH = kGT + KS - 1;
    static constexpr int HWG = kGT + KS;                         // halo-gradient row stride (odd)
    static constexpr int NGMAX = 4;                              // segments per run
    static_assert(MARG >= P - KS && RW >= MARG + KS + 9, "lane reads stay inside the staged row");
    static_assert(kGT - kStrip + PW <= HWG - 1, "window columns inside the halo row");
};

// One lane's share of staging one kernel row (both sides, natural tap order
// v, mirrors applied): element e = lane + 64 k of [2 sides][KS].
template <int KS>
struct SplitRowTaps {
    using S = SplitBwdGeom<KS>;
    static constexpr int NL = (S::NTAP + 63) / 64;
    int src[NL], dst[NL];
    float v[NL];
    __device__ void init(int lane, bool fx, bool fy) {
        const int ri = fy ? KS - 1 : 0;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int e = min(lane + 64 * k, S::NTAP - 1);
            const int side = e >= KS, u = e - side * KS;
            // effective kernel K'_s[i][u]: the stored side s, or side 1 - s
            // mirrored in x
            src[k] = fx ? (1 - side) * KS * KS + ri * KS + KS - 1 - u : side * KS * KS + ri * KS + u;
            dst[k] = side * S::RW + S::MARG + u;
        }
    }
    __device__ void load(const float* __restrict__ entry, int ofs) {
#pragma unroll
        for (int k = 0; k < NL; ++k) v[k] = entry[src[k] + ofs];
    }
    // one dword per tap: its bf16 high part, then its low part
    __device__ void store(u32_alias* st, int lane) const {
#pragma unroll
        for (int k = 0; k < NL; ++k)
            if (64 * k + 64 <= S::NTAP || lane + 64 * k < S::NTAP) st[dst[k]] = split_bf16_bits(v[k]);
    }
};

__device__ inline uint32_t rot_row_left(uint32_t x) {
    // lane l of each row of 16 takes lane (l + 1) mod 16 (DPP row_ror:15)
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x12f, 0xf, 0xf, false);
}

// All kernel rows for a run of NG vertically adjacent segments of one entry
// (segment u at strip rows 16 (rs0 + u) ..).  ga / gl: the lane's x32
// gradient fragments of strip m = lane % 16 of each segment at i = 0 (g_hi
// twice; g_lo then zeros); hrow: the halo row of strip 0 of the top segment
// at i = 0 (16 rs0 + KS - 1); hcol: the lane's halo column at block 0
// (8 strip column + lane % 16).
template <int KS, int NG>
__device__ inline void bank_split_bwd_rows(const float* __restrict__ entry, bool fx, bool fy,
                                           float* hg, float* scratch, int lane,
                                           u32x4_t (&ga)[kSBGroups], u32x4_t (&gl)[kSBGroups],
                                           int hrow, int hcol) {
    using S = SplitBwdGeom<KS>;
    u32_alias* sw = reinterpret_cast<u32_alias*>(scratch);
    const int pl = lane & 15, kg = lane >> 4;
    const int side = kg >> 1, q0 = 4 * (kg & 1);
    // the lane's four taps of block b: dwords ad0 - 16 b .. + 3
    const int ad0 = side * S::RW + S::MARG + KS - 1 - pl + q0;
    // acc: the running halo rows, one 16 x 16 block per segment and window
    // block (row m of segment u: strip (m + i) mod 16's halo row)
    floatx4_t acc[NG][S::NB];
#pragma unroll
    for (int u = 0; u < NG; ++u)
#pragma unroll
        for (int b = 0; b < S::NB; ++b) acc[u][b] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    const int rstep = fy ? -KS : KS;
    SplitRowTaps<KS> taps;
    taps.init(lane, fx, fy);
    taps.load(entry, 0);
    for (int i = 0; i < KS; ++i) {
        __asm__ volatile("" ::: "memory");
        taps.store(sw, lane);
        __asm__ volatile("" ::: "memory");
        if (i + 1 < KS) taps.load(entry, (i + 1) * rstep);
        if (i > 0) {
            // accumulator row m* = (16 - i) mod 16 of every segment finished
            // a halo row (strip 15 at row i - 1), which the same row of the
            // segment below continues: the lowest adds its row into the halo,
            // the others move down one segment, the top one starts from zero
            const int ms = (16 - (i & 15)) & 15;
            const bool mine = kg == (ms >> 2);
            const int rb = (hrow + 16 * (NG - 1) + 16 - i) * S::HWG + hcol;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                if ((ms & 3) != jj) continue;
#pragma unroll
                for (int b = 0; b < S::NB; ++b) {
                    if (mine && 16 * b + pl < S::PW) atomicAdd(&hg[rb + 16 * b], acc[NG - 1][b][jj]);
#pragma unroll
                    for (int u = NG - 1; u > 0; --u) acc[u][b][jj] = mine ? acc[u - 1][b][jj] : acc[u][b][jj];
                    acc[0][b][jj] = mine ? 0.f : acc[0][b][jj];
                }
            }
            // gradient rows move up by one strip
#pragma unroll
            for (int u = 0; u < NG; ++u) {
#pragma unroll
                for (int w = 0; w < 4; ++w) ga[u][w] = rot_row_left(ga[u][w]);
                gl[u][0] = rot_row_left(gl[u][0]);
                gl[u][1] = rot_row_left(gl[u][1]);
            }
        }
#pragma unroll
        for (int b = 0; b < S::NB; ++b) {
            u32x4_t tw;
#pragma unroll
            for (int j = 0; j < 4; ++j) tw[j] = sw[ad0 - 16 * b + j];
            const bf16x8_t t32 = __builtin_bit_cast(bf16x8_t, tw);
#pragma unroll
            for (int u = 0; u < NG; ++u) {
                // g_lo kept as two packed dwords; spread to one per tap here
                const u32x4_t glw = u32x4_t{gl[u][0] & 0xffffu, gl[u][0] >> 16, gl[u][1] & 0xffffu,
                                            gl[u][1] >> 16};
                acc[u][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, ga[u]), t32,
                                                                    acc[u][b], 0, 0, 0);
                acc[u][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, glw), t32,
                                                                    acc[u][b], 0, 0, 0);
            }
        }
    }
    // every accumulator row holds (part of) one halo row: strip
    // n = (m + KS - 1) mod 16 of its segment at the last kernel row, halo row
    // 16 (rs0 + u) + n
#pragma unroll
    for (int u = 0; u < NG; ++u)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int nn = (4 * kg + jj + KS - 1) & 15;
            const int rb = (hrow - (KS - 1) + 16 * u + nn) * S::HWG + hcol;
#pragma unroll
            for (int b = 0; b < S::NB; ++b)
                if (16 * b + pl < S::PW) atomicAdd(&hg[rb + 16 * b], acc[u][b][jj]);
        }
}

template <int KS>
__global__ __launch_bounds__(kRBlock, 2) void render_bank_split_bwd_kernel(const RenderArgs A,
                                                                         const float* __restrict__ bank) {
    using S = SplitBwdGeom<KS>;
    extern __shared__ __align__(16) float hgrad[];                 // [HH][HWG]
    __shared__ uint8_t pm[kSBSlots][kGStrips];                     // pixel masks per batch entry
    __shared__ unsigned segm[kSBSlots];                            // segments holding the entry
    __shared__ int slot_key[kSBSlots];
    __shared__ int chunk_tab[kSBChunks];                           // slot | col << 4 | row << 7 | len << 9
    __shared__ int red[kRBlock / 64];
    __shared__ int n_chunks, next_chunk;
    __shared__ __align__(16) float wscr[kRBlock / 64][S::SCRATCH];
    const int kk = KS * KS;
    const int pad = (KS - 1) / 2;
    const int tilesx = (A.W + kGT - 1) / kGT, tilesy = (A.H + kGT - 1) / kGT;
    const int nt = A.N * tilesx * tilesy;
    const int c = blockIdx.x / nt;                                 // channel slowest
    const int tile = blockIdx.x - c * nt;
    const int n = tile / (tilesx * tilesy);
    const int rem = tile - n * tilesx * tilesy;
    const int y0 = (rem / tilesx) * kGT, x0 = (rem % tilesx) * kGT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float* scr = wscr[wave];
    for (int e = lane; e < S::SCRATCH; e += 64) scr[e] = 0.f;    // margins stay zero
    for (int e = tid; e < S::HH * S::HWG; e += kRBlock) hgrad[e] = 0.f;
    int key[2][kStrip];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int sid = tid + h * kRBlock;
        const int y = y0 + (sid >> 3), xs = x0 + (sid & 7) * kStrip;
#pragma unroll
        for (int q = 0; q < kStrip; ++q)
            key[h][q] = (y < A.H && xs + q < A.W) ? bank_key(A, n, y, xs + q) : 0x7fffffff;
    }
    unsigned done = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < kStrip; ++q)
            if (key[h][q] == 0x7fffffff) done |= 1u << (8 * h + q);
    const int lam = A.lam_of_c[c];
    const size_t plane = (size_t)A.C * A.H * A.W;
    bool more = true;
    while (more) {
        // ---- list a batch of up to kSBSlots entries: pixel masks per strip
        // and the 16-row segments that hold each entry
        if (tid < kSBSlots) segm[tid] = 0u;
        int ns = 0;
        while (ns < kSBSlots) {
            int mine = 0x7fffffff;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < kStrip; ++q)
                    if (!(done & (1u << (8 * h + q)))) mine = min(mine, key[h][q]);
            const int wm = wave_min_int(mine);
            if (lane == 0) red[wave] = wm;
            __syncthreads();
            int k = red[0];
#pragma unroll
            for (int w = 1; w < kRBlock / 64; ++w) k = min(k, red[w]);
            __syncthreads();
            if (k == 0x7fffffff) { more = false; break; }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int sid = tid + h * kRBlock;
                unsigned m = 0;
#pragma unroll
                for (int q = 0; q < kStrip; ++q)
                    if (key[h][q] == k) m |= 1u << q;
                pm[ns][sid] = (uint8_t)m;
                if (m) {
                    atomicOr(&segm[ns], 1u << ((sid & 7) + 8 * (sid >> 7)));
                    done |= m << (8 * h);
                }
            }
            if (tid == 0) slot_key[ns] = k;
            ++ns;
        }
        __syncthreads();
        if (tid == 0) {
            int nc = 0;
            // runs of vertically adjacent segments, column by column
            for (int s2 = 0; s2 < ns; ++s2) {
                const unsigned bits = segm[s2];
                for (int sc = 0; sc < kStrip; ++sc) {
                    int rs = 0;
                    while (rs < 4) {
                        if (!((bits >> (8 * rs + sc)) & 1u)) { ++rs; continue; }
                        int len = 1;
                        while (rs + len < 4 && len < S::NGMAX && ((bits >> (8 * (rs + len) + sc)) & 1u)) ++len;
                        chunk_tab[nc++] = s2 | (sc << 4) | (rs << 7) | (len << 9);
                        rs += len;
                    }
                }
            }
            n_chunks = nc;
            next_chunk = 0;
        }
        __syncthreads();
        const int nch = n_chunks;
        while (true) {
            int j = 0;
            if (lane == 0) j = atomicAdd(&next_chunk, 1);
            j = __builtin_amdgcn_readfirstlane(j);
            if (j >= nch) break;
            const int ct = __builtin_amdgcn_readfirstlane(chunk_tab[j]);
            const int sl = ct & 15, sc = (ct >> 4) & 7, rs0 = (ct >> 7) & 3, cnt = ct >> 9;
            const int k = __builtin_amdgcn_readfirstlane(slot_key[sl]);
            const int fyb = k & 1, fxb = (k >> 1) & 1, fd = k >> 2;
            const float* entry = bank + ((size_t)fd * A.L + lam) * 2 * kk;
            const int pl = lane & 15, kg = lane >> 4;
            const int side = kg >> 1, q0 = 4 * (kg & 1);
            u32x4_t ga[kSBGroups], gl[kSBGroups];
#pragma unroll
            for (int u = 0; u < kSBGroups; ++u) {
                const int tr = 16 * min(rs0 + u, 3) + pl;              // tile strip row of row m = pl
                const unsigned pmk = u < cnt ? pm[sl][tr * 8 + sc] : 0u;
                const int y = min(y0 + tr, A.H - 1);
                const size_t orow = (((size_t)n * 2 * A.C + c) * A.H + y) * A.W + side * plane;
                uint32_t hb[4], lb[4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int q = q0 + jj;
                    const int xq = min(x0 + sc * kStrip + q, A.W - 1);
                    float g = 0.f;
                    if ((pmk >> q) & 1u) {
                        g = A.gout[orow + xq];
                        if (A.bank2d) g *= pass_weight(A, n, y, xq);
                    }
                    const uint32_t bb = split_bf16_bits(g);
                    hb[jj] = bb & 0xffffu;
                    lb[jj] = bb >> 16;
                }
                // k pairs (tap j high, tap j low): g_hi against both, g_lo
                // against the high part only
                ga[u] = u32x4_t{hb[0] * 0x10001u, hb[1] * 0x10001u, hb[2] * 0x10001u, hb[3] * 0x10001u};
                gl[u] = u32x4_t{lb[0] | (lb[1] << 16), lb[2] | (lb[3] << 16), 0u, 0u};
            }
            const int hrow = 16 * rs0 + KS - 1, hcol = sc * kStrip + pl;
            if (cnt == 1) {
                bank_split_bwd_rows<KS, 1>(entry, fxb, fyb, hgrad, scr, lane, ga, gl, hrow, hcol);
            } else if (cnt == 2 || S::NGMAX == 2) {
                bank_split_bwd_rows<KS, 2>(entry, fxb, fyb, hgrad, scr, lane, ga, gl, hrow, hcol);
            } else if constexpr (S::NGMAX == 4) {
                if (cnt == 3) bank_split_bwd_rows<KS, 3>(entry, fxb, fyb, hgrad, scr, lane, ga, gl, hrow, hcol);
                else bank_split_bwd_rows<KS, 4>(entry, fxb, fyb, hgrad, scr, lane, ga, gl, hrow, hcol);
            }
        }
        __syncthreads();
    }
    // fold the tile's halo gradient onto the clamped image pixels
    float* gi = A.gimg + ((size_t)n * A.C + c) * A.H * A.W;
    for (int e = tid; e < S::HH * S::HWG; e += kRBlock) {
        const int R = e / S::HWG, Cc = e - R * S::HWG;
        const float v = hgrad[e];
        if (v == 0.f || Cc >= kGT + KS - 1) continue;
        const int yy = min(max(y0 - pad + R, 0), A.H - 1);
        const int xx = min(max(x0 - pad + Cc, 0), A.W - 1);
        atomicAdd(&gi[(size_t)yy * A.W + xx], v);
    }
}

template <int KS, bool BWD>
static bool launch_bank_fast(const RenderArgs& A, hipStream_t st) {
    if (BWD && A.split) {
        using S = SplitBwdGeom<KS>;
        const size_t shm = (size_t)S::HH * S::HWG * sizeof(float);
        const int tilesx = (A.W + kGT - 1) / kGT, tilesy = (A.H + kGT - 1) / kGT;
        const dim3 grid((unsigned)((long long)A.C * A.N * tilesx * tilesy));
        if (shm > 65536) (void)hipFuncSetAttribute((const void*)render_bank_split_bwd_kernel<KS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        hipLaunchKernelGGL(render_bank_split_bwd_kernel<KS>, grid, dim3(kRBlock), shm, st, A,
                           reinterpret_cast<const float*>(A.psf));
    } else if (BWD) {
        const size_t shm = (size_t)BandGeom<KS>::HH * BandGeom<KS>::HW * sizeof(float);
        const int bandsx = (A.W + kBW - 1) / kBW, bandsy = (A.H + kBR - 1) / kBR;
        const dim3 grid((unsigned)((long long)A.C * A.N * bandsx * bandsy));
        if (shm > 65536) (void)hipFuncSetAttribute((const void*)render_bank_bwd_kernel<KS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        hipLaunchKernelGGL(render_bank_bwd_kernel<KS>, grid, dim3(64), shm, st, A,
                           reinterpret_cast<const float*>(A.psf));
    } else if (A.split) {
        using S = SplitGeom<KS>;
        const size_t shm = (size_t)2 * S::HH * S::HWB * sizeof(uint16_t);
        const int tilesx = (A.W + kGT - 1) / kGT, tilesy = (A.H + kGT - 1) / kGT;
        const dim3 grid((unsigned)((long long)A.C * A.N * tilesx * tilesy));
        if (shm > 65536) (void)hipFuncSetAttribute((const void*)render_bank_split_kernel<KS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        hipLaunchKernelGGL(render_bank_split_kernel<KS>, grid, dim3(kRBlock), shm, st, A,
                           reinterpret_cast<const float*>(A.psf));
    } else {
        using G = GroupGeom<KS>;
        const size_t shm = (size_t)G::HH * G::HW * sizeof(float);
        const int tilesx = (A.W + kGT - 1) / kGT, tilesy = (A.H + kGT - 1) / kGT;
        const dim3 grid((unsigned)((long long)A.C * A.N * tilesx * tilesy));
        if (shm > 65536) (void)hipFuncSetAttribute((const void*)render_bank_fast_kernel<KS, kBankFwd>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        hipLaunchKernelGGL((render_bank_fast_kernel<KS, kBankFwd>), grid, dim3(kRBlock), shm, st, A,
                           reinterpret_cast<const float*>(A.psf), (float*)nullptr);
    }
    return true;
}

template <int KS>
static void launch_bank_kgrad(const RenderArgs& A, float* grad, hipStream_t st) {
    using G = GroupGeom<KS>;
    const size_t shm = (size_t)G::HH * G::HW * sizeof(float);
    const int tilesx = (A.W + kGT - 1) / kGT, tilesy = (A.H + kGT - 1) / kGT;
    const dim3 grid((unsigned)((long long)A.C * A.N * tilesx * tilesy));
    if (shm > 65536) (void)hipFuncSetAttribute((const void*)render_bank_fast_kernel<KS, kBankKGrad>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL((render_bank_fast_kernel<KS, kBankKGrad>), grid, dim3(kRBlock), shm, st, A,
                       (const float*)nullptr, grad);
}

static bool bank_kgrad_pass(const RenderArgs& A, float* grad, hipStream_t st) {
    switch (A.ks) {
        case 21: launch_bank_kgrad<21>(A, grad, st); return true;
        case 31: launch_bank_kgrad<31>(A, grad, st); return true;
        case 33: launch_bank_kgrad<33>(A, grad, st); return true;
        case 41: launch_bank_kgrad<41>(A, grad, st); return true;
        case 63: launch_bank_kgrad<63>(A, grad, st); return true;
        case 65: launch_bank_kgrad<65>(A, grad, st); return true;
        default: return false;
    }
}

template <bool BWD>
static bool try_bank_fast_pass(const RenderArgs& A, hipStream_t st) {
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

// The 2-D bank renders its depth blend in two passes over entry-grouped
// pixels: plane d0 weighted 1 - w (writing the output), then plane d0 + 1
// weighted w (adding to it); the adjoint's passes both add into the image
// gradient.
template <bool BWD>
static bool try_bank_fast(const RenderArgs& A, hipStream_t st) {
    if (A.source != SDIRT_SRC_BANK && A.source != SDIRT_SRC_BANK2D) return false;
    const long long cells = A.bank2d ? (long long)A.F * A.Fy : A.F;
    if (cells * A.D * 4 >= 0x7fffffffLL) return false;
    if (!A.bank2d) return try_bank_fast_pass<BWD>(A, st);
    RenderArgs B = A;
    B.pass = 0;
    if (!try_bank_fast_pass<BWD>(B, st)) return false;
    B.pass = 1;
    return try_bank_fast_pass<BWD>(B, st);
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
    } else if (d->source == SDIRT_SRC_BANK || d->source == SDIRT_SRC_BANK2D) {
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
        if (d->source == SDIRT_SRC_BANK2D) {
            // first-quadrant grid: nearest |2x - W + 1| (exact integer, half
            // pixels) against floor(2 * midpoint / pitch), likewise in y;
            // inverse depths as float32, strictly increasing
            A->bank2d = 1;
            A->Fy = d->bank_fields_y;
            if (A->Fy < 1 || !d->field_y) return SDIRT_EINVAL;
            if (A->Fy > SDIRT_MAX_BANK_F) return SDIRT_EUNSUPPORTED;
            if (!(d->field_radii[0] >= 0)) return SDIRT_EINVAL;
            for (int k = 0; k < A->Fy; ++k) {
                if (!std::isfinite(d->field_y[k]) || !(d->field_y[k] >= 0)) return SDIRT_EINVAL;
                if (k && !(d->field_y[k] > d->field_y[k - 1])) return SDIRT_EINVAL;
            }
            for (int k = 0; k + 1 < A->F; ++k)
                A->t_r[k] = (long long)std::floor((d->field_radii[k] + d->field_radii[k + 1]) / d->pitch);
            for (int k = 0; k + 1 < A->Fy; ++k)
                A->t_y[k] = (long long)std::floor((d->field_y[k] + d->field_y[k + 1]) / d->pitch);
            for (int k = 0; k < A->D; ++k) {
                A->ivk[k] = (float)d->inv_depths[k];
                if (k && !(A->ivk[k] > A->ivk[k - 1])) return SDIRT_EINVAL;
            }
        } else {
            // nearest field radius: R2 (exact integer, half-pixel units)
            // against floor((2 * midpoint / pitch)^2)
            for (int k = 0; k + 1 < A->F; ++k) {
                const double mid = 0.5 * (d->field_radii[k] + d->field_radii[k + 1]);
                const double t = std::floor((2.0 * mid / d->pitch) * (2.0 * mid / d->pitch));
                A->t_r[k] = t < 0 ? -1 : (long long)t;
            }
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
        if (d->bank_math != SDIRT_BANK_FP32 && d->bank_math != SDIRT_BANK_SPLIT_BF16)
            return SDIRT_EINVAL;
        A->split = d->bank_math == SDIRT_BANK_SPLIT_BF16;
    } else {
        return SDIRT_EINVAL;
    }
    A->use_fast = 1;
    A->tiles_x = (d->W + kTW - 1) / kTW;
    A->tiles_y = (d->H + kTH - 1) / kTH;
    // the dense kernels launch up to one workgroup per row of every 8 x 8 tile
    if ((long long)d->N * A->tiles_x * A->tiles_y * kTH > 0xffffffffLL) return SDIRT_EUNSUPPORTED;
    return SDIRT_OK;
}

template <int NC, bool BWD, int MODE, bool BF16>
static void launch_render3(const RenderArgs& A, hipStream_t st) {
    const long long tiles = (long long)A.N * A.tiles_x * A.tiles_y;
    if (BWD) {
        hipLaunchKernelGGL((render_bwd_kernel<NC, MODE, BF16>), dim3((unsigned)tiles), dim3(kRBlock), 0, st, A);
    } else {
        constexpr int kFwdRows = fwd_rows<MODE, BF16>();
        const int hh = kFwdRows + A.ks - 1, hw = kTW + A.ks - 1;
        const size_t shm = (size_t)NC * hh * hw * sizeof(float);
        if (shm > 65536) (void)hipFuncSetAttribute((const void*)render_fwd_kernel<NC, MODE, BF16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        hipLaunchKernelGGL((render_fwd_kernel<NC, MODE, BF16>), dim3((unsigned)(tiles * (kTH / kFwdRows))),
                           dim3(kRBlock), shm, st, A);
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
    if (A.bank2d) return SDIRT_EUNSUPPORTED;           // grouped kernels only
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
    if (A.source != SDIRT_SRC_DENSE && !depth) return SDIRT_EINVAL;
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
    if (A.source != SDIRT_SRC_DENSE && !depth) return SDIRT_EINVAL;
    A.psf = psf; A.depth = depth; A.gout = gout; A.gimg = gimg;
    if ((rc = launch_fill_zero(gimg, (size_t)A.N * A.C * A.H * A.W * sizeof(float), stream)))
        return rc;
    return dispatch_render<true>(A, stream);
}

template <int NC>
static void launch_psf_grad(const RenderArgs& A, void* grad, hipStream_t st) {
#define SDIRT_PSFG(SH, BF)                                                                   \
    do {                                                                                     \
        const int hh = grad_rows<SH>() + A.ks - 1, hw = kTW + A.ks - 1;                      \
        const size_t shm = (size_t)NC * hh * hw * sizeof(float);                            \
        const dim3 grid((unsigned)((long long)A.N * A.tiles_x * A.tiles_y * (kTH / grad_rows<SH>()))); \
        auto k = render_psf_grad_kernel<NC, SH, BF>;                                         \
        if (shm > 65536) (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm); \
        hipLaunchKernelGGL(k, grid, dim3(kRBlock), shm, st, A, grad);                        \
    } while (0)
    if (A.Cp == 1 && A.bf16) SDIRT_PSFG(true, true);
    else if (A.Cp == 1) SDIRT_PSFG(true, false);
    else if (A.bf16) SDIRT_PSFG(false, true);
    else SDIRT_PSFG(false, false);
#undef SDIRT_PSFG
}

int render_psf_backward_impl(const sdirt_render_desc* desc, const float* img, const float* depth,
                             const float* gout, void* grad_psf, hipStream_t stream) {
    RenderArgs A;
    int rc = pack_render(desc, &A);
    if (rc) return rc;
    if (!img || !gout || !grad_psf) return SDIRT_EINVAL;
    if (A.source != SDIRT_SRC_DENSE) {
        // bank sources: gradient with respect to the bank entries,
        // accumulated over the pixels that read them (mirrors undone)
        if (!depth) return SDIRT_EINVAL;
        A.img = img; A.gout = gout; A.depth = depth;
        const long long cells = A.bank2d ? (long long)A.F * A.Fy : A.F;
        if (cells * A.D * 4 >= 0x7fffffffLL) return SDIRT_EUNSUPPORTED;
        if (A.ks != 21 && A.ks != 31 && A.ks != 33 && A.ks != 41 && A.ks != 63 && A.ks != 65)
            return SDIRT_EUNSUPPORTED;
        const size_t n = (size_t)cells * A.D * A.L * 2 * A.ks * A.ks;
        if ((rc = launch_fill_zero(grad_psf, n * sizeof(float), stream))) return rc;
        float* g = reinterpret_cast<float*>(grad_psf);
        for (int pass = 0; pass < (A.bank2d ? 2 : 1); ++pass) {
            RenderArgs B = A;
            B.pass = pass;
            bank_kgrad_pass(B, g, stream);
        }
        return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
    }
    (void)depth;
    const int hh = kTH + A.ks - 1, hw = kTW + A.ks - 1;
    if ((size_t)A.C * hh * hw * sizeof(float) > 160 * 1024) return SDIRT_EUNSUPPORTED;
    A.img = img; A.gout = gout;
    switch (A.C) {
        case 1: launch_psf_grad<1>(A, grad_psf, stream); break;
        case 2: launch_psf_grad<2>(A, grad_psf, stream); break;
        case 3: launch_psf_grad<3>(A, grad_psf, stream); break;
        default: launch_psf_grad<4>(A, grad_psf, stream); break;
    }
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

}  // namespace sdirt
