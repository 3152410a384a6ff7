// Ray-traced DP PSF kernels (Sec. 3.1, Eq. (1)-(3)) for gfx950.
//
// trace_splat: one lane per ray.  A workgroup owns one PSF point and a chunk
// of its pupil grid; every lane samples its pupil point (counter-based
// jitter, concentric map), traces it through the prescription held in
// kernel arguments (scalar loads), splits the landed ray into left/right
// energy and adds it to a [2][ks][ks] float tile in LDS.  The tile is
// flushed once per workgroup with global atomics (non-zero entries only);
// per-point energy statistics are reduced in the workgroup first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.hpp"
#include "pack.hpp"

namespace sdirt {

struct SplatArgs {
    LensArgs lens;
    LambdaArgs lam;
    PointArgs pts;
    SampleArgs smp;
    SensorArgs sen;
    int splat;
    void* out;
    double* stats;
};
static_assert(sizeof(SplatArgs) <= 4000, "kernel arguments too large");

constexpr int kBlock = 256;
// The trace-and-splat workgroup: eight waves (two per SIMD) sharing one LDS
// splat tile, with registers capped for six waves per SIMD, so that three
// workgroups (24 waves) fit per compute unit even at the 33.8 KB tile of
// ks 65 (with 256 lanes and no cap the tile limited a compute unit to 16
// waves; 370 -> 351 ms on the 16-surface lens at ks 65).
constexpr int kTBlock = 512;
constexpr int kTWavesPerSimd = 6;


__device__ inline float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Point data: field (h_x, h_y), depth, wavelength slot.
__device__ inline void point_of(const PointArgs& P, int q, double* hx, double* hy,
                                double* depth, int* slot) {
    if (P.points) {
        const double* p = P.points + 4 * (size_t)q;
        *hx = p[0]; *hy = p[1]; *depth = p[2];
        *slot = (int)p[3];
    } else {
        const int l = q % P.L;
        const int d = (q / P.L) % P.D;
        const int f = q / (P.L * P.D);
        *hx = P.fields[f][0]; *hy = P.fields[f][1];
        *depth = P.depths[d];
        *slot = l;
    }
}

// A weight in [0, 1] as an integer multiple of 2^-32 (round to nearest):
// sums of these are exact and independent of the order of the additions.
__device__ inline unsigned long long fixed_weight(float w) {
    return (unsigned long long)__builtin_rintf(w * 4294967296.0f);
}

template <typename T, int SPLAT, int DP, typename OutT, bool GENERAL>
__global__ __launch_bounds__(kTBlock, kTWavesPerSimd) void trace_splat_kernel(const SplatArgs A) {
    // [2][ks][ks] float32 sums, or (deterministic mode) 64-bit integer sums
    // of weights in units of 2^-32
    extern __shared__ float tile[];
    unsigned long long* tile_q = reinterpret_cast<unsigned long long*>(tile);
    const bool det = A.smp.det != 0;
    __shared__ float red[kTBlock / 64][8];
    __shared__ TraceConsts tc;
    const int ks = A.sen.ks;
    const int kk = ks * ks;
    const int pad = (ks - 1) / 2;
    const int q = blockIdx.x / A.smp.chunks;
    const int chunk = blockIdx.x - q * A.smp.chunks;
    const int tid = threadIdx.x;
    // masked mode: points outside the mask are left as they are (the whole
    // workgroup leaves before its first barrier)
    if (A.pts.mask && A.pts.mask[q] == 0) return;
    for (int i = tid; i < (det ? 4 : 2) * kk; i += kTBlock) tile[i] = 0.0f;

    double hx, hy, depth;
    int slot;
    point_of(A.pts, q, &hx, &hy, &depth, &slot);
    const bool slot_ok = slot >= 0 && slot < A.lam.L;
    slot = slot_ok ? slot : 0;
    const double m = A.pts.m_num / (A.pts.z_ep_ref + depth);
    const double px = hx / m, py = hy / m, pz = -depth;
    const double zep = A.lam.z_ep[slot], rep = A.lam.rho_ep[slot];
    const double* mu = A.lam.mu[slot];
    if (GENERAL) stage_trace_consts(A.lens, mu, &tc, tid);
    const uint32_t key = point_key(A.smp.seed, (uint32_t)q);
    const double ps = A.sen.ps, inv_ps = 1.0 / ps;
    const int nx = A.smp.nx;
    const int n_rays = nx * A.smp.ny;
    const double two_nx = 2.0 / nx, two_ny = 2.0 / A.smp.ny;
    const int r0 = chunk * A.smp.rays_per_chunk;
    const int r1 = min(r0 + A.smp.rays_per_chunk, n_rays);
    float e_vig = 0.f, e_tr = 0.f, e_l = 0.f, e_r = 0.f, e_miss = 0.f, e_out = 0.f;
    __syncthreads();

    // grid cell (ci, cj) of ray r.  Tile order (nx and ny multiples of 8):
    // a wave's 64 rays sample one 8 x 8 patch of the pupil, so vignetting,
    // which cuts the pupil along curves, more often loses whole waves (which
    // then leave the surface loop); the jitter is keyed by the cell, so the
    // rays are those of row order.  Row order: r = cj nx + ci, advanced at
    // the top of each pass by the loop stride kTBlock = step_j nx + step_i
    // with one carry (0 <= ci < nx), starting one stride before the first ray.
    const int step_j = kTBlock / nx, step_i = kTBlock - step_j * nx;
    int cj = (int)(((uint64_t)(uint32_t)(r0 + tid) * A.smp.div_magic) >> A.smp.div_shift);
    int ci = r0 + tid - cj * nx - step_i;
    cj -= step_j;
    if (ci < 0) { ci += nx; --cj; }
    const bool tile8 = A.smp.tile8 != 0;
    const uint32_t lx = (uint32_t)tid & 7u, ly = ((uint32_t)tid >> 3) & 7u;   // cell in the tile
    for (int r = r0 + tid; r < r1 && slot_ok; r += kTBlock) {
        uint32_t cell = (uint32_t)r;
        if (tile8) {
            // the wave's tile: chunks start on whole tiles, so r >> 6 is the
            // same on every lane of a wave (scalar arithmetic)
            const uint32_t t = __builtin_amdgcn_readfirstlane((uint32_t)r >> 6);
            const uint32_t ty = (uint32_t)(((uint64_t)t * A.smp.tdiv_magic) >> A.smp.tdiv_shift);
            ci = (int)(((t - ty * (uint32_t)(nx >> 3)) << 3) | lx);
            cj = (int)((ty << 3) | ly);
            cell = (uint32_t)(cj * nx + ci);
        } else {
            ci += step_i;
            cj += step_j;
            if (ci >= nx) { ci -= nx; ++cj; }
        }
        double x1 = 0.5, x2 = 0.5;
        if (A.smp.jitter) {
            x1 = jitter01(key, cell, 0u);
            x2 = jitter01(key, cell, 1u);
        }
        const double a = -1.0 + (ci + x1) * two_nx;
        const double b = -1.0 + (cj + x2) * two_ny;
        double u, v;
        concentric(a, b, &u, &v);
        const double ex = rep * u, ey = rep * v;
        double ddx = ex - px, ddy = ey - py, ddz = zep - pz;
        const double inv = rsqrt_t<double>(ddx * ddx + ddy * ddy + ddz * ddz);
        Ray<T> ray{(T)ex, (T)ey, (T)zep, (T)(ddx * inv), (T)(ddy * inv), (T)(ddz * inv)};
        const int st = trace_ray<T, NoRec, false, GENERAL, GENERAL>(A.lens, mu, ray, NoRec(), &tc);
        if (st != kAlive) { e_vig += 1.f; continue; }
        e_tr += 1.f;
        const double wu = ((double)ray.x - hx) * inv_ps + pad;
        const double wv = ((double)ray.y - hy) * inv_ps + pad;
        float wl, wr;
        const int jb = (int)floor(wu + 0.5);
        const int ib = (int)floor(wv + 0.5);
        if (DP == SDIRT_DP_SIGMOID) {
            const float dxf = (float)ray.dx, dzf = (float)ray.dz;
            const float sx = dxf * __builtin_amdgcn_rsqf(dxf * dxf + dzf * dzf);
            wl = __builtin_amdgcn_rcpf(1.0f + __expf(-(float)A.sen.sig_k * sx));
            wr = 1.0f - wl;
        } else {
            const double xk = (double)ray.x, yk = (double)ray.y;
            const double xc = hx + (jb - pad) * ps;
            const double yc = hy + (ib - pad) * ps;
            const double tn = (double)ray.dx * rcp_d((double)ray.dz);
            const double h = A.sen.ml_h, f = A.sen.ml_f, w = A.sen.ml_w, rr = A.sen.ml_r;
            const bool inside = (xk - xc) * (xk - xc) + (yk - yc) * (yk - yc) <= rr * rr;
            double xL, xM, xR;
            if (inside) {
                const double g = h / (f - h);
                xL = xc + w - (f * tn - w) * g;
                xM = xc - (f * tn) * g;
                xR = xc - w - (f * tn + w) * g;
            } else {
                xL = xc + w - h * tn;
                xM = xc - h * tn;
                xR = xc - w - h * tn;
            }
            const bool left = xM <= xk && xk < xL;
            const bool right = xR <= xk && xk < xM;
            if (!left && !right) { e_miss += 1.f; continue; }
            wl = left ? 1.f : 0.f;
            wr = right ? 1.f : 0.f;
        }
        if (SPLAT == SDIRT_SPLAT_BOX) {
            if (ib >= 0 && ib < ks && jb >= 0 && jb < ks) {
                const int o = __mul24(ib, ks) + jb;
                if (det) {
                    if (wl != 0.f) atomicAdd(&tile_q[o], fixed_weight(wl));
                    if (wr != 0.f) atomicAdd(&tile_q[kk + o], fixed_weight(wr));
                } else {
                    if (wl != 0.f) atomicAdd(&tile[o], wl);
                    if (wr != 0.f) atomicAdd(&tile[kk + o], wr);
                }
                e_l += wl;
                e_r += wr;
            } else {
                e_out += 1.f;
            }
        } else {
            const double fj = floor(wu), fi = floor(wv);
            const int j0 = (int)fj, i0 = (int)fi;
            const float fx = (float)(wu - fj), fy = (float)(wv - fi);
            const float wt[4] = {(1.f - fy) * (1.f - fx), (1.f - fy) * fx,
                                 fy * (1.f - fx), fy * fx};
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int ii = i0 + (t >> 1), jj = j0 + (t & 1);
                if (ii >= 0 && ii < ks && jj >= 0 && jj < ks) {
                    const int o = ii * ks + jj;
                    if (det) {
                        atomicAdd(&tile_q[o], fixed_weight(wl * wt[t]));
                        atomicAdd(&tile_q[kk + o], fixed_weight(wr * wt[t]));
                    } else {
                        atomicAdd(&tile[o], wl * wt[t]);
                        atomicAdd(&tile[kk + o], wr * wt[t]);
                    }
                    e_l += wl * wt[t];
                    e_r += wr * wt[t];
                } else {
                    e_out += wt[t];
                }
            }
        }
    }
    // workgroup reduction of the statistics
    float vals[6] = {e_vig, e_tr, e_l, e_r, e_miss, e_out};
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const float s = wave_sum(vals[k]);
        if (lane == 0) red[wave][k] = s;
    }
    __syncthreads();
    if (tid == 0 && A.stats && slot_ok) {
        double tot[6] = {0, 0, 0, 0, 0, 0};
        for (int w = 0; w < kTBlock / 64; ++w)
            for (int k = 0; k < 6; ++k) tot[k] += red[w][k];
        double* st = A.stats + 7 * (size_t)q;
        atomicAdd(&st[0], (double)max(r1 - r0, 0));
        for (int k = 0; k < 6; ++k)
            if (tot[k] != 0.0) atomicAdd(&st[k + 1], tot[k]);
    }
    OutT* out = reinterpret_cast<OutT*>(A.out) + (size_t)q * 2 * kk;
    if (det) {
        // the point's only workgroup: exact sums, one store per element
        for (int i = tid; i < 2 * kk; i += kTBlock)
            out[i] = (OutT)((double)tile_q[i] * (1.0 / 4294967296.0));
        return;
    }
    if (A.smp.chunks == 1) {
        // the point's only workgroup: plain stores (the host skips the
        // output's zero fill)
        for (int i = tid; i < 2 * kk; i += kTBlock) out[i] = (OutT)tile[i];
        return;
    }
    for (int i = tid; i < 2 * kk; i += kTBlock) {
        const float v = tile[i];
        if (v != 0.0f) atomicAdd(&out[i], (OutT)v);
    }
}

// Joint normalisation of each point's [2][ks][ks] block (sum or max);
// points outside a mask (if any) are left as they are.
template <typename OutT>
__global__ __launch_bounds__(kBlock) void normalize_kernel(OutT* out, int kk2, int mode,
                                                           const int* mask) {
    if (mask && mask[blockIdx.x] == 0) return;
    __shared__ double red[kBlock / 64];
    OutT* p = out + (size_t)blockIdx.x * kk2;
    double acc = 0.0;
    for (int i = threadIdx.x; i < kk2; i += kBlock) {
        const double v = (double)p[i];
        acc = mode == SDIRT_NORM_SUM ? acc + v : fmax(acc, v);
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(acc, o, 64);
        acc = mode == SDIRT_NORM_SUM ? acc + w : fmax(acc, w);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    double tot = red[0];
    for (int w = 1; w < kBlock / 64; ++w)
        tot = mode == SDIRT_NORM_SUM ? tot + red[w] : fmax(tot, red[w]);
    if (tot > 0.0) {
        const double inv = 1.0 / tot;
        for (int i = threadIdx.x; i < kk2; i += kBlock) p[i] = (OutT)((double)p[i] * inv);
    }
}

// Zero the [P][n_words] blocks of the points with mask != 0.
__global__ void fill_zero_masked_kernel(uint32_t* p, int P, int n_words, const int* mask) {
    const int q = blockIdx.x;
    if (q >= P || mask[q] == 0) return;
    uint32_t* b = p + (size_t)q * n_words;
    for (int i = threadIdx.x; i < n_words; i += blockDim.x) b[i] = 0u;
}

__global__ void fill_zero_kernel(uint32_t* p, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// Per-surface recorder for sdirt_trace_rays.
template <typename T>
struct HitRec {
    double* h;
    __device__ void operator()(int s, const Ray<T>& r) const {
        double* o = h + 6 * s;
        o[0] = r.x; o[1] = r.y; o[2] = r.z; o[3] = r.dx; o[4] = r.dy; o[5] = r.dz;
    }
};

struct RaysArgs {
    LensArgs lens;
    double mu[kMaxS];
    int n;
    const double* o;
    const double* d;
    double* hits;
    int* status;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void trace_rays_kernel(const RaysArgs A) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= A.n) return;
    const double* o = A.o + 3 * (size_t)k;
    const double* d = A.d + 3 * (size_t)k;
    Ray<T> r{(T)o[0], (T)o[1], (T)o[2], (T)d[0], (T)d[1], (T)d[2]};
    double* h = A.hits + (size_t)k * 6 * (A.lens.S + 1);
    const int st = trace_ray<T>(A.lens, A.mu, r, HitRec<T>{h});
    double* hs = h + 6 * A.lens.S;
    hs[0] = r.x; hs[1] = r.y; hs[2] = 0.0; hs[3] = r.dx; hs[4] = r.dy; hs[5] = r.dz;
    A.status[k] = st;
}

// ---- host side -----------------------------------------------------------

int launch_fill_zero(void* p, size_t bytes, hipStream_t stream) {
    const size_t n = bytes / 4;
    if (n == 0) return SDIRT_OK;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, stream,
                       (uint32_t*)p, n);
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

template <typename T, int SPLAT, int DP, typename OutT>
static void launch_splat(const SplatArgs& A, dim3 grid, size_t shm, hipStream_t st, bool general) {
    auto k = general ? trace_splat_kernel<T, SPLAT, DP, OutT, true>
                  : trace_splat_kernel<T, SPLAT, DP, OutT, false>;
    if (shm > 65536) (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL(k, grid, dim3(kTBlock), shm, st, A);
}

template <typename T, typename OutT>
static void dispatch_splat(const SplatArgs& A, dim3 grid, size_t shm, hipStream_t st) {
    const int sp = A.splat, dp = A.sen.dp_mode;
    // spheres, planes and stops only: the branch-free surface loop
    bool general = false;
    for (int s = 0; s < A.lens.S; ++s)
        general = general || kind_of(A.lens, s) == SDIRT_ASPHERE || kind_of(A.lens, s) == SDIRT_IDEAL;
    if (sp == SDIRT_SPLAT_BOX && dp == SDIRT_DP_SIGMOID) launch_splat<T, SDIRT_SPLAT_BOX, SDIRT_DP_SIGMOID, OutT>(A, grid, shm, st, general);
    else if (sp == SDIRT_SPLAT_BOX) launch_splat<T, SDIRT_SPLAT_BOX, SDIRT_DP_MICROLENS, OutT>(A, grid, shm, st, general);
    else if (dp == SDIRT_DP_SIGMOID) launch_splat<T, SDIRT_SPLAT_TENT, SDIRT_DP_SIGMOID, OutT>(A, grid, shm, st, general);
    else launch_splat<T, SDIRT_SPLAT_TENT, SDIRT_DP_MICROLENS, OutT>(A, grid, shm, st, general);
}

// Chunks per point so that the grid holds enough workgroups to fill the
// 256 compute units several times over.
static int chunks_for(int P, int n_rays) {
    const int target = 8192;
    int chunks = (target + P - 1) / P;
    const int max_chunks = std::max(1, n_rays / (kBlock * 4));
    chunks = std::max(1, std::min(chunks, max_chunks));
    return chunks;
}

int trace_dp_psf_impl(const sdirt_lens* lens, const sdirt_sensor* sensor,
                      const sdirt_psf_query* query, void* psf_out,
                      double* stats_out, hipStream_t stream, int chunks_override,
                      const int* mask) {
    if (!psf_out) return SDIRT_EINVAL;
    Resolved R;
    int rc = resolve_lens(lens, &R);
    if (rc) return rc;
    SplatArgs A;
    std::memset(&A, 0, sizeof(A));
    if ((rc = pack_lens(R, &A.lens))) return rc;
    if ((rc = check_query(query, R, &A.pts, &A.smp))) return rc;
    if ((rc = pack_lambdas(R, query->wavelengths, query->n_wavelengths, &A.lam))) return rc;
    if ((rc = check_sensor(sensor, query->ks, &A.sen))) return rc;
    A.splat = query->splat;
    A.out = psf_out;
    A.stats = stats_out;
    const int P = A.pts.P;
    const int n_rays = A.smp.nx * A.smp.ny;
    const int kk = query->ks * query->ks;
    const size_t elt = query->out_dtype == SDIRT_F64 ? 8 : 4;
    A.pts.mask = mask;
    // deterministic mode: one workgroup per point, integer tile
    const int chunks = A.smp.det ? 1
                       : chunks_override > 0 ? std::min(chunks_override, n_rays) : chunks_for(P, n_rays);
    // with one workgroup per point the kernel stores every output element
    // itself; otherwise the chunks add into a zeroed output
    const bool fill = chunks > 1;
    if (mask) {
        // only the masked points' blocks (and statistics) start from zero
        if (P > 0) {
            if (fill)
                hipLaunchKernelGGL(fill_zero_masked_kernel, dim3(P), dim3(kBlock), 0, stream,
                                   (uint32_t*)psf_out, P, (int)(2 * kk * elt / 4), mask);
            if (stats_out)
                hipLaunchKernelGGL(fill_zero_masked_kernel, dim3(P), dim3(64), 0, stream,
                                   (uint32_t*)stats_out, P, 14, mask);
        }
        if (hipGetLastError() != hipSuccess) return SDIRT_ELAUNCH;
    } else {
        if (fill && (rc = launch_fill_zero(psf_out, (size_t)P * 2 * kk * elt, stream))) return rc;
        if (stats_out && (rc = launch_fill_zero(stats_out, (size_t)P * 7 * 8, stream))) return rc;
    }
    A.smp.chunks = chunks;
    A.smp.rays_per_chunk = (n_rays + chunks - 1) / chunks;
    if (A.smp.nx % 8 == 0 && A.smp.ny % 8 == 0) {
        // whole 8 x 8 tiles per chunk (the last chunks may be short or empty)
        A.smp.rays_per_chunk = (A.smp.rays_per_chunk + 63) / 64 * 64;
        A.smp.tile8 = 1;
        div_magic_for((uint32_t)(A.smp.nx / 8), &A.smp.tdiv_magic, &A.smp.tdiv_shift);
    }
    const dim3 grid((unsigned)((long long)chunks * P));
    const size_t shm = (size_t)2 * kk * (A.smp.det ? sizeof(unsigned long long) : sizeof(float));
    const bool f64math = query->math == SDIRT_F64;
    if (query->out_dtype == SDIRT_F64) {
        if (f64math) dispatch_splat<double, double>(A, grid, shm, stream);
        else dispatch_splat<float, double>(A, grid, shm, stream);
    } else {
        if (f64math) dispatch_splat<double, float>(A, grid, shm, stream);
        else dispatch_splat<float, float>(A, grid, shm, stream);
    }
    if (hipGetLastError() != hipSuccess) return SDIRT_ELAUNCH;
    if (query->normalize != SDIRT_NORM_NONE) {
        if (query->out_dtype == SDIRT_F64)
            hipLaunchKernelGGL(normalize_kernel<double>, dim3(P), dim3(kBlock), 0, stream,
                               (double*)psf_out, 2 * kk, query->normalize, mask);
        else
            hipLaunchKernelGGL(normalize_kernel<float>, dim3(P), dim3(kBlock), 0, stream,
                               (float*)psf_out, 2 * kk, query->normalize, mask);
        if (hipGetLastError() != hipSuccess) return SDIRT_ELAUNCH;
    }
    return SDIRT_OK;
}

int trace_rays_impl(const sdirt_lens* lens, double wavelength, int math, int n,
                    const double* o, const double* d, double* hits, int* status,
                    hipStream_t stream) {
    if (!o || !d || !hits || !status || n < 0) return SDIRT_EINVAL;
    if (math != SDIRT_F32 && math != SDIRT_F64) return SDIRT_EUNSUPPORTED;
    Resolved R;
    int rc = resolve_lens(lens, &R);
    if (rc) return rc;
    RaysArgs A;
    std::memset(&A, 0, sizeof(A));
    if ((rc = pack_lens(R, &A.lens))) return rc;
    LambdaArgs LA;
    if ((rc = pack_lambdas(R, &wavelength, 1, &LA))) return rc;
    for (int s = 0; s < R.S; ++s) A.mu[s] = LA.mu[0][s];
    A.n = n; A.o = o; A.d = d; A.hits = hits; A.status = status;
    if (n == 0) return SDIRT_OK;
    const dim3 grid((n + kBlock - 1) / kBlock);
    if (math == SDIRT_F64)
        hipLaunchKernelGGL(trace_rays_kernel<double>, grid, dim3(kBlock), 0, stream, A);
    else
        hipLaunchKernelGGL(trace_rays_kernel<float>, grid, dim3(kBlock), 0, stream, A);
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

}  // namespace sdirt
