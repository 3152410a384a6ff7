// Adjoint of the trace + splat (reverse mode, per-ray recomputation).
//
// Computes dL/dtheta = sum_{q,s,i,j} G[q][s][i][j] dPSF[q][s][i][j]/dtheta for
// the tent splat with the angular (sigmoid) DP response, under frozen
// framing (pupil samples, pupil, window centres and the surviving rays are
// those of the given parameters).  theta per surface: [c, t, conic, a4, a6,
// a8, a10, a12], then the response slope.
//
// One lane per ray.  The lane re-traces its ray forward in float64 (the same
// trace as the forward kernel), keeping the state entering every surface in
// a small per-lane array; it back-propagates the splat's sensitivity to the
// landing point and direction, then sweeps the surfaces in reverse: each
// surface is recomputed locally from its entry state and its adjoint applied
// (vector Snell, sphere / even-asphere intersection with the implicit
// derivative at the Newton root, transfers).  Per-surface parameter
// adjoints are reduced across the wave and added to a float64 LDS vector;
// the workgroup flushes it with one global atomic per parameter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "device_common.hpp"
#include "pack.hpp"

namespace sdirt {

int launch_fill_zero(void* p, size_t bytes, hipStream_t stream);

constexpr int kBBlock = 64;        // one wave per workgroup
constexpr int kPerSurf = 8;

struct BwdArgs {
    LensArgs lens;
    LambdaArgs lam;
    PointArgs pts;
    SampleArgs smp;
    SensorArgs sen;
    const float* grad_psf;
    double* grad;
};
static_assert(sizeof(BwdArgs) <= 4000, "kernel arguments too large");

struct St {
    double x, y, z, dx, dy, dz;
};

// v of a lane moved by one DPP pattern (each 32-bit half); lanes without a
// source read 0
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the wave's 64 lanes, returned on every lane.  Within each row of
// 16 lanes two quad permutations and two row rotations leave the row's sum
// in every lane; two row broadcasts then carry rows 0..2 into the later
// rows, so that lane 63 holds the total.  All steps are VALU data movement
// (no LDS round trips).
__device__ inline double wave_sum_d(double v) {
    v += dpp_move<0xb1>(v);     // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4e>(v);     // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x124>(v);    // row_ror:4
    v += dpp_move<0x128>(v);    // row_ror:8
    v += dpp_move<0x142>(v);    // row_bcast:15
    v += dpp_move<0x143>(v);    // row_bcast:31
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Row sums of two per-lane values at once: on return the even lanes of
// each row of 16 hold the row's sum of a, the odd lanes its sum of b.  The
// first step exchanges a and b within each lane pair (an even lane keeps
// a and receives its odd neighbour's a, and the reverse for b), so the
// three remaining steps carry one value per lane instead of two.
__device__ inline double row_sum_pair(double a, double b, int lane) {
    const bool odd = lane & 1;
    double t = (odd ? b : a) + dpp_move<0xb1>(odd ? a : b);   // quad_perm [1, 0, 3, 2]
    t += dpp_move<0x4e>(t);     // quad_perm [2, 3, 0, 1]
    t += dpp_move<0x124>(t);    // row_ror:4
    t += dpp_move<0x128>(t);    // row_ror:8
    return t;
}

// Adds the wave's sums of a and b into LDS: lanes 0, 16, 32 and 48 add
// their row's sum of a at g[ia] if ua, lanes 1, 17, 33 and 49 their row's
// sum of b at g[ib] if ub.
__device__ inline void lds_add_pair(double* g, double a, int ia, bool ua, double b, int ib, bool ub,
                                    int lane) {
    const double t = row_sum_pair(a, b, lane);
    const bool odd = lane & 1;
    if ((lane & 14) == 0 && (odd ? ub : ua) && t != 0.0) atomicAdd(&g[odd ? ib : ia], t);
}

// Adjoint of vector Snell refraction d' = mu d + g N, g = sqrt(K) - mu cosI,
// K = 1 - mu^2 (1 - cosI^2), cosI = d . N.  Adds to db and nb.
__device__ __forceinline__ void refract_bwd(double mu, const double d[3], const double n[3],
                                   const double ob[3], double db[3], double nb[3]) {
    const double cosI = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
    const double K = 1.0 - mu * mu * (1.0 - cosI * cosI);
    const double sK = sqrt_t<double>(K);
    const double g = sK - mu * cosI;
    const double gb = ob[0] * n[0] + ob[1] * n[1] + ob[2] * n[2];
    for (int k = 0; k < 3; ++k) {
        nb[k] += ob[k] * g;
        db[k] += ob[k] * mu;
    }
    const double Kb = sK > 0.0 ? gb * 0.5 * rcp_d(sK) : 0.0;
    const double cb = -mu * gb + Kb * mu * mu * 2.0 * cosI;
    for (int k = 0; k < 3; ++k) {
        db[k] += cb * n[k];
        nb[k] += cb * d[k];
    }
}

// Sag, dsag/drho, d2sag/drho2 and the parameter derivatives of sag and of
// dsag/drho for an even asphere (conic k, a4..a12) at rho = r^2.
struct SagD {
    double sag, s1, s2;
    double sag_c, sag_k, s1_c, s1_k;
};

__device__ __forceinline__ SagD sag_derivs(const double* co, double c, double rho) {
    const double k = co[0];
    const double a4 = co[1], a6 = co[2], a8 = co[3], a10 = co[4], a12 = co[5];
    const double al = (1.0 + k) * c * c;
    double arg = 1.0 - al * rho;
    arg = arg > 0.0 ? arg : 1e-300;
    const double q = sqrt(arg);
    const double opq = 1.0 + q;
    SagD r;
    r.sag = c * rho / opq + rho * rho * (a4 + rho * (a6 + rho * (a8 + rho * (a10 + rho * a12))));
    r.s1 = c / (2.0 * q) + rho * (2 * a4 + rho * (3 * a6 + rho * (4 * a8 + rho * (5 * a10 + rho * 6 * a12))));
    r.s2 = c * al / (4.0 * q * q * q) +
           (2 * a4 + rho * (6 * a6 + rho * (12 * a8 + rho * (20 * a10 + rho * 30 * a12))));
    r.sag_c = rho / opq + (1.0 + k) * c * c * rho * rho / (q * opq * opq);
    r.sag_k = c * c * c * rho * rho / (2.0 * q * opq * opq);
    r.s1_c = 1.0 / (2.0 * q) + (1.0 + k) * c * c * rho / (2.0 * q * q * q);
    r.s1_k = c * c * c * rho / (4.0 * q * q * q);
    return r;
}

// Reverse of one surface.  `in` is the state entering surface s (frame of
// surface s-1), `ob` the adjoint of its output (hit point in frame s and
// refracted direction).  Writes the adjoint of `in` to `ib` and the
// parameter adjoints [c, t_{s-1}, k, a4..a12] to pg (t_{s-1} at index 1 is
// the thickness of the previous surface).
template <bool GENERAL>
__device__ __forceinline__ void surface_bwd(const LensArgs& L, int s, double mu, const St& in,
                                   const St& ob, St& ib, double pg[kPerSurf]) {
    for (int k = 0; k < kPerSurf; ++k) pg[k] = 0.0;
    const int kind = kind_of(L, s);
    const double c = L.c[s];
    const double tprev = L.tprev[s];
    // ---- forward recompute -------------------------------------------
    const double dx = in.dx, dy = in.dy, dz = in.dz;
    const double z1 = in.z - tprev;
    const double idz = rcp_d(dz);
    const double tau = -z1 * idz;
    const double x1 = in.x + tau * dx, y1 = in.y + tau * dy;
    double D = 0.0, F = 0.0, G = 0.0, den = 1.0, sq = 0.0;
    double xh = x1, yh = y1, zh = 0.0;
    const int slot = aslot_of(L, s);
    const double* co = L.asph[slot > 0 ? slot : 0];   // read only for ASPHERE
    if (kind == SDIRT_SPHERE) {
        F = c * (x1 * x1 + y1 * y1);
        G = dz - c * (x1 * dx + y1 * dy);
        const double disc = G * G - c * F;
        sq = sqrt_t<double>(disc);
        den = G + sq;
        D = F * rcp_d(den);
    } else if (GENERAL && kind == SDIRT_ASPHERE) {
        const double kk = co[0];
        const double FF = c * (x1 * x1 + y1 * y1);
        const double GG = dz - c * (x1 * dx + y1 * dy);
        const double a = c * (1.0 + kk * dz * dz);
        const double disc = GG * GG - a * FF;
        D = disc >= 0.0 ? FF / (GG + sqrt(disc)) : 0.0;
        const Asph<double> SA(co, c);
        for (int it = 0; it < 50; ++it) {
            const double xr = x1 + D * dx, yr = y1 + D * dy;
            double sag, dsag2;
            bool ok;
            asphere_sag<double, true>(SA, xr * xr + yr * yr, &sag, &dsag2, &ok);
            if (!ok) break;
            const double f = D * dz - sag;
            const double fp = dz - dsag2 * (xr * dx + yr * dy);
            const double step = f / fp;
            D -= step;
            if (fabs(step) < 1e-12 * (1.0 + fabs(D))) break;
        }
    }
    if (kind == SDIRT_SPHERE || (GENERAL && kind == SDIRT_ASPHERE)) {
        xh = x1 + D * dx;
        yh = y1 + D * dy;
        zh = D * dz;
    }
    // ---- reverse -------------------------------------------------------
    double xhb = ob.x, yhb = ob.y, zhb = ob.z;
    double db[3] = {0.0, 0.0, 0.0};
    const double d[3] = {dx, dy, dz};
    const double odb[3] = {ob.dx, ob.dy, ob.dz};
    if (kind == SDIRT_STOP) {
        db[0] += odb[0]; db[1] += odb[1]; db[2] += odb[2];
        zhb = 0.0;
    } else if (kind == SDIRT_PLANE) {
        const double n[3] = {0.0, 0.0, 1.0};
        double nb[3] = {0.0, 0.0, 0.0};
        refract_bwd(mu, d, n, odb, db, nb);
        zhb = 0.0;
    } else if (GENERAL && kind == SDIRT_IDEAL) {
        const double tx = dx / dz - xh * c, ty = dy / dz - yh * c;
        const double inv = 1.0 / sqrt(tx * tx + ty * ty + 1.0);
        const double ab = odb[0] * tx + odb[1] * ty + odb[2];
        const double inv3 = inv * inv * inv;
        const double txb = odb[0] * inv - ab * inv3 * tx;
        const double tyb = odb[1] * inv - ab * inv3 * ty;
        db[0] += txb / dz;
        db[1] += tyb / dz;
        db[2] += -(txb * dx + tyb * dy) / (dz * dz);
        xhb += -txb * c;
        yhb += -tyb * c;
        zhb = 0.0;
    } else if (kind == SDIRT_SPHERE) {
        const double n[3] = {-c * xh, -c * yh, 1.0 - c * zh};
        double nb[3] = {0.0, 0.0, 0.0};
        refract_bwd(mu, d, n, odb, db, nb);
        xhb += -c * nb[0];
        yhb += -c * nb[1];
        zhb += -c * nb[2];
        pg[0] += -(xh * nb[0] + yh * nb[1] + zh * nb[2]);
        // xh = x1 + D dx, yh = y1 + D dy, zh = D dz
        const double Db = xhb * dx + yhb * dy + zhb * dz;
        db[0] += xhb * D; db[1] += yhb * D; db[2] += zhb * D;
        double x1b = xhb, y1b = yhb;
        const double iden = rcp_d(den);
        const double Fb0 = Db * iden;
        const double denb = -Db * D * iden;
        double Gb = denb;
        const double sqb = denb;
        const double discb = sq > 0.0 ? sqb * 0.5 * rcp_d(sq) : 0.0;
        Gb += discb * 2.0 * G;
        const double Fb = Fb0 - c * discb;
        pg[0] += -F * discb;
        // G = dz - c (x1 dx + y1 dy)
        db[2] += Gb;
        x1b += -c * dx * Gb; y1b += -c * dy * Gb;
        db[0] += -c * x1 * Gb; db[1] += -c * y1 * Gb;
        pg[0] += -(x1 * dx + y1 * dy) * Gb;
        // F = c (x1^2 + y1^2)
        x1b += Fb * 2.0 * c * x1; y1b += Fb * 2.0 * c * y1;
        pg[0] += Fb * (x1 * x1 + y1 * y1);
        xhb = x1b; yhb = y1b;     // now adjoints of x1, y1
    } else if (GENERAL) {   // ASPHERE
        const double rho = xh * xh + yh * yh;
        const SagD S = sag_derivs(co, c, rho);
        const double nrm = sqrt(4.0 * rho * S.s1 * S.s1 + 1.0);
        const double n[3] = {-2.0 * xh * S.s1 / nrm, -2.0 * yh * S.s1 / nrm, 1.0 / nrm};
        double nb[3] = {0.0, 0.0, 0.0};
        refract_bwd(mu, d, n, odb, db, nb);
        // N = m / |m|, m = (-2 xh s1, -2 yh s1, 1)
        const double ndot = nb[0] * n[0] + nb[1] * n[1] + nb[2] * n[2];
        const double mb0 = (nb[0] - ndot * n[0]) / nrm;
        const double mb1 = (nb[1] - ndot * n[1]) / nrm;
        xhb += mb0 * (-2.0 * S.s1);
        yhb += mb1 * (-2.0 * S.s1);
        const double s1b = mb0 * (-2.0 * xh) + mb1 * (-2.0 * yh);
        double rhob = s1b * S.s2;
        pg[0] += s1b * S.s1_c;
        pg[2] += s1b * S.s1_k;
        double rm = rho;
        for (int m = 1; m <= 5; ++m) {       // d s1 / d a_{2m+2} = (m+1) rho^m
            pg[2 + m] += s1b * (m + 1) * rm;
            rm *= rho;
        }
        xhb += 2.0 * xh * rhob;
        yhb += 2.0 * yh * rhob;
        // xh = x1 + D dx, yh = y1 + D dy, zh = D dz
        const double Db = xhb * dx + yhb * dy + zhb * dz;
        db[0] += xhb * D; db[1] += yhb * D; db[2] += zhb * D;
        double x1b = xhb, y1b = yhb;
        // implicit root of f = D dz - sag(rho(D))
        const double fp = dz - S.s1 * 2.0 * (xh * dx + yh * dy);
        const double lam = -Db / fp;
        x1b += lam * (-S.s1 * 2.0 * xh);
        y1b += lam * (-S.s1 * 2.0 * yh);
        db[0] += lam * (-S.s1 * 2.0 * xh * D);
        db[1] += lam * (-S.s1 * 2.0 * yh * D);
        db[2] += lam * D;
        pg[0] += lam * (-S.sag_c);
        pg[2] += lam * (-S.sag_k);
        double rp = rho * rho;
        for (int m = 0; m < 5; ++m) {        // d sag / d a_{2m+4} = rho^{m+2}
            pg[3 + m] += lam * (-rp);
            rp *= rho;
        }
        xhb = x1b; yhb = y1b;
    }
    // transfer: x1 = x + tau dx, y1 = y + tau dy, tau = -z1/dz, z1 = z - tprev
    const double taub = xhb * dx + yhb * dy;
    db[0] += xhb * tau;
    db[1] += yhb * tau;
    const double z1b = -taub * idz;
    db[2] += taub * z1 * idz * idz;
    ib.x = xhb;
    ib.y = yhb;
    ib.z = z1b;
    ib.dx = db[0];
    ib.dy = db[1];
    ib.dz = db[2];
    pg[1] += -z1b;
}

// The state entering every surface, kept in LDS as float32 (structure of
// arrays: entry (s, k) of lane l at [(NV s + k) * 64 + l], conflict-free):
// x, y, dx, dy and (spheres-and-planes instance) z.  dz is the positive root
// of |d| = 1 (a live ray always travels toward +z).  The general instance,
// whose registers allow more resident waves than its LDS does, rebuilds z
// from the surface the ray left instead of storing it (the hit of surface
// s - 1 in its vertex frame: 0 on planes, stops and ideal lenses, the
// sphere's or the asphere's sag at the stored (x, y); the ray start lies on
// the entrance-pupil plane): ten workgroups per CU instead of eight on a
// 12-surface lens.
template <bool GENERAL>
struct PathRec {
    static constexpr int NV = GENERAL ? 4 : 5;
    float* v;
    int lane;
    __device__ void operator()(int s, const Ray<double>& r) const {
        float* o = v + NV * (s + 1) * 64 + lane;
        o[0] = (float)r.x; o[64] = (float)r.y;
        o[128] = (float)r.dx; o[192] = (float)r.dy;
        if (!GENERAL) o[256] = (float)r.z;
    }
};

template <bool GENERAL>
__device__ inline void path_put(float* v, int s, int lane, const Ray<double>& r) {
    PathRec<GENERAL>{v, lane}(s - 1, r);
}

template <bool GENERAL>
__device__ inline St path_get(const LensArgs& L, const float* v, int s, int lane, double zep) {
    const float* o = v + PathRec<GENERAL>::NV * s * 64 + lane;
    const double x = o[0], y = o[64], dx = o[128], dy = o[192];
    double z = GENERAL ? zep : (double)o[256];
    if (GENERAL && s > 0) {
        const int kind = kind_of(L, s - 1);
        const double c = L.c[s - 1];
        const double rho = x * x + y * y;
        z = 0.0;
        if (kind == SDIRT_SPHERE) {
            // the root near the vertex of c (rho + z^2) - 2 z = 0
            z = c * rho * rcp_d(1.0 + sqrt_t<double>(1.0 - c * c * rho));
        } else if (kind == SDIRT_ASPHERE) {
            const Asph<double> SA(L.asph[aslot_of(L, s - 1)], c);
            double sag, dsag2;
            bool ok;
            asphere_sag<double, false>(SA, rho, &sag, &dsag2, &ok);
            z = sag;
        }
    }
    return St{x, y, z, dx, dy, sqrt_t<double>(1.0 - dx * dx - dy * dy)};
}

// GENERAL = false: spheres, planes and stops only (the forward re-trace then
// takes the branch-free surface loop).
template <bool GENERAL>
__global__ __launch_bounds__(kBBlock) void trace_bwd_kernel(const BwdArgs A) {
    __shared__ double gsh[kPerSurf * kMaxS + 1];
    extern __shared__ float path[];     // [(S + 1) * NV][64]
    const int S = A.lens.S;
    const int np = kPerSurf * S + 1;
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < np; i += kBBlock) gsh[i] = 0.0;
    const int ks = A.sen.ks, kk = ks * ks, pad = (ks - 1) / 2;
    // wave-uniform indices, kept in scalar registers so that the kernel
    // arguments are read with scalar loads (no private copy of them)
    const int q = __builtin_amdgcn_readfirstlane(blockIdx.x / A.smp.chunks);
    const int chunk = __builtin_amdgcn_readfirstlane(blockIdx.x - q * A.smp.chunks);
    const int l = __builtin_amdgcn_readfirstlane(q % A.pts.L);
    const int dix = __builtin_amdgcn_readfirstlane((q / A.pts.L) % A.pts.D);
    const int f = __builtin_amdgcn_readfirstlane(q / (A.pts.L * A.pts.D));
    const double hx = A.pts.fields[f][0], hy = A.pts.fields[f][1];
    const double depth = A.pts.depths[dix];
    const double m = A.pts.m_num / (A.pts.z_ep_ref + depth);
    const double px = hx / m, py = hy / m, pz = -depth;
    const double zep = A.lam.z_ep[l], rep = A.lam.rho_ep[l];
    const double* mu = A.lam.mu[l];
    const uint32_t key = point_key(A.smp.seed, (uint32_t)q);
    const double ps = A.sen.ps, inv_ps = 1.0 / ps;
    const double ksig = A.sen.sig_k;
    const float* Gq = A.grad_psf + (size_t)q * 2 * kk;
    const int nx = A.smp.nx;
    const int n_rays = nx * A.smp.ny;
    const int r0 = chunk * A.smp.rays_per_chunk;
    const int r1 = min(r0 + A.smp.rays_per_chunk, n_rays);
    double g_slope = 0.0;
    __syncthreads();
    for (int base = r0; base < r1; base += kBBlock) {
        const int r = base + tid;
        bool live = r < r1;
        Ray<double> ray{0, 0, 0, 0, 0, 1};
        if (live) {
            const int ci = r % nx, cj = r / nx;
            double x1 = 0.5, x2 = 0.5;
            if (A.smp.jitter) {
                x1 = jitter01(key, (uint32_t)r, 0u);
                x2 = jitter01(key, (uint32_t)r, 1u);
            }
            const double a = -1.0 + 2.0 * (ci + x1) / nx;
            const double b = -1.0 + 2.0 * (cj + x2) / A.smp.ny;
            double u, v;
            concentric(a, b, &u, &v);
            const double ex = rep * u, ey = rep * v;
            const double ddx = ex - px, ddy = ey - py, ddz = zep - pz;
            const double inv = 1.0 / sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
            ray = Ray<double>{ex, ey, zep, ddx * inv, ddy * inv, ddz * inv};
            path_put<GENERAL>(path, 0, lane, ray);
            const int st = trace_ray<double, PathRec<GENERAL>, false, GENERAL>(A.lens, mu, ray,
                                                                             PathRec<GENERAL>{path, lane});
            live = st == kAlive;
        }
        // ---- splat adjoint: dL/dO, dL/dD, dL/dk -----------------------
        St ob{0, 0, 0, 0, 0, 0};
        double gts = 0.0;
        if (live) {
            const double wu = (ray.x - hx) * inv_ps + pad;
            const double wv = (ray.y - hy) * inv_ps + pad;
            const double fj = floor(wu), fi = floor(wv);
            const int j0 = (int)fj, i0 = (int)fi;
            const double fx = wu - fj, fy = wv - fi;
            const double rr = sqrt(ray.dx * ray.dx + ray.dz * ray.dz);
            const double sx = ray.dx / rr;
            const double wl = 1.0 / (1.0 + exp(-ksig * sx));
            const double wr = 1.0 - wl;
            double gu = 0.0, gv = 0.0, glr = 0.0;
            const double wt[4] = {(1 - fy) * (1 - fx), (1 - fy) * fx, fy * (1 - fx), fy * fx};
            const double wtu[4] = {-(1 - fy), (1 - fy), -fy, fy};
            const double wtv[4] = {-(1 - fx), -fx, (1 - fx), fx};
            for (int t = 0; t < 4; ++t) {
                const int ii = i0 + (t >> 1), jj = j0 + (t & 1);
                if (ii >= 0 && ii < ks && jj >= 0 && jj < ks) {
                    const double GL = Gq[ii * ks + jj], GR = Gq[kk + ii * ks + jj];
                    const double gw = wl * GL + wr * GR;
                    gu += gw * wtu[t];
                    gv += gw * wtv[t];
                    glr += (GL - GR) * wt[t];
                }
            }
            const double sig1 = wl * wr;
            g_slope += glr * sig1 * sx;
            const double sxb = glr * sig1 * ksig;
            const double r3 = rr * rr * rr;
            // sensor plane: O = p + tau d, tau = -(z - t_S) / dz (ray holds O)
            const St pl = path_get<GENERAL>(A.lens, path, S, lane, zep);
            const double pz0 = pl.z;
            const double pdx = pl.dx, pdy = pl.dy, pdz = pl.dz;
            const double z1 = pz0 - A.lens.sensor_dist;
            const double tau = -z1 / pdz;
            const double Oxb = gu * inv_ps, Oyb = gv * inv_ps;
            const double taub = Oxb * pdx + Oyb * pdy;
            ob.x = Oxb;
            ob.y = Oyb;
            ob.dx = Oxb * tau + sxb * (ray.dz * ray.dz) / r3;
            ob.dy = Oyb * tau;
            ob.dz = taub * z1 / (pdz * pdz) - sxb * ray.dx * ray.dz / r3;
            const double z1b = -taub / pdz;
            ob.z = z1b;
            gts = -z1b;                        // sensor distance = t of the last surface
        }
        {
            const double red = wave_sum_d(gts);
            if (lane == 0 && red != 0.0) atomicAdd(&gsh[kPerSurf * (S - 1) + 1], red);
        }
        // ---- reverse sweep over the surfaces ---------------------------
        for (int s = S - 1; s >= 0; --s) {
            double pg[kPerSurf];
            St ib{0, 0, 0, 0, 0, 0};
            if (live) {
                const St in = path_get<GENERAL>(A.lens, path, s, lane, zep);
                surface_bwd<GENERAL>(A.lens, s, mu[s], in, ob, ib, pg);
                ob = ib;
            } else {
                for (int k = 0; k < kPerSurf; ++k) pg[k] = 0.0;
            }
            const int kind = kind_of(A.lens, s);
            // c (sphere/asphere) with t_{s-1} (s > 0), then conic and the
            // a's (asphere) in pairs
            const bool has_c = kind == SDIRT_SPHERE || (GENERAL && kind == SDIRT_ASPHERE);
            if (has_c || s > 0)
                lds_add_pair(gsh, pg[0], kPerSurf * s, has_c, pg[1], kPerSurf * (s - 1) + 1, s > 0,
                             lane);
            if (GENERAL && kind == SDIRT_ASPHERE) {
#pragma unroll
                for (int k = 2; k < kPerSurf; k += 2)
                    lds_add_pair(gsh, pg[k], kPerSurf * s + k, true, pg[k + 1], kPerSurf * s + k + 1,
                                 true, lane);
            }
        }
    }
    const double vs = wave_sum_d(g_slope);
    if (lane == 0 && vs != 0.0) atomicAdd(&gsh[np - 1], vs);
    __syncthreads();
    for (int i = tid; i < np; i += kBBlock)
        if (gsh[i] != 0.0) atomicAdd(&A.grad[i], gsh[i]);
}

int trace_backward_impl(const sdirt_lens* lens, const sdirt_sensor* sensor,
                        const sdirt_psf_query* query, const float* grad_psf,
                        double* grad_out, hipStream_t stream) {
    if (!grad_psf || !grad_out) return SDIRT_EINVAL;
    Resolved R;
    int rc = resolve_lens(lens, &R);
    if (rc) return rc;
    BwdArgs A;
    std::memset(&A, 0, sizeof(A));
    if ((rc = pack_lens(R, &A.lens))) return rc;
    if ((rc = check_query(query, R, &A.pts, &A.smp))) return rc;
    if ((rc = pack_lambdas(R, query->wavelengths, query->n_wavelengths, &A.lam))) return rc;
    if ((rc = check_sensor(sensor, query->ks, &A.sen))) return rc;
    if (A.pts.points) return SDIRT_EUNSUPPORTED;              // grid mode only
    if (query->splat != SDIRT_SPLAT_TENT || sensor->dp_mode != SDIRT_DP_SIGMOID ||
        query->normalize != SDIRT_NORM_NONE || query->math != SDIRT_F64)
        return SDIRT_EUNSUPPORTED;
    A.grad_psf = grad_psf;
    A.grad = grad_out;
    const int P = A.pts.P;
    const int n_rays = A.smp.nx * A.smp.ny;
    const int np = kPerSurf * R.S + 1;
    if ((rc = launch_fill_zero(grad_out, (size_t)np * sizeof(double), stream))) return rc;
    int chunks = std::max(1, std::min((16384 + P - 1) / P, n_rays / (kBBlock * 4)));
    A.smp.chunks = chunks;
    A.smp.rays_per_chunk = (n_rays + chunks - 1) / chunks;
    bool general = false;
    for (int s = 0; s < R.S; ++s)
        general = general || R.kind[s] == SDIRT_ASPHERE || R.kind[s] == SDIRT_IDEAL;
    const int nv = general ? PathRec<true>::NV : PathRec<false>::NV;
    const size_t shm = (size_t)(R.S + 1) * nv * kBBlock * sizeof(float);
    hipLaunchKernelGGL(general ? trace_bwd_kernel<true> : trace_bwd_kernel<false>,
                       dim3((unsigned)((long long)chunks * P)),
                       dim3(kBBlock), shm, stream, A);
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

}  // namespace sdirt
