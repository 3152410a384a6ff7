// Device-side building blocks of the DP PSF engine (gfx950, wave64):
// kernel-argument layout of a prescription, the counter-based pupil jitter,
// the concentric pupil map and the per-surface intersect / refract steps of
// the sequential trace (Sec. 3.1).  Templated on the arithmetic type T
// (double by default, float for the fast mode).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/sdirt.h"

namespace sdirt {

constexpr int kMaxS = SDIRT_MAX_SURFACES;
constexpr int kMaxL = SDIRT_MAX_LAMBDAS;
constexpr int kMaxAsph = 8;   // asphere rows per prescription

enum RayStatus : int { kAlive = 0, kMiss = 1, kClip = 2, kTir = 3,
                       kNewton = 4, kInvalid = 5 };

// Prescription as kernel arguments: read with scalar loads in the hot loop.
// code[s] = kind | 0x40 if an asphere's 1 / ((1 + k) c) is nonzero | 0x80 if
// inv_c[s] holds 1/c | (asphere slot << 8) (slot -1
// when not an asphere); a 32-bit word so that it is fetched by a scalar load
// and tested with scalar instructions.
struct LensArgs {
    int S;
    int stop;
    int code[kMaxS];
    double c[kMaxS];            // curvature; 1/f for IDEAL
    double inv_c[kMaxS];        // 1/c for spheres with |c| >= 1e-6 per mm, else 0
    double tprev[kMaxS];        // distance from the previous vertex (0 for s=0)
    double semi2[kMaxS];        // squared clear semi-diameter
    double asph[kMaxAsph][7];   // conic, a4, a6, a8, a10, a12, 1 / ((1 + conic) c) or 0
    double sensor_dist;         // last vertex -> sensor plane
};

__device__ __host__ inline int kind_of(const LensArgs& L, int s) { return L.code[s] & 0x3f; }
__device__ __host__ inline int aslot_of(const LensArgs& L, int s) { return L.code[s] >> 8; }

// Per-wavelength data: index ratios and entrance pupil.
struct LambdaArgs {
    int L;
    double mu[kMaxL][kMaxS];    // n_before / n_after per surface
    double z_ep[kMaxL];
    double rho_ep[kMaxL];
    double lambda[kMaxL];
};

// ---- counter-based jitter: MurmurHash3 fmix32 finaliser chain -----------
__device__ __host__ inline uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

__device__ __host__ inline uint32_t point_key(uint32_t seed, uint32_t q) {
    return fmix32(fmix32(seed ^ 0x9E3779B9u) ^ q);
}

// Uniform number in [0, 1) with 24 random bits for (point key, ray, dim).
__device__ inline double jitter01(uint32_t key, uint32_t ray, uint32_t dim) {
    const uint32_t h = fmix32(key ^ (2u * ray + dim));
    return (double)(h >> 8) * (1.0 / 16777216.0);
}

// Reciprocal from the hardware approximation (v_rcp_f64, ~5e-8 relative)
// refined by one Newton step (~2e-15).
__device__ inline double rcp_d(double v) {
    const double r = __builtin_amdgcn_rcp(v);
    return fma(r, fma(-v, r, 1.0), r);
}

// a * b + c with c in scalar registers: one v_fma_f64.  (Left to itself
// the compiler keeps loop-invariant float64 constants in vector registers
// and evaluates a Horner step as a register copy of the constant followed
// by an accumulating fma.)
__device__ __forceinline__ double fma_sc(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// sin and cos for |x| <= pi/4 from their Taylor series through x^15 and
// x^16 (truncation below 1e-16 on that interval), in float64.  sin is odd
// and cos even bit for bit.
__device__ inline void sincos_quarter(double x, double* s, double* c) {
    const double x2 = x * x;
    double p = -1.0 / 1307674368000.0;           // -1/15!
    p = fma_sc(p, x2, 1.0 / 6227020800.0);       //  1/13!
    p = fma_sc(p, x2, -1.0 / 39916800.0);        // -1/11!
    p = fma_sc(p, x2, 1.0 / 362880.0);           //  1/9!
    p = fma_sc(p, x2, -1.0 / 5040.0);            // -1/7!
    p = fma_sc(p, x2, 1.0 / 120.0);              //  1/5!
    p = fma_sc(p, x2, -1.0 / 6.0);               // -1/3!
    *s = fma(x * x2, p, x);
    double q = 1.0 / 20922789888000.0;           //  1/16!
    q = fma_sc(q, x2, -1.0 / 87178291200.0);     // -1/14!
    q = fma_sc(q, x2, 1.0 / 479001600.0);        //  1/12!
    q = fma_sc(q, x2, -1.0 / 3628800.0);         // -1/10!
    q = fma_sc(q, x2, 1.0 / 40320.0);            //  1/8!
    q = fma_sc(q, x2, -1.0 / 720.0);             // -1/6!
    q = fma_sc(q, x2, 1.0 / 24.0);               //  1/4!
    q = fma(q, x2, -0.5);                        // -1/2!
    *c = fma(x2, q, 1.0);
}

// Shirley-Chiu concentric map of [-1,1]^2 onto the unit disk in float64,
// in a form that commutes exactly with a -> -a and b -> -b:
//   |a| > |b|: phi = (pi/4) b/a, (u, v) = (a cos phi, a sin phi)
//   else:      phi = (pi/4) a/b, (u, v) = (b sin phi, b cos phi)
__device__ inline void concentric(double a, double b, double* u, double* v) {
    const bool wide = fabs(a) > fabs(b);
    const double num = wide ? b : a, den = wide ? a : b;
    const double phi = den != 0.0 ? 0.78539816339744830962 * (num * rcp_d(den)) : 0.0;
    double sn, cs;
    sincos_quarter(phi, &sn, &cs);
    const double p = den * cs, o = den * sn;
    *u = wide ? p : o;
    *v = wide ? o : p;
}

template <typename T>
struct Ray {
    T x, y, z, dx, dy, dz;
};

template <typename T> __device__ inline T tol_newton();
template <> __device__ inline double tol_newton<double>() { return 1e-12; }
template <> __device__ inline float tol_newton<float>() { return 2e-6f; }

// Reciprocal, square root and reciprocal square root.  float64: the hardware
// approximations (v_rcp_f64, v_rsq_f64: ~5e-8 relative on gfx950) refined
// by one Newton step to ~4e-15 (measured over 1e6 arguments in [1e-3, 1e3]),
// far below what the trace needs; no IEEE rounding or denormal handling is
// needed on this path.  float32: the hardware instructions (1 ulp).
template <typename T> __device__ inline T rcp_t(T v);
template <> __device__ inline double rcp_t<double>(double v) { return rcp_d(v); }
template <> __device__ inline float rcp_t<float>(float v) { return __builtin_amdgcn_rcpf(v); }

template <typename T> __device__ inline T rsqrt_t(T v);
template <> __device__ inline double rsqrt_t<double>(double v) {
    const double y = __builtin_amdgcn_rsq(v);
    return y * fma(-0.5 * v * y, y, 1.5);
}
template <> __device__ inline float rsqrt_t<float>(float v) { return __builtin_amdgcn_rsqf(v); }

// sqrt of a non-negative argument (0 for v <= 0): s = v y with the raw
// y ~ 1/sqrt(v), corrected once by s + (y/2)(v - s^2); relative error
// 1.5 e^2 for a raw error e.
template <typename T> __device__ inline T sqrt_t(T v);
template <> __device__ inline double sqrt_t<double>(double v) {
    if (!(v > 0.0)) return 0.0;
    const double y = __builtin_amdgcn_rsq(v);
    const double s = v * y;
    return fma(0.5 * y, fma(-s, s, v), s);
}
template <> __device__ inline float sqrt_t<float>(float v) {
    return v > 0.f ? __builtin_amdgcn_sqrtf(v) : 0.f;
}

// Raw hardware approximations (~5e-8 relative in float64), for quantities
// whose error only slows an iteration down (Newton derivatives).
template <typename T> __device__ inline T rcp_raw(T v);
template <> __device__ inline double rcp_raw<double>(double v) { return __builtin_amdgcn_rcp(v); }
template <> __device__ inline float rcp_raw<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <typename T> __device__ inline T rsq_raw(T v);
template <> __device__ inline double rsq_raw<double>(double v) { return __builtin_amdgcn_rsq(v); }
template <> __device__ inline float rsq_raw<float>(float v) { return __builtin_amdgcn_rsqf(v); }

// sqrt where a negative argument marks a ray that the caller already counts
// as lost: the argument is clamped instead of selected on, and the result
// for such a ray is finite and unused.
template <typename T> __device__ inline T sqrt_live(T v);
template <> __device__ inline double sqrt_live<double>(double v) {
    v = fmax(v, 1e-300);
    const double y = __builtin_amdgcn_rsq(v);
    const double s = v * y;
    return fma(0.5 * y, fma(-s, s, v), s);
}
template <> __device__ inline float sqrt_live<float>(float v) {
    return __builtin_amdgcn_sqrtf(fmaxf(v, 1e-30f));
}

// sqrt of an argument that is positive on every path of a live ray: the
// caller has already marked a ray with a non-positive (or NaN) argument as
// lost, and the NaN it gets here stays in that ray's unused state.
template <typename T> __device__ inline T sqrt_pos(T v);
template <> __device__ inline double sqrt_pos<double>(double v) {
    const double y = __builtin_amdgcn_rsq(v);
    const double s = v * y;
    return fma(0.5 * y, fma(-s, s, v), s);
}
template <> __device__ inline float sqrt_pos<float>(float v) {
    return __builtin_amdgcn_sqrtf(v);
}

// Constants of the trace that depend only on the prescription and the
// wavelength, staged once per workgroup in LDS: float64 has no scalar ALU,
// so evaluated in the per-ray loop they cost vector instructions on every
// surface of every ray.  Per surface m^2 and 1 - m^2 (m the index ratio, the
// latter as fma(-m, m, 1)); per asphere slot (1 + k) c^2, a12, the
// coefficients 4 a4, 6 a6, 8 a8, 10 a10, 12 a12 of twice the sag's slope
// and k c.
struct TraceConsts {
    double sm[kMaxS][2];
    double as[kMaxAsph][8];
};

// Fill the table (threads tid < S each take one surface); the caller
// synchronises the workgroup before the first read.
__device__ inline void stage_trace_consts(const LensArgs& L, const double* mu, TraceConsts* tc,
                                          int tid) {
    if (tid >= L.S) return;
    const double m = mu[tid];
    tc->sm[tid][0] = m * m;
    tc->sm[tid][1] = fma(-m, m, 1.0);
    const int code = L.code[tid];
    if ((code & 0x3f) == SDIRT_ASPHERE) {
        const double* co = L.asph[code >> 8];
        const double c = L.c[tid];
        double* a = tc->as[code >> 8];
        a[0] = (1.0 + co[0]) * c * c;
        a[1] = co[5];
        a[2] = 4.0 * co[1];
        a[3] = 6.0 * co[2];
        a[4] = 8.0 * co[3];
        a[5] = 10.0 * co[4];
        a[6] = 12.0 * co[5];
        a[7] = co[0] * c;
    }
}

// Even-asphere surface constants, read once per surface.  inv_kc =
// 1 / ((1 + k) c) when |(1 + k) c| >= 1e-3 per mm (host), else 0; d4 .. d12
// = 4 a4 .. 12 a12 are the coefficients of twice the slope.
template <typename T>
struct Asph {
    T c, kc2, a4, a6, a8, a10, a12, inv_kc, d4, d6, d8, d10, d12;
    bool iv;    // inv_kc != 0
    __device__ Asph(const double* co, T cc)
        : c(cc), kc2((T(1) + (T)co[0]) * cc * cc), a4((T)co[1]), a6((T)co[2]), a8((T)co[3]),
          a10((T)co[4]), a12((T)co[5]), inv_kc((T)co[6]), d4(T(4) * a4), d6(T(6) * a6),
          d8(T(8) * a8), d10(T(10) * a10), d12(T(12) * a12), iv(co[6] != 0.0) {}
    // the derived constants from a staged table row (TraceConsts::as) and
    // the surface code's flag for a nonzero inv_kc
    __device__ Asph(const double* co, T cc, const double* t, bool iv_)
        : c(cc), kc2((T)t[0]), a4((T)co[1]), a6((T)co[2]), a8((T)co[3]), a10((T)co[4]),
          a12((T)t[1]), inv_kc((T)co[6]), d4((T)t[2]), d6((T)t[3]), d8((T)t[4]), d10((T)t[5]),
          d12((T)t[6]), iv(iv_) {}
};

// Even-asphere sag and twice its derivative in rho = r^2; *ok is false where the
// conic root is imaginary.  EXACT_D: derivative from the refined 1/sqrt;
// otherwise from the raw hardware value (for Newton steps, whose
// convergence a 5e-8 relative error in the slope does not spoil).  The conic
// part c rho / (1 + q), q = sqrt(1 - (1 + k) c^2 rho), equals
// (1 - q) / ((1 + k) c): with that reciprocal from the host it takes no
// division (absolute error about eps / |(1 + k) c| <= 1.1e-13 mm at the
// host's threshold); nearly parabolic or flat surfaces keep the quotient.
template <typename T, bool EXACT_D>
__device__ __forceinline__ void asphere_sag(const Asph<T>& S, T rho, T* sag, T* dsag2, bool* ok) {
    const T arg = T(1) - S.kc2 * rho;
    *ok = arg >= T(0);
    const T a = fmax(arg, T(1e-30));
    const T y = rsq_raw<T>(a);
    const T s0 = a * y;
    const T q = fma(T(0.5) * y, fma(-s0, s0, a), s0);                 // sqrt(a)
    const T iq = EXACT_D ? y * fma(T(-0.5) * a * y, y, T(1.5)) : y;   // 1 / sqrt(a)
    const T conic = S.iv ? fma(-q, S.inv_kc, S.inv_kc)
                                     : S.c * rho * rcp_t<T>(T(1) + q);
    *sag = conic +
           rho * rho * (S.a4 + rho * (S.a6 + rho * (S.a8 + rho * (S.a10 + rho * S.a12))));
    *dsag2 = S.c * iq + rho * (S.d4 + rho * (S.d6 + rho * (S.d8 + rho * (S.d10 + rho * S.d12))));
}

// Sequential trace of one ray through surfaces [0, S): on return r holds
// the vertex-local state after the last surface.  `rec(s, r)` is called
// after each surface (hit point + refracted direction).
// Spheres are intersected straight from the current point: the root of the
// quadratic c t^2 - 2 G t + F = 0 (c |p + t d|^2 - 2 (p_z + t d_z) = 0), whose
// discriminant does not depend on where along the ray p sits, in float64 as
// (G - sqrt(G^2 - cF)) / c with 1/c from the host (absolute error about
// eps G / |c|, below 1e-10 mm for |c| >= 1e-6 per mm), else and in float32 as
// F / (G + sqrt(G^2 - cF));
// aspheres, planes, the stop and ideal lenses first move the ray to the
// vertex plane.
// EXACT: report the first failure's code (ray-level debugging); otherwise
// only whether the ray survived (kAlive or kMiss), which keeps the
// bookkeeping in scalar lane masks, and in the general surface loop a wave
// leaves after the surface where its last ray was lost (rec is then not
// called for the surfaces after it).  GENERAL = false is for prescriptions of
// spheres, planes and stops only: a flat surface is a sphere of curvature 0
// (the quadratic's root is then the plane transfer) and a stop has index
// ratio 1 (the refraction then leaves the direction unchanged), so every
// surface but the aperture stop takes the sphere path, without per-surface
// branches; the aperture stop is a plane transfer and a clip.  TC: the
// derived constants come from the workgroup's staged table tc (the values
// computed here, bit for bit; only the asphere's base-conic start is
// evaluated differently, as one fma with k c).
template <typename T, typename Rec, bool EXACT = true, bool GENERAL = true, bool TC = false>
__device__ __forceinline__ int trace_ray(const LensArgs& L, const double* mu, Ray<T>& r,
                                Rec rec, const TraceConsts* tc = nullptr) {
    int status = kAlive;
    bool alive = true;
#define SDIRT_FAIL(cond, code)                                   \
    do {                                                         \
        if (EXACT) { if ((cond) && status == kAlive) status = (code); } \
        else alive = alive && !(cond);                           \
    } while (0)
    // sphere, or a flat surface as a sphere of curvature 0.  rho2 = x^2 + y^2
    // of the current point on entry, of the hit on return (the clip test's
    // value, reused by the next surface: a transfer along z leaves it).
    auto sphere = [&](const int s, const int code, const T c, const T semi2, T& rho2)
                      __attribute__((always_inline)) {
        const T F = c * fma(r.z, r.z, rho2) - T(2) * r.z;
        const T G = r.dz - c * (r.x * r.dx + r.y * r.dy + r.z * r.dz);
        const T disc = G * G - c * F;
        // a ray that misses the sphere or only grazes it is lost
        SDIRT_FAIL(!(disc > T(0)), kMiss);
        // sqrt(disc) is also the cosine of the incidence angle at the
        // hit: with n = (-c x, -c y, 1 - c z) there, d.n = G - c t
        const T cosI = sqrt_pos<T>(disc);
        T t;
        if (sizeof(T) == sizeof(double) && (code & 0x80))
            t = (G - cosI) * (T)L.inv_c[s];
        else
            t = F * rcp_t<T>(G + cosI);
        r.x += t * r.dx;
        r.y += t * r.dy;
        r.z += t * r.dz;
        rho2 = r.x * r.x + r.y * r.y;
        SDIRT_FAIL(rho2 > semi2, kClip);
        // vector Snell with cos^2 I = disc: K = 1 - m^2 (1 - disc)
        const T m = (T)mu[s];
        const T m2 = TC ? (T)tc->sm[s][0] : m * m;
        const T om2 = TC ? (T)tc->sm[s][1] : fma(-m, m, T(1));
        const T K = fma(m2, disc, om2);
        // total internal reflection, or an exit ray along the surface
        SDIRT_FAIL(!(K > T(0)), kTir);
        const T g = sqrt_pos<T>(K) - m * cosI;
        const T gc = g * c;
        r.dx = fma(-gc, r.x, m * r.dx);
        r.dy = fma(-gc, r.y, m * r.dy);
        r.dz = fma(g, fma(-c, r.z, T(1)), m * r.dz);
    };
    int s0 = 0;
    if (!GENERAL) {
        // spheres and flats only: every surface but the aperture stop takes
        // the sphere path (no per-surface branches); the stop, a plane of
        // index ratio 1, is a transfer and a clip
        T rho2 = r.x * r.x + r.y * r.y;
        auto surf = [&](const int s) __attribute__((always_inline)) {
            r.z -= (T)L.tprev[s];
            SDIRT_FAIL(!(r.dz > T(0)), kInvalid);
            sphere(s, L.code[s], (T)L.c[s], (T)L.semi2[s], rho2);
            rec(s, r);
        };
        const int stop = L.stop;
        for (; s0 < stop; ++s0) surf(s0);
        if (s0 < L.S && (L.code[s0] & 0x3f) == SDIRT_STOP) {
            r.z -= (T)L.tprev[s0];
            SDIRT_FAIL(!(r.dz > T(0)), kInvalid);
            const T tau = -r.z * rcp_t<T>(r.dz);
            r.x += tau * r.dx;
            r.y += tau * r.dy;
            r.z = T(0);
            rho2 = r.x * r.x + r.y * r.y;
            SDIRT_FAIL(rho2 > (T)L.semi2[s0], kClip);
            rec(s0, r);
            ++s0;
        }
        for (; s0 < L.S; ++s0) surf(s0);
    }
    // x^2 + y^2 of the current point, left by every surface at its hit (a
    // transfer along z keeps it)
    T hrho2 = r.x * r.x + r.y * r.y;
    for (int s = s0; GENERAL && s < L.S; ++s) {
        const int code = L.code[s];
        const int kind = code & 0x3f;
        const T c = (T)L.c[s];
        const T semi2 = (T)L.semi2[s];
        r.z -= (T)L.tprev[s];
        SDIRT_FAIL(!(r.dz > T(0)), kInvalid);
        if (kind == SDIRT_SPHERE) {
            sphere(s, code, c, semi2, hrho2);
        } else {
            const T tau = -r.z * rcp_t<T>(r.dz);
            r.x += tau * r.dx;
            r.y += tau * r.dy;
            r.z = T(0);
            if (kind == SDIRT_ASPHERE) {
                const double* co = L.asph[code >> 8];
                const Asph<T> S = TC ? Asph<T>(co, c, tc->as[code >> 8], (code & 0x40) != 0)
                                     : Asph<T>(co, c);
                const T F = c * (r.x * r.x + r.y * r.y);
                const T G = r.dz - c * (r.x * r.dx + r.y * r.dy);
                // c (1 + k dz^2), with k c from the staged table
                const T a = TC ? fma((T)tc->as[code >> 8][7], r.dz * r.dz, c)
                               : c * (T(1) + (T)co[0] * r.dz * r.dz);
                const T disc = G * G - a * F;
                T delta = disc >= T(0) ? F * rcp_t<T>(G + sqrt_live<T>(disc)) : T(0);
                // Converged when the step is below the tolerance, or (float64)
                // below 1e-7 mm while shrinking more than 1000-fold on the
                // previous one: Newton is then in its quadratic regime and the
                // next step would be under r^2 |step| < 1e-13 mm (r the ratio),
                // so that step is skipped.  The tests are evaluated as
                // |step| - tol |delta| < tol (one fma each), and prev holds
                // 1e-3 times the previous |step|.
                // a ray already lost (bookkeeping mode) takes no Newton
                // step: its state is never used, and its iterations, which
                // need not converge, would hold the whole wave
                bool conv = !alive, bad = false;
                T prev = T(1e27);
                for (int it = 0; it < 50 && !conv && !bad; ++it) {
                    const T xr = r.x + delta * r.dx;
                    const T yr = r.y + delta * r.dy;
                    T sag, dsag2;
                    bool ok;
                    asphere_sag<T, false>(S, xr * xr + yr * yr, &sag, &dsag2, &ok);
                    if (!ok) { bad = true; break; }
                    const T f = delta * r.dz - sag;
                    const T fp = r.dz - dsag2 * (xr * r.dx + yr * r.dy);
                    const T step = f * rcp_raw<T>(fp);
                    delta -= step;
                    const T as = fabs(step), ad = fabs(delta);
                    conv = fma(-tol_newton<T>(), ad, as) < tol_newton<T>() ||
                           (sizeof(T) == sizeof(double) && fma(T(-1e-7), ad, as) < T(1e-7) &&
                            as < prev);
                    prev = T(1e-3) * as;
                }
                SDIRT_FAIL(!conv || bad, kNewton);
                r.x += delta * r.dx;
                r.y += delta * r.dy;
                r.z = delta * r.dz;
                const T r2 = r.x * r.x + r.y * r.y;
                hrho2 = r2;
                SDIRT_FAIL(r2 > semi2, kClip);
                T sag, dsag2;
                bool ok;
                asphere_sag<T, true>(S, r2, &sag, &dsag2, &ok);
                // vector Snell at the normal n (-x s', -y s', 1) / |n|, s' =
                // dsag2 (|n|^2 = 1 + r2 s'^2), with the scale applied to the
                // dot product and to the refracted term instead of to n
                const T nx = -r.x * dsag2, ny = -r.y * dsag2;
                const T inv = rsqrt_t<T>(fma(r2, dsag2 * dsag2, T(1)));
                const T m = (T)mu[s];
                const T m2 = TC ? (T)tc->sm[s][0] : m * m;
                const T cosI = fma(r.dx, nx, fma(r.dy, ny, r.dz)) * inv;
                const T K = T(1) - m2 * (T(1) - cosI * cosI);
                SDIRT_FAIL(K < T(0), kTir);
                const T gi = (sqrt_live<T>(K) - m * cosI) * inv;
                r.dx = fma(gi, nx, m * r.dx);
                r.dy = fma(gi, ny, m * r.dy);
                r.dz = fma(m, r.dz, gi);
            } else {
                hrho2 = r.x * r.x + r.y * r.y;
                SDIRT_FAIL(hrho2 > semi2, kClip);
                if (kind == SDIRT_PLANE) {
                    // normal (0, 0, 1): the refracted dz is sqrt(K)
                    const T m = (T)mu[s];
                    const T m2 = TC ? (T)tc->sm[s][0] : m * m;
                    const T K = T(1) - m2 * (T(1) - r.dz * r.dz);
                    SDIRT_FAIL(K < T(0), kTir);
                    r.dx *= m;
                    r.dy *= m;
                    r.dz = sqrt_live<T>(K);
                } else if (kind == SDIRT_IDEAL) {
                    const T idz = rcp_t<T>(r.dz);
                    const T tx = r.dx * idz - r.x * c;
                    const T ty = r.dy * idz - r.y * c;
                    const T inv = rsqrt_t<T>(tx * tx + ty * ty + T(1));
                    r.dx = tx * inv; r.dy = ty * inv; r.dz = inv;
                }
            }
        }
        rec(s, r);
        // a wave whose rays are all lost leaves (vignetting loses whole
        // stretches of the pupil, so this is the common way to lose rays)
        if (!EXACT && !__any(alive)) return kMiss;
    }
    // to the sensor plane
    r.z -= (T)L.sensor_dist;
    SDIRT_FAIL(!(r.dz > T(0)), kInvalid);
    const T tau = -r.z * rcp_t<T>(r.dz);
    r.x += tau * r.dx;
    r.y += tau * r.dy;
    r.z = T(0);
    SDIRT_FAIL(!(isfinite(r.x) && isfinite(r.y)), kInvalid);
#undef SDIRT_FAIL
    return EXACT ? status : (alive ? kAlive : kMiss);
}

struct NoRec {
    template <typename R>
    __device__ void operator()(int, const R&) const {}
};

}  // namespace sdirt
