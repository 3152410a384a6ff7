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
struct LensArgs {
    int S;
    int stop;
    int8_t kind[kMaxS];
    int8_t aslot[kMaxS];        // asphere slot or -1
    double c[kMaxS];            // curvature; 1/f for IDEAL
    double tprev[kMaxS];        // distance from the previous vertex (0 for s=0)
    double semi2[kMaxS];        // squared clear semi-diameter
    double asph[kMaxAsph][6];   // conic, a4, a6, a8, a10, a12
    double sensor_dist;         // last vertex -> sensor plane
};

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

// Shirley-Chiu concentric map of [-1,1]^2 onto the unit disk, in a form
// that commutes exactly with a -> -a and b -> -b.  float32 trigonometry on
// |phi| <= pi/4.
__device__ inline void concentric(double a, double b, double* u, double* v) {
    const float af = (float)a, bf = (float)b;
    if (fabsf(af) > fabsf(bf)) {
        const float phi = 0.785398163397448309616f * (bf / af);
        float s, c;
        sincosf(phi, &s, &c);
        *u = (double)(af * c);
        *v = (double)(af * s);
    } else if (bf != 0.0f) {
        const float phi = 0.785398163397448309616f * (af / bf);
        float s, c;
        sincosf(phi, &s, &c);
        *u = (double)(bf * s);
        *v = (double)(bf * c);
    } else {
        *u = 0.0;
        *v = 0.0;
    }
}

template <typename T>
struct Ray {
    T x, y, z, dx, dy, dz;
};

template <typename T> __device__ inline T tol_newton();
template <> __device__ inline double tol_newton<double>() { return 1e-12; }
template <> __device__ inline float tol_newton<float>() { return 2e-6f; }

// Reciprocal, square root and reciprocal square root from the hardware
// approximations refined by one Newton step.  On gfx950 v_rcp_f64 and
// v_rsq_f64 are accurate to ~5e-8 relative; one step brings them to
// ~4e-15 (measured over 1e6 arguments in [1e-3, 1e3]), far below what the
// trace needs; no IEEE rounding or denormal handling is needed on this path.
template <typename T> __device__ inline T rcp_t(T v);
template <> __device__ inline double rcp_t<double>(double v) {
    const double r = __builtin_amdgcn_rcp(v);
    return fma(r, fma(-v, r, 1.0), r);
}
template <> __device__ inline float rcp_t<float>(float v) { return 1.0f / v; }

template <typename T> __device__ inline T rsqrt_t(T v);
template <> __device__ inline double rsqrt_t<double>(double v) {
    const double y = __builtin_amdgcn_rsq(v);
    return y * fma(-0.5 * v * y, y, 1.5);
}
template <> __device__ inline float rsqrt_t<float>(float v) { return 1.0f / sqrtf(v); }

// sqrt of a non-negative argument (0 -> 0)
template <typename T> __device__ inline T sqrt_t(T v);
template <> __device__ inline double sqrt_t<double>(double v) {
    if (!(v > 0.0)) return 0.0;
    const double y = rsqrt_t<double>(v);
    const double s = v * y;
    return fma(0.5 * y, fma(-s, s, v), s);
}
template <> __device__ inline float sqrt_t<float>(float v) { return v > 0.f ? sqrtf(v) : 0.f; }

// Even-asphere sag and its derivative in rho = r^2.
template <typename T>
__device__ __forceinline__ void asphere_sag(const double* co, T c, T rho, T* sag, T* dsag,
                                   bool* ok) {
    const T k = (T)co[0];
    const T arg = T(1) - (T(1) + k) * c * c * rho;
    *ok = arg >= T(0);
    const T q = sqrt_t<T>(arg >= T(0) ? arg : T(1));
    const T a4 = (T)co[1], a6 = (T)co[2], a8 = (T)co[3], a10 = (T)co[4], a12 = (T)co[5];
    *sag = c * rho / (T(1) + q) +
           rho * rho * (a4 + rho * (a6 + rho * (a8 + rho * (a10 + rho * a12))));
    *dsag = c / (T(2) * q) +
            rho * (T(2) * a4 + rho * (T(3) * a6 + rho * (T(4) * a8 +
                   rho * (T(5) * a10 + rho * T(6) * a12))));
}

// Sequential trace of one ray through surfaces [0, S): on return r holds
// the vertex-local state after the last surface.  `rec(s, r)` is called
// after each surface (hit point + refracted direction).
// EXACT: report the first failure's code (ray-level debugging); otherwise
// only whether the ray survived (kAlive or kMiss), which keeps the
// bookkeeping in scalar lane masks.
template <typename T, typename Rec, bool EXACT = true>
__device__ __forceinline__ int trace_ray(const LensArgs& L, const double* mu, Ray<T>& r,
                                Rec rec) {
    int status = kAlive;
    bool alive = true;
#define SDIRT_FAIL(cond, code)                                   \
    do {                                                         \
        if (EXACT) { if ((cond) && status == kAlive) status = (code); } \
        else alive = alive && !(cond);                           \
    } while (0)
    for (int s = 0; s < L.S; ++s) {
        const int kind = L.kind[s];
        r.z -= (T)L.tprev[s];
        SDIRT_FAIL(!(r.dz > T(0)), kInvalid);
        const T inv_dz = rcp_t<T>(r.dz);
        const T tau = -r.z * inv_dz;
        r.x += tau * r.dx;
        r.y += tau * r.dy;
        r.z = T(0);
        const T c = (T)L.c[s];
        if (kind == SDIRT_SPHERE) {
            const T F = c * (r.x * r.x + r.y * r.y);
            const T G = r.dz - c * (r.x * r.dx + r.y * r.dy);
            const T disc = G * G - c * F;
            SDIRT_FAIL(disc < T(0), kMiss);
            const T delta = F * rcp_t<T>(G + sqrt_t<T>(disc));
            r.x += delta * r.dx;
            r.y += delta * r.dy;
            r.z = delta * r.dz;
        } else if (kind == SDIRT_ASPHERE) {
            const double* co = L.asph[L.aslot[s]];
            const T k = (T)co[0];
            const T F = c * (r.x * r.x + r.y * r.y);
            const T G = r.dz - c * (r.x * r.dx + r.y * r.dy);
            const T a = c * (T(1) + k * r.dz * r.dz);
            const T disc = G * G - a * F;
            T delta = disc >= T(0) ? F * rcp_t<T>(G + sqrt_t<T>(disc)) : T(0);
            bool conv = false, bad = false;
            for (int it = 0; it < 50 && !conv && !bad; ++it) {
                const T xr = r.x + delta * r.dx;
                const T yr = r.y + delta * r.dy;
                T sag, dsag;
                bool ok;
                asphere_sag(co, c, xr * xr + yr * yr, &sag, &dsag, &ok);
                if (!ok) { bad = true; break; }
                const T f = delta * r.dz - sag;
                const T fp = r.dz - dsag * T(2) * (xr * r.dx + yr * r.dy);
                const T step = f * rcp_t<T>(fp);
                delta -= step;
                conv = fabs(step) < tol_newton<T>() * (T(1) + fabs(delta));
            }
            SDIRT_FAIL(!conv || bad, kNewton);
            r.x += delta * r.dx;
            r.y += delta * r.dy;
            r.z = delta * r.dz;
        }
        const T r2 = r.x * r.x + r.y * r.y;
        SDIRT_FAIL(r2 > (T)L.semi2[s], kClip);
        if (kind == SDIRT_SPHERE || kind == SDIRT_ASPHERE || kind == SDIRT_PLANE) {
            T nx, ny, nz;
            if (kind == SDIRT_SPHERE) {
                nx = -c * r.x; ny = -c * r.y; nz = T(1) - c * r.z;
            } else if (kind == SDIRT_ASPHERE) {
                T sag, dsag;
                bool ok;
                asphere_sag(L.asph[L.aslot[s]], c, r2, &sag, &dsag, &ok);
                nx = T(-2) * r.x * dsag; ny = T(-2) * r.y * dsag; nz = T(1);
                const T inv = rsqrt_t<T>(nx * nx + ny * ny + T(1));
                nx *= inv; ny *= inv; nz = inv;
            } else {
                nx = T(0); ny = T(0); nz = T(1);
            }
            const T m = (T)mu[s];
            const T cosI = r.dx * nx + r.dy * ny + r.dz * nz;
            const T K = T(1) - m * m * (T(1) - cosI * cosI);
            SDIRT_FAIL(K < T(0), kTir);
            const T g = sqrt_t<T>(K) - m * cosI;
            r.dx = m * r.dx + g * nx;
            r.dy = m * r.dy + g * ny;
            r.dz = m * r.dz + g * nz;
        } else if (kind == SDIRT_IDEAL) {
            const T idz = rcp_t<T>(r.dz);
            const T tx = r.dx * idz - r.x * c;
            const T ty = r.dy * idz - r.y * c;
            const T inv = rsqrt_t<T>(tx * tx + ty * ty + T(1));
            r.dx = tx * inv; r.dy = ty * inv; r.dz = inv;
        }
        rec(s, r);
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
