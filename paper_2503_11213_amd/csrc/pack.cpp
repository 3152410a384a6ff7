// Argument packing and validation (host, float64).  See pack.hpp.
#include "pack.hpp"

#include <cmath>

namespace sdirt {

int pack_lens(const Resolved& R, LensArgs* A) {
    std::memset(A, 0, sizeof(*A));
    A->S = R.S;
    A->stop = R.stop;
    int nas = 0;
    for (int s = 0; s < R.S; ++s) {
        int slot = -1;
        A->c[s] = R.kind[s] == SDIRT_IDEAL ? 1.0 / R.focal[s] : R.c[s];
        A->inv_c[s] = (R.kind[s] == SDIRT_SPHERE && std::fabs(R.c[s]) >= 1e-6) ? 1.0 / R.c[s] : 0.0;
        A->tprev[s] = s == 0 ? 0.0 : R.t[s - 1];
        A->semi2[s] = R.semi[s] * R.semi[s];
        if (R.kind[s] == SDIRT_ASPHERE) {
            if (nas >= kMaxAsph) return SDIRT_EUNSUPPORTED;
            slot = nas;
            A->asph[nas][0] = R.conic[s];
            for (int m = 0; m < 5; ++m) A->asph[nas][m + 1] = R.asph[5 * s + m];
            // reciprocal of (1 + k) c for the division-free conic sag
            const double kc = (1.0 + R.conic[s]) * R.c[s];
            A->asph[nas][6] = std::fabs(kc) >= 1e-3 ? 1.0 / kc : 0.0;
            ++nas;
        }
        A->code[s] = (R.kind[s] & 0x3f) | (A->inv_c[s] != 0.0 ? 0x80 : 0) |
                     (slot >= 0 && A->asph[slot][6] != 0.0 ? 0x40 : 0) |
                     (int)((unsigned)slot << 8);
    }
    A->sensor_dist = R.sensor_distance;
    return SDIRT_OK;
}

int pack_lambdas(const Resolved& R, const double* lambdas, int L, LambdaArgs* A) {
    if (!lambdas || L < 1) return SDIRT_EINVAL;
    if (L > kMaxL) return SDIRT_EUNSUPPORTED;
    std::memset(A, 0, sizeof(*A));
    A->L = L;
    for (int l = 0; l < L; ++l) {
        const double lam = lambdas[l];
        if (!std::isfinite(lam) || !(lam > 0)) return SDIRT_EINVAL;
        A->lambda[l] = lam;
        for (int m = 0; m <= R.S; ++m)
            if (!(R.index(m, lam) > 0)) return SDIRT_EINVAL;
        // the stop is an aperture only: no refraction there
        for (int s = 0; s < R.S; ++s)
            A->mu[l][s] = R.kind[s] == SDIRT_STOP ? 1.0 : R.index(s, lam) / R.index(s + 1, lam);
        R.pupil(lam, &A->z_ep[l], &A->rho_ep[l]);
        if (!std::isfinite(A->z_ep[l]) || !std::isfinite(A->rho_ep[l]))
            return SDIRT_EINVAL;
    }
    return SDIRT_OK;
}

int check_sensor(const sdirt_sensor* s, int ks, SensorArgs* A) {
    if (!s) return SDIRT_EINVAL;
    if (!std::isfinite(s->pitch) || !(s->pitch > 0)) return SDIRT_EINVAL;
    std::memset(A, 0, sizeof(*A));
    A->ks = ks;
    A->ps = s->pitch;
    A->dp_mode = s->dp_mode;
    if (s->dp_mode == SDIRT_DP_SIGMOID) {
        if (!std::isfinite(s->sigmoid_k)) return SDIRT_EINVAL;
        A->sig_k = s->sigmoid_k;
    } else if (s->dp_mode == SDIRT_DP_MICROLENS) {
        const double h = s->ml_h, f = s->ml_f, w = s->ml_w, r = s->ml_r;
        if (!std::isfinite(h) || !std::isfinite(f) || !std::isfinite(w) ||
            !std::isfinite(r)) return SDIRT_EINVAL;
        if (!(h >= 0) || !(f > h) || !(w > 0) || !(r > 0)) return SDIRT_EINVAL;
        A->ml_h = h * s->pitch;
        A->ml_f = f * s->pitch;
        A->ml_w = w * s->pitch;
        A->ml_r = r * s->pitch;
    } else {
        return SDIRT_EINVAL;
    }
    return SDIRT_OK;
}

void div_magic_for(uint32_t d, uint64_t* magic, uint32_t* shift) {
    // q = (n * m) >> (32 + l) with l = ceil(log2 d), m = ceil(2^(32+l) / d):
    // the error n (m - 2^(32+l)/d) / 2^(32+l) < n / 2^32 < 1/d for n < 2^32,
    // so q = floor(n / d); n < 2^30 and m < 2^33 keep n m below 2^63.
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    *magic = ((1ull << (32 + l)) + d - 1) / d;
    *shift = 32 + l;
}

int check_query(const sdirt_psf_query* q, const Resolved& R, PointArgs* P,
                SampleArgs* S) {
    if (!q) return SDIRT_EINVAL;
    if (q->ks < 1 || (q->ks % 2) == 0) return SDIRT_EINVAL;
    if (q->ks > SDIRT_MAX_KS) return SDIRT_EUNSUPPORTED;
    if (q->rays_x < 1 || q->rays_y < 1) return SDIRT_EINVAL;
    if ((long long)q->rays_x * q->rays_y > (1LL << 30)) return SDIRT_EUNSUPPORTED;
    if (q->splat != SDIRT_SPLAT_BOX && q->splat != SDIRT_SPLAT_TENT) return SDIRT_EINVAL;
    if (q->normalize < SDIRT_NORM_NONE || q->normalize > SDIRT_NORM_MAX) return SDIRT_EINVAL;
    if (q->out_dtype != SDIRT_F32 && q->out_dtype != SDIRT_F64) return SDIRT_EUNSUPPORTED;
    if (q->math != SDIRT_F32 && q->math != SDIRT_F64) return SDIRT_EUNSUPPORTED;
    if (q->deterministic != 0 && q->deterministic != 1) return SDIRT_EINVAL;
    // the integer tile [2][ks][ks] of 64-bit sums plus the kernel's own
    // 128 bytes of statistics scratch within the 160 KB of LDS
    if (q->deterministic && 16LL * q->ks * q->ks > 160LL * 1024 - 256) return SDIRT_EUNSUPPORTED;
    if (!q->wavelengths || q->n_wavelengths < 1) return SDIRT_EINVAL;
    if (q->n_wavelengths > kMaxL) return SDIRT_EUNSUPPORTED;
    std::memset(P, 0, sizeof(*P));
    P->m_num = R.m_num;
    P->z_ep_ref = R.z_ep_ref;
    P->L = q->n_wavelengths;
    if (q->points) {
        if (q->n_points < 1) return SDIRT_EINVAL;
        P->P = q->n_points;
        P->points = q->points;
    } else {
        if (!q->fields || !q->depths) return SDIRT_EINVAL;
        if (q->n_fields < 1 || q->n_depths < 1) return SDIRT_EINVAL;
        if (q->n_fields > kMaxF || q->n_depths > kMaxD) return SDIRT_EUNSUPPORTED;
        P->F = q->n_fields;
        P->D = q->n_depths;
        for (int f = 0; f < P->F; ++f) {
            P->fields[f][0] = q->fields[2 * f];
            P->fields[f][1] = q->fields[2 * f + 1];
            if (!std::isfinite(P->fields[f][0]) || !std::isfinite(P->fields[f][1]))
                return SDIRT_EINVAL;
        }
        for (int d = 0; d < P->D; ++d) {
            P->depths[d] = q->depths[d];
            if (!std::isfinite(P->depths[d]) || !(P->depths[d] > 0)) return SDIRT_EINVAL;
            if (!(P->z_ep_ref + P->depths[d] != 0.0)) return SDIRT_EINVAL;
        }
        const long long PP = (long long)P->F * P->D * P->L;
        if (PP > (1LL << 24)) return SDIRT_EUNSUPPORTED;
        P->P = (int)PP;
    }
    std::memset(S, 0, sizeof(*S));
    S->nx = q->rays_x;
    S->ny = q->rays_y;
    div_magic_for((uint32_t)q->rays_x, &S->div_magic, &S->div_shift);
    S->seed = q->seed;
    S->jitter = q->jitter ? 1 : 0;
    S->det = q->deterministic;
    return SDIRT_OK;
}

}  // namespace sdirt
