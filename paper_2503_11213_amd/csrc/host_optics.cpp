// First-order (paraxial) optics on the host, float64.  See host_optics.hpp.
#include "host_optics.hpp"

#include <cmath>

namespace sdirt {

namespace {

constexpr double kLambdaF = 0.4861327;   // um, hydrogen F line
constexpr double kLambdaD = 0.5875618;   // um, helium d line
constexpr double kLambdaC = 0.6562725;   // um, hydrogen C line

bool finite(double v) { return std::isfinite(v); }

// Two-term Cauchy medium from a material descriptor.
bool cauchy_of(int kind, double p0, double p1, double* a, double* b) {
    if (!finite(p0) || !finite(p1)) return false;
    if (kind == SDIRT_MAT_CAUCHY) {
        *a = p0;
        *b = p1;
    } else if (kind == SDIRT_MAT_ABBE) {
        if (!(p1 > 0.0)) return false;
        // n_F - n_C = (n_d - 1) / V_d and n(lambda_d) = n_d.
        const double inv_f2 = 1.0 / (kLambdaF * kLambdaF);
        const double inv_c2 = 1.0 / (kLambdaC * kLambdaC);
        *b = (p0 - 1.0) / (p1 * (inv_f2 - inv_c2));
        *a = p0 - *b / (kLambdaD * kLambdaD);
    } else {
        return false;
    }
    return true;
}

void mat_mul(const double A[4], const double B[4], double out[4]) {
    double r[4] = {A[0] * B[0] + A[1] * B[2], A[0] * B[1] + A[1] * B[3],
                   A[2] * B[0] + A[3] * B[2], A[2] * B[1] + A[3] * B[3]};
    for (int i = 0; i < 4; ++i) out[i] = r[i];
}

}  // namespace

double Resolved::index(int medium, double lambda) const {
    return mat_a[medium] + mat_b[medium] / (lambda * lambda);
}

// Paraxial power of surface s between media s and s+1.
static double power_of(const Resolved& R, int s, double lambda) {
    if (R.kind[s] == SDIRT_SPHERE || R.kind[s] == SDIRT_ASPHERE)
        return (R.index(s + 1, lambda) - R.index(s, lambda)) * R.c[s];
    if (R.kind[s] == SDIRT_IDEAL) return 1.0 / R.focal[s];
    return 0.0;
}

void Resolved::system_matrix(double lambda, int upto, double M[4]) const {
    M[0] = 1; M[1] = 0; M[2] = 0; M[3] = 1;
    for (int s = 0; s < upto; ++s) {
        const double refr[4] = {1.0, 0.0, -power_of(*this, s, lambda), 1.0};
        mat_mul(refr, M, M);
        const double tt = (s == S - 1) ? sensor_distance : t[s];
        const double tran[4] = {1.0, tt / index(s + 1, lambda), 0.0, 1.0};
        mat_mul(tran, M, M);
    }
}

void Resolved::pupil(double lambda, double* z_ep, double* rho_ep) const {
    // A ray from the axial point z_ep reaches the centre of the stop plane
    // iff A (-z_ep u) + B n0 u = 0, so z_ep = B n0 / A; the pupil height
    // maps to the stop height with magnification A.
    double M[4];
    system_matrix(lambda, stop, M);
    *z_ep = M[1] * index(0, lambda) / M[0];
    *rho_ep = stop_radius / std::fabs(M[0]);
}

int resolve_lens(const sdirt_lens* lens, Resolved* R) {
    if (!lens || !lens->surfaces || !R) return SDIRT_EINVAL;
    const int S = lens->n_surfaces;
    if (S < 1 || S > SDIRT_MAX_SURFACES) return SDIRT_EINVAL;
    if (lens->stop < 0 || lens->stop >= S) return SDIRT_EINVAL;
    if (!finite(lens->f_number) || lens->f_number < 0) return SDIRT_EINVAL;
    if (!finite(lens->focus_depth) || lens->focus_depth < 0) return SDIRT_EINVAL;
    if (!finite(lens->ref_wavelength) || !(lens->ref_wavelength > 0)) return SDIRT_EINVAL;
    R->S = S;
    R->stop = lens->stop;
    R->ref_lambda = lens->ref_wavelength;
    R->kind.assign(S, 0); R->c.assign(S, 0); R->t.assign(S, 0);
    R->semi.assign(S, 0); R->conic.assign(S, 0); R->focal.assign(S, 0);
    R->asph.assign(5 * S, 0);
    R->mat_kind.assign(S + 1, 0); R->mat_a.assign(S + 1, 1.0); R->mat_b.assign(S + 1, 0.0);
    double a, b;
    if (!cauchy_of(lens->object_material, lens->object_p0, lens->object_p1, &a, &b))
        return SDIRT_EINVAL;
    R->mat_a[0] = a; R->mat_b[0] = b;
    for (int s = 0; s < S; ++s) {
        const sdirt_surface& q = lens->surfaces[s];
        if (q.kind < SDIRT_SPHERE || q.kind > SDIRT_IDEAL) return SDIRT_EINVAL;
        if (!finite(q.c) || !finite(q.t) || !finite(q.semi_diameter) ||
            !finite(q.conic) || !finite(q.focal)) return SDIRT_EINVAL;
        for (int m = 0; m < 5; ++m) if (!finite(q.asph[m])) return SDIRT_EINVAL;
        if (!(q.semi_diameter > 0)) return SDIRT_EINVAL;
        if (!cauchy_of(q.material, q.mat_p0, q.mat_p1, &a, &b)) return SDIRT_EINVAL;
        R->mat_a[s + 1] = a; R->mat_b[s + 1] = b;
        R->kind[s] = q.kind;
        R->c[s] = (q.kind == SDIRT_SPHERE || q.kind == SDIRT_ASPHERE) ? q.c : 0.0;
        R->t[s] = q.t;
        R->semi[s] = q.semi_diameter;
        R->conic[s] = q.kind == SDIRT_ASPHERE ? q.conic : 0.0;
        for (int m = 0; m < 5; ++m) R->asph[5 * s + m] = q.kind == SDIRT_ASPHERE ? q.asph[m] : 0.0;
        if (q.kind == SDIRT_IDEAL) {
            if (q.focal == 0.0) return SDIRT_EINVAL;
            R->focal[s] = q.focal;
        }
        if (q.kind == SDIRT_STOP &&
            (R->mat_a[s + 1] != R->mat_a[s] || R->mat_b[s + 1] != R->mat_b[s]))
            return SDIRT_EINVAL;   // an aperture does not change the medium
        if (q.kind == SDIRT_ASPHERE) {
            // the base conic must have a real sag over the clear aperture
            const double rho = q.semi_diameter * q.semi_diameter;
            if (1.0 - (1.0 + q.conic) * q.c * q.c * rho < 0.0) return SDIRT_EINVAL;
        }
    }
    // indices must be positive at the reference wavelength
    for (int m = 0; m <= S; ++m)
        if (!(R->index(m, R->ref_lambda) > 0)) return SDIRT_EINVAL;

    const double lr = R->ref_lambda;
    // effective focal length from the vertex-to-vertex matrix
    R->sensor_distance = R->t[S - 1];
    double M[4] = {1, 0, 0, 1};
    for (int s = 0; s < S; ++s) {
        const double refr[4] = {1.0, 0.0, -power_of(*R, s, lr), 1.0};
        mat_mul(refr, M, M);
        if (s < S - 1) {
            const double tran[4] = {1.0, R->t[s] / R->index(s + 1, lr), 0.0, 1.0};
            mat_mul(tran, M, M);
        }
    }
    const double n_img = R->index(S, lr);
    R->efl = (M[2] != 0.0) ? -n_img / M[2] : INFINITY;
    // image distance after the last vertex: -y n' / (n' u')
    R->bfd = (M[2] != 0.0) ? -M[0] * n_img / M[2] : INFINITY;
    if (lens->focus_depth > 0) {
        const double y = M[0] * lens->focus_depth + M[1] * R->index(0, lr);
        const double w = M[2] * lens->focus_depth + M[3] * R->index(0, lr);
        if (w == 0.0) return SDIRT_EINVAL;
        R->sensor_distance = -y * n_img / w;
    }
    if (!finite(R->sensor_distance) || !(R->sensor_distance > 0)) return SDIRT_EINVAL;
    // stop: resized so the entrance pupil diameter is EFL / N
    R->stop_radius = R->semi[R->stop];
    if (lens->f_number > 0) {
        if (!finite(R->efl)) return SDIRT_EINVAL;
        double Ms[4];
        R->system_matrix(lr, R->stop, Ms);
        R->stop_radius = R->efl / (2.0 * lens->f_number) * std::fabs(Ms[0]);
        R->semi[R->stop] = R->stop_radius;
    }
    R->pupil(lr, &R->z_ep_ref, &R->rho_ep_ref);
    // chief ray from (y_o, -d) toward the pupil centre reaches the sensor at
    // y_o (A z_ep - B n0) / (z_ep + d)
    double Mf[4];
    R->system_matrix(lr, S, Mf);
    R->m_num = Mf[0] * R->z_ep_ref - Mf[1] * R->index(0, lr);
    double z = 0;
    for (int s = 0; s < S - 1; ++s) z += R->t[s];
    R->sensor_z = z + R->sensor_distance;
    if (!finite(R->z_ep_ref) || !finite(R->rho_ep_ref) || !finite(R->m_num))
        return SDIRT_EINVAL;
    return SDIRT_OK;
}

}  // namespace sdirt
