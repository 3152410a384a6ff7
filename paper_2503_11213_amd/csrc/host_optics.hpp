// Host-side first-order optics and argument packing for the DP PSF engine.
// Resolves what the trace needs before any device work: refractive indices
// per wavelength, the stop radius (F-number), the sensor distance (focus),
// the entrance pupil per wavelength (Sec. 3.1: rays aim at samples of the
// image of the stop in object space) and the chief-ray magnification that
// maps an image-plane field point to its object point.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/sdirt.h"

namespace sdirt {

struct Resolved {
    int S = 0, stop = 0;
    std::vector<int> kind;
    std::vector<double> c, t, semi, conic, focal;
    std::vector<double> asph;       // S * 5
    std::vector<int> mat_kind;      // S + 1 media: [0] object side
    std::vector<double> mat_a, mat_b;  // Cauchy A, B of each medium
    double ref_lambda = 0.55;
    double efl = 0, bfd = 0;
    double sensor_distance = 0, stop_radius = 0;
    double z_ep_ref = 0, rho_ep_ref = 0, m_num = 0, sensor_z = 0;

    double index(int medium, double lambda) const;
    // 2x2 matrix on (y, n u) from vertex plane 0 to vertex plane `upto`
    // (before its refraction); upto == S -> sensor plane.
    void system_matrix(double lambda, int upto, double M[4]) const;
    void pupil(double lambda, double* z_ep, double* rho_ep) const;
};

// Validates and resolves a lens; returns SDIRT_OK or SDIRT_EINVAL.
int resolve_lens(const sdirt_lens* lens, Resolved* out);

}  // namespace sdirt
