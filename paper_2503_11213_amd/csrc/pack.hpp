// Packing of host-resolved lens / wavelength / query data into the kernel
// argument structs, and query validation.
#pragma once

#include <cstring>
#include <vector>

#include "device_common.hpp"
#include "host_optics.hpp"

namespace sdirt {

constexpr int kMaxF = SDIRT_MAX_FIELDS;
constexpr int kMaxD = SDIRT_MAX_DEPTHS;

struct PointArgs {
    int P;
    int F, D, L;                 // grid mode (points == nullptr)
    double fields[kMaxF][2];
    double depths[kMaxD];
    const double* points;        // list mode: device [P][4]
    double m_num, z_ep_ref;      // chief-ray magnification constants
    const int* mask;             // device [P] or nullptr: trace only points with mask != 0
};

struct SampleArgs {
    int nx, ny;
    uint32_t seed;
    int jitter;
    int chunks;
    int rays_per_chunk;
    uint64_t div_magic;              // r / nx == (r * div_magic) >> div_shift
    uint32_t div_shift;
    int det;                         // fixed-point tiles, one workgroup per point
    // tile order (nx, ny multiples of 8 and chunks of whole 64-ray tiles):
    // ray r takes cell (8 (t mod nx/8) + r mod 8, 8 (t div nx/8) + (r div 8)
    // mod 8) of the pupil grid, t = r div 64, so a wave's 64 rays sample one
    // 8 x 8 patch of the pupil instead of a 64-cell stretch of one row
    int tile8;
    uint32_t tdiv_shift;             // t / (nx / 8) == (t * tdiv_magic) >> tdiv_shift
    uint64_t tdiv_magic;
};

// Multiplier and shift for exact unsigned division by d of every n < 2^30.
void div_magic_for(uint32_t d, uint64_t* magic, uint32_t* shift);

struct SensorArgs {
    int ks;
    int dp_mode;
    double ps;
    double sig_k;
    double ml_h, ml_f, ml_w, ml_r;   // mm
};

int pack_lens(const Resolved& R, LensArgs* out);
int pack_lambdas(const Resolved& R, const double* lambdas, int L, LambdaArgs* out);
int check_sensor(const sdirt_sensor* s, int ks, SensorArgs* out);
int check_query(const sdirt_psf_query* q, const Resolved& R, PointArgs* pts,
                SampleArgs* smp);

}  // namespace sdirt
