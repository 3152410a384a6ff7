"""The host-side first-order optics (lens validation and resolution: indices,
paraxial matrices, stop resizing, focus, entrance pupil) built with g++
under AddressSanitizer and UndefinedBehaviorSanitizer and driven over
valid, perturbed and invalid prescriptions, on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.join(os.path.dirname(__file__), "..")
CSRC = os.path.join(ROOT, "paper_2503_11213_amd", "csrc")

DRIVER = r"""
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>
#include "host_optics.hpp"

using namespace sdirt;

static uint64_t st = 88172645463325252ull;
static double uni() {                       // xorshift64 in [0, 1)
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    return (st >> 11) * (1.0 / 9007199254740992.0);
}

static sdirt_surface surf(int kind, double c, double t, double semi, double n) {
    sdirt_surface s{};
    s.kind = kind; s.c = c; s.t = t; s.semi_diameter = semi;
    s.material = SDIRT_MAT_CAUCHY; s.mat_p0 = n; s.mat_p1 = n > 1.0 ? 0.004 : 0.0;
    return s;
}

int main() {
    int ok = 0, rejected = 0;
    for (int trial = 0; trial < 4000; ++trial) {
        // a stop and 1..22 spheres / planes / aspheres, perturbed at random;
        // every 7th prescription broken in one field
        const int S = 2 + (int)(uni() * 22);
        std::vector<sdirt_surface> v;
        v.push_back(surf(SDIRT_STOP, 0.0, uni() * 3.0, 5.0 + 10.0 * uni(), 1.0));
        for (int s = 1; s < S; ++s) {
            const int kind = uni() < 0.6 ? SDIRT_SPHERE : (uni() < 0.5 ? SDIRT_PLANE : SDIRT_ASPHERE);
            const bool glass = s % 2 == 1;
            sdirt_surface x = surf(kind, (uni() - 0.5) * 0.08, 0.5 + 6.0 * uni(), 8.0 + 10.0 * uni(),
                                   glass ? 1.45 + 0.3 * uni() : 1.0);
            if (kind == SDIRT_ASPHERE) {
                x.conic = (uni() - 0.5) * 2.0;
                for (int k = 0; k < 5; ++k) x.asph[k] = (uni() - 0.5) * std::pow(10.0, -4.0 - 2.0 * k);
            }
            v.push_back(x);
        }
        v.back().t = 40.0;
        sdirt_lens L{};
        L.n_surfaces = S;
        L.stop = 0;
        L.object_material = SDIRT_MAT_CAUCHY; L.object_p0 = 1.0;
        L.f_number = uni() < 0.5 ? 1.0 + 8.0 * uni() : 0.0;
        L.focus_depth = uni() < 0.5 ? 300.0 + 5000.0 * uni() : 0.0;
        L.ref_wavelength = 0.55;
        switch (trial % 7) {
            case 1: L.stop = S + 3; break;
            case 2: v[S / 2].semi_diameter = -1.0; break;
            case 3: v[1].c = NAN; break;
            case 4: L.n_surfaces = 0; break;
            case 5: L.n_surfaces = SDIRT_MAX_SURFACES + 1; break;
            case 6: L.ref_wavelength = 0.0; break;
            default: break;
        }
        L.surfaces = v.data();
        Resolved R;
        if (resolve_lens(&L, &R) != SDIRT_OK) { ++rejected; continue; }
        for (double lam : {0.45, 0.55, 0.65}) {
            double z = 0, r = 0;
            R.pupil(lam, &z, &r);
            double M[4];
            R.system_matrix(lam, R.S, M);
            (void)z; (void)r; (void)M;
        }
        ++ok;
    }
    std::printf("resolved %d rejected %d\n", ok, rejected);
    return ok > 100 && rejected > 500 ? 0 : 1;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_host_optics_under_asan_ubsan(tmp_path):
    drv = tmp_path / "driver.cpp"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
           str(drv), os.path.join(CSRC, "host_optics.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, (run.stdout + run.stderr)[-3000:]
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
