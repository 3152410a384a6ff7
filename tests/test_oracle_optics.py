"""Pins of the oracle's materials and first-order optics (CPU only)."""
import json
import os

import numpy as np
import pytest

from workloads import lenses
from workloads.lens import Surface, Lens, SPHERE, STOP, cauchy
from oracle import optics, trace as tr

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_cauchy_reproduces_nd_and_dispersion():
    for nd, vd in [(1.83481, 42.7), (1.53110, 55.9), (2.00100, 29.1)]:
        a, b = optics.cauchy_from_abbe(nd, vd)
        n = lambda lam: a + b / lam ** 2
        assert n(optics.LAMBDA_D) == pytest.approx(nd, abs=1e-14)
        assert (nd - 1) / (n(optics.LAMBDA_F) - n(optics.LAMBDA_C)) == pytest.approx(vd, rel=1e-12)


def test_rf50_cauchy_literals_match_conversion():
    for (nd, vd), (a, b) in lenses.RF50_CAUCHY.items():
        a2, b2 = optics.cauchy_from_abbe(nd, vd)
        assert a == pytest.approx(a2, rel=1e-15) and b == pytest.approx(b2, rel=1e-14)


def test_rf50_back_focal_distance_matches_table():
    # The printed last thickness of Table S1 is the infinity-focus sensor
    # distance; the paraxial BFD at the d line must reproduce it to the
    # printed precision.  This also pins the reading "n/V names the medium
    # after the surface".
    L = lenses.rf50()
    assert optics.bfd(L, optics.LAMBDA_D) == pytest.approx(GOLD["rf50_last_thickness_mm"]["value"], abs=0.01)
    efl = optics.efl(L, optics.LAMBDA_D)
    z_ep, r_ep = optics.entrance_pupil(L, optics.LAMBDA_D)
    fno = efl / (2 * r_ep)
    assert 1.8 <= fno < 1.9            # printed as F/1.8
    assert efl == pytest.approx(49.56, abs=0.01)


def test_rf35_back_focal_distance_matches_table():
    L = lenses.rf35()
    assert optics.bfd(L, optics.LAMBDA_D) == pytest.approx(GOLD["rf35_last_thickness_mm"]["value"], abs=0.015)
    efl = optics.efl(L, optics.LAMBDA_D)
    z_ep, r_ep = optics.entrance_pupil(L, optics.LAMBDA_D)
    assert efl / (2 * r_ep) == pytest.approx(GOLD["rf35_f_number"]["value"], abs=0.01)


def test_thick_singlet_closed_form():
    n, R1, R2, d = 1.5168, 51.5, -51.5, 5.0
    phi = (n - 1) * (1 / R1 - 1 / R2 + (n - 1) * d / (n * R1 * R2))
    f = 1 / phi
    L = lenses.singlet()
    assert optics.efl(L, 0.55) == pytest.approx(f, rel=1e-13)
    assert f == pytest.approx(50.6638, abs=1e-4)
    # principal planes: H' lies f (n-1) d / (n R1) before the rear vertex,
    # H lies -f (n-1) d / (n R2) after the front vertex
    dHp = f * (n - 1) * d / (n * R1)
    dH = -f * (n - 1) * d / (n * R2)
    assert optics.bfd(L, 0.55) == pytest.approx(f - dHp, rel=1e-13)
    for depth in (1000.0, 2000.0):
        u = depth + dH
        v = 1.0 / (1.0 / f - 1.0 / u)
        assert optics.image_distance(L, 0.55, depth) == pytest.approx(v - dHp, rel=1e-12)
    P = optics.Prepared(L)
    assert P.sensor_distance == pytest.approx(50.3035, abs=1e-4)
    assert P.stop_radius == pytest.approx(f / 4.0, rel=1e-14)   # f/2, stop = pupil


def test_real_ray_focal_length_equals_paraxial():
    # a real ray close to the axis, parallel to it, crosses the axis at the
    # paraxial focus; -h / tan(u') is the focal length to O(h^2)
    L = lenses.rf50()
    P = optics.Prepared(L)
    h = 1e-4
    o = np.array([[0.0, h, -10.0]])
    d = np.array([[0.0, 0.0, 1.0]])
    res = tr.trace(P, optics.LAMBDA_D, o, d, record=True)
    D = res["D"][0]
    assert res["status"][0] == 0
    efl_real = -h / (D[1] / D[2])
    assert efl_real == pytest.approx(optics.efl(L, optics.LAMBDA_D), rel=1e-7)


def test_entrance_pupil_is_image_of_stop():
    # a near-axis real ray from an off-axis object point aimed at the pupil
    # centre crosses the stop plane at its centre (to first order), and a
    # ray aimed at the pupil edge of a tiny stop grazes the stop edge
    L = lenses.rf50()
    P = optics.Prepared(L)
    lam = 0.55
    z_ep, r_ep = P.pupil(lam)
    for depth in (500.0, 3000.0):
        p = np.array([0.0, 0.01, -depth])
        e = np.array([0.0, 0.0, z_ep])
        d = (e - p) / np.linalg.norm(e - p)
        res = tr.trace(P, lam, e[None], d[None], record=True)
        y_stop = res["hits"][0, L.stop, 1]
        assert abs(y_stop) < 1e-7
    tiny = 1e-3
    z2, r2 = optics.entrance_pupil(L, lam, stop_radius=tiny)
    p = np.array([0.0, 0.0, -2000.0])
    e = np.array([0.0, r2, z2])
    d = (e - p) / np.linalg.norm(e - p)
    res = tr.trace(P, lam, e[None], d[None], record=True)
    assert res["hits"][0, L.stop, 1] == pytest.approx(tiny, rel=1e-5)


def test_ideal_lens_magnification_is_exact():
    L = lenses.ideal(f=50.0, sensor=52.0)
    P = optics.Prepared(L)
    for depth in (500.0, 1234.5, 5000.0):
        assert P.magnification(depth) == pytest.approx(-52.0 / depth, rel=1e-14)
    assert np.allclose(P.object_point((0.0, 0.0), 800.0), [0, 0, -800.0])


def test_f_number_resizes_stop():
    L = lenses.rf50()
    L.f_number = 4.0
    P = optics.Prepared(L)
    z, r = P.pupil(L.ref_wavelength)
    assert P.efl / (2 * r) == pytest.approx(4.0, rel=1e-13)
    assert 2 * P.stop_radius == pytest.approx(7.52, abs=0.01)


def test_phone_lens_focal_length_and_surfaces():
    from workloads.lens import ASPHERE, STOP
    L = lenses.phone_lens_16(0)
    assert optics.efl(L, 0.55) == pytest.approx(4.3, rel=1e-12)
    assert sum(1 for s in L.surfaces if s.kind != STOP) == 16
    assert sum(1 for s in L.surfaces if s.kind == ASPHERE) == 6
    P = optics.Prepared(L)
    z, r = P.pupil(0.55)
    assert P.efl / (2 * r) == pytest.approx(1.8, rel=1e-12)
    # asphere terms stay small against the base sag (Newton starts close)
    for s in L.surfaces:
        if s.kind == ASPHERE:
            rho = s.semi_diameter ** 2
            extra = sum(a * rho ** (m + 2) for m, a in enumerate(s.asph))
            base = s.c * rho / (1 + np.sqrt(1 - s.c * s.c * rho))
            assert abs(extra) <= 0.5 * abs(base) + 2e-3
