"""Pins of the oracle's real-ray trace (CPU only)."""
import copy

import mpmath
import numpy as np
import pytest

from workloads import lenses
from workloads.lens import Surface, Lens, SPHERE, STOP, PLANE, ASPHERE, IDEAL, cauchy, air
from oracle import optics, trace as tr


def _rays(n, rng, z0=-5.0, spread=0.05, r=3.0):
    o = np.zeros((n, 3))
    o[:, 0] = rng.uniform(-r, r, n)
    o[:, 1] = rng.uniform(-r, r, n)
    o[:, 2] = z0
    d = np.zeros((n, 3))
    d[:, 0] = rng.uniform(-spread, spread, n)
    d[:, 1] = rng.uniform(-spread, spread, n)
    d[:, 2] = 1.0
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o, d


def test_plate_lateral_shift_closed_form():
    n, t = 1.6, 5.0
    Lp = lenses.plate(thickness=t, n=n)
    La = lenses.plate(thickness=t, n=1.0)
    Pp, Pa = optics.Prepared(Lp), optics.Prepared(La)
    for theta in (0.05, 0.2, 0.4):
        o = np.array([[0.0, 0.0, 0.0]])
        d = np.array([[np.sin(theta), 0.0, np.cos(theta)]])
        xp = tr.trace(Pp, 0.55, o, d)["O"][0, 0]
        xa = tr.trace(Pa, 0.55, o, d)["O"][0, 0]
        shift = (xa - xp) * np.cos(theta)
        expect = t * np.sin(theta) * (1 - np.cos(theta) / np.sqrt(n * n - np.sin(theta) ** 2))
        assert shift == pytest.approx(expect, rel=1e-12)


def test_ray_through_centre_of_curvature_is_undeviated():
    R = 30.0
    L = Lens(surfaces=[Surface(kind=STOP, c=0, t=1.0, semi_diameter=10.0),
                       Surface(kind=SPHERE, c=1 / R, t=10.0, semi_diameter=10.0,
                               medium=cauchy(1.7, 0.0))], stop=0)
    P = optics.Prepared(L)
    rng = np.random.default_rng(1)
    for _ in range(5):
        e = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), 0.0])
        centre = np.array([0.0, 0.0, 1.0 + R])
        d = (centre - e) / np.linalg.norm(centre - e)
        res = tr.trace(P, 0.55, e[None], d[None], record=True)
        assert np.allclose(res["hits"][0, 1, 3:], d, atol=1e-14)


def _normal(surf, x, y, z):
    if surf.kind == SPHERE:
        return np.stack([-surf.c * x, -surf.c * y, 1 - surf.c * z], axis=1)
    _, ds, _ = tr.asphere_sag(surf, x * x + y * y)
    N = np.stack([-2 * x * ds, -2 * y * ds, np.ones_like(x)], axis=1)
    return N / np.linalg.norm(N, axis=1, keepdims=True)


def test_snell_invariant_and_unit_directions_rf50():
    L = lenses.rf50()
    P = optics.Prepared(L)
    lam = 0.55
    n = optics.indices(L, lam)
    z_ep, r_ep = P.pupil(lam)
    rng = np.random.default_rng(3)
    m = 500
    e = np.stack([rng.uniform(-1, 1, m) * r_ep * 0.7, rng.uniform(-1, 1, m) * r_ep * 0.7,
                  np.full(m, z_ep)], axis=1)
    p = np.array([20.0, -10.0, -1500.0])
    d = (e - p) / np.linalg.norm(e - p, axis=1, keepdims=True)
    res = tr.trace(P, lam, e, d, record=True)
    ok = res["status"] == 0
    assert ok.mean() > 0.9
    hits = res["hits"][ok]
    d_in = d[ok]
    for s, surf in enumerate(L.surfaces):
        d_out = hits[:, s, 3:]
        assert np.allclose(np.linalg.norm(d_out, axis=1), 1.0, atol=1e-14)
        if surf.kind in (SPHERE, ASPHERE):
            N = _normal(surf, hits[:, s, 0], hits[:, s, 1], hits[:, s, 2])
            lhs = n[s] * np.cross(d_in, N)
            rhs = n[s + 1] * np.cross(d_out, N)
            assert np.allclose(lhs, rhs, atol=1e-13)
        d_in = d_out


def test_asphere_hits_are_roots_in_high_precision():
    L = lenses.rf50()
    P = optics.Prepared(L)
    lam = 0.55
    z_ep, r_ep = P.pupil(lam)
    rng = np.random.default_rng(5)
    m = 40
    ang = rng.uniform(0, 2 * np.pi, m)
    rad = r_ep * np.sqrt(rng.uniform(0, 0.8, m))
    e = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.full(m, z_ep)], axis=1)
    p = np.array([5.0, 0.0, -1000.0])
    d = (e - p) / np.linalg.norm(e - p, axis=1, keepdims=True)
    res = tr.trace(P, lam, e, d, record=True)
    mpmath.mp.dps = 50
    for s in (8, 9):
        surf = L.surfaces[s]
        a4, a6, a8, a10, a12 = [mpmath.mpf(v) for v in surf.asph]
        c = mpmath.mpf(surf.c)
        for k in np.nonzero(res["status"] == 0)[0]:
            x, y, z = [mpmath.mpf(float(v)) for v in res["hits"][k, s, :3]]
            rho = x * x + y * y
            sag = c * rho / (1 + mpmath.sqrt(1 - c * c * rho)) + \
                a4 * rho ** 2 + a6 * rho ** 3 + a8 * rho ** 4 + a10 * rho ** 5 + a12 * rho ** 6
            assert abs(float(z - sag)) < 1e-12


def _reversed(L, P):
    """Mirror image z -> -z of the lens traced backwards."""
    S = len(L.surfaces)
    media = [L.object_medium] + [s.medium for s in L.surfaces]
    out = []
    for k in range(S):
        s = L.surfaces[S - 1 - k]
        t_next = P.thickness[S - 2 - k] if k < S - 1 else 10.0
        out.append(Surface(kind=s.kind, c=-s.c, t=t_next, semi_diameter=1e3,
                           medium=media[S - 1 - k], conic=s.conic,
                           asph=tuple(-a for a in s.asph), focal=s.focal))
    return Lens(surfaces=out, stop=0, object_medium=L.surfaces[-1].medium)


def test_trace_is_reversible():
    L = lenses.rf50()
    P = optics.Prepared(L)
    lam = 0.6
    rng = np.random.default_rng(7)
    o, d = _rays(200, rng, z0=-5.0, spread=0.08, r=6.0)
    res = tr.trace(P, lam, o, d, record=True)
    ok = res["status"] == 0
    S = P.S
    Lr = _reversed(L, P)
    Pr = optics.Prepared(Lr)
    last = res["hits"][ok, S - 1]
    # reversed ray in the mirrored frame, starting at the last hit
    o2 = np.stack([last[:, 0], last[:, 1], -last[:, 2]], axis=1)
    d2 = np.stack([-last[:, 3], -last[:, 4], last[:, 5]], axis=1)
    back = tr.trace(Pr, lam, o2, d2, record=True)
    assert np.all(back["status"] == 0)
    first = back["hits"][:, S - 1]
    assert np.allclose(first[:, 0], res["hits"][ok, 0, 0], atol=1e-11)
    assert np.allclose(first[:, 1], res["hits"][ok, 0, 1], atol=1e-11)
    # direction before surface 1 (mirrored back)
    assert np.allclose(-first[:, 3], d[ok, 0], atol=1e-12)
    assert np.allclose(-first[:, 4], d[ok, 1], atol=1e-12)


def test_ideal_lens_images_points_exactly():
    f, depth = 50.0, 1200.0
    s_img = 1.0 / (1.0 / f - 1.0 / depth)
    L = lenses.ideal(f=f, stop_radius=12.0, sensor=s_img)
    P = optics.Prepared(L)
    rng = np.random.default_rng(0)
    for yo in (0.0, 30.0):
        p = np.array([0.0, yo, -depth])
        ang = rng.uniform(0, 2 * np.pi, 300)
        rad = 12.0 * np.sqrt(rng.uniform(0, 1, 300))
        e = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.zeros(300)], axis=1)
        d = (e - p) / np.linalg.norm(e - p, axis=1, keepdims=True)
        O = tr.trace(P, 0.55, e, d)["O"]
        assert np.allclose(O[:, 0], 0.0, atol=1e-12)
        assert np.allclose(O[:, 1], -yo * s_img / depth, atol=1e-11)


def test_thin_lens_circle_of_confusion():
    # config-1 geometry on an aberration-free lens: focus 2 m, object 1 m
    f, rho = 50.0, 12.5
    s_f = 1 / (1 / f - 1 / 2000.0)
    s_o = 1 / (1 / f - 1 / 1000.0)
    L = lenses.ideal(f=f, stop_radius=rho, sensor=s_f)
    P = optics.Prepared(L)
    ang = np.linspace(0, 2 * np.pi, 721)
    e = np.stack([rho * np.cos(ang), rho * np.sin(ang), np.zeros_like(ang)], axis=1)
    p = np.array([0.0, 0.0, -1000.0])
    d = (e - p) / np.linalg.norm(e - p, axis=1, keepdims=True)
    O = tr.trace(P, 0.55, e, d)["O"]
    diam = 2 * np.max(np.linalg.norm(O, axis=1))
    coc = 2 * rho * abs(s_o - s_f) / s_o
    assert diam == pytest.approx(coc, rel=1e-12)
