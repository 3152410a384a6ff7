"""Pins of the oracle's finite-difference gradients (CPU only)."""
import copy

import numpy as np
import pytest

from workloads import lenses
from workloads.lens import Sensor, PsfQuery, SPLAT_TENT, DP_SIGMOID
from oracle import adjoint as A, optics, psf, trace as tr


def _setup(lens=None, ks=21, rays=24):
    if lens is None:
        lens = lenses.rf50()
        lens.f_number = 4.0
        lens.focus_depth = 1000.0
    S = Sensor(pitch=0.02, dp_mode=DP_SIGMOID, sigmoid_k=20.0)
    Q = PsfQuery(fields=[(0.0, 0.0), (3.0, 0.5)], depths=[700.0, 1400.0],
                 wavelengths=[0.5, 0.62], rays_x=rays, rays_y=rays, seed=0,
                 jitter=True, ks=ks, splat=SPLAT_TENT)
    est = A.FrozenEstimator(lens, S, Q)
    G = np.random.default_rng(11).normal(size=(Q.n_points, 2, ks, ks))
    return est, G


def _tent_grad(est, G, dO_fn, dwl_fn):
    """<G, dPSF> from per-ray landing-point derivatives dO (n, 2) and left
    weight derivatives dwl (n,), through the analytic tent and sigmoid."""
    q = est.query
    ps = est.sensor.pitch
    pad = (q.ks - 1) // 2
    total = 0.0
    prep = est.prep
    for idx, ((f, d, l), (e, dirs)) in enumerate(zip(est.points, est.bundles)):
        res = tr.trace(prep, q.wavelengths[l], e, dirs)
        O, D = res["O"], res["D"]
        sx = D[:, 0] / np.sqrt(D[:, 0] ** 2 + D[:, 2] ** 2)
        wl = 1 / (1 + np.exp(-est.sensor.sigmoid_k * sx))
        w = [wl, 1 - wl]
        dO = dO_fn(idx, e, dirs, O, D)
        dwl = dwl_fn(idx, e, dirs, O, D, sx, wl)
        dw = [dwl, -dwl]
        h = q.fields[f]
        u = (O[:, 0] - h[0]) / ps + pad
        v = (O[:, 1] - h[1]) / ps + pad
        du, dv = dO[:, 0] / ps, dO[:, 1] / ps
        j0 = np.floor(u).astype(int); i0 = np.floor(v).astype(int)
        fx, fy = u - j0, v - i0
        taps = [(0, 0, (1 - fy) * (1 - fx), -(1 - fy), -(1 - fx)),
                (0, 1, (1 - fy) * fx, (1 - fy), -fx),
                (1, 0, fy * (1 - fx), -fy, (1 - fx)),
                (1, 1, fy * fx, fy, fx)]
        for (di_, dj_, wt, dwt_du, dwt_dv) in taps:
            ii, jj = i0 + di_, j0 + dj_
            inw = (ii >= 0) & (ii < q.ks) & (jj >= 0) & (jj < q.ks)
            for s in range(2):
                g = np.zeros(len(u))
                g[inw] = G[idx, s, ii[inw], jj[inw]]
                total += np.sum(g * (w[s] * (dwt_du * du + dwt_dv * dv) + dw[s] * wt))
    return total


def test_slope_gradient_closed_form():
    est, G = _setup()
    k = est.sensor.sigmoid_k
    fd = est.fd_gradient(G, rel_step=1e-6, params=[len(est.theta0) - 1])[-1]
    zero = lambda idx, e, d, O, D: np.zeros((len(e), 2))
    ana = _tent_grad(est, G, zero, lambda idx, e, d, O, D, sx, wl: wl * (1 - wl) * sx)
    assert fd == pytest.approx(ana, rel=1e-7)


def test_sensor_distance_gradient_closed_form():
    est, G = _setup()
    p = A.PER_SURFACE * (est.prep.S - 1) + 1      # last thickness = sensor distance
    fd = est.fd_gradient(G, rel_step=1e-7, params=[p])[p]
    slope = lambda idx, e, d, O, D: np.stack([D[:, 0] / D[:, 2], D[:, 1] / D[:, 2]], 1)
    ana = _tent_grad(est, G, slope, lambda *a: np.zeros(len(a[1])))
    assert fd == pytest.approx(ana, rel=1e-6)


@pytest.mark.parametrize("which", ["c3", "t5", "a4_9", "c10"])
def test_fd_matches_per_ray_chain_rule(which):
    est, G = _setup()
    name, s = which.split("_") if "_" in which else (which[0], which[1:])
    s = int(s)
    off = {"c": 0, "t": 1, "a4": 3}[name]
    p = A.PER_SURFACE * s + off
    th0 = est.theta0
    h = 1e-6 * max(abs(th0[p]), {"c": 1e-3, "t": 1.0, "a4": 1e-6}[name])
    fd = est.fd_gradient(G, rel_step=1e-6, params=[p],
                         scale=np.full(len(th0), {"c": 1e-3, "t": 1.0, "a4": 1e-6}[name]))[p]
    cache = {}

    def per_ray(idx, e, d):
        if idx not in cache:
            lam = est.query.wavelengths[est.points[idx][2]]
            outs = []
            for sgn in (1, -1):
                th = th0.copy(); th[p] += sgn * h
                prep, _ = A.with_theta(est.prep, est.sensor, th)
                r = tr.trace(prep, lam, e, d)
                outs.append((r["O"], r["D"]))
            cache[idx] = outs
        return cache[idx]

    def dO(idx, e, d, O, D):
        (Op, _), (Om, _) = per_ray(idx, e, d)
        return (Op - Om) / (2 * h)

    def dwl(idx, e, d, O, D, sx, wl):
        (_, Dp), (_, Dm) = per_ray(idx, e, d)
        k = est.sensor.sigmoid_k
        def w(D):
            return 1 / (1 + np.exp(-k * D[:, 0] / np.sqrt(D[:, 0] ** 2 + D[:, 2] ** 2)))
        return (w(Dp) - w(Dm)) / (2 * h)

    ana = _tent_grad(est, G, dO, dwl)
    # the two differ only by rays whose tent weights cross a pixel-centre kink
    assert fd == pytest.approx(ana, rel=2e-3, abs=1e-6 * abs(ana) + 1e-9)


def test_fd_error_shrinks_quadratically_for_smooth_parameter():
    est, G = _setup()
    p = len(est.theta0) - 1
    exact = est.fd_gradient(G, rel_step=1e-6, params=[p])[p]
    errs = [abs(est.fd_gradient(G, rel_step=r, params=[p])[p] - exact) for r in (4e-2, 2e-2)]
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.1)


def test_per_ray_differences_equal_psf_level_difference():
    # the per-ray form (smooth central differences of landing points plus
    # the tent / response derivatives) is the kink-free limit of the
    # PSF-level central difference
    est, G = _setup()
    for p in (8 * 2 + 0, 8 * 6 + 1, 8 * 8 + 3, len(est.theta0) - 1):
        sens = est.landing_sensitivity(p, 1e-7 * max(abs(est.theta0[p]), 1e-3))
        if p == len(est.theta0) - 1:
            a = est.ray_fd_gradient(G, p, 1.0)
            c = est.fd_gradient_at(G, p, 1e-6 * abs(est.theta0[p]))
        else:
            a = est.ray_fd_gradient(G, p, 1e-6 / sens)
            c = est.fd_gradient_at(G, p, 2e-9 / sens)
        assert c == pytest.approx(a, rel=1e-4)
