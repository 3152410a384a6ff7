"""Pins of the oracle's DP PSF estimator (CPU only)."""
import copy

import numpy as np
import pytest

from workloads import lenses
from workloads.lens import (Sensor, PsfQuery, DP_SIGMOID, DP_MICROLENS,
                            SPLAT_BOX, SPLAT_TENT, NORM_SUM, NORM_MAX)
from oracle import optics, psf, trace as tr


def _query(fields, depths, **kw):
    base = dict(wavelengths=[0.55], rays_x=48, rays_y=48, seed=0, jitter=True,
                ks=41, splat=SPLAT_BOX)
    base.update(kw)
    return PsfQuery(fields=fields, depths=depths, **base)


def _rf50_f4():
    L = lenses.rf50()
    L.f_number = 4.0
    L.focus_depth = 1000.0
    return L


@pytest.mark.parametrize("mode", [DP_SIGMOID, DP_MICROLENS])
@pytest.mark.parametrize("splat", [SPLAT_BOX, SPLAT_TENT])
def test_energy_bookkeeping(mode, splat):
    L = _rf50_f4()
    S = Sensor(pitch=0.02, dp_mode=mode)
    Q = _query([(0.0, 0.0), (3.0, 1.0)], [600.0, 1800.0], splat=splat, ks=15)
    out, st = psf.trace_dp_psf(L, S, Q)
    assert np.allclose(st[:, 0], st[:, 1] + st[:, 2], atol=1e-9)
    assert np.allclose(st[:, 2], st[:, 3] + st[:, 4] + st[:, 5] + st[:, 6], atol=1e-9)
    assert np.allclose(out[:, 0].sum(axis=(1, 2)), st[:, 3], atol=1e-9)
    assert np.allclose(out[:, 1].sum(axis=(1, 2)), st[:, 4], atol=1e-9)
    if mode == DP_MICROLENS and splat == SPLAT_BOX:
        assert np.all(out == np.round(out))
    if mode == DP_SIGMOID:
        assert np.all(st[:, 5] == 0)


@pytest.mark.parametrize("mode", [DP_SIGMOID, DP_MICROLENS])
def test_on_axis_left_right_mirror_symmetry(mode):
    L = _rf50_f4()
    S = Sensor(pitch=0.02, dp_mode=mode)
    Q = _query([(0.0, 0.0)], [600.0, 2500.0], jitter=False, rays_x=64, rays_y=64, ks=25)
    out, _ = psf.trace_dp_psf(L, S, Q)
    for q in range(out.shape[0]):
        Lp, Rp = out[q, 0], out[q, 1]
        if mode == DP_MICROLENS:
            assert np.array_equal(Lp, Rp[:, ::-1])
        else:
            assert np.allclose(Lp, Rp[:, ::-1], atol=1e-10)
        assert Lp.sum() > 0


def test_field_on_x_axis_is_row_symmetric_and_mirror_pair():
    L = _rf50_f4()
    S = Sensor(pitch=0.02, dp_mode=DP_MICROLENS)
    Q = _query([(4.0, 0.0), (-4.0, 0.0)], [700.0], jitter=False, rays_x=64, rays_y=64, ks=25)
    out, _ = psf.trace_dp_psf(L, S, Q)
    assert np.array_equal(out[0, 0], out[0, 0, ::-1, :])
    assert np.array_equal(out[0, 1], out[0, 1, ::-1, :])
    # PSF_L(-h) = flip_cols(PSF_R(h))
    assert np.array_equal(out[1, 0], out[0, 1][:, ::-1])
    assert np.array_equal(out[1, 1], out[0, 0][:, ::-1])


def test_phase_difference_flips_across_focus():
    L = _rf50_f4()
    S = Sensor(pitch=0.02, dp_mode=DP_MICROLENS)
    Q = _query([(0.0, 0.0)], [600.0, 3000.0], ks=41, rays_x=64, rays_y=64)
    out, _ = psf.trace_dp_psf(L, S, Q)
    cols = np.arange(41) - 20
    def cx(p):
        return np.sum(p.sum(axis=0) * cols) / p.sum()
    near = cx(out[0, 0]) - cx(out[0, 1])
    far = cx(out[1, 0]) - cx(out[1, 1])
    assert near * far < 0
    assert abs(near) > 0.5 and abs(far) > 0.2


def test_box_splat_equals_histogram_of_landing_points():
    L = _rf50_f4()
    S = Sensor(pitch=0.02, dp_mode=DP_SIGMOID, sigmoid_k=20.0)
    Q = _query([(2.0, -1.0)], [800.0], ks=21)
    out, st = psf.trace_dp_psf(L, S, Q)
    P = optics.Prepared(L)
    e, d = psf.bundle(P, Q, 0, 0, 0)
    res = tr.trace(P, 0.55, e, d)
    ok = res["status"] == 0
    O, D = res["O"][ok], res["D"][ok]
    sx = D[:, 0] / np.sqrt(D[:, 0] ** 2 + D[:, 2] ** 2)
    wl = 1 / (1 + np.exp(-20.0 * sx))
    edges_x = 2.0 + (np.arange(22) - 10.5) * 0.02
    edges_y = -1.0 + (np.arange(22) - 10.5) * 0.02
    H, _, _ = np.histogram2d(O[:, 1], O[:, 0], bins=[edges_y, edges_x], weights=wl)
    assert np.allclose(out[0, 0], H, atol=1e-9)


def test_tent_splat_preserves_centroid():
    L = _rf50_f4()
    S = Sensor(pitch=0.02, dp_mode=DP_SIGMOID, sigmoid_k=0.0)
    Q = _query([(0.0, 0.0)], [1100.0], ks=41, splat=SPLAT_TENT)
    out, st = psf.trace_dp_psf(L, S, Q)
    assert st[0, 6] == 0                # the whole blur is inside the window
    P = optics.Prepared(L)
    e, d = psf.bundle(P, Q, 0, 0, 0)
    res = tr.trace(P, 0.55, e, d)
    O = res["O"][res["status"] == 0]
    tot = out[0].sum(axis=0)
    j = np.arange(41) - 20
    cx = np.sum(tot.sum(axis=0) * j) / tot.sum() * 0.02
    cy = np.sum(tot.sum(axis=1) * j) / tot.sum() * 0.02
    assert cx == pytest.approx(O[:, 0].mean(), abs=1e-12)
    assert cy == pytest.approx(O[:, 1].mean(), abs=1e-12)


def test_thin_lens_coc_in_pixels():
    # aberration-free lens focused at 2 m, object at 1 m, 4 um pixels:
    # the blur disk of the landing points has the thin-lens CoC diameter
    f, N = 50.0, 2.0
    L = lenses.ideal(f=f, f_number=N, focus_depth=2000.0)
    P = optics.Prepared(L)
    Q = _query([(0.0, 0.0)], [1000.0], rays_x=128, rays_y=128, jitter=False)
    e, d = psf.bundle(P, Q, 0, 0, 0)
    O = tr.trace(P, 0.55, e, d)["O"]
    s_f = 1 / (1 / f - 1 / 2000.0)
    s_o = 1 / (1 / f - 1 / 1000.0)
    coc = (f / N) * abs(s_o - s_f) / s_o
    r = np.linalg.norm(O, axis=1)
    # outermost ring of a 128^2 grid sits at radius 1 - 1/128 of the pupil
    assert 2 * r.max() == pytest.approx(coc * (1 - 1 / 128), rel=1e-9)


@pytest.mark.parametrize("mode", [NORM_SUM, NORM_MAX])
def test_normalisation_is_joint(mode):
    L = _rf50_f4()
    S = Sensor(pitch=0.02)
    Q = _query([(1.0, 0.0)], [900.0], ks=21)
    raw, _ = psf.trace_dp_psf(L, S, Q)
    Q.normalize = mode
    nrm, _ = psf.trace_dp_psf(L, S, Q)
    s = raw[0].sum() if mode == NORM_SUM else raw[0].max()
    assert np.allclose(nrm[0], raw[0] / s, atol=1e-15)
