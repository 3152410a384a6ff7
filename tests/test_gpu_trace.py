"""GPU parity of the ray tracer and the DP PSF estimator against the CPU
oracle (float64), through the C ABI."""
import copy

import numpy as np
import pytest
import torch

from workloads import lenses, configs
from workloads.lens import (Sensor, PsfQuery, Surface, Lens, SPHERE, PLANE, STOP, cauchy,
                            DP_SIGMOID, DP_MICROLENS, SPLAT_BOX, SPLAT_TENT, NORM_SUM,
                            NORM_MAX)
from oracle import optics, psf as opsf, trace as otr
from paper_2503_11213_amd import sdirt, _abi as abi

pytestmark = pytest.mark.gpu

L1_TOL = 1e-3          # energy L1 for identical seeded rays
HIT_TOL = 1e-5         # relative, floor 1 mm


def _rf50_f4():
    L = lenses.rf50()
    L.f_number = 4.0
    L.focus_depth = 1000.0
    return L


def _energy_l1(g, r):
    return np.abs(g - r).sum() / max(np.abs(r).sum(), 1e-300)


def _rays(lens, query, points):
    P = optics.Prepared(lens)
    o, d, lam = [], [], []
    for (f, dd, l) in points:
        e, dirs = opsf.bundle(P, query, f, dd, l)
        o.append(e); d.append(dirs); lam.append(query.wavelengths[l])
    return P, o, d, lam


@pytest.mark.parametrize("which", ["config1", "config2", "rf50_f4"])
def test_trace_rays_hits_match_oracle(which):
    if which == "config1":
        lens, sensor, query = configs.config1()
    elif which == "config2":
        lens, sensor, query = configs.config2(rays=48)
    else:
        lens = _rf50_f4()
        query = PsfQuery(fields=[(0, 0), (10.0, 6.0)], depths=[600.0, 4000.0],
                         wavelengths=[0.55], rays_x=48, rays_y=48, ks=21)
    pts = [(0, 0, 0), (len(query.fields) - 1, len(query.depths) - 1, len(query.wavelengths) - 1)]
    P, os_, ds, lams = _rays(lens, query, pts)
    for o, d, lam in zip(os_, ds, lams):
        ref = otr.trace(P, lam, o, d, record=True)
        hits, st = sdirt.trace_rays(lens, lam, torch.from_numpy(o).cuda(),
                                    torch.from_numpy(d).cuda())
        torch.cuda.synchronize()
        hits, st = hits.cpu().numpy(), st.cpu().numpy()
        assert np.array_equal(st, ref["status"])
        ok = st == 0
        assert ok.mean() > 0.5
        h, r = hits[ok], ref["hits"][ok]
        err = np.abs(h - r) / np.maximum(np.abs(r), 1.0)
        assert err.max() <= HIT_TOL, err.max()


def test_trace_rays_f32_mode_error_budget():
    # the float32 trace is a fast mode; its error on the 12-surface lens is
    # measured here (not the parity path)
    lens, sensor, query = configs.config2(rays=48)
    P, os_, ds, lams = _rays(lens, query, [(10, 5, 1)])
    ref = otr.trace(P, lams[0], os_[0], ds[0], record=True)
    hits, st = sdirt.trace_rays(lens, lams[0], torch.from_numpy(os_[0]).cuda(),
                                torch.from_numpy(ds[0]).cuda(), math=abi.F32)
    hits = hits.cpu().numpy()
    ok = ref["status"] == 0
    err = np.abs(hits[ok] - ref["hits"][ok]) / np.maximum(np.abs(ref["hits"][ok]), 1.0)
    print("float32 trace max rel err", err.max())
    assert err.max() < 2e-4


def test_config1_psf_and_stats_match_oracle():
    lens, sensor, query = configs.config1()
    psf, st = sdirt.trace_dp_psf(lens, sensor, query)
    torch.cuda.synchronize()
    ref, rst = opsf.trace_dp_psf(lens, sensor, query)
    g, gs = psf.cpu().numpy(), st.cpu().numpy()
    assert psf.dtype == torch.float64
    assert _energy_l1(g, ref) <= L1_TOL
    assert np.array_equal(gs[:, :3], rst[:, :3])
    assert np.allclose(gs[:, 3:], rst[:, 3:], rtol=1e-5, atol=1e-2)


@pytest.mark.parametrize("mode", [DP_SIGMOID, DP_MICROLENS])
@pytest.mark.parametrize("splat", [SPLAT_BOX, SPLAT_TENT])
def test_modes_on_aspheric_lens_match_oracle(mode, splat):
    lens = _rf50_f4()
    sensor = Sensor(pitch=0.01, dp_mode=mode, sigmoid_k=20.0)
    query = PsfQuery(fields=[(0.0, 0.0), (8.0, 3.0), (-12.0, -7.5)], depths=[550.0, 1000.0, 9000.0],
                     wavelengths=[0.5, 0.62], rays_x=80, rays_y=72, seed=3, jitter=True,
                     ks=45, splat=splat)
    psf, st = sdirt.trace_dp_psf(lens, sensor, query)
    torch.cuda.synchronize()
    ref, rst = opsf.trace_dp_psf(lens, sensor, query)
    g, gs = psf.cpu().numpy(), st.cpu().numpy()
    for q in range(ref.shape[0]):
        if ref[q].sum() > 0:
            assert _energy_l1(g[q], ref[q]) <= L1_TOL, q
    assert np.array_equal(gs[:, :3], rst[:, :3])
    assert np.allclose(gs[:, 3:], rst[:, 3:], rtol=1e-5, atol=0.05)
    assert np.allclose(gs[:, 0], gs[:, 1] + gs[:, 2])
    assert np.allclose(gs[:, 2], gs[:, 3:].sum(axis=1), rtol=1e-6)


def test_config2_grid_at_reduced_rays_matches_oracle():
    lens, sensor, query = configs.config2(rays=40)
    psf, st = sdirt.trace_dp_psf(lens, sensor, query)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    picks = [(int(rng.integers(32)), int(rng.integers(16)), int(rng.integers(3))) for _ in range(24)]
    ref, rst = opsf.trace_dp_psf(lens, sensor, query, points=picks)
    g, gs = psf.cpu().numpy(), st.cpu().numpy()
    for (f, d, l) in picks:
        q = opsf.point_index(f, d, l, 16, 3)
        if ref[q].sum() > 0:
            assert _energy_l1(g[q], ref[q]) <= L1_TOL, (f, d, l)
        assert np.array_equal(gs[q, :3], rst[q, :3])


def test_config2_full_size_sampled_points():
    # the benchmarked launch: 1536 points x 512^2 rays, ks 63, float32 out
    lens, sensor, query = configs.config2()
    psf, st = sdirt.trace_dp_psf(lens, sensor, query)
    torch.cuda.synchronize()
    picks = [(0, 0, 1), (17, 9, 0), (31, 15, 2)]
    ref, rst = opsf.trace_dp_psf(lens, sensor, query, points=picks)
    g, gs = psf.cpu().numpy(), st.cpu().numpy()
    for (f, d, l) in picks:
        q = opsf.point_index(f, d, l, 16, 3)
        assert _energy_l1(g[q], ref[q]) <= L1_TOL, (f, d, l)
        assert np.array_equal(gs[q, :3], rst[q, :3])
    # properties over every point: bookkeeping and launched rays
    assert np.all(gs[:, 0] == 512 * 512)
    assert np.allclose(gs[:, 0], gs[:, 1] + gs[:, 2])
    assert np.allclose(gs[:, 2], gs[:, 3:].sum(axis=1), rtol=1e-5)
    assert np.allclose(g.sum(axis=(2, 3))[:, 0], gs[:, 3], rtol=1e-4)


@pytest.mark.parametrize("norm", [NORM_SUM, NORM_MAX])
def test_normalisation_matches_oracle(norm):
    lens, sensor, query = configs.config1()
    query.normalize = norm
    psf, _ = sdirt.trace_dp_psf(lens, sensor, query)
    ref, _ = opsf.trace_dp_psf(lens, sensor, query)
    g = psf.cpu().numpy()
    for q in range(ref.shape[0]):
        assert _energy_l1(g[q], ref[q]) <= L1_TOL


def test_on_axis_mirror_symmetry_on_gpu():
    lens = _rf50_f4()
    for mode in (DP_MICROLENS, DP_SIGMOID):
        sensor = Sensor(pitch=0.02, dp_mode=mode)
        query = PsfQuery(fields=[(0.0, 0.0)], depths=[600.0, 2500.0], wavelengths=[0.55],
                         rays_x=128, rays_y=128, jitter=False, ks=25)
        psf, _ = sdirt.trace_dp_psf(lens, sensor, query)
        g = psf.cpu().numpy()
        for q in range(2):
            if mode == DP_MICROLENS:
                assert np.array_equal(g[q, 0], g[q, 1][:, ::-1])
            else:
                assert np.allclose(g[q, 0], g[q, 1][:, ::-1], rtol=1e-5, atol=1e-4)


def test_edge_cases():
    lens, sensor, query = configs.config1()
    # one ray, ks 1
    q = copy.deepcopy(query); q.rays_x = 1; q.rays_y = 1; q.ks = 1
    psf, st = sdirt.trace_dp_psf(lens, sensor, q)
    ref, rst = opsf.trace_dp_psf(lens, sensor, q)
    assert np.allclose(psf.cpu().numpy(), ref, atol=1e-6)
    assert np.array_equal(st.cpu().numpy()[:, :3], rst[:, :3])
    # a field far outside the window: everything outside, zero PSF
    q = copy.deepcopy(query); q.fields = [(0.0, 0.0)]
    L = lenses.singlet(); L.focus_depth = 2000.0
    psf, st = sdirt.trace_dp_psf(L, sensor, q)
    ref, rst = opsf.trace_dp_psf(L, sensor, q)
    assert np.allclose(st.cpu().numpy(), rst, rtol=1e-6, atol=1e-3)
    # all rays vignetted: tiny clear aperture behind the stop
    L = lenses.singlet(); L.surfaces[2].semi_diameter = 1e-4
    psf, st = sdirt.trace_dp_psf(L, sensor, query)
    s = st.cpu().numpy()
    assert np.all(psf.cpu().numpy() == 0) and np.all(s[:, 1] == s[:, 0])
    # ragged ray count not a multiple of the workgroup
    q = copy.deepcopy(query); q.rays_x = 37; q.rays_y = 29
    psf, st = sdirt.trace_dp_psf(lens, sensor, q)
    ref, rst = opsf.trace_dp_psf(lens, sensor, q)
    assert np.array_equal(st.cpu().numpy()[:, :3], rst[:, :3])
    assert _energy_l1(psf.cpu().numpy(), ref) <= L1_TOL


@pytest.mark.parametrize("which", ["plano_convex", "plate"])
def test_flat_surfaces_on_the_spheres_and_flats_path(which):
    # prescriptions of spheres, planes and stops take the branch-free surface
    # loop, where a refracting plane is a sphere of curvature 0 and the stop
    # an index ratio of 1
    if which == "plate":
        # no power: the blur is the stop's shadow, so coarse pixels
        lens, pitch = lenses.plate(), 0.3
        fields = [(0.0, 0.0), (2.0, 1.4)]
    else:
        pitch = 0.006
        lens = Lens(surfaces=[
            Surface(kind=STOP, c=0.0, t=1.0, semi_diameter=8.0),
            Surface(kind=SPHERE, c=1.0 / 31.0, t=4.0, semi_diameter=12.0,
                    medium=cauchy(1.62, 0.012)),
            Surface(kind=PLANE, c=0.0, t=48.0, semi_diameter=12.0)],
            stop=0, f_number=2.8, focus_depth=1500.0)
        fields = [(0.0, 0.0), (1.2, -0.7), (-2.5, 1.5)]
    sensor = Sensor(pitch=pitch, dp_mode=DP_SIGMOID, sigmoid_k=15.0)
    query = PsfQuery(fields=fields, depths=[800.0, 3000.0], wavelengths=[0.48, 0.63],
                     rays_x=96, rays_y=80, seed=5, jitter=True, ks=41)
    psf, st = sdirt.trace_dp_psf(lens, sensor, query)
    ref, rst = opsf.trace_dp_psf(lens, sensor, query)
    g, gs = psf.cpu().numpy(), st.cpu().numpy()
    for q in range(ref.shape[0]):
        if ref[q].sum() > 0:
            assert _energy_l1(g[q], ref[q]) <= L1_TOL, q
    assert np.array_equal(gs[:, :3], rst[:, :3])
    assert np.allclose(gs[:, 3:], rst[:, 3:], rtol=1e-5, atol=0.05)


def test_list_mode_equals_grid_mode():
    lens, sensor, query = configs.config2(rays=32)
    psf, st = sdirt.trace_dp_psf(lens, sensor, query)
    pts = []
    for f, fld in enumerate(query.fields):
        for d, dep in enumerate(query.depths):
            for l in range(3):
                pts.append([fld[0], fld[1], dep, l])
    pts = torch.tensor(pts, dtype=torch.float64, device="cuda")
    psf2, st2 = sdirt.trace_dp_psf(lens, sensor, query, points=pts)
    assert torch.allclose(psf, psf2, rtol=1e-5, atol=1e-5)
    assert torch.equal(st[:, :3], st2[:, :3])


def test_chunking_does_not_change_result():
    lens, sensor, query = configs.config2(rays=64)
    a, sa = sdirt.trace_dp_psf(lens, sensor, query, chunks=1)
    b, sb = sdirt.trace_dp_psf(lens, sensor, query, chunks=7)
    assert torch.allclose(a, b, rtol=1e-5, atol=1e-4)
    assert torch.equal(sa[:, :3], sb[:, :3])


@pytest.mark.parametrize("out_f64", [False, True])
def test_single_chunk_writes_every_element(out_f64):
    # with one workgroup per point the kernel stores the whole tile and the
    # output is not zero-filled first: a buffer full of NaN must come back
    # finite and equal to the (zero-filled, atomically summed) 5-chunk result
    lens, sensor, query = configs.config5(rays=40)
    query.out_f64 = out_f64
    dt = torch.float64 if out_f64 else torch.float32
    shape = (query.n_points, 2, query.ks, query.ks)
    out = torch.full(shape, float("nan"), dtype=dt, device="cuda")
    a, sa = sdirt.trace_dp_psf(lens, sensor, query, chunks=1, out=out)
    b, sb = sdirt.trace_dp_psf(lens, sensor, query, chunks=5)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(a).all())
    assert torch.allclose(a, b, rtol=1e-5, atol=1e-4)
    assert torch.equal(sa[:, :3], sb[:, :3])


def test_paper_psf_map_sampled_pixels():
    # the per-pixel map of the paper's workload (RF50 F/4, microlens DP
    # model, ks 21, 4096 rays): list-mode points at sampled pixels against
    # the oracle.  List point k draws the jitter stream of point index k, so
    # the oracle evaluates point (k, 0, 0) of a grid whose fields all equal
    # that pixel.
    lens, sensor, query, (H, W) = configs.paper_psf_map()
    from workloads import scenes
    dmap = scenes.depth_uniform_inverse(H, W, 500.0, 20000.0, seed=100)
    pts_all = configs.pixel_points(H, W, sensor.pitch, dmap)
    rng = np.random.default_rng(4)
    idx = [0, W - 1, (H // 2) * W + W // 2, H * W - 1] + [int(v) for v in rng.integers(0, H * W, 8)]
    pts = torch.from_numpy(pts_all[idx]).cuda()
    psf, st = sdirt.trace_dp_psf(lens, sensor, query, points=pts)
    g, gs = psf.cpu().numpy(), st.cpu().numpy()
    for k, i in enumerate(idx):
        q = copy.deepcopy(query)
        q.fields = [(pts_all[i, 0], pts_all[i, 1])] * (k + 1)
        q.depths = [pts_all[i, 2]]
        ref, rst = opsf.trace_dp_psf(lens, sensor, q, points=[(k, 0, 0)])
        assert np.array_equal(gs[k, :3], rst[k, :3])
        assert np.array_equal(g[k], np.round(g[k]))         # box + microlens: counts
        if ref[k].sum() > 0:
            assert _energy_l1(g[k], ref[k]) <= L1_TOL


def test_config5_phone_lens_sampled_points():
    # 16 refracting surfaces with six even aspheres, 1 um pixels, ks 65:
    # the full 64 x 32 x 3 grid at reduced rays, sampled points vs the oracle
    lens, sensor, query = configs.config5(rays=48)
    psf, st = sdirt.trace_dp_psf(lens, sensor, query)
    torch.cuda.synchronize()
    picks = [(0, 0, 1), (20, 16, 0), (40, 31, 2), (63, 5, 1), (63, 31, 0)]
    ref, rst = opsf.trace_dp_psf(lens, sensor, query, points=picks)
    g, gs = psf.cpu().numpy(), st.cpu().numpy()
    for (f, d, l) in picks:
        q = opsf.point_index(f, d, l, 32, 3)
        assert np.array_equal(gs[q, :3], rst[q, :3]), (f, d, l)
        if ref[q].sum() > 0:
            assert _energy_l1(g[q], ref[q]) <= L1_TOL, (f, d, l)
    assert np.allclose(gs[:, 0], gs[:, 1] + gs[:, 2])


@pytest.mark.parametrize("splat", [SPLAT_BOX, SPLAT_TENT])
def test_deterministic_mode(splat):
    # integer tiles and one workgroup per point: identical bits from call to
    # call (and from grid to list mode), the same PSFs as the default mode
    # to the rounding of the weights, and the oracle's parity bar
    lens, sensor, query = configs.config2(rays=96)
    query.fields = query.fields[::10]
    query.depths = query.depths[::5]
    query.splat = splat
    query.deterministic = True
    a, sa = sdirt.trace_dp_psf(lens, sensor, query)
    b, sb = sdirt.trace_dp_psf(lens, sensor, query, chunks=5)
    assert torch.equal(a, b) and torch.equal(sa, sb)
    pts = torch.tensor([[f[0], f[1], d, l] for f in query.fields for d in query.depths
                        for l in range(len(query.wavelengths))], dtype=torch.float64, device="cuda")
    c, sc = sdirt.trace_dp_psf(lens, sensor, query, points=pts)
    assert torch.equal(a, c)
    q2 = copy.deepcopy(query)
    q2.deterministic = False
    d, sd = sdirt.trace_dp_psf(lens, sensor, q2)
    assert torch.equal(sa[:, :3], sd[:, :3])
    assert (a - d).abs().sum().item() <= 1e-6 * d.abs().sum().item()
    ref, rst = opsf.trace_dp_psf(lens, sensor, query)
    g = a.cpu().numpy()
    for q in range(g.shape[0]):
        if ref[q].sum() > 0:
            assert _energy_l1(g[q], ref[q]) <= L1_TOL, q
    assert np.array_equal(sa.cpu().numpy()[:, :3], rst[:, :3])
    # normalised, still reproducible
    q3 = copy.deepcopy(query)
    q3.normalize = NORM_SUM
    n1, _ = sdirt.trace_dp_psf(lens, sensor, q3)
    n2, _ = sdirt.trace_dp_psf(lens, sensor, q3)
    assert torch.equal(n1, n2)


@pytest.mark.parametrize("name", ["clip", "tir", "miss", "conic", "invalid", "first_failure"])
def test_failure_status_at_its_closed_form_boundary(name):
    # the status codes of rays just inside / outside each failure condition,
    # against the answer the case's geometry fixes (pinned on the oracle too)
    from workloads import status_cases as sc
    L, o, d, expect = sc.CASES[name]()
    print("status case", name, flush=True)
    hits, status = sdirt.trace_rays(L, 0.55, torch.from_numpy(o).cuda(),
                                    torch.from_numpy(d).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(status.cpu().numpy(), expect), (status.cpu().numpy(), expect)
