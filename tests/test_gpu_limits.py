"""GPU parity at the documented size limits: the largest prescription (24
surfaces) and PSF window (ks 129) of the trace, the largest windows of the
dense render (its LDS image tile), and the largest bank (64 fields x 64
depths x 4 wavelengths), against the CPU oracle through the C ABI."""
import numpy as np
import pytest
import torch

from workloads import scenes
from workloads.lens import (Sensor, PsfQuery, Surface, Lens, SPHERE, PLANE, STOP, cauchy,
                            DP_SIGMOID, SPLAT_BOX)
from oracle import optics, psf as opsf, trace as otr, render as R
from paper_2503_11213_amd import sdirt, _abi as abi

pytestmark = pytest.mark.gpu


def _rel(g, r):
    scale = max(np.abs(r).max(), 1e-30)
    return np.max(np.abs(g - r) / np.maximum(np.abs(r), 1e-3 * scale))


def _lens24():
    # a singlet behind the stop, ten glass plates, a weak air-spaced sphere:
    # SDIRT_MAX_SURFACES rows, all on the spheres-and-flats path
    S = [Surface(kind=STOP, c=0.0, t=0.0, semi_diameter=12.5),
         Surface(kind=SPHERE, c=1.0 / 51.5, t=5.0, semi_diameter=15.0,
                 medium=cauchy(1.5168, 0.0042)),
         Surface(kind=SPHERE, c=-1.0 / 51.5, t=2.0, semi_diameter=15.0)]
    for k in range(10):
        S.append(Surface(kind=PLANE, c=0.0, t=0.8, semi_diameter=14.0,
                         medium=cauchy(1.45 + 0.02 * k, 0.003)))
        S.append(Surface(kind=PLANE, c=0.0, t=0.4, semi_diameter=14.0))
    S.append(Surface(kind=SPHERE, c=1e-3, t=30.0, semi_diameter=14.0))
    return Lens(surfaces=S, stop=0, f_number=2.0, focus_depth=2000.0, name="24 surfaces")


def test_trace_at_the_largest_prescription_and_window():
    lens = _lens24()
    assert len(lens.surfaces) == 24                    # SDIRT_MAX_SURFACES
    sensor = Sensor(pitch=0.008, dp_mode=DP_SIGMOID, sigmoid_k=20.0)
    query = PsfQuery(fields=[(0.0, 0.0), (0.6, 0.3)], depths=[1000.0],
                     wavelengths=[0.486, 0.656], rays_x=64, rays_y=64, seed=4, jitter=True,
                     ks=129, splat=SPLAT_BOX)
    psf, st = sdirt.trace_dp_psf(lens, sensor, query)
    ref, rst = opsf.trace_dp_psf(lens, sensor, query)
    psf, st = psf.cpu().numpy(), st.cpu().numpy()
    assert np.array_equal(st[:, :3], rst[:, :3])
    assert np.abs(psf - ref).sum() / np.abs(ref).sum() <= 1e-3
    assert ref.sum() > 0.5 * rst[:, 0].sum()
    # every surface's hit of one bundle, to the intersection bar
    P = optics.Prepared(lens)
    e, d = opsf.bundle(P, query, 1, 0, 1)
    want = otr.trace(P, 0.656, e, d, record=True)
    hits, status = sdirt.trace_rays(lens, 0.656, torch.from_numpy(e).cuda(), torch.from_numpy(d).cuda())
    hits, status = hits.cpu().numpy(), status.cpu().numpy()
    assert np.array_equal(status, want["status"])
    ok = status == 0
    assert hits.shape[1] == 25 and ok.mean() > 0.9
    err = np.abs(hits[ok] - want["hits"][ok]) / np.maximum(np.abs(want["hits"][ok]), 1.0)
    assert err.max() <= 1e-5


@pytest.mark.parametrize("C,ks", [(1, 129), (3, 109)])
def test_dense_render_at_the_largest_windows(C, ks):
    # the forward stages C (ks + 7)^2 image floats per 8 x 8 tile in LDS:
    # ks 129 at one channel, ks 109 (the largest that fits) at three.  The
    # window is several times the image, so the adjoint folds up to ~10^4
    # clamped taps onto a border pixel: the upstream gradient is taken
    # nonnegative, as with mixed signs the float32 sum's cancellation alone
    # reaches the 1e-4 bar (measured 1.0e-4 at ks 109)
    N, H, W = 1, 12, 21
    rng = np.random.default_rng(ks)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    K = rng.uniform(0, 1, (N, H, W, C, 2, ks, ks)).astype(np.float32)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, psf_channels=C)
    Kt, it = torch.from_numpy(K).cuda(), torch.from_numpy(img).cuda()
    out = sdirt.render_dp(desc, it, Kt)
    assert _rel(out.cpu().numpy(), R.render_dense(img, K)) <= 1e-4
    g = rng.uniform(size=(N, 2 * C, H, W)).astype(np.float32)
    gt = torch.from_numpy(g).cuda()
    gi = sdirt.render_dp_backward(desc, Kt, gt)
    assert _rel(gi.cpu().numpy(), R.render_dense_adjoint(g, K)) <= 1e-4
    gk = sdirt.render_dp_psf_backward(desc, it, gt)
    ref = R.render_dense_psf_adjoint(img, g, C, ks)
    assert np.max(np.abs(gk.cpu().numpy() - ref)) <= 1e-5 * np.abs(ref).max()


def test_dense_render_window_past_the_tile_limit():
    # ks 111 at three channels: the forward's image tile does not fit in LDS
    # (SDIRT_EUNSUPPORTED before any launch); the adjoint, which stages
    # nothing, still runs
    N, C, H, W, ks = 1, 3, 9, 10, 111
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    K = rng.uniform(0, 1, (N, H, W, C, 2, ks, ks)).astype(np.float32)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, psf_channels=C)
    Kt = torch.from_numpy(K).cuda()
    with pytest.raises(abi.SdirtError) as e:
        sdirt.render_dp(desc, torch.from_numpy(img).cuda(), Kt)
    assert e.value.status == abi.EUNSUPPORTED
    g = rng.uniform(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, Kt, torch.from_numpy(g).cuda())
    assert _rel(gi.cpu().numpy(), R.render_dense_adjoint(g, K)) <= 1e-4


def test_largest_bank():
    # 64 field radii x 64 inverse depths x 4 wavelength slots (the key and
    # entry-offset arithmetic at its largest), forward, adjoint and bank
    # gradient on the grouped matrix-core path
    N, C, H, W, ks, F, D, L, ps = 1, 3, 40, 64, 21, 64, 64, 4, 0.01
    rng = np.random.default_rng(77)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    bank = rng.uniform(0, 1, (F, D, L, 2, ks, ks)).astype(np.float32)
    radii = np.linspace(0, np.hypot(W * ps / 2, H * ps / 2), F)
    iv = np.linspace(1 / 5000.0, 1 / 500.0, D)
    dmap = rng.uniform(500.0, 5000.0, size=(N, H, W)).astype(np.float32)
    loc = [3, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK, field_radii=radii,
                                        inv_depths=iv, bank_lambdas=L, lambda_of_channel=loc,
                                        pitch=ps)
    bt, dt, it = (torch.from_numpy(bank).cuda(), torch.from_numpy(dmap).cuda(),
                  torch.from_numpy(img).cuda())
    out = sdirt.render_dp(desc, it, bt, depth=dt)
    assert _rel(out.cpu().numpy(), R.render_bank(img, bank, dmap, radii, iv, loc, ps)) <= 1e-4
    g = rng.normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gt = torch.from_numpy(g).cuda()
    gi = sdirt.render_dp_backward(desc, bt, gt, depth=dt)
    assert _rel(gi.cpu().numpy(), R.render_bank_adjoint(g, bank, dmap, radii, iv, loc, ps)) <= 1e-4
    gb = sdirt.render_dp_psf_backward(desc, it, gt, depth=dt).cpu().numpy()
    ref = R.render_bank_psf_adjoint(img, g, bank.shape, dmap, radii, iv, loc, ps)
    assert np.max(np.abs(gb - ref)) <= 1e-5 * np.abs(ref).max()
