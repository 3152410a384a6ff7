"""GPU parity of the pixel-wise DP renderer and its image adjoint against the
CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from workloads import scenes
from oracle import render as R
from oracle.mlp import to_bf16
from paper_2503_11213_amd import sdirt, _abi as abi

pytestmark = pytest.mark.gpu

REL_TOL = 1e-4


def _rel(g, r):
    scale = max(np.abs(r).max(), 1e-30)
    return np.max(np.abs(g - r) / np.maximum(np.abs(r), 1e-3 * scale))


def _dense(N, C, H, W, ks, Cp, seed, bf16=False):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    K = rng.uniform(0, 1, (N, H, W, Cp, 2, ks, ks)).astype(np.float32)
    if bf16:
        K = to_bf16(K).astype(np.float32)
    return img, K


@pytest.mark.parametrize("shape", [(1, 3, 19, 37, 7, 3), (2, 3, 17, 9, 5, 1),
                                   (1, 1, 8, 8, 1, 1), (1, 2, 23, 21, 9, 2),
                                   (1, 3, 5, 4, 11, 3)])
def test_dense_forward_and_adjoint(shape):
    N, C, H, W, ks, Cp = shape
    img, K = _dense(N, C, H, W, ks, Cp, 1)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, psf_channels=Cp)
    Kt = torch.from_numpy(K).cuda()
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), Kt)
    ref = R.render_dense(img, K)
    assert _rel(out.cpu().numpy(), ref) <= REL_TOL
    g = np.random.default_rng(2).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, Kt, torch.from_numpy(g).cuda())
    gref = R.render_dense_adjoint(g, K)
    assert _rel(gi.cpu().numpy(), gref) <= REL_TOL


def test_dense_bf16_kernels():
    N, C, H, W, ks, Cp = 1, 3, 21, 26, 9, 3
    img, K = _dense(N, C, H, W, ks, Cp, 3, bf16=True)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, psf_channels=Cp, psf_dtype=abi.BF16)
    Kb = torch.from_numpy(K).to(torch.bfloat16).cuda()
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), Kb)
    ref = R.render_dense(img, K)
    assert _rel(out.cpu().numpy(), ref) <= REL_TOL
    g = np.random.default_rng(4).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, Kb, torch.from_numpy(g).cuda())
    assert _rel(gi.cpu().numpy(), R.render_dense_adjoint(g, K)) <= REL_TOL


@pytest.mark.parametrize("shape", [(1, 3, 1, 13, 5, 3), (1, 2, 9, 1, 3, 1),
                                   (2, 3, 12, 11, 7, 3), (1, 1, 3, 17, 9, 1)])
@pytest.mark.parametrize("bf16", [False, True])
def test_dense_thin_images_and_partial_bands(shape, bf16):
    # one-row and one-column images, and heights that end inside a band of the
    # 8 x 8 tile (the forward and the kernel-map gradient give a workgroup one
    # to four rows of a tile): forward, image adjoint and kernel-map gradient
    N, C, H, W, ks, Cp = shape
    img, K = _dense(N, C, H, W, ks, Cp, 5, bf16=bf16)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, psf_channels=Cp,
                                        psf_dtype=abi.BF16 if bf16 else abi.F32)
    Kt = torch.from_numpy(K).cuda()
    if bf16:
        Kt = Kt.to(torch.bfloat16)
    it = torch.from_numpy(img).cuda()
    out = sdirt.render_dp(desc, it, Kt)
    assert _rel(out.cpu().numpy(), R.render_dense(img, K)) <= REL_TOL
    g = np.random.default_rng(6).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gt = torch.from_numpy(g).cuda()
    gi = sdirt.render_dp_backward(desc, Kt, gt)
    assert _rel(gi.cpu().numpy(), R.render_dense_adjoint(g, K)) <= REL_TOL
    gk = sdirt.render_dp_psf_backward(desc, it, gt).float().cpu().numpy()
    ref = R.render_dense_psf_adjoint(img, g, Cp, ks)
    assert gk.shape == ref.shape
    if bf16:
        # the float32 value rounded once to nearest even: within half a bf16
        # ulp (2^-9 relative) of the exact one, plus float32 rounding
        assert np.all(np.abs(gk - ref) <= 2.0 ** -8 * np.abs(ref))
    else:
        assert np.max(np.abs(gk - ref)) <= 1e-6 * np.abs(ref).max()


def _bank_case(N, C, H, W, ks, F, D, L, ps, seed):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    bank = rng.uniform(0, 1, (F, D, L, 2, ks, ks)).astype(np.float32)
    half_diag = np.hypot(W * ps / 2, H * ps / 2)
    radii = np.linspace(0, half_diag, F)
    depths = 1.0 / np.linspace(1 / 5000.0, 1 / 500.0, D)
    dmap = np.stack([scenes.depth_voronoi(H, W, 500.0, 5000.0, seed=100 + n) for n in range(N)])
    return img, bank, radii, 1.0 / depths, dmap


def test_bank_forward_and_adjoint():
    N, C, H, W, ks, F, D, L, ps = 2, 3, 33, 45, 7, 6, 5, 3, 0.01
    img, bank, radii, iv, dmap = _bank_case(N, C, H, W, ks, F, D, L, ps, 5)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps)
    bt, dt = torch.from_numpy(bank).cuda(), torch.from_numpy(dmap).cuda()
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), bt, depth=dt)
    ref = R.render_bank(img, bank, dmap, radii, iv, loc, ps)
    assert _rel(out.cpu().numpy(), ref) <= REL_TOL
    g = np.random.default_rng(6).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, bt, torch.from_numpy(g).cuda(), depth=dt)
    gref = R.render_bank_adjoint(g, bank, dmap, radii, iv, loc, ps)
    assert _rel(gi.cpu().numpy(), gref) <= REL_TOL


def test_bank_full_size_sampled_pixels():
    # the benchmarked launch: one 1680 x 1120 RGB image, 32 x 16 x 3 bank, ks 63
    N, C, H, W, ks, F, D, L, ps = 1, 3, 1120, 1680, 63, 32, 16, 3, 0.00536
    rng = np.random.default_rng(7)
    img = scenes.aif_blobs(H, W, C, n_blobs=300, seed=0)[None]
    bank = rng.uniform(0, 1, (F, D, L, 2, ks, ks)).astype(np.float32)
    radii = np.arange(F) * np.hypot(W * ps / 2, H * ps / 2) / (F - 1)
    iv = np.linspace(1 / 5000.0, 1 / 500.0, D)
    dmap = scenes.depth_voronoi(H, W, 500.0, 5000.0, seed=100)[None]
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps)
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), torch.from_numpy(bank).cuda(),
                          depth=torch.from_numpy(dmap).cuda()).cpu().numpy()
    pix = [(0, 0, 0), (0, H - 1, W - 1), (0, 0, W - 1), (0, 560, 840), (0, 559, 839),
           (0, 17, 1201), (0, 1000, 3)] + [(0, int(rng.integers(H)), int(rng.integers(W)))
                                          for _ in range(40)]
    ref = R.render_bank_pixels(img, bank, dmap, radii, iv, loc, ps, pix)
    got = np.stack([out[n, :, y, x] for (n, y, x) in pix])
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= REL_TOL
    # constant image: every output pixel is its kernel's sum
    one = np.ones((N, C, H, W), dtype=np.float32)
    o1 = sdirt.render_dp(desc, torch.from_numpy(one).cuda(), torch.from_numpy(bank).cuda(),
                         depth=torch.from_numpy(dmap).cuda()).cpu().numpy()
    sums = bank.sum(axis=(-1, -2))          # [F, D, L, 2]
    assert o1.min() >= sums.min() * (1 - 1e-5) and o1.max() <= sums.max() * (1 + 1e-5)


@pytest.mark.parametrize("ks", [21, 31, 33, 41, 63, 65])
def test_bank_grouped_path(ks):
    # every window size of the grouped bank kernels; several 64 x 64
    # (forward) and 32 x 32 (adjoint) tiles with ragged edges, both mirror
    # flips, many entries per tile
    N, C, H, W, F, D, L, ps = 2, 3, 45, 150, 6, 5, 3, 0.01
    img, bank, radii, iv, dmap = _bank_case(N, C, H, W, ks, F, D, L, ps, 9)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps)
    bt, dt = torch.from_numpy(bank).cuda(), torch.from_numpy(dmap).cuda()
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), bt, depth=dt)
    ref = R.render_bank(img, bank, dmap, radii, iv, loc, ps)
    assert _rel(out.cpu().numpy(), ref) <= REL_TOL
    g = np.random.default_rng(10).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, bt, torch.from_numpy(g).cuda(), depth=dt)
    gref = R.render_bank_adjoint(g, bank, dmap, radii, iv, loc, ps)
    assert _rel(gi.cpu().numpy(), gref) <= REL_TOL


def test_bank_entry_per_pixel_noise():
    # white-noise depth: up to 8 entries per 8-pixel strip, so a 64 x 64 tile
    # lists more (strip, entry) items than one batch holds and the forward
    # kernel renders it in several batches
    N, C, H, W, ks, F, D, L, ps = 1, 3, 130, 200, 21, 9, 24, 3, 0.01
    rng = np.random.default_rng(31)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    bank = rng.uniform(0, 1, (F, D, L, 2, ks, ks)).astype(np.float32)
    radii = np.linspace(0, np.hypot(W * ps / 2, H * ps / 2), F)
    iv = np.linspace(1 / 5000.0, 1 / 500.0, D)
    dmap = (1.0 / rng.uniform(1 / 5000.0, 1 / 500.0, (N, H, W))).astype(np.float32)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps)
    bt, dt = torch.from_numpy(bank).cuda(), torch.from_numpy(dmap).cuda()
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), bt, depth=dt)
    assert _rel(out.cpu().numpy(), R.render_bank(img, bank, dmap, radii, iv, loc, ps)) <= REL_TOL
    g = rng.normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, bt, torch.from_numpy(g).cuda(), depth=dt)
    gref = R.render_bank_adjoint(g, bank, dmap, radii, iv, loc, ps)
    assert _rel(gi.cpu().numpy(), gref) <= REL_TOL


@pytest.mark.parametrize("Cp", [3, 1])
def test_dense_adjoint_several_halo_passes(Cp):
    # ks 41: the 48 x 48 halo of an 8 x 8 tile takes two passes of the gather
    N, C, H, W, ks = 1, 3, 13, 21, 41
    img, K = _dense(N, C, H, W, ks, Cp, 7)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, psf_channels=Cp)
    Kt = torch.from_numpy(K).cuda()
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), Kt)
    assert _rel(out.cpu().numpy(), R.render_dense(img, K)) <= REL_TOL
    g = np.random.default_rng(8).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, Kt, torch.from_numpy(g).cuda())
    assert _rel(gi.cpu().numpy(), R.render_dense_adjoint(g, K)) <= REL_TOL


def test_dense_full_size_sampled_pixels():
    # the benchmarked dense launch: 512 x 512 RGB, per-channel 41 x 41 kernels;
    # each sampled output (forward) or input pixel (adjoint) depends only on a
    # (2 pad + 1)^2 neighbourhood, so the oracle runs on that crop (anchored at
    # the image border for border pixels, where clamping folds taps)
    N, C, H, W, ks, Cp = 1, 3, 512, 512, 41, 3
    pad = ks // 2
    rng = np.random.default_rng(21)
    img = rng.random((N, C, H, W), dtype=np.float32)
    K = rng.random((N, H, W, Cp, 2, ks, ks), dtype=np.float32)
    g = rng.normal(size=(N, 2 * C, H, W)).astype(np.float32)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, psf_channels=Cp)
    Kt = torch.from_numpy(K).cuda()
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), Kt).cpu().numpy()
    gi = sdirt.render_dp_backward(desc, Kt, torch.from_numpy(g).cuda()).cpu().numpy()
    del Kt
    picks = [(0, 0), (511, 511), (0, 300), (255, 256), (100, 7), (400, 480), (37, 211)]
    for (y, x) in picks:
        ya = min(max(y - 2 * pad, 0), H - 4 * pad - 1)
        xa = min(max(x - 2 * pad, 0), W - 4 * pad - 1)
        sl = (slice(ya, ya + 4 * pad + 1), slice(xa, xa + 4 * pad + 1))
        ref = R.render_dense(img[:, :, sl[0], sl[1]], K[:, sl[0], sl[1]])
        gref = R.render_dense_adjoint(g[:, :, sl[0], sl[1]], K[:, sl[0], sl[1]])
        assert _rel(out[:, :, y, x], ref[:, :, y - ya, x - xa]) <= REL_TOL, (y, x)
        assert _rel(gi[:, :, y, x], gref[:, :, y - ya, x - xa]) <= REL_TOL, (y, x)


@pytest.mark.parametrize("shape", [(1, 3, 19, 37, 7, 3), (2, 3, 17, 9, 5, 1),
                                   (1, 2, 23, 21, 9, 2), (1, 1, 8, 8, 1, 1)])
def test_dense_kernel_gradient(shape):
    # gradient with respect to the per-pixel kernel map: one product per
    # element (a sum of C products for shared kernels), float32
    N, C, H, W, ks, Cp = shape
    img, _ = _dense(N, C, H, W, ks, Cp, 21)
    g = np.random.default_rng(22).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, psf_channels=Cp)
    gk = sdirt.render_dp_psf_backward(desc, torch.from_numpy(img).cuda(),
                                      torch.from_numpy(g).cuda()).cpu().numpy()
    ref = R.render_dense_psf_adjoint(img, g, Cp, ks)
    assert gk.shape == ref.shape
    assert np.max(np.abs(gk - ref)) <= 1e-6 * max(np.abs(ref).max(), 1e-30)


def test_dense_kernel_gradient_bf16_and_full_size_sample():
    # bf16 kernel map: each element rounded once to nearest even; and the
    # 512 x 512 RGB, 41 x 41 per-channel launch on sampled pixels
    N, C, H, W, ks, Cp = 1, 3, 512, 512, 41, 3
    rng = np.random.default_rng(23)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    g = rng.normal(size=(N, 2 * C, H, W)).astype(np.float32)
    it, gt = torch.from_numpy(img).cuda(), torch.from_numpy(g).cuda()
    pix = [(0, 0), (H - 1, W - 1), (0, W - 1), (200, 311), (17, 500)] + \
          [(int(rng.integers(H)), int(rng.integers(W))) for _ in range(10)]
    pad = (ks - 1) // 2
    for dt in (abi.F32, abi.BF16):
        desc, keep = sdirt.make_render_desc(N, C, H, W, ks, psf_channels=Cp, psf_dtype=dt)
        gk = sdirt.render_dp_psf_backward(desc, it, gt)
        for (y, x) in pix:
            got = gk[0, y, x].float().cpu().numpy()                 # [C, 2, ks, ks]
            rows = np.clip(y + pad - np.arange(ks), 0, H - 1)
            cols = np.clip(x + pad - np.arange(ks), 0, W - 1)
            for c in range(C):
                win = img[0, c][rows][:, cols].astype(np.float64)
                for s in range(2):
                    ref = g[0, s * C + c, y, x] * win
                    if dt == abi.BF16:
                        ref = to_bf16(ref)
                        assert np.max(np.abs(got[c, s] - ref)) <= 1e-6 * np.abs(ref).max()
                    else:
                        assert np.max(np.abs(got[c, s] - ref)) <= 1e-6 * np.abs(ref).max()
        del gk


def _bank2d_case(N, C, H, W, ks, Fx, Fy, D, L, ps, seed, noise=False):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    bank = rng.uniform(0, 1, (Fy, Fx, D, L, 2, ks, ks)).astype(np.float32)
    xs = np.linspace(0, W * ps / 2, Fx)
    ys = np.linspace(0, H * ps / 2, Fy)
    iv = np.linspace(1 / 5000.0, 1 / 500.0, D)
    if noise:
        dmap = (1.0 / rng.uniform(1 / 6000.0, 1 / 400.0, (N, H, W))).astype(np.float32)
    else:
        dmap = np.stack([scenes.depth_voronoi(H, W, 450.0, 5500.0, seed=140 + n)
                         for n in range(N)]).astype(np.float32)
    return img, bank, xs, ys, iv, dmap


@pytest.mark.parametrize("ks,noise", [(21, False), (33, True), (63, False)])
def test_bank2d_forward_and_adjoint(ks, noise):
    # exact-azimuth bank: first-quadrant grid, flips, linear in 1/d (two
    # passes of the grouped kernels); depths beyond both ends of the planes
    N, C, H, W, Fx, Fy, D, L, ps = 2, 3, 45, 150, 5, 4, 4, 3, 0.01
    img, bank, xs, ys, iv, dmap = _bank2d_case(N, C, H, W, ks, Fx, Fy, D, L, ps, 41, noise)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK2D,
                                        field_radii=xs, field_y=ys, inv_depths=iv,
                                        bank_lambdas=L, lambda_of_channel=loc, pitch=ps)
    bt, dt = torch.from_numpy(bank).cuda(), torch.from_numpy(dmap).cuda()
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), bt, depth=dt)
    ref = R.render_bank2d(img, bank, dmap, xs, ys, iv, loc, ps)
    assert _rel(out.cpu().numpy(), ref) <= REL_TOL
    g = np.random.default_rng(42).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, bt, torch.from_numpy(g).cuda(), depth=dt)
    gref = R.render_bank2d_adjoint(g, bank, dmap, xs, ys, iv, loc, ps)
    assert _rel(gi.cpu().numpy(), gref) <= REL_TOL


def test_bank2d_single_plane_and_unsupported_window():
    N, C, H, W, ks, ps = 1, 1, 20, 30, 21, 0.01
    img, bank, xs, ys, iv, dmap = _bank2d_case(N, C, H, W, ks, 3, 2, 1, 1, ps, 43)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK2D,
                                        field_radii=xs, field_y=ys, inv_depths=iv,
                                        bank_lambdas=1, lambda_of_channel=[0], pitch=ps)
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), torch.from_numpy(bank).cuda(),
                          depth=torch.from_numpy(dmap).cuda())
    ref = R.render_bank2d(img, bank, dmap, xs, ys, iv, [0], ps)
    assert _rel(out.cpu().numpy(), ref) <= REL_TOL
    desc7, keep7 = sdirt.make_render_desc(N, C, H, W, 7, source=abi.SRC_BANK2D,
                                          field_radii=xs, field_y=ys, inv_depths=iv,
                                          bank_lambdas=1, lambda_of_channel=[0], pitch=ps)
    with pytest.raises(abi.SdirtError):
        sdirt.render_dp(desc7, torch.from_numpy(img).cuda(), torch.zeros((2, 3, 1, 1, 2, 7, 7)).cuda(),
                        depth=torch.from_numpy(dmap).cuda())


@pytest.mark.parametrize("ks,two_d", [(21, False), (63, False), (33, True), (65, True)])
def test_bank_kernel_gradient(ks, two_d):
    # gradient with respect to the bank entries: per-pixel kernel gradients
    # summed over the pixels reading each entry, mirrors undone, 2-D bank
    # weights applied (matrix-core correlation, atomic accumulation)
    N, C, H, W, L, ps = 1, 3, 45, 150, 3, 0.01
    loc = [2, 1, 0]
    rng = np.random.default_rng(61)
    g = rng.normal(size=(N, 2 * C, H, W)).astype(np.float32)
    if two_d:
        img, bank, xs, ys, iv, dmap = _bank2d_case(N, C, H, W, ks, 4, 3, 3, L, ps, 62)
        desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK2D,
                                            field_radii=xs, field_y=ys, inv_depths=iv,
                                            bank_lambdas=L, lambda_of_channel=loc, pitch=ps)
        ref = R.render_bank2d_psf_adjoint(img, g, bank.shape, dmap, xs, ys, iv, loc, ps)
    else:
        F, D = 6, 5
        img, bank, radii, iv, dmap = _bank_case(N, C, H, W, ks, F, D, L, ps, 63)
        desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                            field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                            lambda_of_channel=loc, pitch=ps)
        ref = R.render_bank_psf_adjoint(img, g, bank.shape, dmap, radii, iv, loc, ps)
    got = sdirt.render_dp_psf_backward(desc, torch.from_numpy(img).cuda(),
                                       torch.from_numpy(g).cuda(),
                                       depth=torch.from_numpy(dmap).cuda()).cpu().numpy()
    assert got.shape == ref.shape
    err = np.max(np.abs(got - ref)) / np.abs(ref).max()
    print("bank kernel gradient max err / max", err)
    assert err <= 1e-5


@pytest.mark.parametrize("bank_math", [0, 1])
def test_bank_config5_full_batch_sampled_pixels(bank_math):
    # the benchmarked launch of the largest workload: 16 RGB 4032 x 3024
    # images, 64 x 32 x 3 bank (ks 65), forward and image adjoint; sampled
    # pixels of images 0 and 15 (corners, both sides of the mirror lines,
    # random) against the oracle's per-pixel bank render and adjoint
    from workloads import configs
    lens, sensor, query = configs.config5(rays=8)
    N, C, H, W, ks = 16, 3, sensor.height_px, sensor.width_px, query.ks
    F, D, L, ps = len(query.fields), len(query.depths), 3, sensor.pitch
    rng = np.random.default_rng(51)
    bank = rng.uniform(0, 1, (F, D, L, 2, ks, ks)).astype(np.float32)
    radii = [f[0] for f in query.fields]
    iv = [1.0 / d for d in query.depths]
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    dms = [scenes.depth_voronoi(H, W, 100.0, 5000.0, seed=200 + k) for k in range(4)]
    dmap = np.stack([dms[k % 4] for k in range(N)])
    loc = list(configs.LAMBDA_OF_RGB)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps, bank_math=bank_math)
    bt, dt = torch.from_numpy(bank).cuda(), torch.from_numpy(dmap).cuda()
    print("config-5 batch: forward, bank_math %d" % bank_math, flush=True)
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), bt, depth=dt)
    cy, cx = (H - 1) // 2, (W - 1) // 2
    pix = []
    for n in (0, N - 1):
        pix += [(n, 0, 0), (n, 0, W - 1), (n, H - 1, 0), (n, H - 1, W - 1),
                (n, cy, cx), (n, cy + 1, cx + 1), (n, cy, cx + 1), (n, cy + 1, cx),
                (n, 5, cx), (n, H - 3, cx + 1), (n, cy, 2), (n, cy + 1, W - 2)]
        pix += [(n, int(rng.integers(H)), int(rng.integers(W))) for _ in range(12)]
    got = np.stack([out[n, :, y, x].cpu().numpy() for (n, y, x) in pix])
    del out
    ref = R.render_bank_pixels(img, bank, dmap, radii, iv, loc, ps, pix)
    err = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()))
    print("config-5 forward max rel err %.2e" % err, flush=True)
    assert err <= REL_TOL
    print("config-5 batch: adjoint", flush=True)
    g = rng.normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, bt, torch.from_numpy(g).cuda(), depth=dt)
    got = np.stack([gi[n, :, y, x].cpu().numpy() for (n, y, x) in pix])
    del gi
    ref = R.render_bank_adjoint_pixels(g, bank, dmap, radii, iv, loc, ps, pix)
    err = np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()))
    print("config-5 adjoint max rel err %.2e" % err, flush=True)
    assert err <= REL_TOL


# ---- split-bf16 bank forward ------------------------------------------------
# Each operand split into bf16 hi + lo, three matrix-core products summed in
# float32: a product's relative error is below 2^-15 (the dropped lo * lo
# term and the residual of each split), so the renders meet the same 1e-4
# bar as the float32 path.

@pytest.mark.parametrize("ks", [21, 31, 33, 41, 63, 65])
def test_bank_split_bf16_forward(ks):
    N, C, H, W, F, D, L, ps = 2, 3, 45, 150, 6, 5, 3, 0.01
    img, bank, radii, iv, dmap = _bank_case(N, C, H, W, ks, F, D, L, ps, 9)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps,
                                        bank_math=abi.BANK_SPLIT_BF16)
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), torch.from_numpy(bank).cuda(),
                          depth=torch.from_numpy(dmap).cuda())
    ref = R.render_bank(img, bank, dmap, radii, iv, loc, ps)
    err = _rel(out.cpu().numpy(), ref)
    print("split-bf16 ks %d rel err %.2e" % (ks, err))
    assert err <= REL_TOL


@pytest.mark.parametrize("ks", [33, 65])
def test_bank2d_split_bf16_forward(ks):
    N, C, H, W, Fx, Fy, D, L, ps = 2, 3, 45, 150, 5, 4, 4, 3, 0.01
    img, bank, xs, ys, iv, dmap = _bank2d_case(N, C, H, W, ks, Fx, Fy, D, L, ps, 41, True)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK2D,
                                        field_radii=xs, field_y=ys, inv_depths=iv,
                                        bank_lambdas=L, lambda_of_channel=loc, pitch=ps,
                                        bank_math=abi.BANK_SPLIT_BF16)
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), torch.from_numpy(bank).cuda(),
                          depth=torch.from_numpy(dmap).cuda())
    ref = R.render_bank2d(img, bank, dmap, xs, ys, iv, loc, ps)
    assert _rel(out.cpu().numpy(), ref) <= REL_TOL


def test_bank_split_bf16_entry_per_pixel_noise_and_delta_kernels():
    # several batches per tile (white-noise depth), and delta kernels whose
    # output must reproduce shifted image values to float32 accuracy
    N, C, H, W, ks, F, D, L, ps = 1, 3, 130, 200, 21, 9, 24, 3, 0.01
    rng = np.random.default_rng(31)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    bank = rng.uniform(0, 1, (F, D, L, 2, ks, ks)).astype(np.float32)
    radii = np.linspace(0, np.hypot(W * ps / 2, H * ps / 2), F)
    iv = np.linspace(1 / 5000.0, 1 / 500.0, D)
    dmap = (1.0 / rng.uniform(1 / 5000.0, 1 / 500.0, (N, H, W))).astype(np.float32)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps,
                                        bank_math=abi.BANK_SPLIT_BF16)
    bt, dt = torch.from_numpy(bank).cuda(), torch.from_numpy(dmap).cuda()
    out = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), bt, depth=dt)
    assert _rel(out.cpu().numpy(), R.render_bank(img, bank, dmap, radii, iv, loc, ps)) <= REL_TOL
    delta = np.zeros_like(bank)
    delta[..., 0, 3, 17] = 1.0          # left: tap (3, 17); right: centre
    delta[..., 1, 10, 10] = 1.0
    o2 = sdirt.render_dp(desc, torch.from_numpy(img).cuda(), torch.from_numpy(delta).cuda(),
                         depth=dt).cpu().numpy()
    ref2 = R.render_bank(img, delta, dmap, radii, iv, loc, ps)
    assert np.max(np.abs(o2 - ref2)) <= 2.0 ** -16 * np.abs(ref2).max()


# ---- split-bf16 bank adjoint ------------------------------------------------
# The image adjoint on the bf16 matrix cores: the gradient and the kernel
# taps split into hi + lo, products g_hi K_hi + g_hi K_lo + g_lo K_hi summed
# in float32.  Each product is off by at most 3 * 2^-18 of its magnitude (the
# dropped lo * lo term and the two split residuals), so with gradients of
# both signs the bound is element-wise against the adjoint of |g| with the
# (nonnegative) kernels: |err| <= 2^-15 * (|g| adjoint |K|).  Relative to the
# result itself the error can exceed 1e-4 where the sum cancels.

SPLIT_BOUND = 2.0 ** -15


def _split_bound(gi, ref, absref):
    ratio = np.abs(gi - ref) / np.maximum(absref, 1e-7 * absref.max())
    return float(ratio.max())

@pytest.mark.parametrize("ks", [21, 31, 33, 41, 63, 65])
def test_bank_split_bf16_adjoint(ks):
    N, C, H, W, F, D, L, ps = 2, 3, 45, 150, 6, 5, 3, 0.01
    img, bank, radii, iv, dmap = _bank_case(N, C, H, W, ks, F, D, L, ps, 9)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps,
                                        bank_math=abi.BANK_SPLIT_BF16)
    g = np.random.default_rng(10).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    print("split-bf16 adjoint ks %d" % ks, flush=True)
    gi = sdirt.render_dp_backward(desc, torch.from_numpy(bank).cuda(), torch.from_numpy(g).cuda(),
                                  depth=torch.from_numpy(dmap).cuda())
    gref = R.render_bank_adjoint(g, bank, dmap, radii, iv, loc, ps)
    gabs = R.render_bank_adjoint(np.abs(g), bank, dmap, radii, iv, loc, ps)
    b = _split_bound(gi.cpu().numpy(), gref, gabs)
    print("split-bf16 adjoint ks %d err / (|g| adjoint K) %.2e" % (ks, b))
    assert b <= SPLIT_BOUND


def test_bank_split_bf16_adjoint_smooth_depth_long_segments():
    # few entries over large regions: full 16-row segments whose diagonals
    # run through every kernel row, several tiles with ragged edges
    N, C, H, W, ks, F, D, L, ps = 1, 3, 200, 270, 65, 3, 2, 3, 0.01
    rng = np.random.default_rng(61)
    bank = rng.uniform(0, 1, (F, D, L, 2, ks, ks)).astype(np.float32)
    radii = np.linspace(0, np.hypot(W * ps / 2, H * ps / 2), F)
    iv = np.array([1 / 3000.0, 1 / 1000.0])
    dmap = np.where(np.arange(W)[None, None, :] < 150, 800.0, 4000.0) * np.ones((N, H, 1))
    dmap = dmap.astype(np.float32)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps,
                                        bank_math=abi.BANK_SPLIT_BF16)
    g = rng.normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, torch.from_numpy(bank).cuda(), torch.from_numpy(g).cuda(),
                                  depth=torch.from_numpy(dmap).cuda())
    gref = R.render_bank_adjoint(g, bank, dmap, radii, iv, loc, ps)
    gabs = R.render_bank_adjoint(np.abs(g), bank, dmap, radii, iv, loc, ps)
    b = _split_bound(gi.cpu().numpy(), gref, gabs)
    print("split-bf16 adjoint smooth depth err / (|g| adjoint K) %.2e" % b)
    assert b <= SPLIT_BOUND


@pytest.mark.parametrize("ks", [21, 65])
def test_bank_split_bf16_adjoint_positive_gradient(ks):
    # nonnegative upstream gradient: sums do not cancel and the relative
    # bar of the float32 path applies element by element
    N, C, H, W, F, D, L, ps = 2, 3, 45, 150, 6, 5, 3, 0.01
    img, bank, radii, iv, dmap = _bank_case(N, C, H, W, ks, F, D, L, ps, 19)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps,
                                        bank_math=abi.BANK_SPLIT_BF16)
    g = np.random.default_rng(20).uniform(0, 1, (N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, torch.from_numpy(bank).cuda(), torch.from_numpy(g).cuda(),
                                  depth=torch.from_numpy(dmap).cuda())
    err = _rel(gi.cpu().numpy(), R.render_bank_adjoint(g, bank, dmap, radii, iv, loc, ps))
    print("split-bf16 adjoint, positive gradient, ks %d rel err %.2e" % (ks, err))
    assert err <= REL_TOL


@pytest.mark.parametrize("ks,noise", [(21, False), (33, True), (65, False)])
def test_bank2d_split_bf16_adjoint(ks, noise):
    N, C, H, W, Fx, Fy, D, L, ps = 2, 3, 45, 150, 5, 4, 4, 3, 0.01
    img, bank, xs, ys, iv, dmap = _bank2d_case(N, C, H, W, ks, Fx, Fy, D, L, ps, 41, noise)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK2D,
                                        field_radii=xs, field_y=ys, inv_depths=iv,
                                        bank_lambdas=L, lambda_of_channel=loc, pitch=ps,
                                        bank_math=abi.BANK_SPLIT_BF16)
    g = np.random.default_rng(42).normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, torch.from_numpy(bank).cuda(), torch.from_numpy(g).cuda(),
                                  depth=torch.from_numpy(dmap).cuda())
    gref = R.render_bank2d_adjoint(g, bank, dmap, xs, ys, iv, loc, ps)
    gabs = R.render_bank2d_adjoint(np.abs(g), bank, dmap, xs, ys, iv, loc, ps)
    assert _split_bound(gi.cpu().numpy(), gref, gabs) <= SPLIT_BOUND


def test_bank_split_bf16_adjoint_noise_and_delta_kernels():
    # white-noise depth (many entries per tile: several batches of entries),
    # and delta kernels, whose adjoint moves each output gradient to one
    # image pixel and must match to float32 accuracy
    N, C, H, W, ks, F, D, L, ps = 1, 3, 130, 200, 21, 9, 24, 3, 0.01
    rng = np.random.default_rng(31)
    bank = rng.uniform(0, 1, (F, D, L, 2, ks, ks)).astype(np.float32)
    radii = np.linspace(0, np.hypot(W * ps / 2, H * ps / 2), F)
    iv = np.linspace(1 / 5000.0, 1 / 500.0, D)
    dmap = (1.0 / rng.uniform(1 / 5000.0, 1 / 500.0, (N, H, W))).astype(np.float32)
    loc = [2, 1, 0]
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv, bank_lambdas=L,
                                        lambda_of_channel=loc, pitch=ps,
                                        bank_math=abi.BANK_SPLIT_BF16)
    dt = torch.from_numpy(dmap).cuda()
    g = rng.normal(size=(N, 2 * C, H, W)).astype(np.float32)
    gi = sdirt.render_dp_backward(desc, torch.from_numpy(bank).cuda(), torch.from_numpy(g).cuda(), depth=dt)
    gref = R.render_bank_adjoint(g, bank, dmap, radii, iv, loc, ps)
    gabs = R.render_bank_adjoint(np.abs(g), bank, dmap, radii, iv, loc, ps)
    assert _split_bound(gi.cpu().numpy(), gref, gabs) <= SPLIT_BOUND
    delta = np.zeros_like(bank)
    delta[..., 0, 3, 17] = 1.0
    delta[..., 1, 10, 10] = 1.0
    g2 = sdirt.render_dp_backward(desc, torch.from_numpy(delta).cuda(), torch.from_numpy(g).cuda(),
                                  depth=dt).cpu().numpy()
    ref2 = R.render_bank_adjoint(g, delta, dmap, radii, iv, loc, ps)
    assert np.max(np.abs(g2 - ref2)) <= 2.0 ** -15 * np.abs(ref2).max()
