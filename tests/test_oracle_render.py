"""Pins of the oracle's pixel-wise DP renderer (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import render as R


def _rand(shape, seed):
    return np.random.default_rng(seed).uniform(0, 1, shape)


def test_centred_delta_is_identity_and_offset_delta_shifts_with_replication():
    N, C, H, W, ks = 1, 3, 9, 11, 5
    img = _rand((N, C, H, W), 0)
    K = np.zeros((N, H, W, 1, 2, ks, ks))
    K[..., 0, 2, 2] = 1.0      # left: centred delta
    K[..., 1, 2, 4] = 1.0      # right: delta two columns right of centre
    out = R.render_dense(img, K)
    assert np.allclose(out[:, :C], img, atol=0)
    # tap (i, j) = (2, 4) reads img[y, clamp(x + 2 - 4)] = img[y, clamp(x - 2)]
    cols = np.clip(np.arange(W) - 2, 0, W - 1)
    assert np.allclose(out[:, C:], img[..., cols], atol=0)


def test_constant_image_gives_kernel_sum():
    N, C, H, W, ks = 2, 3, 7, 6, 5
    K = _rand((N, H, W, C, 2, ks, ks), 1)
    img = np.full((N, C, H, W), 0.75)
    out = R.render_dense(img, K)
    for s in range(2):
        for c in range(C):
            assert np.allclose(out[:, s * C + c], 0.75 * K[:, :, :, c, s].sum(axis=(-1, -2)))


def test_matches_pure_python_loops():
    N, C, H, W, ks = 1, 2, 6, 5, 3
    img = _rand((N, C, H, W), 2)
    K = _rand((N, H, W, C, 2, ks, ks), 3)
    pad = ks // 2
    ref = np.zeros((N, 2 * C, H, W))
    for n in range(N):
        for s in range(2):
            for c in range(C):
                for y in range(H):
                    for x in range(W):
                        acc = 0.0
                        for i in range(ks):
                            for j in range(ks):
                                yy = min(max(y + pad - i, 0), H - 1)
                                xx = min(max(x + pad - j, 0), W - 1)
                                acc += K[n, y, x, c, s, i, j] * img[n, c, yy, xx]
                        ref[n, s * C + c, y, x] = acc
    assert np.allclose(R.render_dense(img, K), ref, atol=1e-14)


def test_matches_torch_unfold_expression():
    # library re-expression: replicate pad, unfold the ks x ks patches, weight
    # each patch by the output pixel's kernel rotated by 180 degrees
    N, C, H, W, ks = 2, 3, 10, 12, 5
    img = _rand((N, C, H, W), 4)
    K = _rand((N, H, W, C, 2, ks, ks), 5)
    pad = ks // 2
    t = torch.from_numpy(img)
    patches = torch.nn.functional.unfold(
        torch.nn.functional.pad(t, (pad, pad, pad, pad), mode="replicate"), ks)
    patches = patches.view(N, C, ks * ks, H * W)                  # [N,C,T,P]
    Kt = torch.from_numpy(K).flip(-1).flip(-2).reshape(N, H * W, C, 2, ks * ks)
    outs = []
    for s in range(2):
        w = Kt[:, :, :, s, :].permute(0, 2, 3, 1)                 # [N,C,T,P]
        outs.append((patches * w).sum(2).view(N, C, H, W))
    ref = torch.cat(outs, 1).numpy()
    assert np.allclose(R.render_dense(img, K), ref, atol=1e-13)


def test_adjoint_dot_product():
    N, C, H, W, ks = 1, 3, 9, 8, 5
    img = _rand((N, C, H, W), 6)
    g = _rand((N, 2 * C, H, W), 7)
    for Cp in (1, C):
        K = _rand((N, H, W, Cp, 2, ks, ks), 8)
        lhs = np.sum(R.render_dense(img, K) * g)
        rhs = np.sum(img * R.render_dense_adjoint(g, K))
        assert lhs == pytest.approx(rhs, rel=1e-13)


def test_bank_lookup_equals_nearest_search():
    H, W, ps = 40, 56, 0.01
    radii = np.linspace(0, 0.3, 7)
    depths = 1.0 / np.linspace(1 / 5000.0, 1 / 500.0, 9)
    rng = np.random.default_rng(9)
    dmap = rng.uniform(500, 5000, (H, W)).astype(np.float32)
    fi, di, mx, my = R.bank_lookup(H, W, dmap, radii, 1 / depths, ps)
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    X = (xx - (W - 1) / 2) * ps
    Y = (yy - (H - 1) / 2) * ps
    rho = np.sqrt(X ** 2 + Y ** 2)
    f_ref = np.argmin(np.abs(rho[..., None] - radii), axis=-1)
    d_ref = np.argmin(np.abs(1.0 / dmap.astype(np.float64)[..., None] - 1 / depths), axis=-1)
    assert np.mean(fi == f_ref) > 0.999
    assert np.array_equal(di, d_ref)
    assert np.array_equal(mx, X < 0) and np.array_equal(my, Y < 0)


def test_bank_render_uses_mirror_rules():
    # a bank whose PSFs are asymmetric deltas; a pixel left of the centre
    # must see the column-flipped, side-swapped kernel
    H, W, ks, ps = 5, 6, 3, 0.01
    bank = np.zeros((2, 1, 1, 2, ks, ks))
    bank[:, 0, 0, 0, 1, 2] = 1.0        # left side: tap to the right
    bank[:, 0, 0, 1, 0, 1] = 1.0        # right side: tap upward
    dmap = np.full((1, H, W), 1000.0)
    K = R.dense_from_bank(bank, dmap, [0.0, 0.02], [1e-3], [0], ps)
    assert K[0, 0, 0, 0, 1, 1, 0] == 1.0      # x<0,y<0: right <- flipped left
    assert K[0, 0, 0, 0, 0, 2, 1] == 1.0      # left <- row-flipped right
    assert K[0, 4, 5, 0, 0, 1, 2] == 1.0      # x>0,y>0: unchanged


@pytest.mark.parametrize("Cp", [1, 3])
def test_kernel_gradient_matches_torch_autograd(Cp):
    # library gradient: torch autograd through the replicate-pad / unfold
    # expression of the render, with respect to the kernels
    N, C, H, W, ks = 1, 3, 9, 11, 5
    img = _rand((N, C, H, W), 11)
    g = _rand((N, 2 * C, H, W), 12) - 0.5
    pad = ks // 2
    K = torch.from_numpy(_rand((N, H, W, Cp, 2, ks, ks), 13)).requires_grad_(True)
    t = torch.from_numpy(img)
    patches = torch.nn.functional.unfold(
        torch.nn.functional.pad(t, (pad, pad, pad, pad), mode="replicate"), ks)
    patches = patches.view(N, C, ks * ks, H * W)
    Kt = K.flip(-1).flip(-2).reshape(N, H * W, Cp, 2, ks * ks)
    outs = []
    for s in range(2):
        w = Kt[:, :, :, s, :].permute(0, 2, 3, 1)                 # [N,Cp,T,P]
        outs.append((patches * w).sum(2).view(N, C, H, W))
    out = torch.cat(outs, 1)
    (out * torch.from_numpy(g)).sum().backward()
    gK = R.render_dense_psf_adjoint(img, g, Cp, ks)
    assert np.allclose(gK, K.grad.numpy(), atol=1e-12)
    # and the adjoint identity against the forward
    D = _rand(K.shape, 14)
    lhs = np.sum(R.render_dense(img, D) * g)
    assert lhs == pytest.approx(np.sum(D * gK), rel=1e-12)


def _delta_bank2d(Fx, Fy, D, ks, i0, j0):
    bank = np.zeros((Fy, Fx, D, 1, 2, ks, ks))
    bank[..., 0, i0, j0] = 1.0
    return bank


def test_bank2d_flip_rules_by_quadrant():
    # a left-side impulse at tap (i0, j0) everywhere: each quadrant shows the
    # image shifted by the mirrored tap on the side the mirror rules give
    H, W, ks, i0, j0 = 12, 14, 5, 1, 3
    pad = ks // 2
    img = _rand((1, 1, H, W), 31)
    depth = np.full((1, H, W), 2000.0, dtype=np.float32)
    bank = _delta_bank2d(2, 2, 1, ks, i0, j0)
    out = R.render_bank2d(img, bank, depth, [0.0, 1.0], [0.0, 1.0], [1 / 2000.0], [0], 0.1)
    for y in range(H):
        for x in range(W):
            mx, my = 2 * x - (W - 1) < 0, 2 * y - (H - 1) < 0
            i = ks - 1 - i0 if my else i0
            j = ks - 1 - j0 if mx else j0
            side = 1 if mx else 0
            src = img[0, 0, min(max(y + pad - i, 0), H - 1), min(max(x + pad - j, 0), W - 1)]
            assert out[0, side, y, x] == pytest.approx(src, abs=1e-14)
            assert out[0, 1 - side, y, x] == 0.0


def test_bank2d_linear_in_inverse_depth():
    # plane 0 an identity kernel, plane 1 zero: the output is (1 - w) img with
    # w the float32 position of 1/depth between the planes (exact here)
    H, W, ks = 6, 7, 3
    img = _rand((1, 1, H, W), 32)
    bank = np.zeros((1, 1, 3, 1, 2, ks, ks))
    bank[0, 0, 0, 0, 0, 1, 1] = 1.0
    iv = [0.25, 1.0, 2.0]                     # planes (1/mm), exact in float32
    for depth, expect in ((4.0, 1.0), (2.0, 2.0 / 3.0), (1.0, 0.0), (8.0, 1.0), (0.5, 0.0)):
        dm = np.full((1, H, W), depth, dtype=np.float32)
        out = R.render_bank2d(img, bank, dm, [0.0], [0.0], iv, [0], 0.1)
        # the centre tap is its own mirror image; the side swaps left of the
        # centre, so the two sides together carry it
        assert np.allclose(out[0, 0] + out[0, 1], expect * img[0, 0], atol=1e-7), depth
    fx, fy, d0, w, _, _ = R.bank2d_lookup(H, W, np.full((H, W), 0.8, dtype=np.float32),
                                           [0.0], [0.0], iv, 0.1)
    assert np.all(d0 == 1) and np.allclose(w, 0.25, atol=1e-7)     # 1/0.8 = 1.25


def test_bank2d_nearest_grid_point_equals_search():
    H, W, pitch = 40, 52, 0.013
    xs, ys = [0.0, 0.071, 0.2, 0.31], [0.0, 0.104, 0.22]
    fx, fy, *_ = R.bank2d_lookup(H, W, np.ones((H, W), dtype=np.float32), xs, ys, [1.0], pitch)
    hx = np.abs((np.arange(W) - (W - 1) / 2) * pitch)
    hy = np.abs((np.arange(H) - (H - 1) / 2) * pitch)
    bx = np.argmin(np.abs(hx[:, None] - np.array(xs)[None]), axis=1)
    by = np.argmin(np.abs(hy[:, None] - np.array(ys)[None]), axis=1)
    assert np.array_equal(fx, np.broadcast_to(bx[None, :], (H, W)))
    assert np.array_equal(fy, np.broadcast_to(by[:, None], (H, W)))


def test_bank_gradients_satisfy_the_adjoint_identity():
    # the render is linear in the bank: <render(B), g> = <B, grad_bank(g)>
    N, C, H, W, ks, L = 1, 2, 10, 13, 5, 2
    img = _rand((N, C, H, W), 51)
    g = _rand((N, 2 * C, H, W), 52) - 0.5
    depth = np.random.default_rng(53).uniform(400, 6000, (N, H, W)).astype(np.float32)
    loc = [1, 0]
    radii, iv = [0.0, 0.03, 0.07], [1 / 5000.0, 1 / 1000.0, 1 / 450.0]
    B = _rand((3, 3, L, 2, ks, ks), 54)
    gB = R.render_bank_psf_adjoint(img, g, B.shape, depth, radii, iv, loc, 0.01)
    lhs = np.sum(R.render_bank(img, B, depth, radii, iv, loc, 0.01) * g)
    assert lhs == pytest.approx(np.sum(B * gB), rel=1e-12)
    xs, ys = [0.0, 0.04], [0.0, 0.02, 0.05]
    B2 = _rand((3, 2, 3, L, 2, ks, ks), 55)
    gB2 = R.render_bank2d_psf_adjoint(img, g, B2.shape, depth, xs, ys, iv, loc, 0.01)
    lhs = np.sum(R.render_bank2d(img, B2, depth, xs, ys, iv, loc, 0.01) * g)
    assert lhs == pytest.approx(np.sum(B2 * gB2), rel=1e-12)


@pytest.mark.parametrize("H,W", [(9, 12), (10, 11)])
def test_bank_pixels_equal_the_bank_render_everywhere(H, W):
    # the per-pixel evaluation used for sampled full-size parity is the bank
    # render itself: every pixel of images with an exact centre row (H odd)
    # or centre column (W odd), all four quadrants and all borders
    N, C, ks, ps = 2, 2, 5, 0.01
    rng = np.random.default_rng(31)
    img = rng.uniform(0, 1, (N, C, H, W))
    bank = rng.uniform(0, 1, (4, 3, 2, 2, ks, ks))
    radii = [0.0, 0.02, 0.04, 0.06]
    iv = [1 / 5000.0, 1 / 2000.0, 1 / 500.0]
    dmap = rng.uniform(500, 5000, (N, H, W)).astype(np.float32)
    loc = [1, 0]
    full = R.render_bank(img, bank, dmap, radii, iv, loc, ps)
    pix = [(n, y, x) for n in range(N) for y in range(H) for x in range(W)]
    got = R.render_bank_pixels(img, bank, dmap, radii, iv, loc, ps, pix)
    ref = np.stack([full[n, :, y, x] for (n, y, x) in pix])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # the lookup reaches every mirror combination in these images
    fi, di, mx, my = R.bank_lookup(H, W, dmap[0], radii, iv, ps)
    assert {(a, b) for a, b in zip(mx.ravel(), my.ravel())} == {(False, False), (False, True),
                                                                (True, False), (True, True)}


@pytest.mark.parametrize("H,W", [(9, 12), (10, 11)])
def test_bank_adjoint_pixels_equal_the_bank_adjoint_everywhere(H, W):
    # the per-pixel image adjoint used for sampled full-size parity is the
    # bank adjoint itself, border pixels (where clamped taps fold) included
    N, C, ks, ps = 2, 2, 5, 0.01
    rng = np.random.default_rng(32)
    g = rng.normal(size=(N, 2 * C, H, W))
    bank = rng.uniform(0, 1, (4, 3, 2, 2, ks, ks))
    radii = [0.0, 0.02, 0.04, 0.06]
    iv = [1 / 5000.0, 1 / 2000.0, 1 / 500.0]
    dmap = rng.uniform(500, 5000, (N, H, W)).astype(np.float32)
    loc = [1, 0]
    full = R.render_bank_adjoint(g, bank, dmap, radii, iv, loc, ps)
    pix = [(n, y, x) for n in range(N) for y in range(H) for x in range(W)]
    got = R.render_bank_adjoint_pixels(g, bank, dmap, radii, iv, loc, ps, pix)
    ref = np.stack([full[n, :, y, x] for (n, y, x) in pix])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
