"""Pins of the oracle's PSF surrogate network (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import mlp

NORM = dict(x_half=4.5, y_half=3.0, iv_lo=1 / 5000, iv_hi=1 / 500, lam_lo=0.486, lam_hi=0.656)


def _params(widths, seed):
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip(widths[:-1], widths[1:]):
        bound = np.sqrt(6.0 / a)
        out.append((rng.uniform(-bound, bound, (b, a)), rng.uniform(-0.1, 0.1, b)))
    return out


def _inputs(B, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-4.5, 4.5, B), rng.uniform(-3, 3, B),
                     rng.uniform(1 / 5000, 1 / 500, B), rng.choice([0.486, 0.55, 0.656], B)], 1)


def _targets(B, n, seed):
    t = np.random.default_rng(seed).uniform(0, 1, (B, n)) ** 4
    return t / t.sum(axis=1, keepdims=True)


def test_encoding_range_and_layout():
    x = _inputs(50, 0)
    f = mlp.encode(x, NORM)
    assert f.shape == (50, 64)
    v = mlp.normalise_inputs(x, NORM)
    assert np.all(np.abs(v) <= 1 + 1e-12)
    assert np.allclose(f[:, 16 * 2 + 2 * 3], np.sin(8 * np.pi * v[:, 2]))
    assert np.allclose(f[:, 16 * 3 + 2 * 7 + 1], np.cos(128 * np.pi * v[:, 3]))


def test_forward_backward_match_torch_autograd():
    widths = [64, 16, 16, 16, 16, 16, 50]
    params = _params(widths, 1)
    x = _inputs(7, 2)
    t = _targets(7, 50, 3)
    p, cache = mlp.forward(params, x, NORM)
    assert np.allclose(p.sum(axis=1), 1.0, atol=1e-14)
    grads = mlp.backward(params, p, cache, t)
    # torch float64 re-expression
    h = torch.from_numpy(mlp.encode(x, NORM))
    tw = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    for li, (W, b) in enumerate(tw):
        h = torch.nn.functional.linear(h, W, b)
        if li < len(tw) - 1:
            h = torch.relu(h)
    pt = torch.softmax(h, dim=1)
    tt = torch.from_numpy(t)
    m = tt.max(dim=1, keepdim=True).values
    lt = (((pt - tt) / m) ** 2).sum(1).mean()
    lt.backward()
    assert np.allclose(pt.detach().numpy(), p, atol=1e-14)
    assert mlp.loss(p, t) == pytest.approx(lt.item(), rel=1e-13)
    for (gW, gb), (W, b) in zip(grads, tw):
        assert np.allclose(gW, W.grad.numpy(), rtol=1e-10, atol=1e-15)
        assert np.allclose(gb, b.grad.numpy(), rtol=1e-10, atol=1e-15)


def test_upstream_gradient_backward_matches_torch_autograd():
    # vector-Jacobian product of the network for an upstream gradient
    # dL/dp (the render's kernel-map gradient): torch autograd of <g, p>
    widths = [64, 16, 16, 16, 16, 16, 50]
    params = _params(widths, 5)
    x = _inputs(9, 6)
    g = np.random.default_rng(7).normal(size=(9, 50))
    p, cache = mlp.forward(params, x, NORM)
    grads = mlp.backward(params, p, cache, g, kind="vjp")
    h = torch.from_numpy(mlp.encode(x, NORM))
    tw = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    for li, (W, b) in enumerate(tw):
        h = torch.nn.functional.linear(h, W, b)
        if li < len(tw) - 1:
            h = torch.relu(h)
    lt = (torch.softmax(h, dim=1) * torch.from_numpy(g)).sum()
    lt.backward()
    assert mlp.loss(p, g, kind="vjp") == pytest.approx(lt.item(), rel=1e-13)
    for (gW, gb), (W, b) in zip(grads, tw):
        assert np.allclose(gW, W.grad.numpy(), rtol=1e-10, atol=1e-15)
        assert np.allclose(gb, b.grad.numpy(), rtol=1e-10, atol=1e-15)
    # a constant upstream gradient has no effect through the softmax
    zero = mlp.backward(params, p, cache, np.full_like(g, 3.0), kind="vjp")
    assert max(np.abs(gW).max() for gW, _ in zero) < 1e-12


def test_width8_finite_differences():
    widths = [64, 8, 8, 8, 8, 8, 12]
    params = _params(widths, 4)
    x = _inputs(5, 5)
    t = _targets(5, 12, 6)
    p, cache = mlp.forward(params, x, NORM)
    grads = mlp.backward(params, p, cache, t)
    rng = np.random.default_rng(0)
    for li in (0, 3, 5):
        W, b = params[li]
        for _ in range(3):
            i, j = rng.integers(W.shape[0]), rng.integers(W.shape[1])
            h = 1e-6
            def L(delta):
                P2 = [(w.copy(), bb.copy()) for w, bb in params]
                P2[li][0][i, j] += delta
                return mlp.loss(mlp.forward(P2, x, NORM)[0], t)
            fd = (L(h) - L(-h)) / (2 * h)
            assert grads[li][0][i, j] == pytest.approx(fd, rel=1e-5, abs=1e-10)


def test_adam_matches_torch():
    params = _params([64, 8, 5], 7)
    rng = np.random.default_rng(8)
    st = mlp.adam_init(params)
    tw = [torch.tensor(a) for Wb in params for a in Wb]
    for w in tw:
        w.requires_grad_(True)
    opt = torch.optim.Adam(tw, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    cur = params
    for step in range(3):
        grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in cur]
        cur = mlp.adam_step(cur, grads, st, 1e-3)
        for w, g in zip(tw, [a for gg in grads for a in gg]):
            w.grad = torch.from_numpy(g)
        opt.step()
    for a, w in zip([a for Wb in cur for a in Wb], tw):
        assert np.allclose(a, w.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(9).normal(size=10000) * 10.0 ** np.random.default_rng(10).integers(-8, 8, 10000)
    ours = mlp.to_bf16(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_kl_loss_and_gradient_match_torch_library():
    # pinned to torch's own KL divergence and soft-target cross entropy
    widths = [64, 16, 16, 16, 16, 16, 50]
    params = _params(widths, 11)
    x = _inputs(6, 12)
    t = _targets(6, 50, 13)
    t[0, :7] = 0.0                      # empty outputs (0 log 0 = 0)
    t /= t.sum(axis=1, keepdims=True)
    p, cache = mlp.forward(params, x, NORM)
    grads = mlp.backward(params, p, cache, t, kind="kl")
    h = torch.from_numpy(mlp.encode(x, NORM))
    tw = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    for li, (W, b) in enumerate(tw):
        h = torch.nn.functional.linear(h, W, b)
        if li < len(tw) - 1:
            h = torch.relu(h)
    tt = torch.from_numpy(t)
    kl = torch.nn.functional.kl_div(torch.log_softmax(h, dim=1), tt, reduction="batchmean")
    assert mlp.loss(p, t, kind="kl") == pytest.approx(kl.item(), rel=1e-12)
    # the cross entropy differs from the KL divergence by the target entropy only
    ce = torch.nn.functional.cross_entropy(h, tt)
    ce.backward()
    for (gW, gb), (W, b) in zip(grads, tw):
        assert np.allclose(gW, W.grad.numpy(), rtol=1e-10, atol=1e-15)
        assert np.allclose(gb, b.grad.numpy(), rtol=1e-10, atol=1e-15)


def _surrogate_case(ks, seed):
    rng = np.random.default_rng(seed)
    N, C, H, W = 1, 2, 11, 14
    img = rng.uniform(0, 1, (N, C, H, W))
    depth = rng.uniform(500, 5000, (N, H, W))
    params = _params([64, 16, 2 * ks * ks], seed)
    return img, depth, params


def test_surrogate_render_uniform_psf_is_half_the_box_mean():
    # zero output layer: every PSF is uniform, 1 / (2 ks^2) per tap, so each
    # side is half the mean of the replicate-padded ks x ks window
    from scipy.ndimage import uniform_filter
    ks = 5
    img, depth, params = _surrogate_case(ks, 1)
    W_out, b_out = params[-1]
    params[-1] = (np.zeros_like(W_out), np.zeros_like(b_out))
    out = mlp.render_surrogate(params, img, depth, [0.5, 0.6], 0.01, NORM, bf16=False)
    for c in range(2):
        box = uniform_filter(img[0, c], size=ks, mode="nearest")
        assert np.allclose(out[0, c], box / 2, atol=1e-12)
        assert np.allclose(out[0, 2 + c], box / 2, atol=1e-12)


@pytest.mark.parametrize("side,i,j", [(0, 2, 2), (1, 0, 0), (1, 4, 1)])
def test_surrogate_render_delta_psf_shifts_the_image(side, i, j):
    # one dominant logit: the PSF is a unit impulse at tap (i, j) of one side,
    # which reads img[clamp(y + pad - i), clamp(x + pad - j)]
    ks, pad = 5, 2
    img, depth, params = _surrogate_case(ks, 2)
    W_out, b_out = params[-1]
    b = np.zeros_like(b_out)
    b[side * ks * ks + i * ks + j] = 200.0
    params[-1] = (np.zeros_like(W_out), b)
    out = mlp.render_surrogate(params, img, depth, [0.5, 0.6], 0.01, NORM, bf16=False)
    H, W = img.shape[2:]
    rows = np.clip(np.arange(H) + pad - i, 0, H - 1)
    cols = np.clip(np.arange(W) + pad - j, 0, W - 1)
    for c in range(2):
        shifted = img[0, c][rows][:, cols]
        assert np.allclose(out[0, side * 2 + c], shifted, atol=1e-12)
        assert np.allclose(out[0, (1 - side) * 2 + c], 0.0, atol=1e-12)


def test_surrogate_pixel_inputs():
    depth = np.full((1, 3, 5), 2000.0)
    x = mlp.pixel_inputs(1, 2, 3, 5, 0.25, depth, [0.5, 0.6])
    assert x.dtype == np.float32
    assert np.array_equal(x[0, 1, :, 0, 0], np.float32([-0.5, -0.25, 0.0, 0.25, 0.5]))
    assert np.array_equal(x[0, :, 2, 1, 1], np.float32([-0.25, 0.0, 0.25]))
    assert np.all(x[..., 2] == np.float32(1.0) / np.float32(2000.0))
    assert np.all(x[..., 0, 3] == np.float32(0.5)) and np.all(x[..., 1, 3] == np.float32(0.6))
