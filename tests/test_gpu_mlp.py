"""GPU parity of the bf16 matrix-core PSF surrogate (forward, loss gradient,
Adam, training) against the CPU oracle's bf16 mirror, through the C ABI."""
import numpy as np
import pytest
import torch

from workloads import scenes
from oracle import mlp as M
from paper_2503_11213_amd import sdirt, _abi as abi
from vjp_bars import vjp_reference, clustered_inputs, compare_flat

pytestmark = pytest.mark.gpu

NORM = dict(x_half=4.5024, y_half=3.0016, iv_lo=1 / 5000, iv_hi=1 / 500, lam_lo=0.486,
            lam_hi=0.656)
REL = 1e-2
# Surrogate render, per output pixel: |out - ref| / max(|ref|, 1e-3) against
# the bf16 mirror's composition.  A rendered pixel is an average of the image
# under the pixel's PSF, so a bf16-level change of a few PSF elements (see
# ELT below) moves it by much less than their own 2^-8; 3e-3 bounds it.
RENDER_ELT = 3e-3


def _desc(n_out=2 * 33 * 33, width=256, n_hidden=5, loss=abi.LOSS_L2MAX):
    return sdirt.make_mlp_desc(n_hidden=n_hidden, width=width, n_out=n_out, n_freq=8, loss=loss,
                               **NORM)


def _params(widths, seed=0):
    layers = scenes.mlp_init(widths, seed)
    flat = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers]).astype(np.float32)
    return layers, flat


def _inputs(B, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-4.5, 4.5, B), rng.uniform(-3, 3, B),
                     rng.uniform(1 / 5000, 1 / 500, B),
                     rng.choice([0.486, 0.55, 0.656], B)], 1).astype(np.float32)


def _targets(B, n, seed):
    t = np.random.default_rng(seed).uniform(0, 1, (B, n)) ** 6
    return (t / t.sum(axis=1, keepdims=True)).astype(np.float32)


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def _oracle_params(layers):
    return [(W.astype(np.float64), b.astype(np.float64)) for W, b in layers]


def test_param_count():
    assert sdirt.mlp_n_params(_desc()) == 839554


@pytest.mark.parametrize("B,ws", [(128, 128), (200, 64)])
def test_forward_matches_bf16_mirror(B, ws):
    widths = [64, 256, 256, 256, 256, 256, 2178]
    layers, flat = _params(widths, 0)
    x = _inputs(B, 1)
    d = _desc()
    ws_t = sdirt.mlp_workspace(d, ws)
    p = sdirt.mlp_forward(d, torch.from_numpy(flat).cuda(), torch.from_numpy(x).cuda(), ws_t, ws)
    p = p.cpu().numpy()
    ref, _ = M.forward(_oracle_params(layers), x.astype(np.float64), NORM, bf16=True)
    assert np.allclose(p.sum(axis=1), 1.0, atol=1e-4)
    print("forward f32 out: max elementwise %.2e, rel L2 %.2e" % (_elementwise(p, ref),
                                                                  _rel_l2(p, ref)))
    assert _elementwise(p, ref) <= ELT
    pb = sdirt.mlp_forward(d, torch.from_numpy(flat).cuda(), torch.from_numpy(x).cuda(), ws_t,
                           ws, out_dtype=abi.BF16).float().cpu().numpy()
    print("forward bf16 out: max elementwise %.2e" % _elementwise(pb, ref))
    assert _elementwise(pb, ref) <= ELT


@pytest.mark.parametrize("loss", ["l2max", "kl"])
def test_gradients_match_bf16_mirror(loss):
    widths = [64, 256, 256, 256, 256, 256, 2178]
    layers, flat = _params(widths, 2)
    B = 256
    x = _inputs(B, 3)
    t = _targets(B, 2178, 4)
    t[:, :100] = 0.0
    t /= t.sum(axis=1, keepdims=True)
    d = _desc(loss=abi.LOSS_KL if loss == "kl" else abi.LOSS_L2MAX)
    ws_t = sdirt.mlp_workspace(d, B)
    g, lval = sdirt.mlp_backward(d, torch.from_numpy(flat).cuda(), torch.from_numpy(x).cuda(),
                                 torch.from_numpy(t).cuda(), ws_t)
    g = g.cpu().numpy()
    P = _oracle_params(layers)
    p, cache = M.forward(P, x.astype(np.float64), NORM, bf16=True)
    ref = M.backward(P, p, cache, t.astype(np.float64), bf16=True, kind=loss)
    assert lval.item() == pytest.approx(M.loss(p, t.astype(np.float64), kind=loss), rel=1e-3)
    off = 0
    for (W, b), (gW, gb) in zip(layers, ref):
        nW = W.size
        assert _rel_l2(g[off:off + nW].reshape(W.shape), gW) <= REL
        off += nW
        assert _rel_l2(g[off:off + b.size], gb) <= REL
        off += b.size
    assert off == g.size


@pytest.mark.parametrize("n,ws,spread", [(200, 128, 0.02), (256, 4096, 0.05)])
def test_vjp_matches_bf16_mirror(n, ws, spread):
    # gradient of sum_rows <g, P(x)> for inputs near one point and an upstream
    # gradient shared by the rows up to 20 % (sums over rows that add up; the
    # independent-row case is the chunk test below)
    widths = [64, 256, 256, 256, 256, 256, 2178]
    layers, flat = _params(widths, 8)
    x = clustered_inputs(n, 9, spread=spread)
    rng = np.random.default_rng(10)
    g = (rng.normal(size=(1, 2178)) + 0.2 * rng.normal(size=(n, 2178))).astype(np.float32)
    d = _desc()
    ws_t = sdirt.mlp_workspace(d, ws)
    grads, val = sdirt.mlp_vjp(d, torch.from_numpy(flat).cuda(), torch.from_numpy(x).cuda(),
                               torch.from_numpy(g).cuda(), ws_t, ws)
    g64 = g.astype(np.float64)
    p, ref = vjp_reference(_oracle_params(layers), x.astype(np.float64), g64, NORM)
    assert abs(val.item() - M.loss(p, g64, kind="vjp")) <= 1e-3 * np.abs(p * g64).sum()
    compare_flat(grads.cpu().numpy(), layers, ref)


def test_vjp_chunks_add_up():
    # rows are independent up to the weight-gradient sums: one chunk, two
    # chunks with a ragged tail padded in the workspace, four chunks with a
    # tail of 8 rows give the same gradient up to float32 summation order
    widths = [64, 256, 256, 256, 256, 256, 2178]
    layers, flat = _params(widths, 13)
    n = 200
    x = torch.from_numpy(_inputs(n, 14)).cuda()
    g = torch.from_numpy(np.random.default_rng(15).normal(size=(n, 2178)).astype(np.float32)).cuda()
    d = _desc()
    pt = torch.from_numpy(flat).cuda()
    res = []
    for ws in (4096, 128, 64):
        gr, val = sdirt.mlp_vjp(d, pt, x, g, sdirt.mlp_workspace(d, ws), ws)
        res.append((gr.cpu().numpy(), val.item()))
    for gr, val in res[1:]:
        assert _rel_l2(gr, res[0][0]) <= 1e-5
        assert val == pytest.approx(res[0][1], rel=1e-5, abs=1e-5)
    # dropping one row is far outside that agreement
    g2 = g.clone()
    g2[137] = 0
    gd, _ = sdirt.mlp_vjp(d, pt, x, g2, sdirt.mlp_workspace(d, 128), 128)
    assert _rel_l2(gd.cpu().numpy(), res[0][0]) > 1e-3


def test_vjp_empty_and_constant_gradient():
    widths = [64, 256, 256, 256, 256, 256, 2178]
    layers, flat = _params(widths, 8)
    d = _desc()
    ws_t = sdirt.mlp_workspace(d, 64)
    pt = torch.from_numpy(flat).cuda()
    e, ev = sdirt.mlp_vjp(d, pt, torch.zeros((0, 4), device="cuda"),
                          torch.zeros((0, 2178), device="cuda"), ws_t, 64)
    assert torch.count_nonzero(e).item() == 0 and ev.item() == 0.0
    # a gradient constant along each row does not pass the softmax
    x = torch.from_numpy(_inputs(100, 11)).cuda()
    g = torch.from_numpy(np.random.default_rng(12).normal(size=(100, 2178)).astype(np.float32)).cuda()
    full, _ = sdirt.mlp_vjp(d, pt, x, g, ws_t, 64)
    const, cv = sdirt.mlp_vjp(d, pt, x, torch.full((100, 2178), 2.5, device="cuda"), ws_t, 64)
    assert cv.item() == pytest.approx(250.0, rel=1e-4)
    assert const.abs().max().item() <= 1e-3 * full.abs().max().item()
    with pytest.raises(abi.SdirtError):
        sdirt.mlp_vjp(d, pt, x, g, ws_t, 100)


def test_adam_matches_oracle():
    widths = [64, 256, 256, 256, 256, 256, 2178]
    layers, flat = _params(widths, 5)
    d = _desc()
    rng = np.random.default_rng(6)
    pt = torch.from_numpy(flat).cuda()
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    P = _oracle_params(layers)
    st = M.adam_init(P)
    for step in range(1, 4):
        g = rng.normal(size=flat.size).astype(np.float32) * 1e-2
        sdirt.mlp_adam(d, pt, m, v, torch.from_numpy(g).cuda(), step, 1e-3)
        grads, off = [], 0
        for W, b in layers:
            grads.append((g[off:off + W.size].reshape(W.shape).astype(np.float64),
                          g[off + W.size:off + W.size + b.size].astype(np.float64)))
            off += W.size + b.size
        P = M.adam_step(P, grads, st, 1e-3)
    ref = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in P])
    assert np.max(np.abs(pt.cpu().numpy() - ref)) <= 1e-6


def test_training_reduces_loss():
    # small dataset of smooth synthetic PSF-like targets; loss must drop
    widths = [64, 256, 256, 256, 256, 256, 2 * 9 * 9]
    d = _desc(n_out=2 * 9 * 9)
    layers, flat = _params(widths, 7)
    n = 4096
    x = _inputs(n, 8)
    yy, xx = np.meshgrid(np.arange(9) - 4, np.arange(9) - 4, indexing="ij")
    sig = 0.8 + 2.0 * (x[:, 2] - NORM["iv_lo"]) / (NORM["iv_hi"] - NORM["iv_lo"])
    cx = 1.5 * x[:, 0] / NORM["x_half"]
    t = np.zeros((n, 2, 9, 9))
    for s, sh in ((0, 1.0), (1, -1.0)):
        t[:, s] = np.exp(-((xx[None] - cx[:, None, None] - sh) ** 2 + yy[None] ** 2) /
                         (2 * sig[:, None, None] ** 2))
    t = t.reshape(n, -1)
    t = (t / t.sum(axis=1, keepdims=True)).astype(np.float32)
    pt = torch.from_numpy(flat).cuda()
    m, v = torch.zeros_like(pt), torch.zeros_like(pt)
    B = 256
    ws_t = sdirt.mlp_workspace(d, B)
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    trace = torch.zeros((600,), device="cuda")
    sdirt.mlp_train(d, pt, m, v, xt, tt, ws_t, B, 0, 600, lr0=1e-3, lr_min=1e-4,
                    total_steps=600, seed=3, loss_trace=trace)
    tr = trace.cpu().numpy()
    assert np.all(np.isfinite(tr))
    assert tr[-50:].mean() < 0.2 * tr[:10].mean()


def test_training_resumes_from_a_checkpoint(tmp_path):
    # train 300 steps in one call; then 150, checkpoint to disk, reload and
    # 150 more: training reductions have a fixed order (no atomics in the
    # gradients), so the resumed run lands on the uninterrupted one's bits
    widths = [64, 256, 256, 256, 256, 256, 2 * 9 * 9]
    d = _desc(n_out=2 * 9 * 9, loss=abi.LOSS_KL)
    layers, flat = _params(widths, 9)
    n, B, steps = 4096, 256, 300
    x = torch.from_numpy(_inputs(n, 10)).cuda()
    t = torch.from_numpy(_targets(n, 2 * 9 * 9, 11)).cuda()
    ws_t = sdirt.mlp_workspace(d, B)

    def fresh():
        p = torch.from_numpy(flat).cuda()
        return p, torch.zeros_like(p), torch.zeros_like(p)

    # a schedule other than the trainer's defaults, which the resumed run
    # must take from the checkpoint
    lr0, lr_min = 2e-3, 3e-5
    runs = []
    for _ in range(2):
        p, m, v = fresh()
        tr = torch.zeros((steps,), device="cuda")
        sdirt.mlp_train(d, p, m, v, x, t, ws_t, B, 0, steps, lr0=lr0, lr_min=lr_min,
                        total_steps=steps, seed=5, loss_trace=tr)
        runs.append((p.cpu(), m.cpu(), v.cpu(), tr.cpu()))
    p, m, v = fresh()
    tr1 = torch.zeros((steps // 2,), device="cuda")
    sdirt.mlp_train(d, p, m, v, x, t, ws_t, B, 0, steps // 2, lr0=lr0, lr_min=lr_min,
                    total_steps=steps, seed=5, loss_trace=tr1)
    path = str(tmp_path / "trainer.safetensors")
    sdirt.mlp_save_checkpoint(path, d, p, m, v, step=steps // 2, seed=5, total_steps=steps,
                              lr0=lr0, lr_min=lr_min, batch=B)
    del p, m, v
    d2, p, m, v, step, seed, total, sched = sdirt.mlp_load_checkpoint(path)
    assert sched == {"lr0": lr0, "lr_min": lr_min, "batch": B}
    B2 = sched["batch"]
    tr2 = torch.zeros((steps - step,), device="cuda")
    sdirt.mlp_train(d2, p, m, v, x, t, sdirt.mlp_workspace(d2, B2), B2, step, steps - step,
                    lr0=sched["lr0"], lr_min=sched["lr_min"], total_steps=total, seed=seed,
                    loss_trace=tr2)
    ref, ref_m, ref_v, ref_tr = runs[0]
    assert all(torch.equal(a, b) for a, b in zip(runs[0][:3], runs[1][:3]))
    assert torch.equal(p.cpu(), ref) and torch.equal(m.cpu(), ref_m) and torch.equal(v.cpu(), ref_v)
    # the reported losses are sums over rows in atomic order: equal to rounding
    resumed = torch.cat([tr1.cpu(), tr2.cpu()])
    assert torch.allclose(resumed, ref_tr, rtol=1e-5, atol=1e-7)


def test_invalid_batch_is_rejected():
    d = _desc()
    with pytest.raises(RuntimeError):
        sdirt.mlp_workspace(d, 100)


@pytest.mark.parametrize("n_out", [99, 64, 130])
def test_fused_forward_output_widths(n_out):
    # odd widths take the 2-byte bf16 store path; 64 is one exact tile; 130
    # leaves a 2-column tail tile
    widths = [64, 256, 256, 256, 256, 256, n_out]
    layers, flat = _params(widths, 12)
    x = _inputs(70, 13)
    d = _desc(n_out=n_out)
    ws_t = sdirt.mlp_workspace(d, 64)
    ref, _ = M.forward(_oracle_params(layers), x.astype(np.float64), NORM, bf16=True)
    for dt in (abi.F32, abi.BF16):
        p = sdirt.mlp_forward(d, torch.from_numpy(flat).cuda(), torch.from_numpy(x).cuda(), ws_t,
                              64, out_dtype=dt).float().cpu().numpy()
        assert _elementwise(p, ref) <= ELT
        assert np.allclose(p.sum(axis=1), 1.0, atol=2e-2 if dt == abi.BF16 else 1e-4)


def test_inference_full_size_sampled_rows():
    # the benchmarked launch: 2^20 rows with a workspace for 65536 (one
    # chunk of activations), ks 33, bf16 out; sampled rows (the 256-row
    # workgroup edges at 65536 among them) against the bf16 mirror,
    # and every row's probabilities summing to one
    from workloads import configs
    n, chunk, n_out = 1 << 20, 65536, 2 * 33 * 33
    norm = configs.config4_desc_kwargs()
    d = sdirt.make_mlp_desc(n_out=n_out, **norm)
    layers, flat = _params([64, 256, 256, 256, 256, 256, n_out], 0)
    _, x = configs.surrogate_points(n, seed=9)
    ws_t = sdirt.mlp_workspace(d, chunk)
    ob = torch.empty((n, n_out), dtype=torch.bfloat16, device="cuda")
    sdirt.mlp_forward(d, torch.from_numpy(flat).cuda(), torch.from_numpy(x).cuda(), ws_t, chunk,
                      out_dtype=abi.BF16, out=ob)
    sums = torch.sum(ob, dim=1, dtype=torch.float32).cpu().numpy()
    assert np.all(np.abs(sums - 1.0) <= 2e-2)
    rng = np.random.default_rng(10)
    rows = np.concatenate([[0, chunk - 1, chunk, n - 1], rng.integers(0, n, 60)])
    got = ob[torch.from_numpy(rows).cuda()].float().cpu().numpy()
    ref, _ = M.forward(_oracle_params(layers), x[rows].astype(np.float64), norm, bf16=True)
    err = _elementwise(got, ref)
    print("full-size inference max elementwise", err, "rel L2", _rel_l2(got, ref))
    assert err <= ELT


@pytest.mark.parametrize("ks,N,C,H,W,ws", [(9, 2, 3, 20, 27, 128), (33, 1, 3, 18, 21, 4096),
                                          (5, 1, 1, 9, 8, 64)])
def test_surrogate_render_matches_oracle(ks, N, C, H, W, ws):
    # per-pixel network PSFs consumed by the renderer in one pass; ragged
    # 8 x 8 tiles, workgroups with idle waves, one and three channels
    widths = [64, 256, 256, 256, 256, 256, 2 * ks * ks]
    layers, flat = _params(widths, 3)
    rng = np.random.default_rng(4)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    depth = rng.uniform(500, 5000, (N, H, W)).astype(np.float32)
    lams = [0.656, 0.55, 0.486][:C]
    pitch = 0.3
    d = _desc(n_out=2 * ks * ks)
    ws_t = sdirt.mlp_workspace(d, ws)
    out = sdirt.mlp_render(d, torch.from_numpy(flat).cuda(), torch.from_numpy(img).cuda(),
                           torch.from_numpy(depth).cuda(), lams, pitch, ws_t, ws)
    got = out.cpu().numpy()
    ref = M.render_surrogate(_oracle_params(layers), img, depth, lams, pitch, NORM, bf16=True)
    err = float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)).max())
    print("surrogate render max per-pixel rel err", err, "rel L2", _rel_l2(got, ref))
    assert err <= RENDER_ELT
    # the two sides together average the window: totals match the box filter
    # of a constant image exactly
    one = torch.ones((N, C, H, W), device="cuda")
    o1 = sdirt.mlp_render(d, torch.from_numpy(flat).cuda(), one, torch.from_numpy(depth).cuda(),
                          lams, pitch, ws_t, ws).cpu().numpy()
    assert np.allclose(o1[:, :C] + o1[:, C:], 1.0, atol=1e-5)


@pytest.mark.parametrize("chunk", [65536, 262144])
def test_surrogate_render_full_size_sampled_pixels(chunk):
    # 1680 x 1120 RGB, ks 33 (5,644,800 pixel rows): with a workspace for
    # 65536 rows (2.8 GB) the activations go in two chunks, with the
    # benchmarked one for 262144 rows in one
    ks, N, C, H, W, ps = 33, 1, 3, 1120, 1680, 0.00536
    widths = [64, 256, 256, 256, 256, 256, 2 * ks * ks]
    layers, flat = _params(widths, 5)
    img = scenes.aif_blobs(H, W, C, n_blobs=300, seed=0)[None]
    depth = scenes.depth_voronoi(H, W, 500.0, 5000.0, seed=100)[None].astype(np.float32)
    lams = [0.656, 0.55, 0.486]
    norm = dict(x_half=W * ps / 2, y_half=H * ps / 2, iv_lo=0.2e-3, iv_hi=2.0e-3,
                lam_lo=0.486, lam_hi=0.656)
    d = sdirt.make_mlp_desc(n_hidden=5, width=256, n_out=2 * ks * ks, n_freq=8, **norm)
    ws_t = sdirt.mlp_workspace(d, chunk)
    out = sdirt.mlp_render(d, torch.from_numpy(flat).cuda(), torch.from_numpy(img).cuda(),
                           torch.from_numpy(depth).cuda(), lams, ps, ws_t, chunk).cpu().numpy()
    x = M.pixel_inputs(N, C, H, W, ps, depth, lams)
    rng = np.random.default_rng(8)
    pix = [(0, 0), (H - 1, W - 1), (0, W - 1), (H - 1, 0), (560, 840), (7, 8)] + \
          [(int(rng.integers(H)), int(rng.integers(W))) for _ in range(30)]
    pad = (ks - 1) // 2
    got, ref = [], []
    for (y, xx) in pix:
        p, _ = M.forward(_oracle_params(layers), x[0, y, xx].astype(np.float64), norm, bf16=True)
        rows = np.clip(y + pad - np.arange(ks), 0, H - 1)
        cols = np.clip(xx + pad - np.arange(ks), 0, W - 1)
        for c in range(C):
            win = img[0, c][rows][:, cols]
            K = p[c].reshape(2, ks, ks)
            ref.append([(K[s] * win).sum() for s in range(2)])
            got.append([out[0, c, y, xx], out[0, C + c, y, xx]])
    got, ref = np.array(got), np.array(ref)
    err = float((np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)).max())
    print("full-size surrogate render max per-pixel rel err", err, "rel L2", _rel_l2(got, ref))
    assert err <= RENDER_ELT


# ---- softmax reference raises (large logit spreads) -----------------------
# The fused heads keep a per-row running reference for the softmax that is
# raised whenever a logit passes it; with the He-initialised weights above a
# row's logits spread over about 10 log2 units and the reference rises once.
# These networks shift the output layer's biases so that the row maxima sit
# in later tiles and in tiles of other waves, with spreads of 80-115 log2
# units, so the reference is raised again and again.  (Scaling the output
# weights up instead would scale the logits' bf16-level differences with
# them, and test the bar rather than the raises.)
#
# Per-element bar against the bf16 mirror: the kernels and the mirror round
# the same operands to bf16; they differ only where a float32 sum lands on
# the other side of a bf16 rounding boundary than the float64 sum (one
# element moves by 2^-8 of itself), plus, for bf16 outputs, the output's own
# rounding (2^-9).  A logit moved by d changes its probability by the factor
# exp(d); the bar allows 2^-5 of the row's largest probability per element.
ELT = 2.0 ** -5


def _shaped_layers(widths, seed, kind):
    layers = scenes.mlp_init(widths, seed)
    W, b = layers[-1]
    n = W.shape[0]
    if kind == "ramp":            # rising bias: maxima in the last tiles, 110 log2 units
        b = b + np.linspace(0.0, 110.0 / np.log2(np.e), n)
    elif kind == "peaks":         # four competing outputs in tiles of three waves;
        b = b - 50.0              # the row decides which wins (~80 log2 units)
        for t in (2, 11, 20, (n - 1) // 64):
            b[min(64 * t + 5, n - 1)] += 50.0
    elif kind == "late_tile":     # only the last 64-output tile is competitive
        b = b - 60.0
        b[64 * ((n - 1) // 64):] += 60.0
    layers[-1] = (W.astype(np.float32), b.astype(np.float32))
    flat = np.concatenate([np.concatenate([Wm.ravel(), bb]) for Wm, bb in layers]).astype(np.float32)
    return layers, flat


def _elementwise(got, ref):
    """max |got - ref| over each row, relative to the row's largest ref."""
    return float(np.max(np.abs(got - ref).max(axis=1) / ref.max(axis=1)))


@pytest.mark.parametrize("kind", ["ramp", "peaks", "late_tile"])
def test_inference_head_softmax_raises(kind):
    widths = [64, 256, 256, 256, 256, 256, 2178]
    layers, flat = _shaped_layers(widths, 40, kind)
    x = _inputs(192, 41)
    d = _desc()
    ws_t = sdirt.mlp_workspace(d, 128)
    ref, cache = M.forward(_oracle_params(layers), x.astype(np.float64), NORM, bf16=True)
    z = cache[-1][1] * np.log2(np.e)
    spread = float(np.median(z.max(axis=1) - z.min(axis=1)))
    print(kind, "median logit spread (log2 units) %.1f" % spread)
    assert spread > 64
    for dt in (abi.F32, abi.BF16):
        p = sdirt.mlp_forward(d, torch.from_numpy(flat).cuda(), torch.from_numpy(x).cuda(), ws_t,
                              128, out_dtype=dt).float().cpu().numpy()
        e = _elementwise(p, ref)
        print(kind, "bf16 out" if dt == abi.BF16 else "f32 out", "max elementwise %.2e" % e,
              "rel L2 %.2e" % _rel_l2(p, ref))
        assert e <= ELT
        assert np.allclose(p.sum(axis=1), 1.0, atol=2e-2 if dt == abi.BF16 else 1e-4)


@pytest.mark.parametrize("kind", ["ramp", "peaks", "late_tile"])
def test_render_head_softmax_raises(kind):
    ks, N, C, H, W, ws = 33, 1, 3, 12, 17, 128
    widths = [64, 256, 256, 256, 256, 256, 2 * ks * ks]
    layers, flat = _shaped_layers(widths, 42, kind)
    rng = np.random.default_rng(43)
    img = rng.uniform(0, 1, (N, C, H, W)).astype(np.float32)
    depth = rng.uniform(500, 5000, (N, H, W)).astype(np.float32)
    lams = [0.656, 0.55, 0.486]
    pitch = 0.3
    d = _desc(n_out=2 * ks * ks)
    out = sdirt.mlp_render(d, torch.from_numpy(flat).cuda(), torch.from_numpy(img).cuda(),
                           torch.from_numpy(depth).cuda(), lams, pitch,
                           sdirt.mlp_workspace(d, ws), ws).cpu().numpy()
    ref = M.render_surrogate(_oracle_params(layers), img, depth, lams, pitch, NORM, bf16=True)
    # these PSFs concentrate on a few taps, so a rendered pixel carries the
    # bf16-level error of its largest PSF elements instead of averaging it
    # out: the per-element PSF bar applies per pixel
    err = float((np.abs(out - ref) / np.maximum(np.abs(ref), 1e-3)).max())
    print(kind, "render max per-pixel rel err %.2e" % err)
    assert err <= ELT
