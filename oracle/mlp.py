"""Oracle: the DP-PSF surrogate network (float64, optional bf16 mirror).
Test infrastructure only.

Sec. 3.2 / Supplement S1.4: an MLP maps a normalised point of the valid
imaging region (image position, depth; here also the wavelength) to the
left and right PSFs, trained with the L2 loss of Eq. (4) on ray-traced
PSFs, with max-normalised targets during training and sum-normalised
outputs at inference.  The synthetic workload fixes the shape: a 64-wide
Fourier encoding, five ReLU layers of width 256 and a 2 x 33 x 33 output
normalised by a joint softmax.  Readings:
  * inputs (h_x, h_y, 1/d, lam) are mapped affinely to [-1, 1] (image
    position by the sensor half-size, the frustum normalisation of Sec. 3.2;
    1/d and lam by their training ranges);
  * encoding gamma(v) = [sin(2^k pi v), cos(2^k pi v)], k = 0..7, for each of
    the four inputs, ordered (input, k, sin/cos);
  * the softmax output is already sum-normalised; the max normalisation of
    the targets enters as the per-sample scale of the squared error:
        loss = mean_b sum_i ((p_bi - t_bi) / max_j t_bj)^2,
    with t the jointly sum-normalised traced PSF ("l2max");
  * alternative training loss (not the paper's): the Kullback-Leibler
    divergence of p from t,  loss = mean_b sum_i t_bi log(t_bi / p_bi)
    (0 log 0 = 0), whose logit gradient (p sum(t) - t) / B does not vanish
    on outputs the network predicts as empty ("kl");
  * optimiser Adam(beta1 0.9, beta2 0.999, eps 1e-8).
bf16 mirror: weights and every GEMM operand are rounded to bfloat16
(round-to-nearest-even, through float32) where the device kernels round
them; sums stay in float64.
"""

import numpy as np

N_FREQ = 8
N_IN = 4
N_FEAT = 2 * N_FREQ * N_IN
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def to_bf16(a):
    """Round to bfloat16 (nearest, ties to even) via float32; returns f64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def normalise_inputs(x, norm):
    """x [B, 4] = (h_x mm, h_y mm, 1/d 1/mm, lam um) -> [-1, 1]^4."""
    x = np.asarray(x, dtype=np.float64)
    v = np.empty_like(x)
    v[:, 0] = x[:, 0] / norm["x_half"]
    v[:, 1] = x[:, 1] / norm["y_half"]
    v[:, 2] = 2.0 * (x[:, 2] - norm["iv_lo"]) / (norm["iv_hi"] - norm["iv_lo"]) - 1.0
    v[:, 3] = 2.0 * (x[:, 3] - norm["lam_lo"]) / (norm["lam_hi"] - norm["lam_lo"]) - 1.0
    return v


def encode(x, norm):
    v = normalise_inputs(x, norm)
    B = v.shape[0]
    out = np.empty((B, N_FEAT))
    for i in range(N_IN):
        for k in range(N_FREQ):
            arg = (2.0 ** k) * np.pi * v[:, i]
            out[:, i * 2 * N_FREQ + 2 * k] = np.sin(arg)
            out[:, i * 2 * N_FREQ + 2 * k + 1] = np.cos(arg)
    return out


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def forward(params, x, norm, bf16=False):
    """params: list of (W [out, in], b [out]).  Returns probabilities
    [B, out] and the cache of layer inputs / pre-activations."""
    rnd = to_bf16 if bf16 else (lambda a: a)
    h = encode(x, norm)
    cache = []
    for li, (W, b) in enumerate(params):
        hin = rnd(h)
        a = hin @ rnd(W).T + b
        cache.append((hin, a))
        h = np.maximum(a, 0.0) if li < len(params) - 1 else a
    return softmax(h), cache


def loss(p, t, kind="l2max"):
    """kind "vjp": t is an upstream gradient dL/dp; the value is the sum
    over rows of <t, p> (not averaged)."""
    if kind == "vjp":
        return float(np.sum(p * t))
    if kind == "kl":
        tl = np.where(t > 0.0, t * np.log(np.where(t > 0.0, t, 1.0)), 0.0)
        return float(np.mean(np.sum(tl - t * np.log(p), axis=1)))
    m = t.max(axis=1, keepdims=True)
    return float(np.mean(np.sum(((p - t) / m) ** 2, axis=1)))


def backward(params, p, cache, t, bf16=False, kind="l2max"):
    """Gradients [(dW, db)] of loss(p, t, kind) through softmax and the layers."""
    rnd = to_bf16 if bf16 else (lambda a: a)
    B = p.shape[0]
    if kind == "vjp":
        # softmax Jacobian applied to the upstream gradient t = dL/dp
        dz = p * (t - np.sum(p * t, axis=1, keepdims=True))
    elif kind == "kl":
        dz = (p * t.sum(axis=1, keepdims=True) - t) / B
    else:
        m = t.max(axis=1, keepdims=True)
        gp = 2.0 * (p - t) / (m * m) / B
        dz = p * (gp - np.sum(p * gp, axis=1, keepdims=True))
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        hin, a = cache[li]
        if li < len(params) - 1:
            dz = dz * (a > 0.0)
        dzr = rnd(dz)
        grads[li] = (dzr.T @ hin, dz.sum(axis=0))
        if li > 0:
            dz = dzr @ rnd(W)
    return grads


def adam_step(params, grads, state, lr):
    """One Adam update in place; state = dict(step, m, v)."""
    state["step"] += 1
    t = state["step"]
    out = []
    for li, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (w, g) in enumerate(((W, gW), (b, gb))):
            m = state["m"][li][j] = ADAM_B1 * state["m"][li][j] + (1 - ADAM_B1) * g
            v = state["v"][li][j] = ADAM_B2 * state["v"][li][j] + (1 - ADAM_B2) * g * g
            mh = m / (1 - ADAM_B1 ** t)
            vh = v / (1 - ADAM_B2 ** t)
            new.append(w - lr * mh / (np.sqrt(vh) + ADAM_EPS))
        out.append(tuple(new))
    return out


def adam_init(params):
    return {"step": 0,
            "m": [[np.zeros_like(W), np.zeros_like(b)] for W, b in params],
            "v": [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]}


def pixel_inputs(N, C, H, W, pitch, depth, wavelengths):
    """Network inputs of every pixel and channel, formed in float32 as the
    surrogate render defines them: h_x = (x - (W - 1) / 2) * pitch, h_y
    likewise, 1/d = 1 / depth (float32 division), lambda_c.  Returns
    [N, H, W, C, 4] float32."""
    f32 = np.float32
    pitch = f32(pitch)
    xs = (np.arange(W, dtype=np.float32) - f32(0.5) * f32(W - 1)) * pitch
    ys = (np.arange(H, dtype=np.float32) - f32(0.5) * f32(H - 1)) * pitch
    depth = np.asarray(depth, dtype=np.float32).reshape(N, H, W)
    x = np.empty((N, H, W, C, 4), dtype=np.float32)
    x[..., 0] = xs[None, None, :, None]
    x[..., 1] = ys[None, :, None, None]
    x[..., 2] = (f32(1.0) / depth)[..., None]
    x[..., 3] = np.asarray(wavelengths, dtype=np.float32)[:C][None, None, None, :]
    return x


def render_surrogate(params, img, depth, wavelengths, pitch, norm, bf16=True):
    """Fig. 2(c) / Sec. 3.2: the all-in-focus image rendered with the PSF the
    network predicts for every pixel and channel: the softmax output of
    forward() read as [2][ks][ks] is that pixel's per-channel kernel of the
    dense renderer (oracle.render.render_dense).  img [N, C, H, W]."""
    from oracle import render as R
    img = np.asarray(img, dtype=np.float64)
    N, C, H, W = img.shape
    x = pixel_inputs(N, C, H, W, pitch, depth, wavelengths)
    p, _ = forward(params, x.reshape(-1, 4).astype(np.float64), norm, bf16=bf16)
    ks = int(round(np.sqrt(p.shape[1] // 2)))
    K = p.reshape(N, H, W, C, 2, ks, ks)
    return R.render_dense(img, K)
