"""Seeded synthetic scenes: all-in-focus RGB images and depth maps that stand
in for the RGBD datasets of Sec. 3.2 / Sec. 6 (not available here).

  * AiF image: sum of Gaussian blobs (sigma log-uniform in [2, 64] px,
    independent per-channel amplitudes) plus 1/f noise, min-max scaled to
    [0, 1] per image;
  * depth map: Voronoi regions, each a 3-D plane (inverse depth affine in the
    pixel coordinates), clipped to the depth range -- piecewise planar like
    indoor scenes; a constant depth map gives the planar scenes of Sec. 5.4.
"""

import numpy as np


def aif_blobs(H, W, C=3, n_blobs=2000, seed=0, noise=0.05):
    rng = np.random.default_rng(seed)
    img = np.zeros((C, H, W), dtype=np.float64)
    sig = np.exp(rng.uniform(np.log(2.0), np.log(64.0), n_blobs))
    cy = rng.uniform(0, H, n_blobs)
    cx = rng.uniform(0, W, n_blobs)
    amp = rng.uniform(0.0, 1.0, (n_blobs, C)) * rng.choice([-1.0, 1.0], (n_blobs, 1))
    for k in range(n_blobs):
        r = int(np.ceil(3 * sig[k]))
        y0, y1 = max(0, int(cy[k]) - r), min(H, int(cy[k]) + r + 1)
        x0, x1 = max(0, int(cx[k]) - r), min(W, int(cx[k]) + r + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        gy = np.exp(-0.5 * ((np.arange(y0, y1) - cy[k]) / sig[k]) ** 2)
        gx = np.exp(-0.5 * ((np.arange(x0, x1) - cx[k]) / sig[k]) ** 2)
        g = np.outer(gy, gx)
        img[:, y0:y1, x0:x1] += amp[k][:, None, None] * g[None]
    # 1/f noise
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.rfftfreq(W)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    f[0, 0] = 1.0
    for c in range(C):
        spec = (rng.normal(size=f.shape) + 1j * rng.normal(size=f.shape)) / f
        spec[0, 0] = 0.0
        n = np.fft.irfft2(spec, s=(H, W))
        img[c] += noise * n / (np.std(n) + 1e-12)
    lo, hi = img.min(), img.max()
    return ((img - lo) / (hi - lo)).astype(np.float32)


def depth_voronoi(H, W, dmin, dmax, n_regions=8, seed=100):
    """Piecewise-planar depth map (mm) in [dmin, dmax]."""
    rng = np.random.default_rng(seed)
    ivmin, ivmax = 1.0 / dmax, 1.0 / dmin
    sy = rng.uniform(0, H, n_regions)
    sx = rng.uniform(0, W, n_regions)
    iv0 = rng.uniform(ivmin, ivmax, n_regions)
    gy = rng.uniform(-0.5, 0.5, n_regions) * (ivmax - ivmin)
    gx = rng.uniform(-0.5, 0.5, n_regions) * (ivmax - ivmin)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    best = np.full((H, W), np.inf)
    lab = np.zeros((H, W), dtype=np.int64)
    for k in range(n_regions):
        d2 = (yy - sy[k]) ** 2 + (xx - sx[k]) ** 2
        m = d2 < best
        best[m] = d2[m]
        lab[m] = k
    iv = iv0[lab] + gy[lab] * (yy / H - 0.5) + gx[lab] * (xx / W - 0.5)
    iv = np.clip(iv, ivmin, ivmax)
    return (1.0 / iv).astype(np.float32)


def depth_uniform_inverse(H, W, dmin, dmax, seed=100):
    """Per-pixel depths uniform in 1/d (independent pixels)."""
    rng = np.random.default_rng(seed)
    iv = rng.uniform(1.0 / dmax, 1.0 / dmin, (H, W))
    return (1.0 / iv).astype(np.float32)


def mlp_init(widths, seed=0):
    """He-uniform weights and small uniform biases, float32, [(W, b)]."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip(widths[:-1], widths[1:]):
        bound = np.sqrt(6.0 / a)
        out.append((rng.uniform(-bound, bound, (b, a)).astype(np.float32),
                    rng.uniform(-0.05, 0.05, b).astype(np.float32)))
    return out
