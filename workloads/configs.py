"""The synthetic workloads: lens, sensor and PSF query of each benchmark
configuration, and the paper's own PSF-map workload (Sec. 5.1 / Table S3).

  config1  singlet, 4 fields x 1 depth x 1 wavelength, 64x64 rays, ks 31
  config2  12-surface double-Gauss-like lens, 32 radial fields x 16 depths
           (uniform in 1/d over 0.5-5 m) x 3 wavelengths, 512x512 rays,
           ks 63, sensor 1680x1120 at 5.36 um; render 1680x1120 RGB
  config3  config-2 lens, 8 x 8 x 3 points, 256x256 rays, ks 41, tent splat
           (differentiation); render 512x512 RGB with a dense 41x41 map
  paper    RF50 (Table S1) at F/4 focused at 1 m, 512x768 px over 24x36 mm,
           microlens DP model (Eq. (S1)), ks 21, 4096 rays, 550 nm
"""

import numpy as np

from .lens import (Sensor, PsfQuery, DP_SIGMOID, DP_MICROLENS, SPLAT_BOX,
                   SPLAT_TENT, NORM_NONE)
from . import lenses

RGB_LAMBDAS = (0.486, 0.550, 0.656)
LAMBDA_OF_RGB = (2, 1, 0)           # R -> 656 nm, G -> 550 nm, B -> 486 nm


def inverse_uniform_depths(dmin, dmax, n):
    """n depths (mm) uniform in 1/d, in increasing 1/d order."""
    iv = np.linspace(1.0 / dmax, 1.0 / dmin, n)
    return [float(1.0 / v) for v in iv]


def config1():
    lens = lenses.singlet(focus_depth=2000.0, f_number=2.0)
    sensor = Sensor(pitch=0.004, dp_mode=DP_SIGMOID, sigmoid_k=20.0)
    query = PsfQuery(fields=[(0.0, 0.0), (0.5, 0.0), (1.0, 0.0), (1.4, 0.0)],
                     depths=[1000.0], wavelengths=[0.55], rays_x=64, rays_y=64,
                     seed=0, jitter=True, ks=31, splat=SPLAT_BOX, out_f64=True)
    return lens, sensor, query


def config2_lens(seed=0):
    lens = lenses.double_gauss_12(seed)
    lens.focus_depth = 2.0 / (1.0 / 500.0 + 1.0 / 5000.0)   # 1/d midpoint
    lens.ref_wavelength = 0.55
    return lens


def config2(rays=512):
    lens = config2_lens()
    W, H, ps = 1680, 1120, 0.00536
    sensor = Sensor(pitch=ps, dp_mode=DP_SIGMOID, sigmoid_k=20.0, width_px=W,
                    height_px=H)
    half_diag = float(np.hypot(W * ps / 2, H * ps / 2))
    fields = [(k * half_diag / 31.0, 0.0) for k in range(32)]
    query = PsfQuery(fields=fields, depths=inverse_uniform_depths(500.0, 5000.0, 16),
                     wavelengths=list(RGB_LAMBDAS), rays_x=rays, rays_y=rays, seed=0,
                     jitter=True, ks=63, splat=SPLAT_BOX, out_f64=False)
    return lens, sensor, query


def config2_bank2d(rays=512, fx=16, fy=11):
    """The 12-surface lens of config2 traced on a first-quadrant 2-D field
    grid (fx x fy points from the centre to the sensor edges, y-major) for
    the exact-azimuth bank render: the same depths, wavelengths and window.
    Returns lens, sensor, query, list-mode points [P][4], x grid, y grid."""
    lens, sensor, query = config2(rays)
    W, H, ps = sensor.width_px, sensor.height_px, sensor.pitch
    xs = [k * (W * ps / 2) / (fx - 1) for k in range(fx)]
    ys = [m * (H * ps / 2) / (fy - 1) for m in range(fy)]
    # list-mode points in bank order [fy][fx][depth][wavelength]
    points = np.array([(x, y, d, l) for y in ys for x in xs for d in query.depths
                       for l in range(len(query.wavelengths))], dtype=np.float64)
    return lens, sensor, query, points, xs, ys


def config3(rays=256):
    lens = config2_lens()
    W, H, ps = 1680, 1120, 0.00536
    sensor = Sensor(pitch=ps, dp_mode=DP_SIGMOID, sigmoid_k=20.0, width_px=W,
                    height_px=H)
    half_diag = float(np.hypot(W * ps / 2, H * ps / 2))
    fields = [(k * half_diag / 7.0, 0.0) for k in range(8)]
    query = PsfQuery(fields=fields, depths=inverse_uniform_depths(500.0, 5000.0, 8),
                     wavelengths=list(RGB_LAMBDAS), rays_x=rays, rays_y=rays, seed=0,
                     jitter=True, ks=41, splat=SPLAT_TENT, normalize=NORM_NONE,
                     out_f64=False)
    return lens, sensor, query


def paper_psf_map():
    """RF50 at F/4, focus 1 m, 512 x 768 pixels over 24 x 36 mm, microlens
    DP pixels, ks 21, 4096 rays per PSF, 550 nm (Sec. 5.1)."""
    lens = lenses.rf50()
    lens.f_number = 4.0
    lens.focus_depth = 1000.0
    lens.ref_wavelength = 0.55
    H, W = 512, 768
    ps = 36.0 / W
    sensor = Sensor(pitch=ps, dp_mode=DP_MICROLENS, width_px=W, height_px=H)
    query = PsfQuery(fields=[(0.0, 0.0)], depths=[1000.0], wavelengths=[0.55],
                     rays_x=64, rays_y=64, seed=0, jitter=True, ks=21,
                     splat=SPLAT_BOX, out_f64=False)
    return lens, sensor, query, (H, W)


def pixel_points(H, W, ps, depth_map, slot=0):
    """List-mode points (h_x, h_y, depth, slot) for every pixel, row-major."""
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    hx = (xx - (W - 1) / 2.0) * ps
    hy = (yy - (H - 1) / 2.0) * ps
    return np.stack([hx.ravel(), hy.ravel(), np.asarray(depth_map, dtype=np.float64).ravel(),
                     np.full(H * W, float(slot))], axis=1)


def config4_desc_kwargs():
    """Normalisation ranges of the surrogate inputs for the 12-surface lens
    workload: image half-size, 1/d in [0.2, 2] per metre, 486-656 nm."""
    W, H, ps = 1680, 1120, 0.00536
    return dict(x_half=W * ps / 2, y_half=H * ps / 2, iv_lo=0.2e-3, iv_hi=2.0e-3,
                lam_lo=RGB_LAMBDAS[0], lam_hi=RGB_LAMBDAS[-1])


def surrogate_points(n, seed):
    """Random PSF points over the sensor and the depth range of the MLP
    workload: returns list-mode points [n][4] (h_x, h_y, depth, slot) and
    the matching MLP inputs [n][4] (h_x, h_y, 1/d, lambda)."""
    k = config4_desc_kwargs()
    rng = np.random.default_rng(seed)
    hx = rng.uniform(-k["x_half"], k["x_half"], n)
    hy = rng.uniform(-k["y_half"], k["y_half"], n)
    iv = rng.uniform(k["iv_lo"], k["iv_hi"], n)
    slot = rng.integers(0, len(RGB_LAMBDAS), n)
    lam = np.asarray(RGB_LAMBDAS)[slot]
    pts = np.stack([hx, hy, 1.0 / iv, slot.astype(np.float64)], 1)
    x = np.stack([hx, hy, iv, lam], 1).astype(np.float32)
    return pts, x


def config4(rays=512):
    """Lens, sensor and query template (ks 33, SUM-normalised) of the MLP
    surrogate workload; points come from surrogate_points."""
    lens = config2_lens()
    W, H, ps = 1680, 1120, 0.00536
    sensor = Sensor(pitch=ps, dp_mode=DP_SIGMOID, sigmoid_k=20.0, width_px=W, height_px=H)
    from .lens import NORM_SUM
    query = PsfQuery(fields=[(0.0, 0.0)], depths=[1000.0], wavelengths=list(RGB_LAMBDAS),
                     rays_x=rays, rays_y=rays, seed=1, jitter=True, ks=33, splat=SPLAT_BOX,
                     normalize=NORM_SUM, out_f64=False)
    return lens, sensor, query


def pixel_inputs(H, W, ps, depth_map, lambdas=RGB_LAMBDAS):
    """MLP inputs for every pixel and channel of an image, row-major in
    (y, x, channel) with channel c at wavelength lambdas[c]: [H*W*C][4]."""
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    hx = ((xx - (W - 1) / 2.0) * ps).ravel()
    hy = ((yy - (H - 1) / 2.0) * ps).ravel()
    iv = 1.0 / np.asarray(depth_map, dtype=np.float64).ravel()
    C = len(lambdas)
    x = np.empty((H * W, C, 4), dtype=np.float32)
    x[:, :, 0] = hx[:, None]
    x[:, :, 1] = hy[:, None]
    x[:, :, 2] = iv[:, None]
    x[:, :, 3] = np.asarray(lambdas)[None, :]
    return x.reshape(-1, 4)


def config5(rays=1024):
    """Smartphone-like 16-surface aspheric lens (EFL 4.3 mm, f/1.8); sensor
    4032 x 3024 at 1.0 um; 64 radial fields to the half-diagonal x 32 depths
    uniform in 1/d over 0.1-5 m (focus at the 1/d midpoint) x 3 wavelengths;
    ks 65, box splat, sigmoid response."""
    from . import lenses as _l
    lens = _l.phone_lens_16(0)
    lens.focus_depth = 2.0 / (1.0 / 100.0 + 1.0 / 5000.0)
    lens.ref_wavelength = 0.55
    W, H, ps = 4032, 3024, 0.001
    sensor = Sensor(pitch=ps, dp_mode=DP_SIGMOID, sigmoid_k=20.0, width_px=W, height_px=H)
    half_diag = float(np.hypot(W * ps / 2, H * ps / 2))
    fields = [(k * half_diag / 63.0, 0.0) for k in range(64)]
    query = PsfQuery(fields=fields, depths=inverse_uniform_depths(100.0, 5000.0, 32),
                     wavelengths=list(RGB_LAMBDAS), rays_x=rays, rays_y=rays, seed=0,
                     jitter=True, ks=65, splat=SPLAT_BOX, out_f64=False)
    return lens, sensor, query
