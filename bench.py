"""Benchmark of the DP-PSF hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step = the whole hot path over one batch of the 12-surface lens workload
(32 radial fields x 16 depths x 3 wavelengths = 1536 DP PSFs, 512 x 512 rays
each, ks 63, sensor 1680 x 1120 at 5.36 um):
  1. trace_dp_psf  -- pupil sampling, sequential trace, DP split, box splat;
  2. render_dp     -- 1680 x 1120 RGB image rendered from that PSF bank and a
                      piecewise-planar depth map (bank source);
  3. render_dp_backward -- image adjoint of the same render.
Inputs (lens, image, depth map, upstream gradient) are resident on the GPU
before timing starts.  Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("rays·surfaces/s and DP PSFs/s; render Mpix/s; fwd+bwd vs fwd time; "
          "MLP vs trace PSFs/s")
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Algorithmic FLOPs of the float64 trace (add/mul = 1, fma = 2, div/sqrt = 1):
# per refracting spherical surface 56 (transfer 7, intersection 20, clip 3,
# normal 4, vector Snell 22), per aperture-only surface 10, and 60 per ray for
# pupil sampling, sensor transfer, DP split and binning.
FLOP_SPHERE, FLOP_STOP, FLOP_RAY = 56, 10, 60


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def timed(fn, stream, reps):
    import torch
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    e.synchronize()
    return s.elapsed_time(e) / reps


def cpu_baseline(lens, sensor, query, img, dmap, radii, iv, loc, ps, total_rs,
                 H, W):
    """The float64 oracle on a bounded sample of the same step, scaled to
    the full step and reported in rays*surfaces/s."""
    import numpy as np
    import oracle.psf as opsf
    import oracle.render as orender
    n_surf = 12
    picks = [(f, (5 * f) % 16, f % 3) for f in range(0, 32, 3)]
    t0 = time.perf_counter()
    bank, _ = opsf.trace_dp_psf(lens, sensor, query, points=picks)
    t_trace = time.perf_counter() - t0
    sample_rays = len(picks) * query.n_rays
    crop = 96
    ks = query.ks
    bank6 = bank.reshape(len(query.fields), len(query.depths), len(query.wavelengths), 2, ks, ks)
    y0, x0 = H // 2 - crop // 2, W // 2 - crop // 2
    pix = [(0, y, x) for y in range(y0, y0 + crop) for x in range(x0, x0 + crop)]
    t0 = time.perf_counter()
    orender.render_bank_pixels(img, bank6, dmap, radii, iv, loc, ps, pix)
    t_render = time.perf_counter() - t0
    # the image adjoint reads the same kernels once more: same cost model
    est_step = (t_trace * (query.n_points * query.n_rays) / sample_rays +
                2.0 * t_render * (H * W) / len(pix))
    return {"value": total_rs / est_step, "unit": "rays*surfaces/s", "cores": 1,
            "kind": "oracle",
            "sample": ("float64 NumPy oracle, one process: %d of 1536 PSF points at "
                       "512x512 rays (%.1f s) and a %dx%d-pixel crop of the bank "
                       "render (%.1f s, counted twice for forward + adjoint); step "
                       "time extrapolated linearly to %.0f s" %
                       (len(picks), t_trace, crop, crop, t_render, est_step))}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from workloads import configs, scenes
    from paper_2503_11213_amd import sdirt, _abi as abi

    torch.cuda.init()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    lens, sensor, query = configs.config2()
    H, W, ps = sensor.height_px, sensor.width_px, sensor.pitch
    img_np = scenes.aif_blobs(H, W, 3, n_blobs=2000, seed=0)[None]
    dmap_np = scenes.depth_voronoi(H, W, 500.0, 5000.0, seed=100)[None]
    img = torch.from_numpy(img_np).to(dev)
    dmap = torch.from_numpy(dmap_np).to(dev)
    gout = torch.from_numpy(np.random.default_rng(1).normal(
        size=(1, 6, H, W)).astype(np.float32)).to(dev)
    radii = [f[0] for f in query.fields]
    iv = [1.0 / d for d in query.depths]
    loc = list(configs.LAMBDA_OF_RGB)
    desc, keep = sdirt.make_render_desc(1, 3, H, W, query.ks, source=abi.SRC_BANK,
                                        field_radii=radii, inv_depths=iv,
                                        bank_lambdas=3, lambda_of_channel=loc, pitch=ps)
    P = query.n_points
    bank = torch.empty((P, 2, query.ks, query.ks), dtype=torch.float32, device=dev)
    stats = torch.empty((P, 7), dtype=torch.float64, device=dev)
    out = torch.empty((1, 6, H, W), dtype=torch.float32, device=dev)
    gimg = torch.empty((1, 3, H, W), dtype=torch.float32, device=dev)

    def trace():
        sdirt.trace_dp_psf(lens, sensor, query, out=bank, stats=False)

    def render():
        sdirt.render_dp(desc, img, bank, depth=dmap, out=out)

    def render_bwd():
        sdirt.render_dp_backward(desc, bank, gout, depth=dmap, grad_img=gimg)

    def step():
        trace()
        render()
        render_bwd()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps

    # per-kernel averages with HIP events on the launch stream
    reps = max(2, args.steps)
    ms_trace = timed(trace, stream, reps)
    ms_render = timed(render, stream, reps)
    ms_rbwd = timed(render_bwd, stream, reps)
    _, st = sdirt.trace_dp_psf(lens, sensor, query, out=bank, stats=True)
    st = st.cpu().numpy()

    n_rays = P * query.n_rays
    n_surf = sum(1 for s in lens.surfaces if s.kind != 2)      # refracting
    n_stop = len(lens.surfaces) - n_surf
    rs = n_rays * n_surf
    value = rs / (ms_step * 1e-3)
    flop = n_rays * (FLOP_SPHERE * n_surf + FLOP_STOP * n_stop + FLOP_RAY)
    achieved = flop / (ms_trace * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "rays*surfaces/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "12-surface double-Gauss-like lens (seed 0, f/2, focus 0.909 m); "
                               "32 radial fields x 16 depths (0.5-5 m, uniform 1/d) x 3 "
                               "wavelengths = 1536 DP PSFs, 512x512 rays each, ks 63, "
                               "sigmoid DP response, box splat; render + image adjoint of a "
                               "1680x1120 RGB image from the PSF bank",
                   "psfs": P, "rays_per_psf": query.n_rays, "surfaces": n_surf,
                   "ks": query.ks, "image": [H, W, 3]},
        "roofline": {"kernel": "trace_splat_kernel<double, box, sigmoid, float>",
                     "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": None,
                     "flop_per_launch": flop},
        "trace": {"ms": ms_trace, "rays_surfaces_per_s": rs / (ms_trace * 1e-3),
                  "psfs_per_s": P / (ms_trace * 1e-3),
                  "in_window_energy_fraction": float((st[:, 3] + st[:, 4]).sum() / st[:, 0].sum()),
                  "transmitted_fraction": float(st[:, 2].sum() / st[:, 0].sum())},
        "render": {"fwd_ms": ms_render, "bwd_ms": ms_rbwd,
                   "fwd_mpix_per_s": H * W / (ms_render * 1e-3) / 1e6,
                   "fwd_plus_bwd_over_fwd": (ms_render + ms_rbwd) / ms_render},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(lens, sensor, query, img_np, dmap_np, radii,
                                            iv, loc, ps, rs, H, W)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
