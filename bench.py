"""Benchmark of the DP-PSF hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step = the whole hot path over one batch of the largest workload, the
16-surface aspheric phone lens (EFL 4.3 mm, f/1.8; sensor 4032 x 3024 at
1.0 um): 64 radial fields x 32 depths (0.1-5 m, uniform in 1/d) x 3
wavelengths = 6144 DP PSFs of 1024 x 1024 rays each, ks 65:
  1. trace_dp_psf  -- pupil sampling, sequential trace (10 spheres, the stop,
                      6 even aspheres), DP split, box splat;
  2. render_dp     -- a batch of 16 RGB 4032 x 3024 images rendered from that
                      PSF bank and piecewise-planar depth maps (bank source);
  3. render_dp_backward -- image adjoint of the same render.
Inputs (lens, images, depth maps, upstream gradient) are resident on the GPU
before timing starts.  Prints one JSON line; the other parts of the metric
(the 12-surface lens step, trace adjoint, dense render, surrogate network,
the paper's PSF-map workload, the exact-azimuth bank) ride along in it.
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
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
# three bf16 products per float32 product on the split path
PEAK_SPLIT_BF16_TFLOPS = PEAK_BF16_MFMA_TFLOPS / 3

# Algorithmic FLOPs of the float64 trace (add/mul = 1, fma = 2, div/sqrt/
# rsqrt = 1), counted on the surfaces a ray reaches alive:
#   60 per launched ray: pupil sampling, sensor transfer, DP split, binning;
#   56 per spherical surface (transfer 7, intersection 20, clip 3, normal 4,
#      vector Snell 22); 10 per aperture stop (transfer and clip);
#   78 per even asphere (transfer to the vertex plane 5, base-conic start 19,
#      hit point 5, clip 4, sag slope at the hit 14, unit normal 12, vector
#      Snell 19) plus 48 per Newton iteration (ray point 4, rho 3, sag 20,
#      slope 11, residual 2, derivative 6, step 2).
FLOP_RAY, FLOP_SPHERE, FLOP_STOP, FLOP_ASPH, FLOP_NEWTON = 60, 56, 10, 78, 48
FLOP_OF_KIND = {0: FLOP_SPHERE, 1: FLOP_STOP, 2: FLOP_STOP, 3: FLOP_ASPH, 4: FLOP_STOP}

# Fraction of launched rays alive at each surface and Newton iterations per
# launched ray (summed over the aspheres, at the kernels' stopping rule),
# counted by tests/flop_counts.py on the oracle (64 x 64 rays at 96 of the
# workload's points) and checked against it by tests/test_flop_model.py.
TRACE_COUNTS = {
    "config5": {"alive": [1.0, 0.9861, 0.9659, 0.9659, 0.9173, 0.9173, 0.9173, 0.8989,
                          0.8695, 0.829, 0.8278, 0.8278, 0.8278, 0.8278, 0.8278, 0.8278,
                          0.8278],
                "newton_per_ray": 10.937},
    "config2": {"alive": [1.0, 1.0, 1.0, 0.9998, 0.9998, 0.9998, 0.9998, 0.9929, 0.9929,
                          0.9929, 0.9928, 0.9928, 0.9928],
                "newton_per_ray": 0.0},
    # the paper's PSF map (RF50, microlens DP pixels): 12 x 8 pixel
    # positions x 8 depths, all counted (tests/flop_counts.py)
    "paper_map": {"alive": [1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.979, 0.979, 0.978, 0.9762, 0.9762,
                            0.9762],
                  "newton_per_ray": 5.083},
}


def trace_flop_per_ray(kinds, alive, newton_per_ray):
    """Algorithmic FLOPs per launched ray of a prescription (surface kinds),
    given the alive fraction per surface and Newton iterations per ray."""
    return (FLOP_RAY + FLOP_NEWTON * newton_per_ray +
            sum(a * FLOP_OF_KIND[k] for k, a in zip(kinds, alive)))


# HBM bytes of one trace launch of the headline step, from two rocprofv3
# --pmc runs of `bench.py --pmc-target` (FETCH_SIZE, then WRITE_SIZE), each
# scaled by what the counter reads on a 1 GiB device copy in the same run.
# The figure holds for the kernel sources with this digest only; otherwise
# traffic is null.
TRACE_SOURCES = ("paper_2503_11213_amd/csrc/device_common.hpp",
                 "paper_2503_11213_amd/csrc/trace.hip",
                 "paper_2503_11213_amd/csrc/pack.hpp",
                 "paper_2503_11213_amd/csrc/pack.cpp")
TRACE_TRAFFIC = {"sources_sha256": "c268f48ee4b5955ec676ca7f5660fd2a7b0f8862440f38ee56f6a5c0343b227e",
                 "bytes": 2.542562e8}    # FETCH 9.645e6 B + WRITE 2.4461e8 B


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRACE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--pmc-target", default=None,
                    choices=["calib", "trace", "trace_c2", "trace_paper", "trace_bwd", "render",
                             "render_bwd",
                             "render_split",
                             "render_split_bwd", "dense",
                             "mlp_head", "mlp_render"],
                    help="for counter runs: a 1 GiB device copy (calibration of the memory "
                         "counters), then one launch of the named kernel; prints nothing")
    return ap.parse_args()


def timed(fn, stream, reps):
    import torch
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    e.synchronize()
    return s.elapsed_time(e) / reps


def _oracle_trace_point(args):
    """One PSF point through the float64 oracle (a pool worker's task);
    returns its time only (the bank it fills is not sent back)."""
    lens, sensor, query, point = args
    import oracle.psf as opsf
    t0 = time.perf_counter()
    opsf.trace_dp_psf(lens, sensor, query, points=[point])
    return time.perf_counter() - t0


def _oracle_render_rows(args):
    """Bank-render pixels of an image crop through the float64 oracle (a
    pool worker's task); the bank is the workload's shape, zero-filled here
    (the oracle's cost does not depend on the kernel values)."""
    img, dmap, bank_shape, radii, iv, loc, ps, pix = args
    import numpy as np
    import oracle.render as orender
    bank6 = np.zeros(bank_shape)
    t0 = time.perf_counter()
    orender.render_bank_pixels(img, bank6, dmap, radii, iv, loc, ps, pix)
    return time.perf_counter() - t0


def cpu_baseline(lens, sensor, query, step_rs, img1, dmap1, n_images):
    """The float64 oracle on a bounded sample of the step, timed on the
    host's cores (a process pool, one PSF point or pixel block per task) and
    on one core, scaled to the whole step, in the step's unit."""
    import multiprocessing as mp
    import numpy as np
    import copy
    cores = min(len(os.sched_getaffinity(0)), 16)
    F, D, L = len(query.fields), len(query.depths), len(query.wavelengths)
    picks = [(f, (7 * f + 3 * k) % D, (f + k) % L) for f in range(0, F, 2) for k in range(2)]
    # 512 x 512 of each point's 1024 x 1024 rays: the oracle's cost is
    # linear in the ray count (whole-bundle array operations)
    q = copy.copy(query)
    q.rays_x = q.rays_y = 512
    ray_scale = query.n_rays / q.n_rays
    H, W = dmap1.shape
    ks = query.ks
    bank_shape = (F, D, L, 2, ks, ks)
    radii = [f[0] for f in query.fields]
    iv = [1.0 / d for d in query.depths]
    from workloads import configs
    loc = list(configs.LAMBDA_OF_RGB)
    # render sample: 8 x 128 pixels per process, inside a 256 x 256 crop of
    # the image and depth map away from its borders (a pixel's cost does not
    # depend on where it is)
    cy, cx = H // 2 - 128, W // 2 - 128
    crop_img = np.ascontiguousarray(img1[None, :, cy:cy + 256, cx:cx + 256])
    crop_dm = np.ascontiguousarray(dmap1[None, cy:cy + 256, cx:cx + 256])
    blocks = [[(0, y, x) for y in range(64 + 8 * k, 72 + 8 * k) for x in range(64, 192)]
              for k in range(cores)]
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_trace_point, [(lens, sensor, q, p) for p in picks])
        t_trace = time.perf_counter() - t0
        args = [(crop_img, crop_dm, bank_shape, radii, iv, loc, sensor.pitch, blk)
                for blk in blocks]
        t0 = time.perf_counter()
        pool.map(_oracle_render_rows, args)
        t_render = time.perf_counter() - t0
    for k, v in env.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    # one core: one PSF point and one pixel block in this process
    t1_trace = _oracle_trace_point((lens, sensor, q, picks[0]))
    t1_render = _oracle_render_rows(args[0])
    n_pix_sample = sum(len(b) for b in blocks)
    full_pixels = n_images * H * W
    # forward and image adjoint read the same kernels: twice the forward
    est = (t_trace * ray_scale * query.n_points / len(picks) +
           2.0 * t_render * full_pixels / n_pix_sample)
    est1 = (t1_trace * ray_scale * query.n_points +
            2.0 * t1_render * full_pixels / len(blocks[0]))
    return {"value": step_rs / est, "unit": "rays*surfaces/s", "cores": cores,
            "kind": "oracle",
            "one_core_value": step_rs / est1,
            "sample": ("float64 NumPy oracle in a pool of %d processes: %d of %d PSF points "
                       "at 512x512 of their 1024x1024 rays (%.1f s) and %d pixels of the bank "
                       "render (%.1f s, counted twice for forward + adjoint), scaled linearly "
                       "to the step's %d PSFs x 1024^2 rays and %d x %dx%d pixels: %.0f s per "
                       "step; one core (one point %.2f s, %d pixels %.2f s): %.0f s per step" %
                       (cores, len(picks), query.n_points, t_trace, n_pix_sample, t_render,
                        query.n_points, n_images, W, H, est, t1_trace, len(blocks[0]),
                        t1_render, est1))}


def extras(dev, stream):
    """The other parts of the metric, each timed with HIP events on the
    launch stream: trace adjoint (fwd+bwd vs fwd), dense render (HBM-bound),
    MLP vs trace PSFs/s at ks 33, and the paper's own PSF-map workload."""
    import numpy as np
    import torch
    from workloads import configs, scenes
    from paper_2503_11213_amd import sdirt, _abi as abi
    out = {}
    # 1. adjoint of trace + splat, 8 x 8 x 3 points, 256^2 rays, ks 41, tent
    lens, sensor, query = configs.config3()
    psf, _ = sdirt.trace_dp_psf(lens, sensor, query, stats=False)
    G = torch.randn_like(psf)
    f = lambda: sdirt.trace_dp_psf(lens, sensor, query, out=psf, stats=False)
    b = lambda: sdirt.trace_dp_psf_backward(lens, sensor, query, G)
    f(); b()
    tf, tb = timed(f, stream, 3), timed(b, stream, 3)
    out["adjoint"] = {"workload": "12-surface lens, 192 PSFs x 256^2 rays, ks 41, tent splat",
                      "fwd_ms": tf, "bwd_ms": tb, "fwd_plus_bwd_over_fwd": (tf + tb) / tf}
    print("adjoint done", file=sys.stderr, flush=True)
    # 2. dense render: 512 x 512 RGB, per-channel 41 x 41 kernels, float32
    N, C, H, W, ks = 1, 3, 512, 512, 41
    K = torch.rand((N, H, W, C, 2, ks, ks), device=dev)
    img = torch.rand((N, C, H, W), device=dev)
    gout = torch.randn((N, 2 * C, H, W), device=dev)
    desc, keep = sdirt.make_render_desc(N, C, H, W, ks)
    o = sdirt.render_dp(desc, img, K)
    gi = sdirt.render_dp_backward(desc, K, gout)
    tf = timed(lambda: sdirt.render_dp(desc, img, K, out=o), stream, 3)
    tb = timed(lambda: sdirt.render_dp_backward(desc, K, gout, grad_img=gi), stream, 3)
    # gradient with respect to the kernel map (written once: 10.6 GB)
    gK = torch.empty_like(K)
    sdirt.render_dp_psf_backward(desc, img, gout, grad_psf=gK)
    tk = timed(lambda: sdirt.render_dp_psf_backward(desc, img, gout, grad_psf=gK), stream, 3)
    nbytes = K.numel() * 4
    out["render_dense"] = {"workload": "512x512 RGB, dense per-pixel per-channel 41x41 f32 map",
                           "fwd_ms": tf, "bwd_ms": tb, "fwd_gbs": nbytes / tf / 1e6,
                           "bwd_gbs": nbytes / tb / 1e6, "fwd_hbm_frac": nbytes / tf / 1e6 / PEAK_HBM_GBS,
                           "fwd_plus_bwd_over_fwd": (tf + tb) / tf,
                           "mpix_per_s": H * W / tf / 1e3,
                           "kernel_grad_ms": tk, "kernel_grad_gbs": nbytes / tk / 1e6,
                           "kernel_grad_hbm_frac": nbytes / tk / 1e6 / PEAK_HBM_GBS}
    del K, gK, gout, gi, o
    print("dense render done", file=sys.stderr, flush=True)
    # 3. the trained surrogate (workloads/surrogate_ks33.safetensors, written by
    #    the surrogate workflow: 200k traced PSFs, 20k steps) against tracing
    #    at ks 33 on the 12-surface lens: its error on fresh points against
    #    8192^2-ray traces, its speed against tracing at the ray count of the
    #    same error, and the network with the tracer as fallback at <= 2 %
    out["mlp_vs_trace"] = surrogate_vs_trace(dev, stream)
    desc, params, _ = sdirt.mlp_load_weights(
        os.path.join(ROOT, "workloads", "surrogate_ks33.safetensors"), device=dev)
    ws = sdirt.mlp_workspace(desc, 65536)
    # 3b. the surrogate workload end to end: per-pixel MLP PSFs (bf16, one per
    #     pixel and wavelength) for a batch of 8 images of 1680 x 1120 RGB,
    #     each image's dense map then rendered (24.6 GB per image)
    H4, W4, ps4 = 1120, 1680, 0.00536
    img4 = torch.from_numpy(scenes.aif_blobs(H4, W4, 3, n_blobs=2000, seed=0)[None]).to(dev)
    dmaps4 = [scenes.depth_voronoi(H4, W4, 500.0, 5000.0, seed=100 + k) for k in range(8)]
    kmap = torch.empty((H4 * W4 * 3, 2178), dtype=torch.bfloat16, device=dev)
    o4 = torch.empty((1, 6, H4, W4), device=dev)
    desc4, keep4 = sdirt.make_render_desc(1, 3, H4, W4, 33, psf_channels=3, psf_dtype=abi.BF16)
    lam_rgb = [configs.RGB_LAMBDAS[i] for i in configs.LAMBDA_OF_RGB]    # image channel -> wavelength
    xin = [torch.from_numpy(configs.pixel_inputs(H4, W4, ps4, dm, lambdas=lam_rgb)).to(dev)
           for dm in dmaps4]

    def pipeline():
        for k in range(8):
            sdirt.mlp_forward(desc, params, xin[k], ws, 65536, out_dtype=abi.BF16, out=kmap)
            sdirt.render_dp(desc4, img4, kmap, out=o4)

    pipeline()
    t_pipe = timed(pipeline, stream, 1)
    t_r4 = timed(lambda: sdirt.render_dp(desc4, img4, kmap, out=o4), stream, 2)
    del kmap, xin, ws
    # the same images through the fused surrogate render (no PSF map in
    # memory), 262144-row chunks
    dm4 = [torch.from_numpy(dm[None]).to(dev) for dm in dmaps4]
    ws = sdirt.mlp_workspace(desc, 262144)

    def fused():
        for k in range(8):
            sdirt.mlp_render(desc, params, img4, dm4[k], lam_rgb, ps4, ws, 262144, out=o4)

    fused()
    t_fused = timed(fused, stream, 1)
    rows = 8 * H4 * W4 * 3
    head_flop = rows * 2.0 * (64 * 256 + 4 * 256 * 256 + 256 * 2178 + 2178)
    out["mlp_render_batch"] = {
        "workload": "8 x 1680x1120 RGB rendered with per-pixel per-wavelength MLP PSFs "
                    "(2x33x33), fused: PSFs consumed in registers",
        "ms": t_fused, "mpix_per_s": 8 * H4 * W4 / (t_fused * 1e-3) / 1e6,
        "tflops": head_flop / (t_fused * 1e-3) / 1e12,
        "mfma_frac": head_flop / (t_fused * 1e-3) / 2.5e15,
        "unfused_ms": t_pipe,
        "unfused_note": "MLP -> dense bf16 map in HBM (24.6 GB per image) -> render_dp",
        "unfused_render_ms_per_image": t_r4,
        "unfused_render_gbs": H4 * W4 * 3 * 2178 * 2 / (t_r4 * 1e-3) / 1e9}
    del ws, dm4
    print("mlp done", file=sys.stderr, flush=True)
    # 4. the paper's PSF-map workload: RF50 at F/4, 512 x 768 pixels, one
    #    microlens-model DP PSF per pixel (ks 21, 4096 rays)
    lens, sensor, query, (H, W) = configs.paper_psf_map()
    dmap = scenes.depth_uniform_inverse(H, W, 500.0, 20000.0, seed=100)
    pts = torch.from_numpy(configs.pixel_points(H, W, sensor.pitch, dmap)).to(dev)
    pm = torch.empty((H * W, 2, 21, 21), device=dev)
    tr = lambda: sdirt.trace_dp_psf(lens, sensor, query, points=pts, out=pm, stats=False)
    tr()
    t_map = timed(tr, stream, 2)
    img = torch.rand((1, 3, H, W), device=dev)
    desc, keep = sdirt.make_render_desc(1, 3, H, W, 21, psf_channels=1)
    ro = sdirt.render_dp(desc, img, pm)
    # three rounds of three launches (the median is reported: a single
    # round right after the surrogate sections has read 40x slow)
    t_rounds = [timed(lambda: sdirt.render_dp(desc, img, pm, out=ro), stream, 3) for _ in range(3)]
    t_r = sorted(t_rounds)[1]
    mdesc = sdirt.make_mlp_desc(n_out=2 * 21 * 21, x_half=18.0, y_half=12.0, iv_lo=1 / 20000.0,
                                iv_hi=1 / 500.0, lam_lo=0.5, lam_hi=0.6)
    layers = scenes.mlp_init([64, 256, 256, 256, 256, 256, 882], seed=0)
    params = torch.from_numpy(np.concatenate([np.concatenate([Wt.ravel(), bt]) for Wt, bt in layers]).astype(np.float32)).to(dev)
    xi = torch.from_numpy(np.stack([pts[:, 0].cpu().numpy(), pts[:, 1].cpu().numpy(),
                                    1.0 / pts[:, 2].cpu().numpy(), np.full(H * W, 0.55)], 1).astype(np.float32)).to(dev)
    ws = sdirt.mlp_workspace(mdesc, 65536)
    mo = torch.empty((H * W, 882), dtype=torch.float32, device=dev)
    inf = lambda: sdirt.mlp_forward(mdesc, params, xi, ws, 65536, out=mo)
    inf()
    t_inf = timed(inf, stream, 3)
    c = TRACE_COUNTS["paper_map"]
    flop_map = H * W * query.n_rays * trace_flop_per_ray([s_.kind for s_ in lens.surfaces],
                                                         c["alive"], c["newton_per_ray"])
    out["paper_psf_map"] = {
        "workload": "RF50 (Table S1) F/4, focus 1 m, 512x768 px over 24x36 mm, microlens DP "
                    "model, ks 21, 4096 rays/PSF, 393216 PSFs, depth uniform in 1/d 0.5-20 m",
        "trace_map_s": t_map * 1e-3, "paper_trace_map_s": 801.544,
        "trace_flop_per_ray": flop_map / (H * W * query.n_rays),
        "trace_tflops": flop_map / (t_map * 1e-3) / 1e12,
        "trace_fp64_frac": flop_map / (t_map * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
        "mlp_map_s": t_inf * 1e-3, "paper_mlp_map_s": 0.395,
        "render_s": t_r * 1e-3, "render_rounds_ms": t_rounds, "paper_render_s": 0.2,
        "paper_hardware": "i7-12700K + RTX 3090 (Sec. 5.1)"}
    print("paper workload done", file=sys.stderr, flush=True)
    # 4b. exact-azimuth bank: the 12-surface lens traced on a 16 x 11
    #     first-quadrant field grid, then the 1680 x 1120 RGB render and its
    #     adjoint with flips and depth interpolation
    lens, sensor, query, pts2, xs, ys = configs.config2_bank2d()
    H, W, ps = sensor.height_px, sensor.width_px, sensor.pitch
    P2 = pts2.shape[0]
    pts2 = torch.from_numpy(pts2).to(dev)
    b2 = torch.empty((P2, 2, query.ks, query.ks), dtype=torch.float32, device=dev)
    tr = lambda: sdirt.trace_dp_psf(lens, sensor, query, points=pts2, out=b2, stats=False)
    tr()
    t_tr = timed(tr, stream, 2)
    img2 = torch.from_numpy(scenes.aif_blobs(H, W, 3, n_blobs=2000, seed=0)[None]).to(dev)
    dm2 = torch.from_numpy(scenes.depth_voronoi(H, W, 500.0, 5000.0, seed=100)[None]).to(dev)
    desc2, keep2 = sdirt.make_render_desc(1, 3, H, W, query.ks, source=abi.SRC_BANK2D,
                                          field_radii=xs, field_y=ys,
                                          inv_depths=[1.0 / d for d in query.depths],
                                          bank_lambdas=3, lambda_of_channel=list(configs.LAMBDA_OF_RGB),
                                          pitch=ps)
    o2 = sdirt.render_dp(desc2, img2, b2, depth=dm2)
    g2 = torch.randn_like(o2)
    gi2 = sdirt.render_dp_backward(desc2, b2, g2, depth=dm2)
    tf = timed(lambda: sdirt.render_dp(desc2, img2, b2, depth=dm2, out=o2), stream, 3)
    tb = timed(lambda: sdirt.render_dp_backward(desc2, b2, g2, depth=dm2, grad_img=gi2), stream, 3)
    gb2 = torch.empty_like(b2)
    kg2 = lambda: sdirt.render_dp_psf_backward(desc2, img2, g2, depth=dm2, grad_psf=gb2)
    kg2()
    tk2 = timed(kg2, stream, 3)
    out["bank2d"] = {"workload": "12-surface lens, 16 x 11 first-quadrant fields x 16 depths x 3 "
                                 "wavelengths (8448 PSFs, 512^2 rays, ks 63); 1680x1120 RGB "
                                 "render + adjoint with flips and linear 1/d interpolation",
                     "trace_ms": t_tr, "psfs_per_s": P2 / (t_tr * 1e-3),
                     "render_fwd_ms": tf, "render_bwd_ms": tb, "bank_grad_ms": tk2}
    del b2, o2, g2, gi2, gb2
    print("bank2d done", file=sys.stderr, flush=True)
    # 5. the 12-surface spherical lens: 32 radial fields x 16 depths x 3
    #    wavelengths (1536 PSFs, 512^2 rays, ks 63), then a 1680 x 1120 RGB
    #    render from that bank and its image adjoint
    out["config2"] = config2_step(dev, stream)
    print("12-surface lens done", file=sys.stderr, flush=True)
    return out


def surrogate_vs_trace(dev, stream):
    import copy
    import numpy as np
    import torch
    from workloads import configs
    from paper_2503_11213_amd import sdirt, _abi as abi
    from paper_2503_11213_amd.surrogate import trace_points, energy_l1
    desc, params, meta = sdirt.mlp_load_weights(
        os.path.join(ROOT, "workloads", "surrogate_ks33.safetensors"), device=dev)
    lens, sensor, query = configs.config4()
    n_eval = 512
    hp, hx = configs.surrogate_points(n_eval, seed=21)       # points the training never saw
    hp_t, hx_t = torch.from_numpy(hp).to(dev), torch.from_numpy(hx).to(dev)
    ref = trace_points(lens, sensor, query, hp_t, rays=8192, chunk=256)
    ws = sdirt.mlp_workspace(desc, 4096)
    e_net = float(energy_l1(sdirt.mlp_forward(desc, params, hx_t, ws, 4096), ref).mean())
    ray_counts = (256, 512, 1024)
    e_tr = {r: float(energy_l1(trace_points(lens, sensor, query, hp_t, rays=r), ref).mean())
            for r in ray_counts}
    # throughput: the network on 2^20 rows (bf16 out), tracing 16384 points
    nrow = 1 << 20
    _, xr = configs.surrogate_points(nrow, seed=22)
    xr = torch.from_numpy(xr).to(dev)
    ob = torch.empty((nrow, desc.n_out), dtype=torch.bfloat16, device=dev)
    wsb = sdirt.mlp_workspace(desc, 65536)
    inf = lambda: sdirt.mlp_forward(desc, params, xr, wsb, 65536, out_dtype=abi.BF16, out=ob)
    inf()
    t_net = timed(inf, stream, 3)
    net_rate = nrow / (t_net * 1e-3)
    tp, _ = configs.surrogate_points(16384, seed=23)
    tp = torch.from_numpy(tp).to(dev)
    tbuf = torch.empty((16384, 2 * 33 * 33), device=dev)
    rate = {}
    for r in ray_counts:
        q = copy.copy(query)
        q.rays_x = q.rays_y = r
        f = lambda: sdirt.trace_dp_psf(lens, sensor, q, points=tp, out=tbuf.view(-1, 2, 33, 33),
                                       stats=False)
        f()
        rate[r] = 16384 / (timed(f, stream, 2) * 1e-3)
    matched = min([r for r in ray_counts if e_tr[r] <= e_net], default=None)
    # the network with the tracer (1024^2 rays) as fallback, by the held-out
    # error per inverse-depth band stored with the weights, bar 2 %
    edges, errs = meta["band_edges_inv_mm"], meta["band_energy_l1"]
    q1k = copy.copy(query)
    q1k.rays_x = q1k.rays_y = 1024
    ph, src = sdirt.psf_hybrid(desc, params, lens, sensor, q1k, hp_t, edges, errs, 0.02, ws, 4096)
    e_h = float(energy_l1(ph.view(n_eval, -1), ref).mean())
    hyb = lambda: sdirt.psf_hybrid(desc, params, lens, sensor, q1k, tp, edges, errs, 0.02, ws,
                                   4096, out=tbuf.view(-1, 2, 33, 33))
    _, src_t = hyb()
    h_rate = 16384 / (timed(hyb, stream, 2) * 1e-3)
    flop = nrow * 2.0 * (64 * 256 + 4 * 256 * 256 + 256 * 2178)
    return {"workload": "ks 33, 12-surface lens; trained network (%s); %d fresh points against "
                        "8192^2-ray traces; network rate on 2^20 rows (bf16 out), tracing and "
                        "fallback rates on 16384 points" % (meta.get("loss", "kl"), n_eval),
            "network_energy_l1": e_net,
            "trace_energy_l1": {str(r): e for r, e in e_tr.items()},
            "network_psfs_per_s": net_rate,
            "trace_psfs_per_s": {str(r): v for r, v in rate.items()},
            "trace_rays_at_network_error": matched,
            "speedup_at_network_error": net_rate / rate[matched] if matched else None,
            "mlp_tflops": flop / (t_net * 1e-3) / 1e12,
            "mlp_mfma_frac": flop / (t_net * 1e-3) / 2.5e15,
            "fallback": {"bar": 0.02, "tracer_rays": 1024 * 1024,
                         "energy_l1": e_h, "traced_fraction": float(src.float().mean()),
                         "traced_fraction_rate_points": float(src_t.float().mean()),
                         "psfs_per_s": h_rate,
                         "speedup_over_tracing_at_2pc": h_rate / rate[1024],
                         "tracing_energy_l1_at_1024": e_tr[1024]}}


def config2_step(dev, stream, reps=5):
    import numpy as np
    import torch
    from workloads import configs, scenes
    from paper_2503_11213_amd import sdirt, _abi as abi
    lens, sensor, query = configs.config2()
    H, W, ps = sensor.height_px, sensor.width_px, sensor.pitch
    img = torch.from_numpy(scenes.aif_blobs(H, W, 3, n_blobs=2000, seed=0)[None]).to(dev)
    dmap = torch.from_numpy(scenes.depth_voronoi(H, W, 500.0, 5000.0, seed=100)[None]).to(dev)
    gout = torch.from_numpy(np.random.default_rng(1).normal(
        size=(1, 6, H, W)).astype(np.float32)).to(dev)
    desc, keep = sdirt.make_render_desc(1, 3, H, W, query.ks, source=abi.SRC_BANK,
                                        field_radii=[f[0] for f in query.fields],
                                        inv_depths=[1.0 / d for d in query.depths],
                                        bank_lambdas=3, lambda_of_channel=list(configs.LAMBDA_OF_RGB),
                                        pitch=ps, bank_math=abi.BANK_SPLIT_BF16)
    P = query.n_points
    bank = torch.empty((P, 2, query.ks, query.ks), dtype=torch.float32, device=dev)
    out = torch.empty((1, 6, H, W), dtype=torch.float32, device=dev)
    gimg = torch.empty((1, 3, H, W), dtype=torch.float32, device=dev)
    tr = lambda: sdirt.trace_dp_psf(lens, sensor, query, out=bank, stats=False)
    rf = lambda: sdirt.render_dp(desc, img, bank, depth=dmap, out=out)
    rb = lambda: sdirt.render_dp_backward(desc, bank, gout, depth=dmap, grad_img=gimg)
    tr(); rf(); rb()
    t_tr, t_rf, t_rb = timed(tr, stream, reps), timed(rf, stream, reps), timed(rb, stream, reps)
    gbank = torch.empty_like(bank)
    kg = lambda: sdirt.render_dp_psf_backward(desc, img, gout, depth=dmap, grad_psf=gbank)
    kg()
    t_kg = timed(kg, stream, reps)
    _, st = sdirt.trace_dp_psf(lens, sensor, query, out=bank, stats=True)
    st = st.cpu().numpy()
    kinds = [s_.kind for s_ in lens.surfaces]
    n_surf = sum(1 for k in kinds if k != 2)
    rays = P * query.n_rays
    c = TRACE_COUNTS["config2"]
    flop = rays * trace_flop_per_ray(kinds, c["alive"], c["newton_per_ray"])
    return {"workload": "12-surface double-Gauss-like lens (seed 0, f/2, focus 0.909 m); 32 "
                        "radial fields x 16 depths (0.5-5 m, uniform 1/d) x 3 wavelengths = "
                        "1536 DP PSFs, 512x512 rays each, ks 63, sigmoid response, box splat; "
                        "render + image adjoint of a 1680x1120 RGB image from the PSF bank",
            "step_ms": t_tr + t_rf + t_rb,
            "rays_surfaces_per_s_step": rays * n_surf / ((t_tr + t_rf + t_rb) * 1e-3),
            "trace_ms": t_tr, "trace_rays_surfaces_per_s": rays * n_surf / (t_tr * 1e-3),
            "trace_psfs_per_s": P / (t_tr * 1e-3),
            "trace_tflops": flop / (t_tr * 1e-3) / 1e12,
            "trace_fp64_frac": flop / (t_tr * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "in_window_energy_fraction": float((st[:, 3] + st[:, 4]).sum() / st[:, 0].sum()),
            "render_fwd_ms": t_rf, "render_bwd_ms": t_rb,
            "render_fwd_mpix_per_s": H * W / (t_rf * 1e-3) / 1e6,
            "render_fwd_plus_bwd_over_fwd": (t_rf + t_rb) / t_rf,
            "bank_grad_ms": t_kg}


def pmc_target(name, dev):
    """One launch of a kernel for a profiler counter pass, after a 1 GiB
    device copy whose FETCH_SIZE / WRITE_SIZE scale the memory counters:
      calib       sdirt_calib_fma64, 2^20 threads x 1000 iterations
                  (8.39e9 float64 FMAs);
      trace       the step's trace (16-surface aspheric lens, 6144 PSFs);
      trace_c2    the 12-surface lens trace (1536 PSFs x 512^2 rays, ks 63);
      trace_paper the paper's PSF map (RF50, 393,216 PSFs x 4096 rays);
      trace_bwd   the adjoint of the trace (12-surface lens, 192 PSFs x
                  256^2 rays, ks 41, tent splat), after its forward;
      render, render_bwd  the step's bank render and image adjoint;
      render_split, render_split_bwd  the step's bank render and image
                  adjoint on the split-bf16 matrix cores;
      dense       dense render of 512 x 512 RGB with a 41 x 41 f32 map,
                  its image adjoint and its kernel-map gradient;
      mlp_head    surrogate inference of 2^20 rows (ks 33, bf16 out);
      mlp_render  fused surrogate render of one 1680 x 1120 RGB image (ks 33,
                  trained weights)."""
    import ctypes as C
    import numpy as np
    import torch
    from workloads import configs, scenes
    from paper_2503_11213_amd import sdirt, _abi as abi
    src = torch.ones((1 << 28,), dtype=torch.float32, device=dev)
    torch.empty_like(src).copy_(src)
    del src
    torch.cuda.synchronize()
    if name == "calib":
        out = torch.empty((1 << 20,), dtype=torch.float64, device=dev)
        abi.check("sdirt_calib_fma64", abi.lib().sdirt_calib_fma64(
            1 << 20, 1000, C.c_void_p(out.data_ptr()),
            C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    elif name == "trace":
        lens, sensor, query = configs.config5()
        sdirt.trace_dp_psf(lens, sensor, query, stats=False)
    elif name == "trace_c2":
        lens, sensor, query = configs.config2()
        sdirt.trace_dp_psf(lens, sensor, query, stats=False)
    elif name == "trace_bwd":
        lens, sensor, query = configs.config3()
        psf, _ = sdirt.trace_dp_psf(lens, sensor, query, stats=False)
        g = torch.from_numpy(np.random.default_rng(5).standard_normal(tuple(psf.shape))
                             .astype(np.float32)).to(dev)
        sdirt.trace_dp_psf_backward(lens, sensor, query, g)
    elif name == "trace_paper":
        lens, sensor, query, (H, W) = configs.paper_psf_map()
        dmap = scenes.depth_uniform_inverse(H, W, 500.0, 20000.0, seed=100)
        pts = torch.from_numpy(configs.pixel_points(H, W, sensor.pitch, dmap)).to(dev)
        sdirt.trace_dp_psf(lens, sensor, query, points=pts, stats=False)
    elif name in ("render", "render_bwd", "render_split", "render_split_bwd"):
        lens, sensor, query = configs.config5()
        bank, _ = sdirt.trace_dp_psf(lens, sensor, query, stats=False)
        H, W, N = sensor.height_px, sensor.width_px, 16
        img = torch.from_numpy(scenes.aif_blobs(H, W, 3, n_blobs=2000, seed=0)).to(dev)
        img = img.unsqueeze(0).expand(N, -1, -1, -1).contiguous()
        dms = [torch.from_numpy(scenes.depth_voronoi(H, W, 100.0, 5000.0, seed=200 + k)).to(dev)
               for k in range(4)]
        dmap = torch.stack([dms[k % 4] for k in range(N)])
        desc, keep = sdirt.make_render_desc(N, 3, H, W, query.ks, source=abi.SRC_BANK,
                                            field_radii=[f[0] for f in query.fields],
                                            inv_depths=[1.0 / d for d in query.depths],
                                            bank_lambdas=3,
                                            lambda_of_channel=list(configs.LAMBDA_OF_RGB),
                                            pitch=sensor.pitch,
                                            bank_math=abi.BANK_SPLIT_BF16 if "split" in name
                                            else abi.BANK_FP32)
        if name in ("render", "render_split"):
            sdirt.render_dp(desc, img, bank, depth=dmap)
        else:
            g = torch.randn((N, 6, H, W), device=dev)
            sdirt.render_dp_backward(desc, bank, g, depth=dmap)
    elif name == "dense":
        N, C_, H, W, ks = 1, 3, 512, 512, 41
        K = torch.rand((N, H, W, C_, 2, ks, ks), device=dev)
        img = torch.rand((N, C_, H, W), device=dev)
        desc, keep = sdirt.make_render_desc(N, C_, H, W, ks)
        sdirt.render_dp(desc, img, K)
        gout = torch.randn((N, 2 * C_, H, W), device=dev)
        sdirt.render_dp_backward(desc, K, gout)
        sdirt.render_dp_psf_backward(desc, img, gout, grad_psf=torch.empty_like(K))
    elif name == "mlp_head":
        desc = sdirt.make_mlp_desc(n_out=2 * 33 * 33, **configs.config4_desc_kwargs())
        layers = scenes.mlp_init([64, 256, 256, 256, 256, 256, 2178], seed=0)
        params = torch.from_numpy(np.concatenate([np.concatenate([Wt.ravel(), bt])
                                                  for Wt, bt in layers]).astype(np.float32)).to(dev)
        _, x = configs.surrogate_points(1 << 20, seed=3)
        ws = sdirt.mlp_workspace(desc, 1 << 20)
        sdirt.mlp_forward(desc, params, torch.from_numpy(x).to(dev), ws, 1 << 20,
                          out_dtype=abi.BF16)
    elif name == "mlp_render":
        desc, params, _ = sdirt.mlp_load_weights(
            os.path.join(ROOT, "workloads", "surrogate_ks33.safetensors"), device=dev)
        H4, W4, ps4 = 1120, 1680, 0.00536
        img = torch.from_numpy(scenes.aif_blobs(H4, W4, 3, n_blobs=2000, seed=0)[None]).to(dev)
        dm = torch.from_numpy(scenes.depth_voronoi(H4, W4, 500.0, 5000.0, seed=100)[None]).to(dev)
        lam_rgb = [configs.RGB_LAMBDAS[i] for i in configs.LAMBDA_OF_RGB]
        ws = sdirt.mlp_workspace(desc, 262144)
        sdirt.mlp_render(desc, params, img, dm, lam_rgb, ps4, ws, 262144)
    torch.cuda.synchronize()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from workloads import configs, scenes
    from paper_2503_11213_amd import sdirt, _abi as abi

    torch.cuda.init()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    if args.pmc_target:
        pmc_target(args.pmc_target, dev)
        return
    lens, sensor, query = configs.config5()
    P, ks = query.n_points, query.ks
    bank = torch.empty((P, 2, ks, ks), dtype=torch.float32, device=dev)
    H, W, N = sensor.height_px, sensor.width_px, 16
    # the batch: one all-in-focus image and four depth maps, each used four
    # times (the render's cost does not depend on the image content)
    img1_np = scenes.aif_blobs(H, W, 3, n_blobs=2000, seed=0)
    dms_np = [scenes.depth_voronoi(H, W, 100.0, 5000.0, seed=200 + k) for k in range(4)]
    img1 = torch.from_numpy(img1_np).to(dev)
    img = img1.unsqueeze(0).expand(N, -1, -1, -1).contiguous()
    del img1
    dms = [torch.from_numpy(d).to(dev) for d in dms_np]
    dmap = torch.stack([dms[k % 4] for k in range(N)])
    del dms
    gout = torch.randn((N, 6, H, W), device=dev, generator=torch.Generator(dev).manual_seed(1))
    desc, keep = sdirt.make_render_desc(N, 3, H, W, ks, source=abi.SRC_BANK,
                                        field_radii=[f[0] for f in query.fields],
                                        inv_depths=[1.0 / d for d in query.depths],
                                        bank_lambdas=3, lambda_of_channel=list(configs.LAMBDA_OF_RGB),
                                        pitch=sensor.pitch, bank_math=abi.BANK_SPLIT_BF16)
    out = torch.empty((N, 6, H, W), dtype=torch.float32, device=dev)
    gimg = torch.empty((N, 3, H, W), dtype=torch.float32, device=dev)

    def trace():
        sdirt.trace_dp_psf(lens, sensor, query, out=bank, stats=False)

    def render():
        sdirt.render_dp(desc, img, bank, depth=dmap, out=out)

    def render_bwd():
        sdirt.render_dp_backward(desc, bank, gout, depth=dmap, grad_img=gimg)

    for _ in range(args.warmup):
        trace()
        render()
        render_bwd()
    torch.cuda.synchronize()
    # the timed steps, with HIP events on the launch stream around each of
    # the step's three calls
    laps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        evs[0].record(stream)
        trace()
        evs[1].record(stream)
        render()
        evs[2].record(stream)
        render_bwd()
        evs[3].record(stream)
        laps.append(evs)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    ms_trace = float(np.mean([e[0].elapsed_time(e[1]) for e in laps]))
    ms_render = float(np.mean([e[1].elapsed_time(e[2]) for e in laps]))
    ms_rbwd = float(np.mean([e[2].elapsed_time(e[3]) for e in laps]))
    _, st = sdirt.trace_dp_psf(lens, sensor, query, out=bank, stats=True)
    st = st.cpu().numpy()

    kinds = [s.kind for s in lens.surfaces]
    n_surf = sum(1 for k in kinds if k != 2)          # refracting surfaces
    rays = P * query.n_rays
    rs = rays * n_surf
    value = rs / (ms_step * 1e-3)
    c = TRACE_COUNTS["config5"]
    flop_ray = trace_flop_per_ray(kinds, c["alive"], c["newton_per_ray"])
    flop = rays * flop_ray
    achieved = flop / (ms_trace * 1e-3) / 1e12
    npx = N * H * W
    render_flop = npx * 4.0 * 3 * ks * ks
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "rays*surfaces/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "16-surface aspheric phone lens (seeded even aspheres to r^10, "
                               "EFL 4.3 mm, f/1.8, focus 0.196 m); 64 radial fields x 32 "
                               "depths (0.1-5 m, uniform 1/d) x 3 wavelengths = 6144 DP PSFs, "
                               "1024x1024 rays each, ks 65, sigmoid DP response, box splat; "
                               "render + image adjoint of 16 RGB 4032x3024 images (1.0 um "
                               "pixels) from the PSF bank and piecewise-planar depth maps",
                   "psfs": P, "rays_per_psf": query.n_rays, "surfaces": n_surf,
                   "ks": ks, "images": [N, 3, H, W]},
        "roofline": {"kernel": "trace_splat_kernel<double, box, sigmoid, float, general surface loop>",
                     "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": (TRACE_TRAFFIC["bytes"]
                                 if TRACE_TRAFFIC["sources_sha256"] == sources_digest() else None),
                     "flop_per_launch": flop, "flop_per_ray": flop_ray,
                     "launch_ms": ms_trace},
        "trace": {"ms": ms_trace, "rays_surfaces_per_s": rs / (ms_trace * 1e-3),
                  "psfs_per_s": P / (ms_trace * 1e-3),
                  "in_window_energy_fraction": float((st[:, 3] + st[:, 4]).sum() / st[:, 0].sum()),
                  "transmitted_fraction": float(st[:, 2].sum() / st[:, 0].sum())},
        "render": {"arithmetic": "split-bf16 matrix cores (hi*hi + hi*lo + lo*hi, float32 accumulation)",
                   "fwd_ms": ms_render, "bwd_ms": ms_rbwd,
                   "fwd_mpix_per_s": npx / (ms_render * 1e-3) / 1e6,
                   "fwd_tflops": render_flop / (ms_render * 1e-3) / 1e12,
                   "fwd_split_bf16_frac": render_flop / (ms_render * 1e-3) / 1e12 / PEAK_SPLIT_BF16_TFLOPS,
                   "bwd_tflops": render_flop / (ms_rbwd * 1e-3) / 1e12,
                   "bwd_split_bf16_frac": render_flop / (ms_rbwd * 1e-3) / 1e12 / PEAK_SPLIT_BF16_TFLOPS,
                   "fwd_plus_bwd_over_fwd": (ms_render + ms_rbwd) / ms_render},
    }
    # the same render on the float32 matrix cores, for comparison
    desc32, keep32 = sdirt.make_render_desc(N, 3, H, W, ks, source=abi.SRC_BANK,
                                            field_radii=[f[0] for f in query.fields],
                                            inv_depths=[1.0 / d for d in query.depths],
                                            bank_lambdas=3, lambda_of_channel=list(configs.LAMBDA_OF_RGB),
                                            pitch=sensor.pitch, bank_math=abi.BANK_FP32)
    sdirt.render_dp(desc32, img, bank, depth=dmap, out=out)
    sdirt.render_dp_backward(desc32, bank, gout, depth=dmap, grad_img=gimg)
    t32f = timed(lambda: sdirt.render_dp(desc32, img, bank, depth=dmap, out=out), stream, 2)
    t32b = timed(lambda: sdirt.render_dp_backward(desc32, bank, gout, depth=dmap, grad_img=gimg), stream, 2)
    line["render"]["fp32_mfma"] = {"fwd_ms": t32f, "bwd_ms": t32b,
                                   "fwd_frac": render_flop / (t32f * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS,
                                   "bwd_frac": render_flop / (t32b * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS}
    del img, dmap, gout, out, gimg
    torch.cuda.empty_cache()
    if not args.no_extras:
        line.update(extras(dev, stream))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(lens, sensor, query, rs, img1_np, dms_np[0], N)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
