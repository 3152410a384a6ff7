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

# HBM bytes of one trace launch, from two rocprofv3 --pmc runs of
# `bench.py --pmc-target` (FETCH_SIZE, then WRITE_SIZE), each scaled by what
# the counter reads on a 1 GiB device copy in the same run.  The figure holds
# for the kernel sources with this digest only; otherwise traffic is null.
TRACE_SOURCES = ("paper_2503_11213_amd/csrc/device_common.hpp",
                 "paper_2503_11213_amd/csrc/trace.hip",
                 "paper_2503_11213_amd/csrc/pack.hpp",
                 "paper_2503_11213_amd/csrc/pack.cpp")
TRACE_TRAFFIC = {"sources_sha256": "efd856cf901a745ab96df7348f5a220c028fac42a5e373f8b7523e19ea27af8a",
                 "bytes": 65716014}


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
    ap.add_argument("--pmc-target", action="store_true",
                    help="for counter runs: a 1 GiB device copy (calibration), then one "
                         "trace_dp_psf call of the step; prints nothing")
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
    picks = [(f, (5 * f + 3 * k) % 16, (f + k) % 3) for f in range(32) for k in range(2)]
    t0 = time.perf_counter()
    bank, _ = opsf.trace_dp_psf(lens, sensor, query, points=picks)
    t_trace = time.perf_counter() - t0
    sample_rays = len(picks) * query.n_rays
    crop = 160
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
    # 3. MLP inference vs tracing at ks 33 (12-surface lens, 512^2 rays)
    lens, sensor, query = configs.config4()
    pts, x = configs.surrogate_points(65536, seed=3)
    pts_t = torch.from_numpy(pts).to(dev)
    tq = torch.empty((65536, 2, 33, 33), device=dev)
    tr = lambda: sdirt.trace_dp_psf(lens, sensor, query, points=pts_t, out=tq, stats=False)
    tr()
    t_trace = timed(tr, stream, 2)
    desc = sdirt.make_mlp_desc(n_out=2 * 33 * 33, **configs.config4_desc_kwargs())
    layers = scenes.mlp_init([64, 256, 256, 256, 256, 256, 2178], seed=0)
    params = torch.from_numpy(np.concatenate([np.concatenate([Wt.ravel(), bt]) for Wt, bt in layers]).astype(np.float32)).to(dev)
    nrow = 1 << 20
    xb = torch.from_numpy(np.tile(x, (nrow // 65536, 1))).to(dev)
    ob = torch.empty((nrow, 2178), dtype=torch.bfloat16, device=dev)
    ws = sdirt.mlp_workspace(desc, 65536)
    inf = lambda: sdirt.mlp_forward(desc, params, xb, ws, 65536, out_dtype=abi.BF16, out=ob)
    inf()
    t_mlp = timed(inf, stream, 2)
    flop = nrow * 2.0 * (64 * 256 + 4 * 256 * 256 + 256 * 2178)
    out["mlp_vs_trace"] = {"workload": "ks 33, 12-surface lens; trace 65536 PSFs x 512^2 rays; "
                                       "MLP 2^20 PSFs, bf16 out",
                           "trace_psfs_per_s": 65536 / (t_trace * 1e-3),
                           "mlp_psfs_per_s": nrow / (t_mlp * 1e-3),
                           "speedup": (nrow / t_mlp) / (65536 / t_trace),
                           "mlp_tflops": flop / (t_mlp * 1e-3) / 1e12,
                           "mlp_mfma_frac": flop / (t_mlp * 1e-3) / 2.5e15}
    del xb, ob, tq
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
    t_r = timed(lambda: sdirt.render_dp(desc, img, pm, out=ro), stream, 3)
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
    out["paper_psf_map"] = {
        "workload": "RF50 (Table S1) F/4, focus 1 m, 512x768 px over 24x36 mm, microlens DP "
                    "model, ks 21, 4096 rays/PSF, 393216 PSFs, depth uniform in 1/d 0.5-20 m",
        "trace_map_s": t_map * 1e-3, "paper_trace_map_s": 801.544,
        "mlp_map_s": t_inf * 1e-3, "paper_mlp_map_s": 0.395,
        "render_s": t_r * 1e-3, "paper_render_s": 0.2,
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
    # 5. smartphone-like 16-surface aspheric lens: 64 x 32 x 3 PSFs, 1024^2
    #    rays each, ks 65; then its render batch: 16 RGB 4032 x 3024 images
    #    (one AiF image, four depth maps, each used four times) from that
    #    bank, forward plus image adjoint
    lens, sensor, query = configs.config5()
    b5 = torch.empty((query.n_points, 2, 65, 65), device=dev)
    tr = lambda: sdirt.trace_dp_psf(lens, sensor, query, out=b5, stats=False)
    tr()
    t5 = timed(tr, stream, 2)
    n_surf = sum(1 for s_ in lens.surfaces if s_.kind != 2)
    out["phone_lens_trace"] = {
        "workload": "16-surface aspheric lens (EFL 4.3 mm, f/1.8), 6144 PSFs x 1024^2 rays, ks 65",
        "ms": t5, "psfs_per_s": query.n_points / (t5 * 1e-3),
        "rays_surfaces_per_s": query.n_points * query.n_rays * n_surf / (t5 * 1e-3)}
    H5, W5, N5 = sensor.height_px, sensor.width_px, 16
    img1 = torch.from_numpy(scenes.aif_blobs(H5, W5, 3, n_blobs=2000, seed=0)).to(dev)
    imgs = img1.unsqueeze(0).expand(N5, -1, -1, -1).contiguous()
    del img1
    dms = [torch.from_numpy(scenes.depth_voronoi(H5, W5, 100.0, 5000.0, seed=200 + k)).to(dev)
           for k in range(4)]
    dmap5 = torch.stack([dms[k % 4] for k in range(N5)])
    del dms
    desc5, keep5 = sdirt.make_render_desc(N5, 3, H5, W5, query.ks, source=abi.SRC_BANK,
                                          field_radii=[f[0] for f in query.fields],
                                          inv_depths=[1.0 / d for d in query.depths],
                                          bank_lambdas=3, lambda_of_channel=list(configs.LAMBDA_OF_RGB),
                                          pitch=sensor.pitch)
    o5 = torch.empty((N5, 6, H5, W5), device=dev)
    g5 = torch.randn((N5, 6, H5, W5), device=dev)
    gi5 = torch.empty_like(imgs)
    rf = lambda: sdirt.render_dp(desc5, imgs, b5, depth=dmap5, out=o5)
    rb = lambda: sdirt.render_dp_backward(desc5, b5, g5, depth=dmap5, grad_img=gi5)
    rf()
    rb()
    tf, tb = timed(rf, stream, 2), timed(rb, stream, 2)
    npx = N5 * H5 * W5
    out["phone_lens_render"] = {
        "workload": "16 x 4032x3024 RGB from the 6144-PSF bank (ks 65), forward + image adjoint",
        "fwd_ms": tf, "bwd_ms": tb, "fwd_mpix_per_s": npx / (tf * 1e-3) / 1e6,
        "fwd_tflops": npx * 4.0 * 3 * query.ks ** 2 / (tf * 1e-3) / 1e12,
        "fwd_plus_bwd_over_fwd": (tf + tb) / tf}
    del imgs, dmap5, o5, g5, gi5, b5
    print("phone lens done", file=sys.stderr, flush=True)
    return out


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
    lens, sensor, query = configs.config2()
    if args.pmc_target:
        src = torch.ones((1 << 28,), dtype=torch.float32, device=dev)
        torch.empty_like(src).copy_(src)
        sdirt.trace_dp_psf(lens, sensor, query)
        torch.cuda.synchronize()
        return
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
    # gradient with respect to the bank (not part of the step: the chain to
    # the tracer's adjoint for end-to-end lens optimisation)
    gbank = torch.empty_like(bank)
    kgrad = lambda: sdirt.render_dp_psf_backward(desc, img, gout, depth=dmap, grad_psf=gbank)
    kgrad()
    ms_kgrad = timed(kgrad, stream, reps)
    del gbank
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
        "roofline": {"kernel": "trace_splat_kernel<double, box, sigmoid, float, spheres and flats>",
                     "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": (TRACE_TRAFFIC["bytes"]
                                 if TRACE_TRAFFIC["sources_sha256"] == sources_digest() else None),
                     "flop_per_launch": flop},
        "trace": {"ms": ms_trace, "rays_surfaces_per_s": rs / (ms_trace * 1e-3),
                  "psfs_per_s": P / (ms_trace * 1e-3),
                  "in_window_energy_fraction": float((st[:, 3] + st[:, 4]).sum() / st[:, 0].sum()),
                  "transmitted_fraction": float(st[:, 2].sum() / st[:, 0].sum())},
        "render": {"fwd_ms": ms_render, "bwd_ms": ms_rbwd,
                   "fwd_mpix_per_s": H * W / (ms_render * 1e-3) / 1e6,
                   "fwd_plus_bwd_over_fwd": (ms_render + ms_rbwd) / ms_render,
                   "bank_grad_ms": ms_kgrad},
    }
    if not args.no_extras:
        line.update(extras(dev, stream))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(lens, sensor, query, img_np, dmap_np, radii,
                                            iv, loc, ps, rs, H, W)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
