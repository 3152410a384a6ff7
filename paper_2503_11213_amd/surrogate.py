"""PSF surrogate workflow on the GPU (orchestration of C-ABI calls only).

Sec. 3.2 / Supplement S1.4: ray-traced DP PSFs at random points of the
valid imaging region are the training set of an MLP that then predicts the
PSF of every pixel of a depth map, which feeds the pixel-wise renderer; the
tracer at many rays remains the reference for the network's error.

    python -m paper_2503_11213_amd.surrogate [--samples N] [--steps S]

traces the training set, trains (Kullback-Leibler loss by default; the
paper's L2 loss with --loss l2max), measures the held-out energy L1 against
high-ray traces (8192^2 rays: their own noise is ~0.1 %), the error of
plain tracing at several ray counts against the same reference, the paper's
per-element L1 / L2 figures, times MLP inference against tracing at the
same window size and prints one JSON line.
"""

import argparse
import json
import time

import numpy as np
import torch

from . import sdirt, _abi as abi


def trace_points(lens, sensor, query, pts, rays=None, chunk=65536, stats=False):
    """SUM-normalised traced PSFs [n][2 ks ks] (float32, device) at list-mode
    points (device float64 [n][4]); with stats=True also the per-point
    energy statistics [n][7] (before normalisation)."""
    import copy
    q = copy.copy(query)
    if rays is not None:
        q.rays_x = q.rays_y = int(rays)
    n = pts.shape[0]
    kk2 = 2 * q.ks * q.ks
    out = torch.empty((n, kk2), dtype=torch.float32, device=pts.device)
    st = torch.empty((n, 7), dtype=torch.float64, device=pts.device) if stats else None
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        view = out[a:b].view(b - a, 2, q.ks, q.ks)
        _, s_ = sdirt.trace_dp_psf(lens, sensor, q, points=pts[a:b].contiguous(), out=view,
                                   stats=stats)
        if stats:
            st[a:b] = s_
    return (out, st) if stats else out


def band_report(err, iv, hx, hy, in_window, x_half, y_half, iv_lo, iv_hi, n_bands=9):
    """Mean and median energy L1 of the network per band of inverse depth and
    per band of field radius, with the mean in-window energy fraction of the
    reference there (below 1 where the blur disc spills out of the window)."""
    import numpy as np
    rep = {"inverse_depth": [], "field_radius": []}
    edges = np.linspace(iv_lo, iv_hi, n_bands + 1)
    for k in range(n_bands):
        m = (iv >= edges[k]) & (iv <= edges[k + 1])
        if m.any():
            rep["inverse_depth"].append({
                "iv_per_m": [float(edges[k] * 1e3), float(edges[k + 1] * 1e3)],
                "points": int(m.sum()), "l1_mean": float(err[m].mean()),
                "l1_median": float(np.median(err[m])),
                "in_window": float(in_window[m].mean())})
    rad = np.hypot(hx / x_half, hy / y_half) / np.sqrt(2.0)
    redges = np.linspace(0.0, 1.0, 6)
    for k in range(5):
        m = (rad >= redges[k]) & (rad <= redges[k + 1])
        if m.any():
            rep["field_radius"].append({
                "relative": [float(redges[k]), float(redges[k + 1])],
                "points": int(m.sum()), "l1_mean": float(err[m].mean()),
                "in_window": float(in_window[m].mean())})
    return rep


def energy_l1(pred, ref):
    """Per-PSF energy L1: sum |pred - ref| / sum ref."""
    return (pred.float() - ref).abs().sum(dim=1) / ref.sum(dim=1).clamp_min(1e-30)


def main():
    from workloads import configs, scenes
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=200000)
    ap.add_argument("--heldout", type=int, default=1000)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--reference-rays", type=int, default=8192)
    ap.add_argument("--loss", choices=["kl", "l2max"], default="kl")
    ap.add_argument("--save", default=None, help="write the trained weights (safetensors)")
    args = ap.parse_args()
    dev = torch.device("cuda", 0)
    lens, sensor, query = configs.config4()
    desc = sdirt.make_mlp_desc(n_hidden=5, width=256, n_out=2 * query.ks ** 2, n_freq=8,
                               loss=abi.LOSS_KL if args.loss == "kl" else abi.LOSS_L2MAX,
                               **configs.config4_desc_kwargs())
    rec = {}
    # training set
    pts, x = configs.surrogate_points(args.samples, seed=1)
    pts_t = torch.from_numpy(pts).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    targets = trace_points(lens, sensor, query, pts_t)
    torch.cuda.synchronize()
    t_trace = time.perf_counter() - t0
    rec["dataset"] = {"psfs": args.samples, "rays": query.n_rays, "ks": query.ks,
                      "trace_s": t_trace, "trace_psfs_per_s": args.samples / t_trace}
    print("traced %d PSFs in %.2f s" % (args.samples, t_trace), flush=True)
    x_t = torch.from_numpy(x).to(dev)
    # training
    layers = scenes.mlp_init([64, 256, 256, 256, 256, 256, desc.n_out], seed=0)
    flat = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers]).astype(np.float32)
    params = torch.from_numpy(flat).to(dev)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    ws = sdirt.mlp_workspace(desc, args.batch)
    trace = torch.zeros((args.steps,), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chunk = 2000
    for s0 in range(0, args.steps, chunk):
        n = min(chunk, args.steps - s0)
        sdirt.mlp_train(desc, params, m, v, x_t, targets, ws, args.batch, s0, n, lr0=args.lr,
                        lr_min=1e-5, total_steps=args.steps, seed=7,
                        loss_trace=trace[s0:s0 + n])
        torch.cuda.synchronize()
        print("step %d loss %.4e" % (s0 + n, trace[s0 + n - 1].item()), flush=True)
    t_train = time.perf_counter() - t0
    rec["train"] = {"steps": args.steps, "batch": args.batch, "seconds": t_train,
                    "ms_per_step": t_train * 1e3 / args.steps,
                    "loss_first": float(trace[:10].mean()), "loss_last": float(trace[-100:].mean())}
    del targets
    torch.cuda.empty_cache()
    # held-out error, against the tracer at more rays
    hpts, hx = configs.surrogate_points(args.heldout, seed=2)
    hpts_t = torch.from_numpy(hpts).to(dev)
    reference, ref_st = trace_points(lens, sensor, query, hpts_t, rays=args.reference_rays,
                                     chunk=4096, stats=True)
    hx_t = torch.from_numpy(hx).to(dev)
    ws_inf = sdirt.mlp_workspace(desc, 4096)
    pred = sdirt.mlp_forward(desc, params, hx_t, ws_inf, 4096)
    e_mlp = energy_l1(pred, reference)
    st = ref_st.cpu().numpy()
    kw = configs.config4_desc_kwargs()
    rec["bands"] = band_report(e_mlp.cpu().numpy(), hx[:, 2].astype(np.float64), hx[:, 0],
                               hx[:, 1], (st[:, 3] + st[:, 4]) / st[:, 0], kw["x_half"],
                               kw["y_half"], kw["iv_lo"], kw["iv_hi"])
    if args.save:
        # the weights, with the held-out error per inverse-depth band (the
        # table the network-with-tracer-fallback entry point routes by)
        b = rec["bands"]["inverse_depth"]
        sdirt.mlp_save_weights(args.save, desc, params, {
            "samples": args.samples, "steps": args.steps, "batch": args.batch, "lr": args.lr,
            "loss": args.loss, "heldout_energy_l1_mean": float(e_mlp.mean()),
            "heldout_points": args.heldout, "reference_rays": args.reference_rays ** 2,
            "band_edges_inv_mm": [x["iv_per_m"][0] * 1e-3 for x in b] + [b[-1]["iv_per_m"][1] * 1e-3],
            "band_energy_l1": [x["l1_mean"] for x in b],
            "band_points": [x["points"] for x in b]})
    kk2 = pred.shape[1]
    rec["heldout"] = {"points": args.heldout, "reference_rays": args.reference_rays ** 2,
                      "mlp_energy_l1_mean": float(e_mlp.mean()),
                      "mlp_energy_l1_median": float(e_mlp.median()),
                      # the paper's Table S3 figures: mean |p - t| and (p - t)^2 per element
                      "mlp_l1_per_element": float((pred.float() - reference).abs().mean()),
                      "mlp_l2_per_element": float(((pred.float() - reference) ** 2).mean()),
                      "outputs_per_psf": kk2}
    # plain tracing: error against the same reference and speed, per ray count
    rec["trace_error"] = {}
    for rays in (128, 256, 512, 1024, 2048):
        same = trace_points(lens, sensor, query, hpts_t, rays=rays)
        rec["trace_error"][str(rays)] = float(energy_l1(same, reference).mean())
    print("held-out energy L1: mlp %.4f; trace %s" % (rec["heldout"]["mlp_energy_l1_mean"],
                                                   rec["trace_error"]), flush=True)
    # throughput at ks 33: MLP inference vs tracing (512^2 rays)
    nb = 1 << 20
    xb = x_t[:nb] if x_t.shape[0] >= nb else x_t.repeat((nb + x_t.shape[0] - 1) // x_t.shape[0], 1)[:nb]
    out = torch.empty((nb, desc.n_out), dtype=torch.bfloat16, device=dev)
    ws_big = sdirt.mlp_workspace(desc, 65536)
    sdirt.mlp_forward(desc, params, xb, ws_big, 65536, out_dtype=abi.BF16, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sdirt.mlp_forward(desc, params, xb, ws_big, 65536, out_dtype=abi.BF16, out=out)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    flop = nb * 2.0 * sum(a * b for a, b in [(64, 256)] + [(256, 256)] * 4 + [(256, desc.n_out)])
    mlp_rate = nb / t_inf
    del out, xb, ws_big
    # tracing speed per ray count (65536 PSFs each)
    tpts = torch.from_numpy(configs.surrogate_points(65536, seed=5)[0]).to(dev)
    trace_rate = {}
    for rays in rec["trace_error"]:
        trace_points(lens, sensor, query, tpts[:4096], rays=int(rays))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        trace_points(lens, sensor, query, tpts, rays=int(rays))
        torch.cuda.synchronize()
        trace_rate[rays] = 65536 / (time.perf_counter() - t0)
    e_m = rec["heldout"]["mlp_energy_l1_mean"]

    def rays_for(err):
        ok = [int(r) for r, e in rec["trace_error"].items() if e <= err]
        return str(min(ok)) if ok else None

    r_same, r_2pc = rays_for(e_m), rays_for(0.02)
    rec["throughput"] = {
        "mlp_psfs_per_s": mlp_rate, "mlp_tflops": flop / t_inf / 1e12,
        "trace_psfs_per_s": trace_rate,
        "speedup_vs_trace_512": mlp_rate / trace_rate["512"],
        "trace_rays_at_mlp_error": r_same,
        "speedup_at_mlp_error": mlp_rate / trace_rate[r_same] if r_same else None,
        "trace_rays_at_2pc": r_2pc,
        "mlp_rate_over_trace_rate_at_2pc": mlp_rate / trace_rate[r_2pc] if r_2pc else None}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
