"""PSF surrogate workflow on the GPU (orchestration of C-ABI calls only).

Sec. 3.2 / Supplement S1.4: ray-traced DP PSFs at random points of the
valid imaging region are the training set of an MLP that then predicts the
PSF of every pixel of a depth map, which feeds the pixel-wise renderer; the
tracer stays the judge of the network's error.

    python -m paper_2503_11213_amd.surrogate [--samples N] [--steps S]

traces the training set, trains, measures the held-out energy L1 against
high-ray traces, times MLP inference against tracing at the same window
size, renders one image through the MLP PSF map and prints one JSON line.
"""

import argparse
import json
import time

import numpy as np
import torch

from . import sdirt, _abi as abi


def trace_points(lens, sensor, query, pts, rays=None, chunk=65536):
    """SUM-normalised traced PSFs [n][2 ks ks] (float32, device) at list-mode
    points (device float64 [n][4])."""
    import copy
    q = copy.copy(query)
    if rays is not None:
        q.rays_x = q.rays_y = int(rays)
    n = pts.shape[0]
    kk2 = 2 * q.ks * q.ks
    out = torch.empty((n, kk2), dtype=torch.float32, device=pts.device)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        view = out[a:b].view(b - a, 2, q.ks, q.ks)
        sdirt.trace_dp_psf(lens, sensor, q, points=pts[a:b].contiguous(), out=view, stats=False)
    return out


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
    ap.add_argument("--judge-rays", type=int, default=2048)
    ap.add_argument("--render", action="store_true")
    args = ap.parse_args()
    dev = torch.device("cuda", 0)
    lens, sensor, query = configs.config4()
    desc = sdirt.make_mlp_desc(n_hidden=5, width=256, n_out=2 * query.ks ** 2, n_freq=8,
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
    # held-out error, judged by the tracer at more rays
    hpts, hx = configs.surrogate_points(args.heldout, seed=2)
    hpts_t = torch.from_numpy(hpts).to(dev)
    judge = trace_points(lens, sensor, query, hpts_t, rays=args.judge_rays)
    same = trace_points(lens, sensor, query, hpts_t)
    hx_t = torch.from_numpy(hx).to(dev)
    ws_inf = sdirt.mlp_workspace(desc, 4096)
    pred = sdirt.mlp_forward(desc, params, hx_t, ws_inf, 4096)
    e_mlp = energy_l1(pred, judge)
    e_trace = energy_l1(same, judge)
    rec["heldout"] = {"points": args.heldout, "judge_rays": args.judge_rays ** 2,
                      "mlp_energy_l1_mean": float(e_mlp.mean()),
                      "mlp_energy_l1_median": float(e_mlp.median()),
                      "trace512_energy_l1_mean": float(e_trace.mean())}
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
    rec["throughput"] = {"mlp_psfs_per_s": nb / t_inf, "mlp_tflops": flop / t_inf / 1e12,
                         "trace_psfs_per_s": rec["dataset"]["trace_psfs_per_s"],
                         "speedup": (nb / t_inf) / rec["dataset"]["trace_psfs_per_s"]}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
