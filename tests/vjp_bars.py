"""Parity bars for the network's vector-Jacobian product against the
oracle's bf16 mirror (test helper, no GPU use)."""
import numpy as np

from oracle import mlp as M

REL = 1e-2


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def vjp_bars(P, x, g, norm):
    """Oracle gradients (bf16 mirror) of sum_rows <g, P(x)> and a bar per
    tensor.  The kernels round at the mirror's points but sum in float32
    where the mirror sums in float64, so a small fraction of their bf16
    roundings falls on the other side of the mirror's, and each such flip
    perturbs the layers below it.  The mirror's own rounding moves every
    value, so the kernels stay well inside the mirror's distance from plain
    float64 arithmetic (measured: 0.2-0.3 of it).  Where sums over rows
    cancel (upstream gradients of mixed sign) that distance exceeds REL;
    the bar is the larger of REL and half of it."""
    pb, cb = M.forward(P, x, norm, bf16=True)
    rb = M.backward(P, pb, cb, g, bf16=True, kind="vjp")
    pf, cf = M.forward(P, x, norm, bf16=False)
    rf = M.backward(P, pf, cf, g, bf16=False, kind="vjp")
    bars = []
    for (bW, bb), (fW, fb) in zip(rb, rf):
        bars += [max(REL, 0.5 * _rel_l2(bW, fW)), max(REL, 0.5 * _rel_l2(bb, fb))]
    return pb, rb, bars


def compare_flat(flat_grads, layers, ref, bars):
    off, errs = 0, []
    for (W, b), (gW, gb) in zip(layers, ref):
        errs.append(_rel_l2(flat_grads[off:off + W.size].reshape(W.shape), gW))
        off += W.size
        errs.append(_rel_l2(flat_grads[off:off + b.size], gb))
        off += b.size
    assert off == flat_grads.size
    print("rel L2 per tensor", [round(float(e), 5) for e in errs])
    print("bars", [round(float(b), 5) for b in bars])
    for e, b in zip(errs, bars):
        assert e <= b, (errs, bars)
