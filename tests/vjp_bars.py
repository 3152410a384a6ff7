"""Parity bar for the network's vector-Jacobian product against the oracle's
bf16 mirror (test helper, no GPU use).

The kernels round to bf16 at the same points as the mirror and differ from
it only where float32 summation (against the mirror's float64) moves a value
across a bf16 rounding boundary: one element then changes by 2^-8 of itself
and the change propagates through the layers below.  For upstream gradients
whose rows add up rather than cancel, the weight and bias gradients stay
within REL = 1e-2 (relative L2 per tensor) of the mirror.  Where row sums
cancel (independent upstream gradients of mixed sign over inputs spread
across the field), the mirror itself moves up to 12 % away from float64
arithmetic and no fixed bar of this size is meaningful; that case is covered
only by the chunk-sum consistency test.  The parity tests therefore use
inputs clustered around one point and upstream gradients sharing most of
their values, and `vjp_reference` checks that the chosen inputs are of that
kind: the mirror lies within 2.5e-2 of float64 arithmetic on every tensor."""
import numpy as np

from oracle import mlp as M

REL = 1e-2
COHERENT = 2.5e-2


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def vjp_reference(P, x, g, norm):
    """Oracle (bf16 mirror) softmax outputs and gradients of
    sum_rows <g, P(x)>; asserts that the rows do not cancel."""
    pb, cb = M.forward(P, x, norm, bf16=True)
    rb = M.backward(P, pb, cb, g, bf16=True, kind="vjp")
    pf, cf = M.forward(P, x, norm, bf16=False)
    rf = M.backward(P, pf, cf, g, bf16=False, kind="vjp")
    for (bW, bb), (fW, fb) in zip(rb, rf):
        assert _rel_l2(bW, fW) <= COHERENT and _rel_l2(bb, fb) <= COHERENT, \
            "test inputs whose row sums cancel"
    return pb, rb


def clustered_inputs(n, seed, centre=(1.3, -0.7, 1.0 / 1500.0, 0.55), spread=0.03):
    """n network inputs (h_x, h_y, 1/d, lambda) close to one point."""
    rng = np.random.default_rng(seed)
    x = np.tile(np.asarray(centre, dtype=np.float64), (n, 1))
    x[:, 0] += spread * rng.normal(size=n)
    x[:, 1] += spread * rng.normal(size=n)
    x[:, 2] *= 1.0 + spread * rng.normal(size=n)
    return x.astype(np.float32)


def compare_flat(flat_grads, layers, ref):
    off, errs = 0, []
    for (W, b), (gW, gb) in zip(layers, ref):
        errs.append(_rel_l2(flat_grads[off:off + W.size].reshape(W.shape), gW))
        off += W.size
        errs.append(_rel_l2(flat_grads[off:off + b.size], gb))
        off += b.size
    assert off == flat_grads.size
    print("rel L2 per tensor", [round(float(e), 5) for e in errs])
    assert max(errs) <= REL, errs
