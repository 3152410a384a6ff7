"""Inputs of the trace's algorithmic FLOP model, counted on the oracle
(test helper, CPU only): per surface the fraction of launched rays that
reach it alive, and the mean number of Newton iterations per launched ray
summed over the even aspheres.  Iterations are counted by the stopping rule
of the kernels (a step below 1e-12 (1 + |Delta|), or below 1e-7 (1 + |Delta|)
and 1000 times smaller than the step before: Newton is then in its quadratic
regime and the next step would be below 1e-13 mm), from the step sizes the
oracle's own iteration takes on the same rays.

    python tests/flop_counts.py     # prints the constants for bench.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import optics, psf as opsf, trace as tr   # noqa: E402


def kernel_rule_iterations(steps):
    """steps [iterations, 2, n] (|step|, |Delta|) -> iterations per ray."""
    n = steps.shape[2]
    its = np.zeros(n)
    done = np.zeros(n, dtype=bool)
    prev = np.full(n, 1e30)
    for k in range(steps.shape[0]):
        a, dl = steps[k, 0], steps[k, 1]
        live = ~np.isnan(a) & ~done
        sc = 1.0 + dl
        stop = live & ((a < 1e-12 * sc) | ((a < 1e-7 * sc) & (a < 1e-3 * prev)))
        its[live] = k + 1
        done |= stop | np.isnan(a)
        prev = np.where(np.isnan(a), prev, a)
    return its


def sample_points(query, per_axis=(8, 4)):
    F, D, L = len(query.fields), len(query.depths), len(query.wavelengths)
    return [(f, d, l) for f in range(0, F, max(1, F // per_axis[0]))
            for d in range(0, D, max(1, D // per_axis[1])) for l in range(L)]


def count(lens, query, per_axis=(8, 4)):
    """(alive fraction per surface, Newton iterations per launched ray) over
    the sample of per_axis[0] fields x per_axis[1] depths x all wavelengths."""
    P = optics.Prepared(lens)
    S = len(lens.surfaces)
    n, alive, its = 0, np.zeros(S), 0.0
    for p in sample_points(query, per_axis):
        e, d = opsf.bundle(P, query, *p)
        log = {}
        tr.trace(P, query.wavelengths[p[2]], e, d, log=log)
        n += e.shape[0]
        for s in range(S):
            alive[s] += log["alive"][s].sum()
        for s, st in log.get("steps", {}).items():
            its += kernel_rule_iterations(st)[log["alive"][s]].sum()
    return alive / n, its / n


def paper_map_sample():
    """The paper's PSF-map workload (one PSF per pixel, list mode) as a grid
    sample for count(): 12 x 8 pixel positions over the sensor and 8 depths
    (all 768 points counted: per_axis=(96, 8))
    uniform in 1/d over the map's 0.5-20 m (its depth map draws each pixel's
    depth independently from that distribution), at the workload's 64 x 64
    rays per PSF."""
    import copy
    from workloads import configs
    lens, sensor, query, (H, W) = configs.paper_psf_map()
    q = copy.copy(query)
    xs = (np.linspace(0.0, W - 1, 12) - (W - 1) / 2.0) * sensor.pitch
    ys = (np.linspace(0.0, H - 1, 8) - (H - 1) / 2.0) * sensor.pitch
    q.fields = [(float(x), float(y)) for y in ys for x in xs]
    q.depths = list(1.0 / np.linspace(1.0 / 500.0, 1.0 / 20000.0, 8))
    return lens, q


if __name__ == "__main__":
    from workloads import configs
    for name, fn in (("config5", configs.config5), ("config2", configs.config2)):
        lens, sensor, query = fn(rays=64)
        a, it = count(lens, query)
        print(name, [round(float(v), 4) for v in a], round(float(it), 3))
    lens, q = paper_map_sample()
    a, it = count(lens, q, per_axis=(96, 8))
    print("paper_map", [round(float(v), 4) for v in a], round(float(it), 3))
