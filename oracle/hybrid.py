"""Oracle: DP PSFs from the surrogate network with the ray tracer as its
fallback (float64).  Test infrastructure only.

Sec. 3.2 / Supplement S1.4: the network is trained on ray-traced PSFs, and
the tracer stays the reference that judges the network's error.  Reading
(the paper does not combine the two at query time): given the network's
measured error per band of inverse depth, a point takes the network's PSF
when its band's error is within a bar, and is ray traced otherwise (also
when its inverse depth lies outside every band).  Band b holds
edges[b] <= 1/d < edges[b+1], the last band including its upper edge, with
1/d in float64.  The network input of a point is (h_x, h_y, 1/d, lambda)
rounded to float32, as the network's own inputs are.
"""

import copy

import numpy as np

from . import mlp as M, psf as P


def route(depths, band_edges, band_error, max_error):
    """1 where a point is traced, 0 where it takes the network's PSF."""
    iv = 1.0 / np.asarray(depths, dtype=np.float64)
    edges = np.asarray(band_edges, dtype=np.float64)
    err = np.asarray(band_error, dtype=np.float64)
    n = len(err)
    traced = np.ones(iv.shape, dtype=np.int32)
    inside = (iv >= edges[0]) & (iv <= edges[n])
    b = np.zeros(iv.shape, dtype=np.int64)
    for k in range(1, n):
        b += iv >= edges[k]
    traced[inside] = (err[b[inside]] > max_error).astype(np.int32)
    return traced


def network_inputs(points, wavelengths):
    """(h_x, h_y, 1/d, lambda) in float32 for list points [P][4]."""
    pts = np.asarray(points, dtype=np.float64)
    lam = np.asarray(wavelengths, dtype=np.float64)[pts[:, 3].astype(np.int64)]
    return np.stack([pts[:, 0], pts[:, 1], 1.0 / pts[:, 2], lam], 1).astype(np.float32)


def trace_list_point(lens, sensor, query, point, k):
    """The traced PSF of list point k (its pupil jitter is the stream of
    point index k): point (k, 0, 0) of a grid whose fields all equal it."""
    q = copy.deepcopy(query)
    q.fields = [(float(point[0]), float(point[1]))] * (k + 1)
    q.depths = [float(point[2])]
    q.wavelengths = [query.wavelengths[int(point[3])]]
    psf, _ = P.trace_dp_psf(lens, sensor, q, points=[(k, 0, 0)])
    return psf[k]


def psf_hybrid(params, norm, lens, sensor, query, points, band_edges, band_error, max_error,
               bf16=True):
    """PSFs [P][2][ks][ks] and the routing [P] (1 traced)."""
    pts = np.asarray(points, dtype=np.float64)
    traced = route(pts[:, 2], band_edges, band_error, max_error)
    x = network_inputs(pts, query.wavelengths).astype(np.float64)
    p, _ = M.forward(params, x, norm, bf16=bf16)
    ks = query.ks
    out = p.reshape(len(pts), 2, ks, ks).copy()
    for k in np.nonzero(traced)[0]:
        out[k] = trace_list_point(lens, sensor, query, pts[k], int(k))
    return out, traced
