"""Pins of the oracle's network-with-tracer-fallback composition (CPU)."""
import numpy as np

from oracle import hybrid as Hy, psf as P
from workloads import configs


def test_route_band_edges_and_outside_points():
    edges = [1e-4, 2e-4, 5e-4, 1e-3]
    err = [0.01, 0.30, 0.01]
    # depths on the edges go to the band above; the last band keeps its
    # upper edge; points outside every band are traced
    depths = 1.0 / np.array([1e-4, 1.5e-4, 2e-4, 4e-4, 5e-4, 1e-3, 5e-5, 2e-3])
    got = Hy.route(depths, edges, err, 0.02)
    assert got.tolist() == [0, 0, 1, 1, 0, 0, 1, 1]
    assert Hy.route(depths, edges, err, np.inf).tolist() == [0, 0, 0, 0, 0, 0, 1, 1]
    assert Hy.route(depths, edges, err, 0.0).tolist() == [1] * 8


def test_all_traced_equals_the_list_mode_trace():
    # with a bar below every band's error the composition is the tracer's:
    # list point k is grid point (k, 0, 0) of a grid of copies of it
    lens, sensor, query = configs.config4(rays=16)
    query.ks = 9
    pts = np.array([[0.3, -0.2, 1500.0, 1], [1.0, 0.5, 800.0, 0]])
    from workloads import scenes
    layers = scenes.mlp_init([64, 256, 256, 256, 256, 256, 2 * 81], seed=0)
    params = [(W.astype(np.float64), b.astype(np.float64)) for W, b in layers]
    out, tr = Hy.psf_hybrid(params, configs.config4_desc_kwargs(), lens, sensor, query, pts,
                            [2e-4, 2e-3], [0.5], 0.0)
    assert tr.tolist() == [1, 1]
    for k in range(2):
        q = query.__class__(**{**query.__dict__})
        q.fields = [(pts[k, 0], pts[k, 1])] * (k + 1)
        q.depths = [pts[k, 2]]
        q.wavelengths = [query.wavelengths[int(pts[k, 3])]]
        ref, _ = P.trace_dp_psf(lens, sensor, q, points=[(k, 0, 0)])
        assert np.array_equal(out[k], ref[k])
        assert abs(out[k].sum() - 1.0) < 1e-12          # SUM-normalised
