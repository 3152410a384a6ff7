"""GPU parity of the network-with-tracer-fallback PSF entry point against
the oracle's composition, through the C ABI: the routing bit for bit, the
traced PSFs to the tracer's bar, the network's PSFs to the network's bar."""
import numpy as np
import pytest
import torch

from workloads import configs, scenes
from oracle import hybrid as Hy
from paper_2503_11213_amd import sdirt, _abi as abi

pytestmark = pytest.mark.gpu

L1_TOL = 1e-3            # energy L1 of traced PSFs for identical seeded rays
ELT = 2.0 ** -5          # network PSFs: per element, of the row's largest value


def _case(n, seed, ks):
    lens, sensor, query = configs.config4(rays=32)
    query.ks = ks
    kw = configs.config4_desc_kwargs()
    rng = np.random.default_rng(seed)
    iv = rng.uniform(kw["iv_lo"], kw["iv_hi"], n)
    iv[:2] = [kw["iv_lo"] * 0.5, kw["iv_hi"] * 1.5]      # outside every band: traced
    pts = np.stack([rng.uniform(-kw["x_half"], kw["x_half"], n),
                    rng.uniform(-kw["y_half"], kw["y_half"], n), 1.0 / iv,
                    rng.integers(0, 3, n).astype(np.float64)], 1)
    edges = list(np.linspace(kw["iv_lo"], kw["iv_hi"], 5))
    errors = [0.01, 0.08, 0.015, 0.3]                     # bands 0 and 2 under the bar
    return lens, sensor, query, kw, pts, edges, errors


@pytest.mark.parametrize("n,ws,ks", [(70, 64, 9), (150, 128, 15)])
def test_hybrid_matches_the_oracle_composition(n, ws, ks):
    lens, sensor, query, kw, pts, edges, errors = _case(n, 61, ks)
    layers = scenes.mlp_init([64, 256, 256, 256, 256, 256, 2 * ks * ks], seed=62)
    flat = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers]).astype(np.float32)
    desc = sdirt.make_mlp_desc(n_hidden=5, width=256, n_out=2 * ks * ks, n_freq=8, **kw)
    psf, src = sdirt.psf_hybrid(desc, torch.from_numpy(flat).cuda(), lens, sensor, query,
                                torch.from_numpy(pts).cuda(), edges, errors, 0.02,
                                sdirt.mlp_workspace(desc, ws), ws)
    got, gsrc = psf.cpu().numpy(), src.cpu().numpy()
    params = [(W.astype(np.float64), b.astype(np.float64)) for W, b in layers]
    ref, rsrc = Hy.psf_hybrid(params, kw, lens, sensor, query, pts, edges, errors, 0.02)
    assert np.array_equal(gsrc, rsrc)
    assert 0 < rsrc.sum() < n                              # both sources in use
    for k in range(n):
        if rsrc[k]:
            l1 = np.abs(got[k] - ref[k]).sum() / ref[k].sum()
            assert l1 <= L1_TOL, (k, l1)
        else:
            e = np.abs(got[k] - ref[k]).max() / ref[k].max()
            assert e <= ELT, (k, e)
    assert np.allclose(got.reshape(n, -1).sum(axis=1), 1.0, atol=1e-4)


def test_hybrid_all_network_and_all_traced():
    ks, n, ws = 9, 70, 64
    lens, sensor, query, kw, pts, edges, errors = _case(n, 63, ks)
    pts[:2, 2] = 1500.0                                    # every point inside a band
    layers = scenes.mlp_init([64, 256, 256, 256, 256, 256, 2 * ks * ks], seed=64)
    flat = torch.from_numpy(np.concatenate([np.concatenate([W.ravel(), b])
                                            for W, b in layers]).astype(np.float32)).cuda()
    desc = sdirt.make_mlp_desc(n_hidden=5, width=256, n_out=2 * ks * ks, n_freq=8, **kw)
    ws_t = sdirt.mlp_workspace(desc, ws)
    pt = torch.from_numpy(pts).cuda()
    net, s1 = sdirt.psf_hybrid(desc, flat, lens, sensor, query, pt, edges, errors, 1e9, ws_t, ws)
    assert int(s1.sum()) == 0
    x = torch.from_numpy(Hy.network_inputs(pts, query.wavelengths)).cuda()
    direct = sdirt.mlp_forward(desc, flat, x, ws_t, ws)
    assert torch.equal(net.reshape(n, -1), direct)
    tr, s2 = sdirt.psf_hybrid(desc, flat, lens, sensor, query, pt, edges, errors, 0.0, ws_t, ws)
    assert int(s2.sum()) == n
    ref, _ = sdirt.trace_dp_psf(lens, sensor, query, points=pt, stats=False)
    assert torch.allclose(tr, ref, rtol=1e-6, atol=1e-7)
