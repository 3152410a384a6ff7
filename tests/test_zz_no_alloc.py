"""The allocation-free surrogate inference entry point against the one with
a caller workspace, through the C ABI: two calls in a row (the second with
fewer rows, so the static array holds the first call's contents), f32 and
bf16 outputs, and the size limit of the static array."""
import numpy as np
import pytest
import torch

from workloads import scenes
from paper_2503_11213_amd import sdirt, _abi as abi

pytestmark = pytest.mark.gpu

NORM = dict(x_half=4.5024, y_half=3.0016, iv_lo=1 / 5000, iv_hi=1 / 500, lam_lo=0.486,
            lam_hi=0.656)


def _net(n_out, seed):
    layers = scenes.mlp_init([64, 256, 256, 256, 256, 256, n_out], seed)
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers]).astype(np.float32)


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-4.5, 4.5, n), rng.uniform(-3, 3, n),
                     rng.uniform(1 / 5000, 1 / 500, n),
                     rng.choice([0.486, 0.55, 0.656], n)], 1).astype(np.float32)


@pytest.mark.parametrize("n_out,dt", [(2 * 33 * 33, abi.F32), (2 * 33 * 33, abi.BF16),
                                      (2 * 21 * 21, abi.F32)])
def test_noalloc_forward_matches_workspace_forward(n_out, dt):
    d = sdirt.make_mlp_desc(n_hidden=5, width=256, n_out=n_out, n_freq=8, **NORM)
    params = torch.from_numpy(_net(n_out, 3)).cuda()
    ws = sdirt.mlp_workspace(d, 4096)
    # 70000 rows: more than one chunk of the static array (a ragged tail);
    # then 700 rows, which reuses the array the first call left behind
    for n, seed in ((70000, 4), (700, 5)):
        print("noalloc n_out %d dtype %d rows %d" % (n_out, dt, n), flush=True)
        x = torch.from_numpy(_inputs(n, seed)).cuda()
        ref = sdirt.mlp_forward(d, params, x, ws, 4096, out_dtype=dt)
        got = sdirt.mlp_forward_noalloc(d, params, x, out_dtype=dt)
        torch.cuda.synchronize()
        # the same kernels on independent rows: identical bits
        assert torch.equal(got, ref)
        assert torch.isfinite(got.float()).all()


def test_noalloc_rejects_networks_beyond_the_static_array():
    # 40000 outputs: the bf16 output layer alone is 20 MB, beyond the 16 MiB
    # array; width 512 has no fused kernels
    d = sdirt.make_mlp_desc(n_hidden=5, width=256, n_out=40000, n_freq=8, **NORM)
    params = torch.zeros((sdirt.mlp_n_params(d),), device="cuda")
    x = torch.zeros((64, 4), device="cuda")
    with pytest.raises(abi.SdirtError) as e:
        sdirt.mlp_forward_noalloc(d, params, x)
    assert e.value.status == abi.ESCRATCH
    d2 = sdirt.make_mlp_desc(n_hidden=5, width=512, n_out=2 * 9 * 9, n_freq=8, **NORM)
    p2 = torch.zeros((sdirt.mlp_n_params(d2),), device="cuda")
    with pytest.raises(abi.SdirtError) as e:
        sdirt.mlp_forward_noalloc(d2, p2, x)
    assert e.value.status == abi.EUNSUPPORTED
