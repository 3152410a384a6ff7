"""C-ABI host layer on the CPU: the library loads, exports every declared
symbol, resolves lenses like the oracle and rejects invalid arguments before
any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from workloads import lenses, configs
from workloads.lens import Sensor, PsfQuery, DP_MICROLENS
from oracle import optics
from paper_2503_11213_amd import _abi as abi, sdirt

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "sdirt.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdirt_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = abi.lib()
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert lib.sdirt_version() >= 1
    assert lib.sdirt_status_string(abi.EINVAL) == b"invalid argument"


def exported_symbols():
    """sdirt_* functions the built library exports (its dynamic symbol table)."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    return sorted({ln.split()[-1] for ln in out.splitlines()
                   if len(ln.split()) == 3 and ln.split()[1] == "T" and
                   ln.split()[-1].startswith("sdirt_")})


def test_library_exports_only_declared_symbols():
    # the header is the whole boundary: nothing callable that it does not declare
    exported = exported_symbols()
    declared = set(declared_symbols())
    assert len(exported) >= 10
    assert [n for n in exported if n not in declared] == []
    assert set(abi.SIGNATURES) == declared


def _lenses():
    L1 = lenses.rf50(); L1.f_number = 4.0; L1.focus_depth = 1000.0
    return [lenses.singlet(), L1, configs.config2_lens(), lenses.rf35(),
            lenses.ideal(f=50.0, f_number=2.0, focus_depth=2000.0)]


@pytest.mark.parametrize("idx", range(5))
def test_resolve_lens_matches_oracle(idx):
    lens = _lenses()[idx]
    info = sdirt.resolve_lens(lens)
    P = optics.Prepared(lens)
    assert info["efl"] == pytest.approx(P.efl, rel=1e-12)
    assert info["sensor_distance"] == pytest.approx(P.sensor_distance, rel=1e-12)
    assert info["stop_radius"] == pytest.approx(P.stop_radius, rel=1e-12)
    assert info["z_ep"] == pytest.approx(P.z_ep_ref, rel=1e-12, abs=1e-12)
    assert info["m_num"] == pytest.approx(P._m_num, rel=1e-12)
    assert info["sensor_z"] == pytest.approx(P.sensor_z, rel=1e-12)
    for lam in (0.486, 0.55, 0.656):
        z, r = sdirt.pupil(lens, lam)
        zo, ro = P.pupil(lam)
        assert z == pytest.approx(zo, rel=1e-12, abs=1e-12)
        assert r == pytest.approx(ro, rel=1e-12)


def _call_trace(lens, sensor, query, out_ptr=0x1000):
    L, k1 = sdirt.make_lens(lens)
    s = sdirt.make_sensor(sensor)
    q, k2 = sdirt.make_query(query)
    return abi.lib().sdirt_trace_dp_psf(C.byref(L), C.byref(s), C.byref(q),
                                        C.c_void_p(out_ptr), C.c_void_p(0), C.c_void_p(0))


def test_invalid_lenses_are_rejected():
    lens, sensor, query = configs.config1()
    bad = []
    L = lenses.singlet(); L.stop = 7; bad.append(L)
    L = lenses.singlet(); L.surfaces[1].c = float("nan"); bad.append(L)
    L = lenses.singlet(); L.surfaces[1].semi_diameter = -1.0; bad.append(L)
    L = lenses.ideal(); L.surfaces[1].focal = 0.0; bad.append(L)
    L = lenses.rf50(); L.surfaces[8].conic = 50.0; bad.append(L)      # no real sag
    L = lenses.singlet(); L.ref_wavelength = 0.0; bad.append(L)
    L = lenses.singlet(); L.surfaces = []; bad.append(L)
    for lens in bad:
        assert _call_trace(lens, sensor, query) == abi.EINVAL


def test_invalid_queries_are_rejected():
    lens, sensor, query = configs.config1()
    import copy
    q = copy.deepcopy(query); q.ks = 30
    assert _call_trace(lens, sensor, q) == abi.EINVAL
    q = copy.deepcopy(query); q.ks = 131
    assert _call_trace(lens, sensor, q) == abi.EUNSUPPORTED
    q = copy.deepcopy(query); q.depths = [-5.0]
    assert _call_trace(lens, sensor, q) == abi.EINVAL
    q = copy.deepcopy(query); q.rays_x = 0
    assert _call_trace(lens, sensor, q) == abi.EINVAL
    q = copy.deepcopy(query); q.wavelengths = [0.5, 0.6, 0.7, 0.8, 0.9]
    assert _call_trace(lens, sensor, q) == abi.EUNSUPPORTED
    q = copy.deepcopy(query); q.wavelengths = [float("nan")]
    assert _call_trace(lens, sensor, q) == abi.EINVAL
    s = Sensor(pitch=0.004, dp_mode=DP_MICROLENS, ml_h=1.5, ml_f=1.44)
    assert _call_trace(lens, s, query) == abi.EINVAL
    s = Sensor(pitch=0.0)
    assert _call_trace(lens, s, query) == abi.EINVAL
    assert _call_trace(lens, sensor, query, out_ptr=0) == abi.EINVAL
    # deterministic mode: a flag, and its integer tile must fit in LDS
    q = copy.deepcopy(query); q.deterministic = True; q.ks = 103
    assert _call_trace(lens, sensor, q) == abi.EUNSUPPORTED
    qs, keep = sdirt.make_query(query)
    qs.deterministic = 2
    L, keepl = sdirt.make_lens(lens)
    rc = abi.lib().sdirt_trace_dp_psf(C.byref(L), C.byref(sdirt.make_sensor(sensor)), C.byref(qs),
                                      C.c_void_p(1), C.c_void_p(0), C.c_void_p(0))
    assert rc == abi.EINVAL


def test_invalid_render_descs_are_rejected():
    lib = abi.lib()
    def call(desc):
        return lib.sdirt_render_dp(C.byref(desc), C.c_void_p(0x1000), C.c_void_p(0x1000),
                                   C.c_void_p(0x1000), C.c_void_p(0x1000), C.c_void_p(0))
    d, k = sdirt.make_render_desc(1, 3, 16, 16, 4)
    assert call(d) == abi.EINVAL
    d, k = sdirt.make_render_desc(1, 5, 16, 16, 5)
    assert call(d) == abi.EUNSUPPORTED
    d, k = sdirt.make_render_desc(1, 3, 16, 16, 5, psf_channels=2)
    assert call(d) == abi.EINVAL
    d, k = sdirt.make_render_desc(1, 3, 16, 16, 5, source=abi.SRC_BANK,
                                  field_radii=[0.0, 0.2, 0.1], inv_depths=[1e-3, 2e-3],
                                  bank_lambdas=3, lambda_of_channel=[2, 1, 0], pitch=0.01)
    assert call(d) == abi.EINVAL
    d, k = sdirt.make_render_desc(1, 3, 16, 16, 5, source=abi.SRC_BANK,
                                  field_radii=[0.0, 0.1], inv_depths=[1e-3, 2e-3],
                                  bank_lambdas=2, lambda_of_channel=[2, 1, 0], pitch=0.01)
    assert call(d) == abi.EINVAL
    assert lib.sdirt_render_dp(C.byref(d), C.c_void_p(0), C.c_void_p(0), C.c_void_p(0),
                               C.c_void_p(0), C.c_void_p(0)) == abi.EINVAL
    # 8 N ceil(H / 8) ceil(W / 8) past 2^32 - 1 (the dense kernels' grid):
    # rejected before any launch
    d, k = sdirt.make_render_desc(4096, 3, 4096, 4096, 5)
    assert call(d) == abi.EUNSUPPORTED
    assert lib.sdirt_render_dp_psf_backward(C.byref(d), C.c_void_p(0x1000), C.c_void_p(0),
                                            C.c_void_p(0x1000), C.c_void_p(0x1000),
                                            C.c_void_p(0)) == abi.EUNSUPPORTED


def test_n_params():
    assert sdirt.n_params(configs.config2_lens()) == 8 * 13 + 1


def test_mlp_desc_validation():
    lib = abi.lib()
    n = C.c_longlong()
    d = sdirt.make_mlp_desc(n_hidden=5, width=256, n_out=2178, n_freq=8, x_half=4.5,
                            y_half=3.0, iv_lo=2e-4, iv_hi=2e-3, lam_lo=0.486, lam_hi=0.656)
    assert lib.sdirt_mlp_n_params(C.byref(d), C.byref(n)) == abi.OK
    assert n.value == 839554
    d.loss = abi.LOSS_KL
    assert lib.sdirt_mlp_n_params(C.byref(d), C.byref(n)) == abi.OK
    d.loss = 7
    assert lib.sdirt_mlp_n_params(C.byref(d), C.byref(n)) == abi.EINVAL
    d.loss = abi.LOSS_L2MAX
    d.width = 100
    assert lib.sdirt_mlp_n_params(C.byref(d), C.byref(n)) == abi.EINVAL


def test_surrogate_render_argument_validation():
    # rejected on the host before any device work
    lib = abi.lib()
    d = sdirt.make_mlp_desc(n_hidden=5, width=256, n_out=2178, n_freq=8, x_half=4.5,
                            y_half=3.0, iv_lo=2e-4, iv_hi=2e-3, lam_lo=0.486, lam_hi=0.656)
    p = C.c_void_p(16)     # never dereferenced: the call fails before any launch

    def call(rd, ws=64, ptr=p):
        return lib.sdirt_mlp_render(C.byref(d), ptr, C.byref(rd), ptr, ptr, ptr, ptr, ws, None)

    good = dict(N=1, C=3, H=8, W=8, ks=33, pitch=0.005)
    def desc(**kw):
        a = dict(good); a.update(kw)
        rd = abi.MlpRenderDesc(a["N"], a["C"], a["H"], a["W"], a["ks"], a["pitch"])
        for c in range(4):
            rd.wavelength[c] = 0.55
        return rd
    assert call(desc(ks=31)) == abi.EINVAL                 # 2 ks^2 != n_out
    assert call(desc(C=5)) == abi.EUNSUPPORTED
    assert call(desc(N=0)) == abi.EINVAL
    assert call(desc(pitch=-1.0)) == abi.EINVAL
    assert call(desc(), ws=100) == abi.EINVAL              # not a multiple of 64
    assert call(desc(), ptr=None) == abi.EINVAL
    rd = desc(); rd.wavelength[1] = float("nan")
    assert call(rd) == abi.EINVAL


@pytest.mark.parametrize("idx", [1, 2])
def test_lens_theta_round_trip(idx):
    # the autograd wrapper's parameter vector: a lens rebuilt from its own
    # theta (stop radius and sensor distance fixed, no f-number or focus)
    # resolves to the same first-order data
    from paper_2503_11213_amd.autograd import lens_theta, lens_at, PER_SURFACE
    lens = _lenses()[idx]
    sensor = Sensor(pitch=0.005, sigmoid_k=17.0)
    th = lens_theta(lens, sensor)
    S = len(lens.surfaces)
    assert th.shape == (PER_SURFACE * S + 1,)
    assert th.shape[0] == sdirt.n_params(lens)
    a = sdirt.resolve_lens(lens)
    assert th[PER_SURFACE * (S - 1) + 1].item() == a["sensor_distance"]
    assert th[-1].item() == 17.0
    l2, s2 = lens_at(lens, sensor, th)
    assert l2.f_number == 0.0 and l2.focus_depth == 0.0 and s2.sigmoid_k == 17.0
    b = sdirt.resolve_lens(l2)
    for k in ("efl", "sensor_distance", "stop_radius", "z_ep", "rho_ep", "m_num", "sensor_z"):
        assert b[k] == pytest.approx(a[k], rel=1e-12, abs=1e-12), k
    with pytest.raises(ValueError):
        lens_at(lens, sensor, th[:-1])


def test_trainer_checkpoint_round_trip(tmp_path):
    # parameters, Adam moments, step, seed, schedule and network description
    # survive a save / load unchanged (host tensors; no device work)
    import torch
    d = sdirt.make_mlp_desc(n_hidden=3, width=64, n_out=50, n_freq=8, x_half=2.0, y_half=1.0,
                            iv_lo=1e-4, iv_hi=2e-3, lam_lo=0.45, lam_hi=0.7, loss=abi.LOSS_KL)
    n = sdirt.mlp_n_params(d)
    g = torch.Generator().manual_seed(0)
    p, m, v = (torch.randn(n, generator=g) for _ in range(3))
    path = str(tmp_path / "trainer.safetensors")
    sdirt.mlp_save_checkpoint(path, d, p, m, v, step=1234, seed=77, total_steps=5000,
                              lr0=1.5e-3, lr_min=2.5e-5, batch=1024)
    d2, p2, m2, v2, step, seed, total, sched = sdirt.mlp_load_checkpoint(path, device="cpu")
    assert torch.equal(p, p2) and torch.equal(m, m2) and torch.equal(v, v2)
    assert (step, seed, total) == (1234, 77, 5000)
    assert sched == {"lr0": 1.5e-3, "lr_min": 2.5e-5, "batch": 1024}
    for name, _ in abi.MlpDesc._fields_:
        assert getattr(d2, name) == getattr(d, name), name


def test_committed_surrogate_weights_load():
    # the trained network bench.py times: its description, parameter count and
    # the held-out error table the fallback routes by (host only)
    desc, params, meta = sdirt.mlp_load_weights(
        os.path.join(os.path.dirname(__file__), "..", "workloads", "surrogate_ks33.safetensors"),
        device="cpu")
    assert (desc.n_hidden, desc.width, desc.n_out, desc.n_freq) == (5, 256, 2178, 8)
    assert params.numel() == sdirt.mlp_n_params(desc) == 839554
    assert len(meta["band_edges_inv_mm"]) == len(meta["band_energy_l1"]) + 1
    assert all(b > a for a, b in zip(meta["band_edges_inv_mm"], meta["band_edges_inv_mm"][1:]))
