"""Python binding of the C ABI (argument marshalling only).

Every function here fills the C structs of include/sdirt.h from plain
Python descriptions (any object with the attribute names of the lens /
sensor / query fields), allocates outputs as torch device tensors and calls
the library on torch's current stream.  No step of the computation runs in
Python or in torch.
"""

import ctypes as C
import json

import torch

from . import _abi as abi


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _expect(t, name, dtype, numel, required=True):
    """Raise ValueError unless t is a contiguous device tensor of the given
    dtype and element count (the layout the C call will read or write)."""
    if t is None:
        if required:
            raise ValueError("%s is required" % name)
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != numel:
        raise ValueError("%s must hold %d elements, got %d" % (name, numel, t.numel()))


def _psf_layout(desc):
    """(dtype, element count) of the kernels a render descriptor reads."""
    ks2 = 2 * desc.ks * desc.ks
    if desc.source == abi.SRC_DENSE:
        dt = torch.bfloat16 if desc.psf_dtype == abi.BF16 else torch.float32
        return dt, desc.N * desc.H * desc.W * desc.psf_channels * ks2
    n = desc.bank_fields * desc.bank_depths * desc.bank_lambdas * ks2
    if desc.source == abi.SRC_BANK2D:
        n *= desc.bank_fields_y
    return torch.float32, n


def _check_render(desc, psf=None, depth=None, img=None, out=None, grad_out=None,
                  grad_img=None, grad_psf=None):
    N, C_, H, W = desc.N, desc.C, desc.H, desc.W
    pdt, pn = _psf_layout(desc)
    _expect(psf, "psf", pdt, pn, required=False)
    _expect(grad_psf, "grad_psf", pdt, pn, required=False)
    _expect(depth, "depth", torch.float32, N * H * W, required=desc.source != abi.SRC_DENSE)
    _expect(img, "img", torch.float32, N * C_ * H * W, required=False)
    _expect(grad_img, "grad_img", torch.float32, N * C_ * H * W, required=False)
    _expect(out, "out", torch.float32, N * 2 * C_ * H * W, required=False)
    _expect(grad_out, "grad_out", torch.float32, N * 2 * C_ * H * W, required=False)


def _material(m):
    kind, p0, p1 = m
    return int(kind), float(p0), float(p1)


def make_lens(lens):
    """C struct for a lens description; returns (struct, keepalive)."""
    S = len(lens.surfaces)
    arr = (abi.Surface * S)()
    for i, s in enumerate(lens.surfaces):
        k, p0, p1 = _material(s.medium)
        arr[i].kind = int(s.kind)
        arr[i].material = k
        arr[i].mat_p0 = p0
        arr[i].mat_p1 = p1
        arr[i].c = float(s.c)
        arr[i].t = float(s.t)
        arr[i].semi_diameter = float(s.semi_diameter)
        arr[i].conic = float(getattr(s, "conic", 0.0))
        for m, a in enumerate(getattr(s, "asph", (0.0,) * 5)):
            arr[i].asph[m] = float(a)
        arr[i].focal = float(getattr(s, "focal", 0.0))
    L = abi.Lens()
    L.n_surfaces = S
    L.stop = int(lens.stop)
    L.surfaces = C.cast(arr, C.POINTER(abi.Surface))
    k, p0, p1 = _material(lens.object_medium)
    L.object_material, L.object_p0, L.object_p1 = k, p0, p1
    L.f_number = float(lens.f_number)
    L.focus_depth = float(lens.focus_depth)
    L.ref_wavelength = float(lens.ref_wavelength)
    return L, arr


def make_sensor(sensor):
    s = abi.Sensor()
    s.pitch = float(sensor.pitch)
    s.dp_mode = int(sensor.dp_mode)
    s.sigmoid_k = float(sensor.sigmoid_k)
    s.ml_h, s.ml_f, s.ml_w, s.ml_r = (float(sensor.ml_h), float(sensor.ml_f),
                                      float(sensor.ml_w), float(sensor.ml_r))
    return s


def _darr(vals):
    vals = [float(v) for v in vals]
    return (C.c_double * max(1, len(vals)))(*vals)


def make_query(query, math=abi.F64, points=None):
    """C struct for a PSF query; `points` (device float64 [P][4]) selects list
    mode.  Returns (struct, keepalive)."""
    q = abi.PsfQuery()
    keep = []
    flat = [v for f in query.fields for v in f]
    fa, da, la = _darr(flat), _darr(query.depths), _darr(query.wavelengths)
    keep += [fa, da, la]
    q.n_fields = len(query.fields)
    q.n_depths = len(query.depths)
    q.n_wavelengths = len(query.wavelengths)
    q.fields = C.cast(fa, C.POINTER(C.c_double))
    q.depths = C.cast(da, C.POINTER(C.c_double))
    q.wavelengths = C.cast(la, C.POINTER(C.c_double))
    if points is not None:
        q.n_points = int(points.shape[0])
        q.points = points.data_ptr()
        keep.append(points)
    q.rays_x = int(query.rays_x)
    q.rays_y = int(query.rays_y)
    q.seed = int(query.seed) & 0xFFFFFFFF
    q.jitter = 1 if query.jitter else 0
    q.ks = int(query.ks)
    q.splat = int(query.splat)
    q.normalize = int(query.normalize)
    q.out_dtype = abi.F64 if query.out_f64 else abi.F32
    q.math = int(math)
    q.deterministic = 1 if getattr(query, "deterministic", False) else 0
    return q, keep


def resolve_lens(lens):
    L, keep = make_lens(lens)
    info = abi.LensInfo()
    abi.check("sdirt_resolve_lens", abi.lib().sdirt_resolve_lens(C.byref(L), C.byref(info)))
    return {n: getattr(info, n) for n, _ in abi.LensInfo._fields_}


def pupil(lens, wavelength):
    L, keep = make_lens(lens)
    z, r = C.c_double(), C.c_double()
    abi.check("sdirt_pupil", abi.lib().sdirt_pupil(C.byref(L), float(wavelength),
                                                   C.byref(z), C.byref(r)))
    return z.value, r.value


def n_params(lens):
    L, keep = make_lens(lens)
    return abi.lib().sdirt_n_params(C.byref(L))


def trace_rays(lens, wavelength, o, d, math=abi.F64):
    """Per-surface hits [n][S+1][6] (float64) and status [n] (int32)."""
    assert o.is_cuda and d.is_cuda and o.dtype == torch.float64 and d.dtype == torch.float64
    o = o.contiguous()
    d = d.contiguous()
    n = o.shape[0]
    L, keep = make_lens(lens)
    S = len(lens.surfaces)
    hits = torch.empty((n, S + 1, 6), dtype=torch.float64, device=o.device)
    status = torch.empty((n,), dtype=torch.int32, device=o.device)
    rc = abi.lib().sdirt_trace_rays(C.byref(L), float(wavelength), int(math), n,
                                    _dptr(o), _dptr(d), _dptr(hits), _dptr(status),
                                    _stream())
    abi.check("sdirt_trace_rays", rc)
    return hits, status


def trace_dp_psf(lens, sensor, query, math=abi.F64, points=None, out=None,
                 stats=True, chunks=None, device="cuda"):
    """DP PSFs [P][2][ks][ks] and stats [P][7] on the device."""
    L, keep = make_lens(lens)
    s = make_sensor(sensor)
    q, keep2 = make_query(query, math, points)
    P = q.n_points if points is not None else q.n_fields * q.n_depths * q.n_wavelengths
    dt = torch.float64 if query.out_f64 else torch.float32
    if points is not None:
        _expect(points, "points", torch.float64, 4 * P)
    if out is None:
        out = torch.empty((P, 2, query.ks, query.ks), dtype=dt, device=device)
    _expect(out, "out", dt, P * 2 * query.ks * query.ks)
    st = torch.empty((P, 7), dtype=torch.float64, device=out.device) if stats else None
    if chunks is None:
        rc = abi.lib().sdirt_trace_dp_psf(C.byref(L), C.byref(s), C.byref(q),
                                          _dptr(out), _dptr(st), _stream())
    else:
        rc = abi.lib().sdirt_trace_dp_psf_chunks(C.byref(L), C.byref(s), C.byref(q),
                                                 _dptr(out), _dptr(st), int(chunks),
                                                 _stream())
    abi.check("sdirt_trace_dp_psf", rc)
    return out, st


def trace_dp_psf_backward(lens, sensor, query, grad_psf, math=abi.F64):
    """Gradient [8 S + 1] (float64) of <grad_psf, PSF> w.r.t. the lens
    parameters and the response slope."""
    L, keep = make_lens(lens)
    s = make_sensor(sensor)
    q, keep2 = make_query(query, math)
    P = q.n_fields * q.n_depths * q.n_wavelengths
    g = grad_psf.contiguous().float()
    _expect(g, "grad_psf", torch.float32, P * 2 * query.ks * query.ks)
    n = abi.lib().sdirt_n_params(C.byref(L))
    out = torch.empty((n,), dtype=torch.float64, device=g.device)
    rc = abi.lib().sdirt_trace_dp_psf_backward(C.byref(L), C.byref(s), C.byref(q),
                                               _dptr(g), _dptr(out), _stream())
    abi.check("sdirt_trace_dp_psf_backward", rc)
    return out


def make_render_desc(N, C_, H, W, ks, source=abi.SRC_DENSE, psf_channels=None,
                     psf_dtype=abi.F32, field_radii=None, inv_depths=None,
                     bank_lambdas=1, lambda_of_channel=None, pitch=0.0, field_y=None,
                     bank_math=abi.BANK_FP32):
    """Render descriptor; for the banks, field_radii is the radial grid
    (SRC_BANK) or the x grid (SRC_BANK2D, with field_y the y grid)."""
    d = abi.RenderDesc()
    d.N, d.C, d.H, d.W, d.ks = int(N), int(C_), int(H), int(W), int(ks)
    d.source = int(source)
    d.psf_channels = int(psf_channels if psf_channels is not None else C_)
    d.psf_dtype = int(psf_dtype)
    d.bank_math = int(bank_math)
    keep = []
    if source == abi.SRC_BANK2D:
        fy = _darr(field_y)
        keep.append(fy)
        d.bank_fields_y = len(field_y)
        d.field_y = C.cast(fy, C.POINTER(C.c_double))
    if source in (abi.SRC_BANK, abi.SRC_BANK2D):
        fr, iv = _darr(field_radii), _darr(inv_depths)
        keep += [fr, iv]
        d.bank_fields = len(field_radii)
        d.bank_depths = len(inv_depths)
        d.bank_lambdas = int(bank_lambdas)
        d.field_radii = C.cast(fr, C.POINTER(C.c_double))
        d.inv_depths = C.cast(iv, C.POINTER(C.c_double))
        loc = lambda_of_channel if lambda_of_channel is not None else [0] * C_
        for c in range(C_):
            d.lambda_of_channel[c] = int(loc[c])
        d.pitch = float(pitch)
    return d, keep


def render_dp(desc, img, psf, depth=None, out=None):
    """out [N][2C][H][W] float32."""
    img = img.contiguous()
    if out is None:
        out = torch.empty((desc.N, 2 * desc.C, desc.H, desc.W), dtype=torch.float32,
                          device=img.device)
    _check_render(desc, psf=psf, depth=depth, img=img, out=out)
    rc = abi.lib().sdirt_render_dp(C.byref(desc), _dptr(img),
                                   _dptr(psf), _dptr(depth), _dptr(out), _stream())
    abi.check("sdirt_render_dp", rc)
    return out


def render_dp_backward(desc, psf, grad_out, depth=None, grad_img=None):
    grad_out = grad_out.contiguous()
    if grad_img is None:
        grad_img = torch.empty((desc.N, desc.C, desc.H, desc.W), dtype=torch.float32,
                               device=grad_out.device)
    _check_render(desc, psf=psf, depth=depth, grad_out=grad_out, grad_img=grad_img)
    rc = abi.lib().sdirt_render_dp_backward(C.byref(desc), _dptr(psf), _dptr(depth),
                                            _dptr(grad_out), _dptr(grad_img), _stream())
    abi.check("sdirt_render_dp_backward", rc)
    return grad_img


# ---- PSF surrogate MLP ------------------------------------------------------

def render_dp_psf_backward(desc, img, grad_out, depth=None, grad_psf=None):
    """Gradient of the render with respect to its kernels: the dense map
    [N][H][W][Cp][2][ks][ks] (the descriptor's kernel dtype) or the bank in
    its own layout (float32; depth required)."""
    img = img.contiguous()
    grad_out = grad_out.contiguous()
    if grad_psf is None:
        ks = desc.ks
        if desc.source == abi.SRC_DENSE:
            dt = torch.bfloat16 if desc.psf_dtype == abi.BF16 else torch.float32
            shape = (desc.N, desc.H, desc.W, desc.psf_channels, 2, ks, ks)
        elif desc.source == abi.SRC_BANK2D:
            dt = torch.float32
            shape = (desc.bank_fields_y, desc.bank_fields, desc.bank_depths, desc.bank_lambdas,
                     2, ks, ks)
        else:
            dt = torch.float32
            shape = (desc.bank_fields, desc.bank_depths, desc.bank_lambdas, 2, ks, ks)
        grad_psf = torch.empty(shape, dtype=dt, device=img.device)
    _check_render(desc, depth=depth, img=img, grad_out=grad_out, grad_psf=grad_psf)
    rc = abi.lib().sdirt_render_dp_psf_backward(C.byref(desc), _dptr(img), _dptr(depth),
                                                _dptr(grad_out), _dptr(grad_psf), _stream())
    abi.check("sdirt_render_dp_psf_backward", rc)
    return grad_psf


def make_mlp_desc(n_hidden=5, width=256, n_out=2 * 33 * 33, n_freq=8, x_half=1.0,
                  y_half=1.0, iv_lo=0.0, iv_hi=1.0, lam_lo=0.4, lam_hi=0.7,
                  loss=abi.LOSS_L2MAX):
    d = abi.MlpDesc()
    d.loss = int(loss)
    d.n_hidden, d.width, d.n_out, d.n_freq = int(n_hidden), int(width), int(n_out), int(n_freq)
    d.x_half, d.y_half = float(x_half), float(y_half)
    d.iv_lo, d.iv_hi = float(iv_lo), float(iv_hi)
    d.lam_lo, d.lam_hi = float(lam_lo), float(lam_hi)
    return d


def mlp_n_params(desc):
    n = C.c_longlong()
    abi.check("sdirt_mlp_n_params", abi.lib().sdirt_mlp_n_params(C.byref(desc), C.byref(n)))
    return n.value


def mlp_workspace(desc, batch, device="cuda"):
    n = C.c_size_t()
    abi.check("sdirt_mlp_workspace_size",
              abi.lib().sdirt_mlp_workspace_size(C.byref(desc), int(batch), C.byref(n)))
    return torch.empty((n.value,), dtype=torch.uint8, device=device)


def _check_mlp(desc, params, workspace=None, ws_batch=None):
    _expect(params, "params", torch.float32, mlp_n_params(desc))
    if workspace is not None:
        n = C.c_size_t()
        abi.check("sdirt_mlp_workspace_size",
                  abi.lib().sdirt_mlp_workspace_size(C.byref(desc), int(ws_batch), C.byref(n)))
        if workspace.numel() * workspace.element_size() < n.value or not workspace.is_cuda:
            raise ValueError("workspace must be a device buffer of at least %d bytes" % n.value)


def mlp_forward(desc, params, x, workspace, ws_batch, out_dtype=abi.F32, out=None):
    n = x.shape[0]
    x = x.contiguous()
    dt = torch.bfloat16 if out_dtype == abi.BF16 else torch.float32
    if out is None:
        out = torch.empty((n, desc.n_out), dtype=dt, device=x.device)
    _check_mlp(desc, params, workspace, ws_batch)
    _expect(x, "x", torch.float32, 4 * n)
    _expect(out, "out", dt, n * desc.n_out)
    rc = abi.lib().sdirt_mlp_forward(C.byref(desc), _dptr(params), int(n), _dptr(x),
                                     _dptr(out), int(out_dtype), _dptr(workspace),
                                     int(ws_batch), _stream())
    abi.check("sdirt_mlp_forward", rc)
    return out


def mlp_forward_noalloc(desc, params, x, out_dtype=abi.F32, out=None):
    """mlp_forward without a workspace: the library's static scratch array
    holds the working memory (allocation-free; calls that overlap on one
    device race).  Width-256 networks only."""
    n = x.shape[0]
    x = x.contiguous()
    dt = torch.bfloat16 if out_dtype == abi.BF16 else torch.float32
    if out is None:
        out = torch.empty((n, desc.n_out), dtype=dt, device=x.device)
    _check_mlp(desc, params)
    _expect(x, "x", torch.float32, 4 * n)
    _expect(out, "out", dt, n * desc.n_out)
    rc = abi.lib().sdirt_mlp_forward_noalloc(C.byref(desc), _dptr(params), int(n), _dptr(x),
                                             _dptr(out), int(out_dtype), _stream())
    abi.check("sdirt_mlp_forward_noalloc", rc)
    return out


def psf_hybrid(desc, params, lens, sensor, query, points, band_edges, band_error, max_error,
               workspace, ws_batch, out=None):
    """PSFs [P][2][ks][ks] (float32) of list-mode points (device float64
    [P][4]) from the network where its measured error per inverse-depth band
    is at most max_error, ray traced elsewhere; returns (psf, source) with
    source [P] int32 (0 network, 1 traced)."""
    P = int(points.shape[0])
    ks = int(query.ks)
    _check_mlp(desc, params, workspace, ws_batch)
    _expect(points, "points", torch.float64, 4 * P)
    if out is None:
        out = torch.empty((P, 2, ks, ks), dtype=torch.float32, device=points.device)
    _expect(out, "out", torch.float32, P * 2 * ks * ks)
    src = torch.empty((P,), dtype=torch.int32, device=points.device)
    L, keep = make_lens(lens)
    s = make_sensor(sensor)
    q, keep2 = make_query(query, abi.F64, points)
    edges, errs = _darr(band_edges), _darr(band_error)
    rc = abi.lib().sdirt_psf_hybrid(C.byref(desc), _dptr(params), C.byref(L), C.byref(s),
                                    C.byref(q), len(band_error), edges, errs, float(max_error),
                                    _dptr(out), _dptr(src), _dptr(workspace), int(ws_batch),
                                    _stream())
    abi.check("sdirt_psf_hybrid", rc)
    return out, src


def mlp_render(desc, params, img, depth, wavelengths, pitch, workspace, ws_batch, out=None):
    """Surrogate render: img [N][C][H][W] f32 rendered with the network's PSF
    for every pixel and channel (depth [N][H][W] mm, wavelengths [C] um,
    pitch mm); returns out [N][2C][H][W] f32."""
    assert img.is_cuda and img.dtype == torch.float32 and depth.dtype == torch.float32
    N, C_, H, W = img.shape
    assert tuple(depth.shape[-2:]) == (H, W) and depth.numel() == N * H * W
    ks = int(round((desc.n_out // 2) ** 0.5))
    rd = abi.MlpRenderDesc(N, C_, H, W, ks, float(pitch))
    for c, lam in enumerate(wavelengths):
        rd.wavelength[c] = float(lam)
    img = img.contiguous()
    depth = depth.contiguous()
    if out is None:
        out = torch.empty((N, 2 * C_, H, W), dtype=torch.float32, device=img.device)
    _check_mlp(desc, params, workspace, ws_batch)
    _expect(out, "out", torch.float32, N * 2 * C_ * H * W)
    rc = abi.lib().sdirt_mlp_render(C.byref(desc), _dptr(params), C.byref(rd),
                                    _dptr(img), _dptr(depth),
                                    _dptr(out), _dptr(workspace), int(ws_batch), _stream())
    abi.check("sdirt_mlp_render", rc)
    return out


def mlp_backward(desc, params, x, target, workspace):
    B = int(x.shape[0])
    x = x.contiguous()
    target = target.contiguous()
    _check_mlp(desc, params, workspace, B)
    _expect(x, "x", torch.float32, 4 * B)
    _expect(target, "target", torch.float32, B * desc.n_out)
    grads = torch.empty_like(params)
    loss = torch.empty((1,), dtype=torch.float32, device=params.device)
    rc = abi.lib().sdirt_mlp_backward(C.byref(desc), _dptr(params), B,
                                      _dptr(x), _dptr(target),
                                      _dptr(grads), _dptr(loss), _dptr(workspace), _stream())
    abi.check("sdirt_mlp_backward", rc)
    return grads, loss


def mlp_vjp(desc, params, x, grad_psf, workspace, ws_batch):
    """Gradient of sum_rows <grad_psf, P(x)> with respect to the parameters
    (float32 [n_params]) and that sum ([1])."""
    n = int(x.shape[0])
    x = x.contiguous()
    grad_psf = grad_psf.contiguous()
    _check_mlp(desc, params, workspace, ws_batch)
    _expect(x, "x", torch.float32, 4 * n)
    _expect(grad_psf, "grad_psf", torch.float32, n * desc.n_out)
    grads = torch.empty_like(params)
    value = torch.empty((1,), dtype=torch.float32, device=params.device)
    rc = abi.lib().sdirt_mlp_vjp(C.byref(desc), _dptr(params), n, _dptr(x),
                                 _dptr(grad_psf), _dptr(grads), _dptr(value),
                                 _dptr(workspace), int(ws_batch), _stream())
    abi.check("sdirt_mlp_vjp", rc)
    return grads, value


def mlp_adam(desc, params, m, v, grads, step, lr):
    n = mlp_n_params(desc)
    for t, name in ((params, "params"), (m, "m"), (v, "v"), (grads, "grads")):
        _expect(t, name, torch.float32, n)
    rc = abi.lib().sdirt_mlp_adam(C.byref(desc), _dptr(params), _dptr(m), _dptr(v),
                                  _dptr(grads), int(step), float(lr), _stream())
    abi.check("sdirt_mlp_adam", rc)


def mlp_train_step(desc, params, m, v, x, target, workspace, step, lr, loss_out=None):
    """One step on the batch (x, target): forward, loss gradient and the Adam
    update of step `step` (from 1); params, m and v are updated in place."""
    B = int(x.shape[0])
    n = mlp_n_params(desc)
    for t, name in ((params, "params"), (m, "m"), (v, "v")):
        _expect(t, name, torch.float32, n)
    _check_mlp(desc, params, workspace, B)
    _expect(x, "x", torch.float32, 4 * B)
    _expect(target, "target", torch.float32, B * desc.n_out)
    _expect(loss_out, "loss_out", torch.float32, 1, required=False)
    rc = abi.lib().sdirt_mlp_train_step(C.byref(desc), _dptr(params), _dptr(m), _dptr(v),
                                        int(step), float(lr), B, _dptr(x), _dptr(target),
                                        _dptr(loss_out), _dptr(workspace), _stream())
    abi.check("sdirt_mlp_train_step", rc)


def mlp_train(desc, params, m, v, x_all, t_all, workspace, batch, step0, n_steps,
              lr0=1e-3, lr_min=1e-5, total_steps=None, seed=1, loss_trace=None):
    total = int(total_steps if total_steps is not None else step0 + n_steps)
    n = mlp_n_params(desc)
    for t, name in ((params, "params"), (m, "m"), (v, "v")):
        _expect(t, name, torch.float32, n)
    _check_mlp(desc, params, workspace, batch)
    _expect(x_all, "x_all", torch.float32, 4 * int(x_all.shape[0]))
    _expect(t_all, "t_all", torch.float32, int(x_all.shape[0]) * desc.n_out)
    _expect(loss_trace, "loss_trace", torch.float32, int(n_steps), required=False)
    rc = abi.lib().sdirt_mlp_train(C.byref(desc), _dptr(params), _dptr(m), _dptr(v),
                                   int(step0), int(n_steps), float(lr0), float(lr_min), total,
                                   int(batch), int(x_all.shape[0]), _dptr(x_all), _dptr(t_all),
                                   int(seed) & 0xFFFFFFFF, _dptr(loss_trace),
                                   _dptr(workspace), _stream())
    abi.check("sdirt_mlp_train", rc)


# ---- trainer checkpoints ------------------------------------------------------

def mlp_save_checkpoint(path, desc, params, m, v, step, seed, total_steps, lr0, lr_min, batch):
    """Trainer state to a safetensors file: the float32 master parameters and
    Adam moments, and as metadata the next step, the data seed, the learning
    rate schedule (lr0, lr_min, total_steps), the batch size and the network
    description.  sdirt_mlp_train draws its batches by a counter hash of
    (seed, step, row) and sets the learning rate from the step and the
    schedule, so with these a resumed run continues the interrupted one."""
    from safetensors.torch import save_file
    meta = {"step": str(int(step)), "seed": str(int(seed)), "total_steps": str(int(total_steps)),
            "lr0": repr(float(lr0)), "lr_min": repr(float(lr_min)), "batch": str(int(batch)),
            "desc": json.dumps({n: getattr(desc, n) for n, _ in desc._fields_})}
    save_file({"params": params.detach().float().cpu().contiguous(),
               "m": m.detach().float().cpu().contiguous(),
               "v": v.detach().float().cpu().contiguous()}, path, metadata=meta)


def mlp_load_checkpoint(path, device="cuda"):
    """(desc, params, m, v, step, seed, total_steps, schedule) from
    mlp_save_checkpoint; schedule = {"lr0", "lr_min", "batch"}."""
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        meta = f.metadata()
        t = {k: f.get_tensor(k).to(device) for k in f.keys()}
    dd = json.loads(meta["desc"])
    desc = abi.MlpDesc()
    for n, _ in abi.MlpDesc._fields_:
        setattr(desc, n, dd[n])
    schedule = {"lr0": float(meta["lr0"]), "lr_min": float(meta["lr_min"]),
                "batch": int(meta["batch"])}
    return (desc, t["params"], t["m"], t["v"], int(meta["step"]), int(meta["seed"]),
            int(meta["total_steps"]), schedule)


def mlp_save_weights(path, desc, params, meta=None):
    """Trained network weights to a safetensors file: the float32 parameter
    vector, the network description and free-form metadata (JSON)."""
    from safetensors.torch import save_file
    m = {"desc": json.dumps({n: getattr(desc, n) for n, _ in desc._fields_}),
         "meta": json.dumps(meta or {})}
    save_file({"params": params.detach().float().cpu().contiguous()}, path, metadata=m)


def mlp_load_weights(path, device="cuda"):
    """(desc, params, meta) from mlp_save_weights."""
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        md = f.metadata()
        params = f.get_tensor("params").to(device)
    dd = json.loads(md["desc"])
    desc = abi.MlpDesc()
    for n, _ in abi.MlpDesc._fields_:
        setattr(desc, n, dd[n])
    return desc, params, json.loads(md["meta"])
