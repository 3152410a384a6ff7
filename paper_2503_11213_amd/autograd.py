"""torch.autograd wrappers of the library's forward and adjoint entry points
(argument marshalling only; every step runs in the library's kernels).

* ``TraceDPPSF``: DP PSFs (Eq. (3), Sec. 3.1) as a function of the lens
  parameter vector theta; the backward is the trace adjoint.
* ``RenderDP``: the pixel-wise dual-pixel render (Sec. 3.2; the output
  pixel's PSF convolved with the clamped image) as a function of the image
  and of its kernels (a dense per-pixel map or a traced bank); the backward
  is the image adjoint and the gradient with respect to the kernels.
* ``MlpPSF``: the surrogate network's PSFs (Sec. 3.2) as a function of its
  parameters; the backward is the network's vector-Jacobian product.

Chained, they give the gradient of an image-space loss with respect to the
lens prescription and the DP response slope, or to the network's weights.
theta follows the trace adjoint's order: per surface [c, t, conic, a4, a6,
a8, a10, a12] (t of the last surface is the sensor distance), then the
sigmoid slope k.  The gradient is that of the estimator at frozen framing:
pupil samples, pupil, window centres and the set of surviving rays are
those of the current theta, as the trace adjoint defines them.
"""

import copy

import torch

from . import sdirt, _abi as abi

PER_SURFACE = 8


def lens_theta(lens, sensor):
    """theta (float64, CPU) of a lens description; the last thickness is
    the resolved sensor distance (from the focus depth when one is set)."""
    info = sdirt.resolve_lens(lens)
    S = len(lens.surfaces)
    th = []
    for s, surf in enumerate(lens.surfaces):
        t = info["sensor_distance"] if s == S - 1 else surf.t
        th += [surf.c, t, getattr(surf, "conic", 0.0)]
        th += list(getattr(surf, "asph", (0.0,) * 5))
    th.append(sensor.sigmoid_k)
    return torch.tensor(th, dtype=torch.float64)


def lens_at(lens, sensor, theta):
    """Copies of the lens and sensor descriptions carrying theta.  The stop
    keeps the radius resolved for `lens` and the sensor sits at theta's last
    thickness: neither is re-derived from an f-number or a focus depth."""
    info = sdirt.resolve_lens(lens)
    th = [float(v) for v in theta.detach().cpu().tolist()]
    S = len(lens.surfaces)
    if len(th) != PER_SURFACE * S + 1:
        raise ValueError("theta has %d entries, the lens needs %d" % (len(th), PER_SURFACE * S + 1))
    l2 = copy.deepcopy(lens)
    for s, surf in enumerate(l2.surfaces):
        b = PER_SURFACE * s
        surf.c = th[b]
        surf.t = th[b + 1]
        surf.conic = th[b + 2]
        surf.asph = tuple(th[b + 3:b + 8])
    l2.surfaces[l2.stop].semi_diameter = info["stop_radius"]
    l2.f_number = 0.0
    l2.focus_depth = 0.0
    s2 = copy.copy(sensor)
    s2.sigmoid_k = th[-1]
    return l2, s2


class TraceDPPSF(torch.autograd.Function):
    """psf = TraceDPPSF.apply(theta, lens, sensor, query[, math]).

    query must use the TENT splat, no normalisation and the grid of fields x
    depths x wavelengths (the adjoint's modes); sensor the SIGMOID response.
    """

    @staticmethod
    def forward(ctx, theta, lens, sensor, query, math=abi.F64):
        l2, s2 = lens_at(lens, sensor, theta)
        psf, _ = sdirt.trace_dp_psf(l2, s2, query, math=math, stats=False)
        ctx.args = (l2, s2, query, math)
        ctx.theta_meta = (theta.device, theta.dtype)
        return psf

    @staticmethod
    def backward(ctx, grad_psf):
        l2, s2, query, math = ctx.args
        g = sdirt.trace_dp_psf_backward(l2, s2, query, grad_psf, math=math)
        dev, dt = ctx.theta_meta
        return g.to(device=dev, dtype=dt), None, None, None, None


class RenderDP(torch.autograd.Function):
    """out = RenderDP.apply(img, psf, desc, depth).

    desc from sdirt.make_render_desc (keep its keep-alive list while the
    graph lives); depth is required for the bank sources.  The kernel
    gradient has the shape of psf (the bank's float32 layout for the banks,
    the map's dtype for a dense map).
    """

    @staticmethod
    def forward(ctx, img, psf, desc, depth=None):
        out = sdirt.render_dp(desc, img, psf, depth=depth)
        ctx.desc = desc
        ctx.save_for_backward(img, psf, depth)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        img, psf, depth = ctx.saved_tensors
        desc = ctx.desc
        g_img = g_psf = None
        if ctx.needs_input_grad[0]:
            g_img = sdirt.render_dp_backward(desc, psf, grad_out, depth=depth)
        if ctx.needs_input_grad[1]:
            g_psf = sdirt.render_dp_psf_backward(desc, img, grad_out, depth=depth)
            g_psf = g_psf.reshape(psf.shape)
        return g_img, g_psf, None, None


class MlpPSF(torch.autograd.Function):
    """psf = MlpPSF.apply(params, x, desc, workspace, ws_batch): float32
    [n_rows][n_out] softmax outputs of the network for the inputs x
    [n_rows][4]; the gradient flows to params only."""

    @staticmethod
    def forward(ctx, params, x, desc, workspace, ws_batch):
        psf = sdirt.mlp_forward(desc, params, x, workspace, ws_batch, out_dtype=abi.F32)
        ctx.desc, ctx.workspace, ctx.ws_batch = desc, workspace, ws_batch
        ctx.save_for_backward(params, x)
        return psf

    @staticmethod
    def backward(ctx, grad_psf):
        params, x = ctx.saved_tensors
        g, _ = sdirt.mlp_vjp(ctx.desc, params, x, grad_psf.float(), ctx.workspace, ctx.ws_batch)
        return g, None, None, None, None
