"""Oracle: gradients of traced DP PSFs by central finite differences
(float64).  Test infrastructure only.

The paper does not differentiate its simulator; differentiable lens tracers
are the setting it builds on (Sec. 2 and Sec. 3.1).  What is differentiated
here is the PSF estimator itself (pupil sampling, trace, angular DP
response, tent splat) under frozen framing: the pupil samples (ray origins
and directions), the entrance pupil, the window centres and the set of rays
that survive the trace are those of the base parameters; only the lens
surfaces, the sensor distance and the response slope move.

Parameter vector theta (8 S + 1 entries), per surface s:
    [c_s, t_s, k_s, a4_s, a6_s, a8_s, a10_s, a12_s]
(curvature, thickness to the next vertex -- for the last surface the sensor
distance --, conic and even-asphere coefficients; conic and a's act on
ASPHERE surfaces only, curvature on SPHERE/ASPHERE only), followed by the
slope k of the angular left/right response.  The contraction computed is
    dL/dtheta_p = sum_{q,s,i,j} G[q,s,i,j] dPSF[q,s,i,j]/dtheta_p
for a given upstream gradient G.
"""

import copy

import numpy as np

from workloads.lens import SPHERE, ASPHERE, DP_SIGMOID
from . import optics, psf as P, trace as tr

PER_SURFACE = 8


def n_params(S):
    return PER_SURFACE * S + 1


def get_theta(prep, sensor):
    S = prep.S
    th = np.zeros(n_params(S))
    for s, surf in enumerate(prep.lens.surfaces):
        b = PER_SURFACE * s
        th[b + 0] = surf.c
        th[b + 1] = prep.thickness[s]
        th[b + 2] = surf.conic
        th[b + 3:b + 8] = surf.asph
    th[-1] = sensor.sigmoid_k
    return th


def active_mask(prep):
    """Which entries of theta the estimator depends on."""
    S = prep.S
    m = np.zeros(n_params(S), dtype=bool)
    for s, surf in enumerate(prep.lens.surfaces):
        b = PER_SURFACE * s
        m[b + 1] = True
        if surf.kind in (SPHERE, ASPHERE):
            m[b + 0] = True
        if surf.kind == ASPHERE:
            m[b + 2:b + 8] = True
    m[-1] = True
    return m


def with_theta(prep, sensor, theta):
    """Copies of the prepared lens and sensor with theta applied, keeping
    pupil, stop radius and object points of the base (frozen framing)."""
    p2 = copy.copy(prep)
    lens = copy.deepcopy(prep.lens)
    for s, surf in enumerate(lens.surfaces):
        b = PER_SURFACE * s
        surf.c = float(theta[b + 0])
        surf.conic = float(theta[b + 2])
        surf.asph = tuple(float(a) for a in theta[b + 3:b + 8])
    p2.lens = lens
    p2.thickness = np.array(theta[1::PER_SURFACE][:prep.S], dtype=np.float64)
    p2.sensor_distance = float(p2.thickness[-1])
    s2 = copy.copy(sensor)
    s2.sigmoid_k = float(theta[-1])
    return p2, s2


class FrozenEstimator:
    """The TENT + SIGMOID PSF estimator of a query at fixed framing."""

    def __init__(self, lens, sensor, query):
        assert sensor.dp_mode == DP_SIGMOID
        self.prep = optics.Prepared(lens)
        self.sensor = sensor
        self.query = query
        F, D, L = len(query.fields), len(query.depths), len(query.wavelengths)
        self.points = [(f, d, l) for f in range(F) for d in range(D) for l in range(L)]
        self.bundles = []
        for (f, d, l) in self.points:
            e, dirs = P.bundle(self.prep, query, f, d, l)
            res = tr.trace(self.prep, query.wavelengths[l], e, dirs)
            alive = res["status"] == tr.ALIVE
            self.bundles.append((e[alive], dirs[alive]))
        self.theta0 = get_theta(self.prep, sensor)

    def psfs(self, theta):
        prep, sensor = with_theta(self.prep, self.sensor, theta)
        q = self.query
        out = np.zeros((len(self.points), 2, q.ks, q.ks))
        for idx, ((f, d, l), (e, dirs)) in enumerate(zip(self.points, self.bundles)):
            res = tr.trace(prep, q.wavelengths[l], e, dirs)
            alive = np.ones(e.shape[0], dtype=bool)
            out[idx], _ = P.split_and_bin(res["O"], res["D"], alive, q.fields[f],
                                          sensor, q.ks, q.splat)
        return out

    def landing_sensitivity(self, p, h):
        """Largest |dO/dtheta_p| over all rays (central differences of the
        landing points, which are smooth in theta)."""
        th0 = self.theta0
        q = self.query
        best = 0.0
        for sgn_pair in [(h, -h)]:
            outs = []
            for dh in sgn_pair:
                th = th0.copy(); th[p] += dh
                prep, _ = with_theta(self.prep, self.sensor, th)
                outs.append([tr.trace(prep, q.wavelengths[l], e, d)["O"]
                             for (f, dd, l), (e, d) in zip(self.points, self.bundles)])
            for a, b in zip(*outs):
                best = max(best, float(np.max(np.abs(a - b))) / (2 * h))
        return best

    def fd_gradient_at(self, G, p, h):
        """Central difference of <G, PSF(theta)> in parameter p with step h.
        The tent splat is piecewise bilinear in the landing point, so the
        step must move every landing point by much less than pitch / rays
        for the difference to resolve the derivative rather than kinks."""
        th0 = self.theta0
        tp = th0.copy(); tp[p] += h
        tm = th0.copy(); tm[p] -= h
        return (np.sum(G * self.psfs(tp)) - np.sum(G * self.psfs(tm))) / (2 * h)

    def ray_fd_gradient(self, G, p, h):
        """<G, dPSF/dtheta_p> with the finite difference taken per ray: each
        ray's landing point O and direction D are smooth in theta, so their
        central differences converge as h^2; the tent and response
        derivatives are then applied to them (the limit h -> 0 of the
        PSF-level difference, without the pixel-centre kinks)."""
        q = self.query
        ps = self.sensor.pitch
        k = self.sensor.sigmoid_k
        pad = (q.ks - 1) // 2
        th0 = self.theta0
        slope = p == len(th0) - 1
        total = 0.0
        prep0, _ = with_theta(self.prep, self.sensor, th0)
        for idx, ((f, d, l), (e, dirs)) in enumerate(zip(self.points, self.bundles)):
            lam = q.wavelengths[l]
            r0 = tr.trace(prep0, lam, e, dirs)
            O, D = r0["O"], r0["D"]
            if slope:
                dO = np.zeros_like(O)
                dD = np.zeros_like(D)
            else:
                tp = th0.copy(); tp[p] += h
                tm = th0.copy(); tm[p] -= h
                rp = tr.trace(with_theta(self.prep, self.sensor, tp)[0], lam, e, dirs)
                rm = tr.trace(with_theta(self.prep, self.sensor, tm)[0], lam, e, dirs)
                dO = (rp["O"] - rm["O"]) / (2 * h)
                dD = (rp["D"] - rm["D"]) / (2 * h)
            rr = np.sqrt(D[:, 0] ** 2 + D[:, 2] ** 2)
            sx = D[:, 0] / rr
            wl = 1.0 / (1.0 + np.exp(-k * sx))
            sig1 = wl * (1.0 - wl)
            dsx = (D[:, 2] ** 2 * dD[:, 0] - D[:, 0] * D[:, 2] * dD[:, 2]) / rr ** 3
            dwl = sig1 * sx if slope else sig1 * k * dsx
            w = (wl, 1.0 - wl)
            dw = (dwl, -dwl)
            hx, hy = q.fields[f]
            u = (O[:, 0] - hx) / ps + pad
            v = (O[:, 1] - hy) / ps + pad
            du, dv = dO[:, 0] / ps, dO[:, 1] / ps
            j0 = np.floor(u).astype(np.int64)
            i0 = np.floor(v).astype(np.int64)
            fx, fy = u - j0, v - i0
            taps = [(0, 0, (1 - fy) * (1 - fx), -(1 - fy), -(1 - fx)),
                    (0, 1, (1 - fy) * fx, (1 - fy), -fx),
                    (1, 0, fy * (1 - fx), -fy, (1 - fx)),
                    (1, 1, fy * fx, fy, fx)]
            for (a, b, wt, wtu, wtv) in taps:
                ii, jj = i0 + a, j0 + b
                inw = (ii >= 0) & (ii < q.ks) & (jj >= 0) & (jj < q.ks)
                for sd in range(2):
                    g = np.zeros(len(u))
                    g[inw] = G[idx, sd, ii[inw], jj[inw]]
                    total += np.sum(g * (w[sd] * (wtu * du + wtv * dv) + dw[sd] * wt))
        return total

    def fd_gradient(self, G, rel_step=1e-6, params=None, scale=None):
        """Central differences of <G, PSF(theta)> for each parameter."""
        th0 = self.theta0
        mask = active_mask(self.prep)
        grad = np.zeros_like(th0)
        idx = np.nonzero(mask)[0] if params is None else params
        for p in idx:
            sc = 1.0 if scale is None else scale[p]
            h = rel_step * max(abs(th0[p]), sc)
            tp = th0.copy(); tp[p] += h
            tm = th0.copy(); tm[p] -= h
            grad[p] = (np.sum(G * self.psfs(tp)) - np.sum(G * self.psfs(tm))) / (2 * h)
        return grad
