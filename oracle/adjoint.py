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
