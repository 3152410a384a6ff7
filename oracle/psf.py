"""Oracle: DP PSFs of a (field, depth, wavelength) grid (float64).
Test infrastructure only.

Eq. (3): PSF_L(i, j) = sum_k A_k delta_{L,k}(i, j) with unit ray energy
A_k = 1 and delta the unit impulse into the left sub-pixel of DP pixel
(i, j); PSF_R likewise.  The window is ks x ks pixels of pitch ps centred on
the field point h (the image-plane position of the object point); pixel
(i, j) covers y in h_y + [(i - pad - 1/2) ps, (i - pad + 1/2) ps) and x
likewise with j, pad = (ks - 1) / 2, row i toward +y and column j toward +x.

Splat rules
  BOX  (the paper's unit impulse): the ray's left/right energy goes to the
       pixel that contains its landing point;
  TENT (differentiable variant, not in the paper): the energy is shared
       bilinearly by the four pixel centres around the landing point.
The microlens model decides the sub-pixel from the containing pixel, then
the splat distributes the ray's unit energy to that side.

Per-point statistics (energies):
  [launched, vignetted (miss / clip / TIR / Newton / invalid), transmitted,
   left in window, right in window, missed sub-pixel, outside window]
with launched = vignetted + transmitted and
transmitted = left + right + missed + outside.

Normalisation (Sec. 3.2 / Supplement S1.4): SUM divides L and R jointly by
their total, MAX jointly by their largest pixel.
"""

import numpy as np

from workloads.lens import (DP_SIGMOID, DP_MICROLENS, SPLAT_BOX, SPLAT_TENT,
                            NORM_NONE, NORM_SUM, NORM_MAX)
from . import optics, pupil, trace as tr, dp

N_STATS = 7


def point_index(f, d, l, D, L):
    return (f * D + d) * L + l


def bundle(prep, query, f, d, l):
    """Rays of one PSF point: origins on the pupil plane and directions."""
    q = point_index(f, d, l, len(query.depths), len(query.wavelengths))
    lam = query.wavelengths[l]
    p = prep.object_point(query.fields[f], query.depths[d])
    z_ep, rho_ep = prep.pupil(lam)
    return pupil.pupil_rays(p, z_ep, rho_ep, query.rays_x, query.rays_y,
                            query.seed, q, query.jitter)


def split_and_bin(O, D, alive, h, sensor, ks, splat):
    """Accumulate one bundle's landed rays into (2, ks, ks) and stats."""
    ps = sensor.pitch
    pad = (ks - 1) // 2
    psf = np.zeros((2, ks, ks))
    st = np.zeros(N_STATS)
    n = O.shape[0]
    st[0] = n
    st[1] = n - np.count_nonzero(alive)
    st[2] = np.count_nonzero(alive)
    O = O[alive]
    D = D[alive]
    # continuous window coordinates: pixel centre (i, j) <-> (v, u) = (i, j)
    u = (O[:, 0] - h[0]) / ps + pad
    v = (O[:, 1] - h[1]) / ps + pad
    jb = np.floor(u + 0.5).astype(np.int64)
    ib = np.floor(v + 0.5).astype(np.int64)
    if sensor.dp_mode == DP_SIGMOID:
        wl, wr = dp.sigmoid_weights(D, sensor.sigmoid_k)
        energy = np.ones(O.shape[0])
    elif sensor.dp_mode == DP_MICROLENS:
        xc = h[0] + (jb - pad) * ps
        yc = h[1] + (ib - pad) * ps
        side = dp.microlens_side(O[:, 0], O[:, 1], xc, yc, D[:, 0] / D[:, 2],
                                 ps, sensor.ml_h, sensor.ml_f, sensor.ml_w,
                                 sensor.ml_r)
        wl = (side == dp.LEFT).astype(np.float64)
        wr = (side == dp.RIGHT).astype(np.float64)
        missed = side == dp.MISSED
        st[5] = np.count_nonzero(missed)
        energy = (~missed).astype(np.float64)
    else:
        raise ValueError("dp mode")
    if splat == SPLAT_BOX:
        taps = [(ib, jb, np.ones(O.shape[0]))]
    elif splat == SPLAT_TENT:
        j0 = np.floor(u).astype(np.int64)
        i0 = np.floor(v).astype(np.int64)
        fx = u - j0
        fy = v - i0
        taps = [(i0, j0, (1 - fy) * (1 - fx)), (i0, j0 + 1, (1 - fy) * fx),
                (i0 + 1, j0, fy * (1 - fx)), (i0 + 1, j0 + 1, fy * fx)]
    else:
        raise ValueError("splat")
    for (ii, jj, wt) in taps:
        inw = (ii >= 0) & (ii < ks) & (jj >= 0) & (jj < ks)
        np.add.at(psf[0], (ii[inw], jj[inw]), (wl * wt)[inw])
        np.add.at(psf[1], (ii[inw], jj[inw]), (wr * wt)[inw])
        st[3] += np.sum((wl * wt)[inw])
        st[4] += np.sum((wr * wt)[inw])
        st[6] += np.sum((energy * wt)[~inw])
    return psf, st


def normalize(psf, mode):
    if mode == NORM_NONE:
        return psf
    if mode == NORM_SUM:
        s = psf.sum()
    elif mode == NORM_MAX:
        s = psf.max()
    else:
        raise ValueError("normalize")
    return psf / s if s > 0 else psf


def trace_dp_psf(lens, sensor, query, points=None):
    """PSFs [P, 2, ks, ks] and stats [P, 7] for the query grid
    P = F x D x L (point index (f D + d) L + l).  `points`, if given, is a
    list of (f, d, l) to compute; the other rows stay zero."""
    prep = optics.Prepared(lens)
    F, D, L = len(query.fields), len(query.depths), len(query.wavelengths)
    ks = query.ks
    out = np.zeros((F * D * L, 2, ks, ks))
    stats = np.zeros((F * D * L, N_STATS))
    if points is None:
        points = [(f, d, l) for f in range(F) for d in range(D) for l in range(L)]
    for (f, d, l) in points:
        q = point_index(f, d, l, D, L)
        e, dirs = bundle(prep, query, f, d, l)
        res = tr.trace(prep, query.wavelengths[l], e, dirs)
        alive = res["status"] == tr.ALIVE
        psf, st = split_and_bin(res["O"], res["D"], alive, query.fields[f],
                                sensor, ks, query.splat)
        out[q] = normalize(psf, query.normalize)
        stats[q] = st
    return out, stats
