"""Oracle: real-ray sequential trace (float64).  Test infrastructure only.

Sec. 3.1: each ray of the set A leaves the object point, is refracted at
every lens surface by Snell's law using the lens parameters, and reaches the
sensor plane with landing point O_k and direction D_k.  The paper gives no
intersection or sag rules; the ones below are the standard sequential-trace
definitions for the surface types of Table S1 (sphere, aperture plane, even
asphere with conic and a4..a12), plus an ideal (paraxial) surface for tests.

Per surface, in the local frame of its vertex (z along the axis):
  1. transfer the ray to the vertex plane z = 0;
  2. intersect
       plane / stop / ideal : already on z = 0,
       sphere  : c(x^2+y^2+z^2) - 2z = 0; from the vertex plane the nearer
                 root is  Delta = F / (G + sqrt(G^2 - c F)),
                 F = c (x^2 + y^2),  G = d_z - c (x d_x + y d_y);
                 a negative discriminant is a miss,
       asphere : z = sag(rho), rho = x^2 + y^2,
                 sag = c rho / (1 + sqrt(1 - (1+k) c^2 rho))
                       + a4 rho^2 + a6 rho^3 + a8 rho^4 + a10 rho^5 + a12 rho^6,
                 Newton on f(Delta) = Delta d_z - sag(rho(Delta)) started at
                 the root of the base conic;
  3. clip against the clear semi-diameter (the stop's radius for the stop);
  4. refract with mu = n_before / n_after by the vector form of Snell's law
       cos I = d . N,  K = 1 - mu^2 (1 - cos^2 I)   (K < 0: total internal
       reflection),  d' = mu d + (sqrt(K) - mu cos I) N,
     N the unit normal on the side the ray travels to; an ideal surface of
     focal length f maps the tangents (t_x, t_y) -> (t_x - x/f, t_y - y/f).
After the last surface the ray is carried to the sensor plane.
"""

import numpy as np

from workloads.lens import SPHERE, PLANE, STOP, ASPHERE, IDEAL

ALIVE, MISS, CLIP, TIR, NEWTON, INVALID = 0, 1, 2, 3, 4, 5

NEWTON_TOL = 1e-12
NEWTON_MAXIT = 50


def asphere_sag(surf, rho):
    """Even-asphere sag and its derivative with respect to rho = r^2.
    Returns (sag, dsag/drho, ok) with ok false where the conic root is
    imaginary."""
    c, k = surf.c, surf.conic
    a4, a6, a8, a10, a12 = surf.asph
    arg = 1.0 - (1.0 + k) * c * c * rho
    ok = arg >= 0.0
    q = np.sqrt(np.where(ok, arg, 1.0))
    sag = c * rho / (1.0 + q) + rho ** 2 * (a4 + rho * (a6 + rho * (a8 + rho * (a10 + rho * a12))))
    dsag = c / (2.0 * q) + rho * (2 * a4 + rho * (3 * a6 + rho * (4 * a8 + rho * (5 * a10 + rho * 6 * a12))))
    return sag, dsag, ok


def _intersect_asphere(surf, x, y, dx, dy, dz, status, steps_log=None):
    c, k = surf.c, surf.conic
    F = c * (x * x + y * y)
    G = dz - c * (x * dx + y * dy)
    a = c * (1.0 + k * dz * dz)
    disc = G * G - a * F
    delta = np.where(disc >= 0.0, F / (G + np.sqrt(np.maximum(disc, 0.0))), 0.0)
    conv = np.zeros(x.shape, dtype=bool)
    bad = np.zeros(x.shape, dtype=bool)
    steps = []                      # (|step|, |Delta|) per iteration (NaN once a ray stopped)
    for _ in range(NEWTON_MAXIT):
        xr = x + delta * dx
        yr = y + delta * dy
        rho = xr * xr + yr * yr
        sag, dsag, ok = asphere_sag(surf, rho)
        f = delta * dz - sag
        fp = dz - dsag * 2.0 * (xr * dx + yr * dy)
        step = f / fp
        active = ~conv & ~bad
        bad |= active & ~ok
        upd = active & ok
        delta = np.where(upd, delta - step, delta)
        steps.append(np.stack([np.where(upd, np.abs(step), np.nan),
                               np.where(upd, np.abs(delta), np.nan)]))
        conv |= upd & (np.abs(step) < NEWTON_TOL)
        if np.all(conv | bad):
            break
    if steps_log is not None:
        steps_log.append(np.array(steps))
    status[(~conv | bad) & (status == ALIVE)] = NEWTON
    xr = x + delta * dx
    yr = y + delta * dy
    return delta, xr, yr


def _refract(d, N, mu, status):
    """Vector Snell refraction; N unit, oriented along the travel side."""
    cosI = np.sum(d * N, axis=1)
    K = 1.0 - mu * mu * (1.0 - cosI * cosI)
    tir = K < 0.0
    status[tir & (status == ALIVE)] = TIR
    sq = np.sqrt(np.maximum(K, 0.0))
    return mu * d + (sq - mu * cosI)[:, None] * N


def trace(prep, lam, o, d, record=False, log=None):
    """Trace rays (global origin o, unit direction d; z = 0 at vertex 1).

    Returns dict with landing point O (n, 2) on the sensor, direction D
    (n, 3), status (n,) and, if record, hits (n, S+1, 6): per surface the
    vertex-local hit point (x, y, z) and the direction after refraction;
    the last entry is the sensor plane.

    log: optional dict that receives log["alive"][s], the rays still alive
    when they reach surface s (after its transfer), and for every asphere
    log["steps"][s], the |step| and the updated |Delta| of each Newton
    iteration per ray ([iterations, 2, n], NaN once a ray stopped).  Bookkeeping only: the trace
    is unchanged.
    """
    lens = prep.lens
    S = prep.S
    mu = prep.mu(lam)
    o = np.asarray(o, dtype=np.float64)
    d = np.array(d, dtype=np.float64)
    n = o.shape[0]
    x, y, z = o[:, 0].copy(), o[:, 1].copy(), o[:, 2].copy()
    status = np.zeros(n, dtype=np.int32)
    hits = np.zeros((n, S + 1, 6)) if record else None
    with np.errstate(all="ignore"):
        for s in range(S):
            surf = lens.surfaces[s]
            if s > 0:
                z = z - prep.thickness[s - 1]
            dx, dy, dz = d[:, 0], d[:, 1], d[:, 2]
            status[(dz <= 0.0) & (status == ALIVE)] = INVALID
            if log is not None:
                log.setdefault("alive", []).append(status == ALIVE)
            tau = -z / dz
            x = x + tau * dx
            y = y + tau * dy
            z = np.zeros(n)
            if surf.kind == SPHERE:
                c = surf.c
                F = c * (x * x + y * y)
                G = dz - c * (x * dx + y * dy)
                disc = G * G - c * F
                status[(disc < 0.0) & (status == ALIVE)] = MISS
                delta = F / (G + np.sqrt(np.maximum(disc, 0.0)))
                x = x + delta * dx
                y = y + delta * dy
                z = delta * dz
            elif surf.kind == ASPHERE:
                steps = [] if log is not None else None
                delta, x, y = _intersect_asphere(surf, x, y, dx, dy, dz, status, steps)
                if log is not None:
                    log.setdefault("steps", {})[s] = steps[0]
                z = delta * dz
            r2 = x * x + y * y
            semi = prep.semi[s]
            status[(r2 > semi * semi) & (status == ALIVE)] = CLIP
            if surf.kind == SPHERE:
                N = np.stack([-surf.c * x, -surf.c * y, 1.0 - surf.c * z], axis=1)
                d = _refract(d, N, mu[s], status)
            elif surf.kind == ASPHERE:
                _, dsag, ok = asphere_sag(surf, r2)
                N = np.stack([-2.0 * x * dsag, -2.0 * y * dsag, np.ones(n)], axis=1)
                N /= np.linalg.norm(N, axis=1, keepdims=True)
                d = _refract(d, N, mu[s], status)
            elif surf.kind == PLANE:
                N = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))
                d = _refract(d, N, mu[s], status)
            elif surf.kind == IDEAL:
                tx = d[:, 0] / d[:, 2] - x / surf.focal
                ty = d[:, 1] / d[:, 2] - y / surf.focal
                d = np.stack([tx, ty, np.ones(n)], axis=1)
                d /= np.linalg.norm(d, axis=1, keepdims=True)
            # STOP: aperture only, no refraction
            if record:
                hits[:, s, 0], hits[:, s, 1], hits[:, s, 2] = x, y, z
                hits[:, s, 3:] = d
        z = z - prep.sensor_distance
        dz = d[:, 2]
        status[(dz <= 0.0) & (status == ALIVE)] = INVALID
        tau = -z / dz
        x = x + tau * d[:, 0]
        y = y + tau * d[:, 1]
        bad = ~np.isfinite(x) | ~np.isfinite(y)
        status[bad & (status == ALIVE)] = INVALID
    if record:
        hits[:, S, 0], hits[:, S, 1], hits[:, S, 2] = x, y, 0.0
        hits[:, S, 3:] = d
    return {"O": np.stack([x, y], axis=1), "D": d, "status": status,
            "hits": hits}
