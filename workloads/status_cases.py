"""Rays placed just inside and just outside the failure conditions of a
sequential trace, with the status each must end with.  The geometry of each
case fixes its answer in closed form:

  clip : a ray parallel to the axis keeps its height through a plane or a
         sphere, so it meets the clear semi-diameter rho exactly at height
         rho (kept) and is clipped just above it;
  TIR  : leaving glass of index n into air through a plane, the refracted
         ray exists iff sin(theta) <= 1/n (critical angle);
  miss : a ray parallel to the axis at height h meets a sphere of radius R
         iff h <= |R|;
  conic: an even asphere's sag is defined only while (1+k) c^2 r^2 <= 1, so a
         ray parallel to the axis beyond r = 1/(|c| sqrt(1+k)) has no root;
  invalid: a ray that does not advance along the axis (d_z <= 0);
  first failure: a ray that misses the first surface and would also be
         clipped by a later one keeps the first code.

Inputs only (lenses, rays, expected codes); no trace arithmetic here.
Status codes: 0 alive, 1 miss, 2 clip, 3 total internal reflection,
4 asphere root failure, 5 invalid direction."""

import numpy as np

from workloads.lens import Lens, Surface, STOP, PLANE, SPHERE, ASPHERE, cauchy, air

ALIVE, MISS, CLIP, TIR, NEWTON, INVALID = 0, 1, 2, 3, 4, 5
EPS = 1e-9


def _parallel(heights, z0=-1.0):
    h = np.asarray(heights, dtype=np.float64)
    o = np.stack([np.zeros_like(h), h, np.full_like(h, z0)], 1)
    d = np.tile([0.0, 0.0, 1.0], (len(h), 1))
    return o, d


def clip_case():
    """Stop of radius 2 then a sphere of clear radius 1.5."""
    L = Lens(surfaces=[Surface(kind=STOP, c=0.0, t=2.0, semi_diameter=2.0),
                       Surface(kind=SPHERE, c=1 / 40.0, t=30.0, semi_diameter=1.5,
                               medium=cauchy(1.5, 0.0)),
                       Surface(kind=PLANE, c=0.0, t=20.0, semi_diameter=10.0, medium=air())],
             stop=0)
    h = [0.0, 1.5, np.nextafter(1.5, 2.0), 1.5 * (1 + EPS), 2.0, np.nextafter(2.0, 3.0),
         -2.0 * (1 + EPS)]
    o, d = _parallel(h)
    expect = [ALIVE, ALIVE, CLIP, CLIP, CLIP, CLIP, CLIP]
    return L, o, d, np.array(expect)


def tir_case(n=1.5):
    """Object space of glass (index n), a plane exit into air."""
    L = Lens(surfaces=[Surface(kind=STOP, c=0.0, t=1.0, semi_diameter=100.0,
                               medium=cauchy(n, 0.0)),
                       Surface(kind=PLANE, c=0.0, t=5.0, semi_diameter=100.0, medium=air())],
             stop=0, object_medium=cauchy(n, 0.0))
    sc = 1.0 / n
    s = np.array([0.0, 0.3, sc * (1 - EPS), sc * (1 + EPS), 0.9])
    o = np.zeros((len(s), 3))
    o[:, 2] = -1.0
    d = np.stack([s, np.zeros_like(s), np.sqrt(1 - s * s)], 1)
    return L, o, d, np.array([ALIVE, ALIVE, ALIVE, TIR, TIR])


def miss_case(R=10.0):
    """A convex sphere of radius R (clear radius 2R) into glass."""
    L = Lens(surfaces=[Surface(kind=STOP, c=0.0, t=1.0, semi_diameter=100.0),
                       Surface(kind=SPHERE, c=1 / R, t=40.0, semi_diameter=2 * R,
                               medium=cauchy(1.5, 0.0))], stop=0)
    h = [0.0, 0.5 * R, R * (1 - EPS), R * (1 + EPS), -R * (1 + EPS), 1.5 * R]
    o, d = _parallel(h)
    return L, o, d, np.array([ALIVE, ALIVE, ALIVE, MISS, MISS, MISS])


def conic_case(c=0.1, k=0.25):
    """An even asphere (conic k, small a4) whose sag ends at r = 1/(c sqrt(1+k)),
    with its clear aperture just inside that radius (a prescription whose sag
    is undefined inside its clear aperture is invalid): rays beyond it fail
    the root search before the clip test."""
    r_end = 1.0 / (c * np.sqrt(1.0 + k))
    L = Lens(surfaces=[Surface(kind=STOP, c=0.0, t=1.0, semi_diameter=100.0),
                       Surface(kind=ASPHERE, c=c, t=40.0, semi_diameter=0.999 * r_end,
                               medium=cauchy(1.5, 0.0), conic=k,
                               asph=(1e-6, 0.0, 0.0, 0.0, 0.0))], stop=0)
    h = [0.0, 0.5 * r_end, 0.9 * r_end, 1.05 * r_end, 1.5 * r_end]
    o, d = _parallel(h)
    return L, o, d, np.array([ALIVE, ALIVE, ALIVE, NEWTON, NEWTON])


def invalid_case():
    L = Lens(surfaces=[Surface(kind=STOP, c=0.0, t=1.0, semi_diameter=100.0),
                       Surface(kind=PLANE, c=0.0, t=5.0, semi_diameter=100.0)], stop=0)
    o = np.array([[0.0, 0.0, -1.0]] * 3)
    d = np.array([[0.0, 1.0, 0.0], [0.0, 0.6, -0.8], [0.0, 0.6, 0.8]])
    return L, o, d, np.array([INVALID, INVALID, ALIVE])


def first_failure_case():
    """A sphere of radius 5 then a stop of radius 1: the edge ray misses the
    sphere first."""
    L = Lens(surfaces=[Surface(kind=SPHERE, c=1 / 5.0, t=8.0, semi_diameter=20.0,
                               medium=cauchy(1.5, 0.0)),
                       Surface(kind=STOP, c=0.0, t=10.0, semi_diameter=1.0,
                               medium=cauchy(1.5, 0.0))], stop=1)
    o, d = _parallel([0.0, 4.0, 6.0])
    return L, o, d, np.array([ALIVE, CLIP, MISS])


CASES = {"clip": clip_case, "tir": tir_case, "miss": miss_case, "conic": conic_case,
         "invalid": invalid_case, "first_failure": first_failure_case}
