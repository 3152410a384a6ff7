"""Oracle: materials, paraxial optics, entrance pupil, focus and object
points (float64).  Test infrastructure only.

The paper fixes the lens by its prescription table (Table S1 / S2 columns:
radius, thickness, n/V of the following medium, clear diameter, conic,
a4..a12), traces rays from an object point toward samples of the entrance
pupil, the image of the aperture stop in object space (Sec. 3.1), and uses
a focus distance and an F-number (Sec. 5.1).  It is silent on how the
pupil, the focus and the object point of a field are found; the readings
below are the standard first-order (paraxial) ones:

  * n/V -> Cauchy n(lam) = A + B/lam^2 through the d, F and C lines;
  * the entrance pupil is the paraxial image of the stop through the
    surfaces before it;
  * an F-number rescales the stop so that the pupil diameter is EFL/N;
  * focus moves the sensor to the paraxial image of an on-axis point;
  * a field is an image-plane point h; its object point at depth d is
    h / m(d), with m(d) the chief-ray magnification onto the sensor plane.
"""

import numpy as np

from workloads.lens import (SPHERE, PLANE, STOP, ASPHERE, IDEAL, MAT_ABBE,
                            MAT_CAUCHY)

LAMBDA_F = 0.4861327   # um, hydrogen F line
LAMBDA_D = 0.5875618   # um, helium d line
LAMBDA_C = 0.6562725   # um, hydrogen C line


def cauchy_from_abbe(nd, vd):
    """Two-term Cauchy coefficients that reproduce n_d at the d line and the
    principal dispersion n_F - n_C = (n_d - 1)/V_d."""
    b = (nd - 1.0) / (vd * (LAMBDA_F ** -2 - LAMBDA_C ** -2))
    a = nd - b / LAMBDA_D ** 2
    return a, b


def index_of(medium, lam):
    kind, p0, p1 = medium
    if kind == MAT_ABBE:
        a, b = cauchy_from_abbe(p0, p1)
    elif kind == MAT_CAUCHY:
        a, b = p0, p1
    else:
        raise ValueError("unknown material kind %r" % (kind,))
    return a + b / lam ** 2


def indices(lens, lam):
    """n[0] = object medium; n[s+1] = medium after surface s."""
    n = [index_of(lens.object_medium, lam)]
    for s in lens.surfaces:
        n.append(index_of(s.medium, lam))
    return np.array(n, dtype=np.float64)


def surface_power(surf, n_before, n_after):
    """Paraxial power of one surface (1/mm)."""
    if surf.kind in (SPHERE, ASPHERE):
        return (n_after - n_before) * surf.c
    if surf.kind == IDEAL:
        return 1.0 / surf.focal
    return 0.0


def refraction_matrix(phi):
    return np.array([[1.0, 0.0], [-phi, 1.0]])


def transfer_matrix(t, n):
    return np.array([[1.0, t / n], [0.0, 1.0]])


def system_matrix(lens, lam, upto, thicknesses=None):
    """2x2 matrix acting on (y, n*u) from the vertex plane of surface 0
    (object side, before any refraction) to the vertex plane of surface
    `upto`, before its refraction.  `upto == len(surfaces)` means the sensor
    plane, using the last thickness (or `thicknesses[-1]`)."""
    n = indices(lens, lam)
    t = [s.t for s in lens.surfaces] if thicknesses is None else thicknesses
    M = np.eye(2)
    for s in range(upto):
        surf = lens.surfaces[s]
        M = refraction_matrix(surface_power(surf, n[s], n[s + 1])) @ M
        M = transfer_matrix(t[s], n[s + 1]) @ M
    return M


def after_last_matrix(lens, lam):
    """Matrix from the vertex plane of surface 0 to just after the last
    surface's refraction (still in its vertex plane)."""
    n = indices(lens, lam)
    M = np.eye(2)
    S = len(lens.surfaces)
    for s in range(S):
        surf = lens.surfaces[s]
        M = refraction_matrix(surface_power(surf, n[s], n[s + 1])) @ M
        if s < S - 1:
            M = transfer_matrix(surf.t, n[s + 1]) @ M
    return M


def efl(lens, lam):
    """Effective focal length n'/Phi with Phi = -C of the vertex-to-vertex
    system matrix."""
    M = after_last_matrix(lens, lam)
    n_img = indices(lens, lam)[-1]
    if M[1, 0] == 0.0:
        return np.inf                      # afocal (no power)
    return -n_img / M[1, 0]


def image_distance(lens, lam, depth):
    """Distance from the last vertex to the paraxial image of the on-axis
    point at `depth` (mm before vertex 1; np.inf for infinity)."""
    M = after_last_matrix(lens, lam)
    n = indices(lens, lam)
    if np.isinf(depth):
        y, w = M @ np.array([1.0, 0.0])
    else:
        y, w = M @ np.array([depth, n[0]])     # slope 1 from (0, -depth)
    return -y * n[-1] / w


def bfd(lens, lam):
    return image_distance(lens, lam, np.inf)


def entrance_pupil(lens, lam, stop_radius=None):
    """(z_EP, rho_EP): the paraxial image of the stop in object space.
    With [[A, B], [C, D]] the matrix from vertex plane 0 to the stop plane, a
    ray from the axial point z_EP reaches the stop centre iff
    z_EP = B n_0 / A, and the pupil magnification is A."""
    M = system_matrix(lens, lam, lens.stop)
    n0 = indices(lens, lam)[0]
    A, B = M[0, 0], M[0, 1]
    rs = lens.surfaces[lens.stop].semi_diameter if stop_radius is None else stop_radius
    return B * n0 / A, rs / abs(A)


class Prepared:
    """Per-lens first-order data at the reference wavelength, plus the
    resolved stop radius and sensor distance; mirrors what a consumer must
    fix before tracing (stop size, sensor position)."""

    def __init__(self, lens):
        lr = lens.ref_wavelength
        self.lens = lens
        self.S = len(lens.surfaces)
        self.efl = efl(lens, lr)
        M = system_matrix(lens, lr, lens.stop)
        A = M[0, 0]
        if lens.f_number > 0:
            rho_ep = self.efl / (2.0 * lens.f_number)
            self.stop_radius = rho_ep * abs(A)
        else:
            self.stop_radius = lens.surfaces[lens.stop].semi_diameter
        if lens.focus_depth > 0:
            self.sensor_distance = image_distance(lens, lr, lens.focus_depth)
        else:
            self.sensor_distance = lens.surfaces[-1].t
        self.thickness = np.array([s.t for s in lens.surfaces], dtype=np.float64)
        self.thickness[-1] = self.sensor_distance
        self.vertex_z = np.concatenate([[0.0], np.cumsum(self.thickness[:-1])])
        self.sensor_z = self.vertex_z[-1] + self.sensor_distance
        self.semi = np.array([s.semi_diameter for s in lens.surfaces])
        self.semi[lens.stop] = self.stop_radius
        # chief-ray magnification constants at the reference wavelength
        z_ep, _ = entrance_pupil(lens, lr, self.stop_radius)
        Ms = system_matrix(lens, lr, self.S, self.thickness)
        n0 = indices(lens, lr)[0]
        self.z_ep_ref = z_ep
        self._m_num = Ms[0, 0] * z_ep - Ms[0, 1] * n0

    def pupil(self, lam):
        return entrance_pupil(self.lens, lam, self.stop_radius)

    def magnification(self, depth):
        """Chief-ray (aimed at the pupil centre) magnification from the plane
        at `depth` onto the sensor plane."""
        return self._m_num / (self.z_ep_ref + depth)

    def object_point(self, field, depth):
        m = self.magnification(depth)
        return np.array([field[0] / m, field[1] / m, -depth])

    def mu(self, lam):
        """Index ratios n_before / n_after for every surface."""
        n = indices(self.lens, lam)
        return n[:-1] / n[1:]
