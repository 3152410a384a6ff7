"""Lens prescriptions: the two tables printed in the supplement, the test
lenses used by the oracle pins, and seeded generators for synthetic lenses.

Everything here is data.  Paraxial quantities (focal length, pupils, focus)
are computed by the consumers, never here.
"""

import numpy as np

from .lens import (Surface, Lens, SPHERE, PLANE, STOP, ASPHERE, IDEAL, air,
                   abbe, cauchy)


def _row(kind, radius, t, mat, diameter, asph=(0, 0, 0, 0, 0), conic=0.0):
    c = 0.0 if (radius is None or radius == 0) else 1.0 / radius
    return Surface(kind=kind, c=c, t=t, semi_diameter=diameter / 2.0,
                   medium=mat if mat is not None else air(), conic=conic,
                   asph=tuple(float(a) for a in asph))


def rf50():
    """Canon RF50mm F/1.8, Table S1 of the supplement (reference lens).

    Row order, radius, thickness, n_d/V_d of the following medium, clear
    diameter and the a4..a12 coefficients of surfaces 9 and 10 as printed.
    The last thickness (25.67 mm) is the infinity-focus sensor distance.
    """
    S = [
        _row(SPHERE, 28.621, 4.20, abbe(1.83481, 42.7), 29.99),
        _row(SPHERE, 68.136, 0.18, None, 28.48),
        _row(SPHERE, 17.772, 6.70, abbe(1.79952, 42.2), 23.90),
        _row(SPHERE, 59.525, 1.10, abbe(1.80518, 25.4), 20.78),
        _row(SPHERE, 11.427, 5.27, None, 16.78),
        _row(STOP, None, 6.20, None, 16.24),
        _row(SPHERE, -16.726, 0.90, abbe(1.67270, 32.1), 14.95),
        _row(SPHERE, -29.829, 0.83, None, 15.46),
        _row(ASPHERE, -25.000, 2.95, abbe(1.53110, 55.9), 15.52,
             asph=(-4.12032e-05, -2.90015e-07, -4.67119e-09, 7.90646e-11,
                   -9.28470e-13)),
        _row(ASPHERE, -18.373, 0.98, None, 18.14,
             asph=(-2.41619e-05, -3.29146e-07, 1.91098e-10, -9.28593e-13,
                   -2.29193e-13)),
        _row(SPHERE, 280.004, 4.60, abbe(1.73400, 51.5), 24.43),
        _row(SPHERE, -34.002, 25.67, None, 25.71),
    ]
    return Lens(surfaces=S, stop=5, name="RF50 (Table S1)")


def rf35():
    """Canon RF35mm F/1.8, Table S2 of the supplement (isolation lens)."""
    S = [
        _row(SPHERE, 800.000, 1.00, abbe(1.80810, 22.8), 27.80),
        _row(SPHERE, 33.296, 1.92, None, 25.64),
        _row(SPHERE, 103.801, 3.11, abbe(2.00100, 29.1), 25.57),
        _row(SPHERE, -86.901, 4.09, None, 25.07),
        _row(SPHERE, -47.674, 1.30, abbe(1.51742, 52.4), 20.44),
        _row(SPHERE, 17.367, 5.73, abbe(1.90043, 37.4), 21.60),
        _row(SPHERE, 777.674, 3.72, None, 21.26),
        _row(STOP, None, 3.62, None, 20.16),
        _row(SPHERE, 64.497, 2.12, abbe(1.69680, 55.5), 19.04),
        _row(SPHERE, -262.934, 3.56, None, 18.69),
        _row(ASPHERE, -35.963, 1.30, abbe(1.58313, 59.4), 17.10,
             asph=(-4.61997e-05, -9.22837e-08, -4.60687e-10, 1.65555e-13, 0)),
        _row(SPHERE, -93.550, 0.13, None, 17.19),
        _row(SPHERE, -84.988, 6.26, abbe(1.88300, 40.8), 17.29),
        _row(SPHERE, -12.701, 1.00, abbe(1.85478, 24.8), 18.97),
        _row(SPHERE, 135.000, 5.27, None, 22.77),
        _row(SPHERE, 800.000, 7.35, abbe(1.90043, 37.4), 31.72),
        _row(SPHERE, -28.799, 0.95, None, 33.14),
        _row(SPHERE, -109.518, 2.86, abbe(1.69680, 55.5), 34.06),
        _row(SPHERE, -53.092, 11.79, None, 34.38),
        _row(SPHERE, -29.766, 1.70, abbe(1.59270, 35.3), 33.78),
        _row(SPHERE, -114.300, 11.66, None, 36.27),
    ]
    return Lens(surfaces=S, stop=7, name="RF35 (Table S2)")


def singlet(focus_depth=2000.0, f_number=2.0, n=1.5168):
    """Equi-convex singlet R1 = +51.5 mm, R2 = -51.5 mm, 5 mm thick, constant
    index, with the aperture stop in the vertex plane of surface 1."""
    S = [
        Surface(kind=STOP, c=0.0, t=0.0, semi_diameter=12.5),
        Surface(kind=SPHERE, c=1.0 / 51.5, t=5.0, semi_diameter=15.0,
                medium=cauchy(n, 0.0)),
        Surface(kind=SPHERE, c=-1.0 / 51.5, t=50.0, semi_diameter=15.0),
    ]
    return Lens(surfaces=S, stop=0, f_number=f_number, focus_depth=focus_depth,
                name="singlet R=+-51.5 t=5")


def ideal(f=50.0, stop_radius=12.5, sensor=50.0, focus_depth=0.0,
          f_number=0.0):
    """Aberration-free test lens: one IDEAL surface (a paraxial thin lens that
    bends every ray exactly by its paraxial rule) with the stop in its plane."""
    S = [
        Surface(kind=STOP, c=0.0, t=0.0, semi_diameter=stop_radius),
        Surface(kind=IDEAL, c=0.0, t=sensor, semi_diameter=1e3, focal=f),
    ]
    return Lens(surfaces=S, stop=0, f_number=f_number,
                focus_depth=focus_depth, name="ideal f=%g" % f)


def plate(thickness=5.0, n=1.5, sensor=10.0, stop_radius=5.0):
    """Plane-parallel plate behind a stop (no focusing power)."""
    S = [
        Surface(kind=STOP, c=0.0, t=2.0, semi_diameter=stop_radius),
        Surface(kind=PLANE, c=0.0, t=thickness, semi_diameter=50.0,
                medium=cauchy(n, 0.0)),
        Surface(kind=PLANE, c=0.0, t=sensor, semi_diameter=50.0),
    ]
    return Lens(surfaces=S, stop=0, name="plate")


# Cauchy coefficients (A, B; B in um^2) of the six RF50 glasses, converted
# once from the printed n_d/V_d by the d/F/C-line rule.  A non-GPU test checks
# these literals against the oracle's conversion of Table S1.
RF50_CAUCHY = {
    (1.83481, 42.7): (1.8051545406110556, 0.010237920699160174),
    (1.79952, 42.2): (1.770781653986178, 0.009921306686087651),
    (1.80518, 25.4): (1.757095605617708, 0.016600121080456897),
    (1.67270, 32.1): (1.6409121405888856, 0.010974086746684115),
    (1.53110, 55.9): (1.5166884935038145, 0.00497526808565919),
    (1.73400, 51.5): (1.712381093702121, 0.007463470566325907),
}


def double_gauss_12(seed=0):
    """Seeded 6-element, 12-surface spherical lens around an f = 50 mm design.

    Recipe: Table S1 with the two aspheres made spherical and the cemented
    surface 4 split into two surfaces 0.05 mm apart (glass / air / glass),
    giving six separate elements; then every radius is scaled by a uniform
    factor in [0.98, 1.02], every thickness by [0.95, 1.05] and each glass's
    Cauchy A and B by [0.99, 1.01], all drawn from one seeded generator.
    The stop is resized to f/2 and the sensor focused by the consumer.
    """
    rng = np.random.default_rng(seed)
    base = rf50().surfaces
    rows = []
    for i, s in enumerate(base):
        s = Surface(kind=SPHERE if s.kind == ASPHERE else s.kind, c=s.c,
                    t=s.t, semi_diameter=s.semi_diameter, medium=s.medium)
        if i == 3:
            # Split the cemented interface: glass(1.79952) | 0.05 air | glass.
            rows.append(Surface(kind=SPHERE, c=s.c, t=0.05,
                                semi_diameter=s.semi_diameter, medium=air()))
            rows.append(s)
        else:
            rows.append(s)
    out = []
    for s in rows:
        kind, c, t, sd, med = s.kind, s.c, s.t, s.semi_diameter, s.medium
        if kind == SPHERE:
            c = c / rng.uniform(0.98, 1.02)
        t = t * rng.uniform(0.95, 1.05)
        if med[0] == 1:     # abbe -> literal Cauchy of the base glass
            a0, b0 = RF50_CAUCHY[(med[1], med[2])]
            med = cauchy(a0 * rng.uniform(0.99, 1.01),
                         b0 * rng.uniform(0.99, 1.01))
        out.append(Surface(kind=kind, c=c, t=t, semi_diameter=sd, medium=med))
    return Lens(surfaces=out, stop=6, f_number=2.0, name="dgauss12 seed=%d" % seed)


# Paraxial focal length of the unscaled 16-surface design below is
# 51.99701660498591 mm at 0.55 um (asphere terms do not change it); the
# literal scale brings it to 4.3 mm.  A non-GPU test checks the result.
PHONE16_SCALE = 4.3 / 51.99701660498591


def phone_lens_16(seed=0, aperture_scale=1.3):
    """Seeded smartphone-like lens: 8 elements, 16 refracting surfaces, even
    aspheres up to r^10, EFL 4.3 mm, f/1.8.

    Recipe: the six elements of Table S1 (cemented surface 4 split by a
    0.05 mm air gap; the a12 terms of surfaces 9 and 10 dropped), followed by
    two weak plastic menisci (Cauchy 1.4905/0.0047 and 1.5700/0.0100) whose
    four surfaces carry seeded a4..a10 (|a4| <= 3e-7, |a6| <= 1e-9,
    |a8| <= 5e-12, |a10| <= 2e-14 in the unscaled millimetre units: at most
    ~12 um of sag at 12 mm); clear semi-diameters enlarged by
    `aperture_scale` (capped at 0.9 |R|) to pass the wider sensor diagonal;
    then every length scaled by PHONE16_SCALE.  The stop is resized to f/1.8
    and the sensor focused by the consumer.
    """
    import copy
    rng = np.random.default_rng(seed)
    rows = []
    for i, s in enumerate(rf50().surfaces):
        s = copy.deepcopy(s)
        if s.kind == ASPHERE:
            s.asph = tuple(s.asph[:4]) + (0.0,)
        if i == 3:
            gap = copy.deepcopy(s)
            gap.medium = air()
            gap.t = 0.05
            rows.append(gap)
        rows.append(s)
    rows[-1].t = 2.0

    def asph():
        return (rng.uniform(-3e-7, 3e-7), rng.uniform(-1e-9, 1e-9),
                rng.uniform(-5e-12, 5e-12), rng.uniform(-2e-14, 2e-14), 0.0)

    rows.append(Surface(kind=ASPHERE, c=-1 / 40.0, t=1.0, semi_diameter=13.5,
                        medium=cauchy(1.4905, 0.0047), asph=asph()))
    rows.append(Surface(kind=ASPHERE, c=-1 / 45.0, t=1.0, semi_diameter=14.0, asph=asph()))
    rows.append(Surface(kind=ASPHERE, c=1 / 100.0, t=1.0, semi_diameter=14.5,
                        medium=cauchy(1.5700, 0.0100), asph=asph()))
    rows.append(Surface(kind=ASPHERE, c=1 / 90.0, t=10.0, semi_diameter=14.5, asph=asph()))
    k = PHONE16_SCALE
    out = []
    for s in rows:
        sd = s.semi_diameter
        if s.kind != STOP:
            sd = aperture_scale * sd
            if s.c != 0:
                sd = min(sd, 0.9 / abs(s.c))
        out.append(Surface(kind=s.kind, c=s.c / k, t=s.t * k, semi_diameter=sd * k,
                           medium=s.medium, conic=s.conic,
                           asph=tuple(a / k ** (2 * m + 3) for m, a in enumerate(s.asph))))
    return Lens(surfaces=out, stop=6, f_number=1.8, name="phone16 seed=%d" % seed)
