"""Closed-form pins of the oracle trace's failure rules (CPU only): rays
just inside and just outside the clear semi-diameter, the critical angle,
the sphere's edge and the asphere's conic domain end with the status their
geometry fixes (workloads/status_cases.py states each case)."""
import numpy as np
import pytest

from workloads import status_cases as sc
from oracle import optics, trace as tr


@pytest.mark.parametrize("name", sorted(sc.CASES))
def test_failure_status_at_its_closed_form_boundary(name):
    L, o, d, expect = sc.CASES[name]()
    res = tr.trace(optics.Prepared(L), 0.55, o, d)
    assert np.array_equal(res["status"], expect), (res["status"], expect)


def test_refraction_below_the_critical_angle_is_snell():
    # the surviving rays of the TIR case leave with sin(theta') = n sin(theta)
    n = 1.5
    L, o, d, expect = sc.tir_case(n)
    res = tr.trace(optics.Prepared(L), 0.55, o, d)
    alive = expect == sc.ALIVE
    assert np.allclose(res["D"][alive, 0], n * d[alive, 0], rtol=1e-14, atol=0)
    assert np.allclose(res["D"][alive, 2], np.sqrt(1 - (n * d[alive, 0]) ** 2),
                       rtol=1e-6, atol=1e-12)


def test_edge_ray_of_the_sphere_meets_it_at_the_equator():
    # a parallel ray just inside |R| hits close to z = R (local frame)
    R = 10.0
    L, o, d, expect = sc.miss_case(R)
    res = tr.trace(optics.Prepared(L), 0.55, o, d, record=True)
    k = 2                                       # h = R (1 - 1e-9)
    z = res["hits"][k, 1, 2]
    # z = R - sqrt(R^2 - h^2), sqrt(R^2 - h^2) = R sqrt(2e-9) to first order
    assert z == pytest.approx(R - R * np.sqrt(2e-9), rel=1e-6)
