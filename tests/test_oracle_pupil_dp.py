"""Pins of the oracle's pupil sampling and dual-pixel split (CPU only)."""
import numpy as np
import pytest

from oracle import pupil, dp


def test_fmix32_is_a_bijection_on_a_block():
    x = np.arange(1 << 20, dtype=np.uint64)
    h = pupil.fmix32(x)
    assert len(np.unique(h)) == len(x)
    assert np.all(h < (1 << 32))


def test_fmix32_matches_integer_reference():
    # plain Python integers, 32-bit wrap written out
    def ref(h):
        h ^= h >> 16
        h = (h * 0x85EBCA6B) & 0xFFFFFFFF
        h ^= h >> 13
        h = (h * 0xC2B2AE35) & 0xFFFFFFFF
        h ^= h >> 16
        return h
    xs = [0, 1, 2, 0xDEADBEEF, 0xFFFFFFFF, 123456789]
    assert [int(v) for v in pupil.fmix32(np.array(xs, dtype=np.uint64))] == [ref(x) for x in xs]


def test_jitter_is_uniform():
    u = np.concatenate([pupil.jitter(0, q, np.arange(20000), dim) for q in range(5) for dim in (0, 1)])
    assert u.min() >= 0.0 and u.max() < 1.0
    hist, _ = np.histogram(u, bins=64, range=(0, 1))
    exp = len(u) / 64
    chi2 = np.sum((hist - exp) ** 2 / exp)
    assert chi2 < 120        # 63 dof, p ~ 1e-5
    assert abs(u.mean() - 0.5) < 5e-3


def test_concentric_map_matches_textbook_form_and_bounds():
    rng = np.random.default_rng(0)
    a = rng.uniform(-1, 1, 100000)
    b = rng.uniform(-1, 1, 100000)
    u, v = pupil.concentric_disk(a, b)
    # textbook form: r = a, phi = pi/4 b/a  or  r = b, phi = pi/2 - pi/4 a/b
    m = np.abs(a) > np.abs(b)
    r = np.where(m, a, b)
    phi = np.where(m, np.pi / 4 * b / a, np.pi / 2 - np.pi / 4 * a / b)
    assert np.allclose(u, r * np.cos(phi), atol=1e-14)
    assert np.allclose(v, r * np.sin(phi), atol=1e-14)
    assert np.all(u * u + v * v <= 1.0 + 1e-15)


def test_concentric_map_preserves_area_and_mirrors_exactly():
    a, b = pupil.square_samples(256, 256, 0, 0, jittered=False)
    u, v = pupil.concentric_disk(a, b)
    assert np.mean(u * u + v * v) == pytest.approx(0.5, abs=2e-5)
    u2, v2 = pupil.concentric_disk(-a, b)
    assert np.array_equal(u2, -u) and np.array_equal(v2, v)
    u3, v3 = pupil.concentric_disk(a, -b)
    assert np.array_equal(u3, u) and np.array_equal(v3, -v)
    # every ray of a jittered grid lies in its own cell
    a, b = pupil.square_samples(64, 32, 5, 3, jittered=True)
    r = np.arange(64 * 32)
    assert np.all(np.floor((a + 1) / 2 * 64) == r % 64)
    assert np.all(np.floor((b + 1) / 2 * 32) == r // 64)


def test_microlens_rule_equals_micro_trace():
    rng = np.random.default_rng(0)
    ps = 0.005
    n = 1_000_000
    xc, yc = 0.0, 0.0
    xk = rng.uniform(-0.5 * ps, 0.5 * ps, n)
    yk = rng.uniform(-0.5 * ps, 0.5 * ps, n)
    t = rng.uniform(-0.6, 0.6, n)
    s1 = dp.microlens_side(xk, yk, xc, yc, t, ps)
    s2 = dp.microlens_side_by_microtrace(xk, yk, xc, yc, t, ps)
    assert np.count_nonzero(s1 != s2) <= 5      # only exact-boundary rounding
    assert np.count_nonzero(s1 == dp.LEFT) > 0 and np.count_nonzero(s1 == dp.RIGHT) > 0


def test_microlens_interval_width_and_zero_depth():
    ps = 1.0
    h, f, w = 0.78, 1.44, 0.30
    xk = np.linspace(-2, 2, 400001)
    side = dp.microlens_side(xk, np.zeros_like(xk), 0.0, 0.0, np.full_like(xk, 0.1), ps)
    inside = np.abs(xk) <= 0.5
    dx = xk[1] - xk[0]
    width_L = np.count_nonzero((side == dp.LEFT) & inside) * dx
    assert width_L == pytest.approx(w * f / (f - h), abs=2 * dx)   # 0.6545 ps
    assert w * f / (f - h) == pytest.approx(0.6545, abs=1e-4)
    # h -> 0: the split depends on position only
    t = np.random.default_rng(1).uniform(-1, 1, xk.size)
    s0 = dp.microlens_side(xk, np.zeros_like(xk), 0.0, 0.0, t, ps, h=0.0)
    assert np.all(s0[(xk >= 0) & (xk < w)] == dp.LEFT)
    assert np.all(s0[(xk >= -w) & (xk < 0)] == dp.RIGHT)
    assert np.all(s0[(xk >= w) | (xk < -w)] == dp.MISSED)


def test_sigmoid_limits():
    rng = np.random.default_rng(0)
    D = rng.normal(size=(1000, 3))
    D[:, 2] = np.abs(D[:, 2]) + 0.1
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    wl, wr = dp.sigmoid_weights(D, 0.0)
    assert np.all(wl == 0.5) and np.all(wr == 0.5)
    wl, wr = dp.sigmoid_weights(D, 1e6)
    assert np.array_equal(wl > 0.5, D[:, 0] > 0)
    wl, wr = dp.sigmoid_weights(D, 20.0)
    assert np.allclose(wl + wr, 1.0, atol=1e-15)
