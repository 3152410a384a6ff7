"""Oracle: entrance-pupil sampling (float64, jitter hash in uint32).
Test infrastructure only.

Sec. 3.1 builds a set of n rays from the object point p toward n points
sampled densely on the entrance pupil, each ray carrying unit energy (the
unit impulse of Eq. (3)).  The paper does not say how the pupil is sampled;
the reading here is a stratified (jittered) n_x x n_y grid on the square
[-1, 1]^2 carried onto the unit disk by the Shirley-Chiu concentric map
(area preserving, so every ray represents the same pupil area), then scaled
to the pupil radius.

The jitter is a counter-based hash: the finaliser of MurmurHash3 (fmix32,
A. Appleby, public domain) chained over (seed, point, ray, dimension):
    k1 = fmix32(seed ^ 0x9E3779B9)
    k2 = fmix32(k1 ^ point)
    h  = fmix32(k2 ^ (2 * ray + dim))
    xi = (h >> 8) * 2^-24            in [0, 1)
"""

import numpy as np

M32 = np.uint64(0xFFFFFFFF)


def fmix32(h):
    """MurmurHash3 32-bit finaliser on uint32 arrays (computed in uint64 and
    masked, so overflow wraps exactly as in 32-bit unsigned arithmetic)."""
    h = np.asarray(h, dtype=np.uint64) & M32
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & M32
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & M32
    h ^= h >> np.uint64(16)
    return h


def point_key(seed, point):
    k1 = fmix32(np.uint64(seed) ^ np.uint64(0x9E3779B9))
    return fmix32(k1 ^ np.uint64(point))


def jitter(seed, point, ray, dim):
    """Uniform numbers in [0, 1) with 24 random bits."""
    k2 = point_key(seed, point)
    h = fmix32(k2 ^ (np.uint64(2) * np.asarray(ray, dtype=np.uint64) + np.uint64(dim)))
    return (h >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def square_samples(nx, ny, seed, point, jittered=True):
    """Stratified samples (a, b) in [-1, 1]^2 for rays r = 0 .. nx*ny-1:
    cell column i = r mod nx, row j = r div nx."""
    r = np.arange(nx * ny, dtype=np.int64)
    i = (r % nx).astype(np.float64)
    j = (r // nx).astype(np.float64)
    if jittered:
        x1 = jitter(seed, point, r, 0)
        x2 = jitter(seed, point, r, 1)
    else:
        x1 = np.full(r.shape, 0.5)
        x2 = np.full(r.shape, 0.5)
    a = -1.0 + 2.0 * (i + x1) / nx
    b = -1.0 + 2.0 * (j + x2) / ny
    return a, b


def concentric_disk(a, b):
    """Shirley-Chiu concentric map of the square [-1,1]^2 onto the unit disk,
    written so that it commutes exactly with a -> -a and b -> -b:
      |a| > |b|:  phi = (pi/4) b/a,  (u, v) = (a cos phi, a sin phi)
      otherwise:  phi = (pi/4) a/b,  (u, v) = (b sin phi, b cos phi)
    and (0, 0) -> (0, 0)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    u = np.zeros_like(a)
    v = np.zeros_like(a)
    m1 = np.abs(a) > np.abs(b)
    m2 = (~m1) & (b != 0)
    phi1 = (np.pi / 4.0) * b[m1] / a[m1]
    u[m1] = a[m1] * np.cos(phi1)
    v[m1] = a[m1] * np.sin(phi1)
    phi2 = (np.pi / 4.0) * a[m2] / b[m2]
    u[m2] = b[m2] * np.sin(phi2)
    v[m2] = b[m2] * np.cos(phi2)
    return u, v


def pupil_rays(p, z_ep, rho_ep, nx, ny, seed, point, jittered=True):
    """Ray bundle from object point p toward the entrance pupil samples.
    Returns origins on the pupil plane (n, 3) and unit directions (n, 3).
    The ray is the line through p and the pupil sample; starting it on the
    pupil plane is the same ray."""
    a, b = square_samples(nx, ny, seed, point, jittered)
    u, v = concentric_disk(a, b)
    e = np.stack([rho_ep * u, rho_ep * v, np.full(u.shape, z_ep)], axis=1)
    d = e - np.asarray(p, dtype=np.float64)[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return e, d
