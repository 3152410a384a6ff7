"""Oracle: pixel-wise DP rendering (float64).  Test infrastructure only.

Sec. 3.2 and Supplement S1.3: every output pixel is the all-in-focus image
convolved with that pixel's own left and right PSF (a local, shift-variant
convolution), the image edges are extended by replication, and the output
stacks the left image's C channels before the right image's.  Following the
corrected kernel orientation of S1.3 (the kernel is flipped before the
unfolded patch is weighted), the operation is a true convolution with the
output pixel's kernel:

    out[n, s C + c, y, x] = sum_{i, j} K[n, y, x, c', s, i, j]
                            * img[n, c, clamp(y + pad - i), clamp(x + pad - j)]

with pad = (ks - 1) / 2, s = 0 (left) / 1 (right), clamp to [0, H-1] and
[0, W-1], and c' = c for per-channel kernels or 0 for a kernel shared by
all channels.  No normalisation happens inside.

Kernel sources
  dense : K given per pixel, [N][H][W][Cp][2][ks][ks];
  bank  : K taken from a traced bank [F][Dn][L][2][ks][ks] of PSFs on radial
          fields along +x, per pixel: nearest field radius (compared as the
          exact integer R2 = (2x - W + 1)^2 + (2y - H + 1)^2 in half-pixel
          units against precomputed squared midpoints), nearest inverse
          depth (the float depth compared with the depths of the inverse-
          depth midpoints), channel c -> wavelength slot lam_of_c[c]; pixels
          left of the centre use the mirror image (columns flipped, left and
          right swapped), pixels below it flip rows.  This lookup is an
          approximation for pixels off the x axis (it ignores azimuth).
  bank2d: a first-quadrant 2-D grid with linear interpolation in inverse
          depth (see the section at the end).
"""

import numpy as np


def _shifted(img2d, di, dj):
    """img2d[clamp(y + di), clamp(x + dj)] for every (y, x)."""
    H, W = img2d.shape
    rows = np.clip(np.arange(H) + di, 0, H - 1)
    cols = np.clip(np.arange(W) + dj, 0, W - 1)
    return img2d[rows][:, cols]


def render_dense(img, K):
    """img [N, C, H, W]; K [N, H, W, Cp, 2, ks, ks] -> out [N, 2C, H, W]."""
    img = np.asarray(img, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    N, C, H, W = img.shape
    Cp, ks = K.shape[3], K.shape[-1]
    pad = (ks - 1) // 2
    out = np.zeros((N, 2 * C, H, W))
    for n in range(N):
        for c in range(C):
            cp = c if Cp == C else 0
            for i in range(ks):
                for j in range(ks):
                    src = _shifted(img[n, c], pad - i, pad - j)
                    for s in range(2):
                        out[n, s * C + c] += K[n, :, :, cp, s, i, j] * src
    return out


def render_dense_adjoint(grad_out, K):
    """Transpose of render_dense with respect to the image."""
    g = np.asarray(grad_out, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    N, C2, H, W = g.shape
    C = C2 // 2
    Cp, ks = K.shape[3], K.shape[-1]
    pad = (ks - 1) // 2
    gin = np.zeros((N, C, H, W))
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for n in range(N):
        for c in range(C):
            cp = c if Cp == C else 0
            for i in range(ks):
                rows = np.clip(yy + pad - i, 0, H - 1)
                for j in range(ks):
                    cols = np.clip(xx + pad - j, 0, W - 1)
                    contrib = sum(K[n, :, :, cp, s, i, j] * g[n, s * C + c]
                                  for s in range(2))
                    np.add.at(gin[n, c], (rows, cols), contrib)
    return gin


def render_dense_psf_adjoint(img, grad_out, Cp, ks):
    """Transpose of render_dense with respect to the kernels (the render is
    linear in K): [N, H, W, Cp, 2, ks, ks], kernel channel c' collecting the
    image channels that read it (c' = c per channel, 0 when shared)."""
    img = np.asarray(img, dtype=np.float64)
    g = np.asarray(grad_out, dtype=np.float64)
    N, C, H, W = img.shape
    pad = (ks - 1) // 2
    gK = np.zeros((N, H, W, Cp, 2, ks, ks))
    for n in range(N):
        for c in range(C):
            cp = c if Cp == C else 0
            for i in range(ks):
                for j in range(ks):
                    src = _shifted(img[n, c], pad - i, pad - j)
                    for s in range(2):
                        gK[n, :, :, cp, s, i, j] += g[n, s * C + c] * src
    return gK


def bank_thresholds(field_radii, inv_depths, pitch):
    """Squared-radius thresholds in half-pixel units (floored) and depth
    thresholds for the nearest-entry bank lookup."""
    r = np.asarray(field_radii, dtype=np.float64)
    mid_r = 0.5 * (r[:-1] + r[1:])
    t_r = np.floor((2.0 * mid_r / pitch) ** 2)
    iv = np.asarray(inv_depths, dtype=np.float64)
    mid_iv = 0.5 * (iv[:-1] + iv[1:])
    t_z = 1.0 / mid_iv
    return t_r, t_z


def bank_lookup(H, W, depth, field_radii, inv_depths, pitch):
    """Per pixel: field index, depth index, mirror-x flag, mirror-y flag.
    depth is [H, W] (float32 values, compared exactly in float64)."""
    t_r, t_z = bank_thresholds(field_radii, inv_depths, pitch)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.int64), np.arange(W, dtype=np.int64),
                         indexing="ij")
    X2 = 2 * xx - (W - 1)
    Y2 = 2 * yy - (H - 1)
    R2 = (X2 * X2 + Y2 * Y2).astype(np.float64)
    fi = np.zeros((H, W), dtype=np.int64)
    for t in t_r:
        fi += (R2 > t)
    z = np.asarray(depth, dtype=np.float64)
    di = np.zeros((H, W), dtype=np.int64)
    for t in t_z:
        di += (z < t)
    return fi, di, X2 < 0, Y2 < 0


def dense_from_bank(bank, depth_maps, field_radii, inv_depths, lam_of_c, pitch):
    """Expand a bank [F][Dn][L][2][ks][ks] to the dense per-pixel kernels
    [N][H][W][C][2][ks][ks] chosen by the lookup rule above."""
    bank = np.asarray(bank, dtype=np.float64)
    N, H, W = depth_maps.shape
    C = len(lam_of_c)
    ks = bank.shape[-1]
    K = np.zeros((N, H, W, C, 2, ks, ks))
    for n in range(N):
        fi, di, mx, my = bank_lookup(H, W, depth_maps[n], field_radii, inv_depths, pitch)
        for y in range(H):
            for x in range(W):
                for c in range(C):
                    k = bank[fi[y, x], di[y, x], lam_of_c[c]]
                    if mx[y, x]:
                        k = k[::-1, :, ::-1]     # swap L/R, flip columns
                    if my[y, x]:
                        k = k[:, ::-1, :]        # flip rows
                    K[n, y, x, c] = k
    return K


def render_bank(img, bank, depth_maps, field_radii, inv_depths, lam_of_c, pitch):
    K = dense_from_bank(bank, depth_maps, field_radii, inv_depths, lam_of_c, pitch)
    return render_dense(img, K)


def render_bank_adjoint(grad_out, bank, depth_maps, field_radii, inv_depths,
                        lam_of_c, pitch):
    K = dense_from_bank(bank, depth_maps, field_radii, inv_depths, lam_of_c, pitch)
    return render_dense_adjoint(grad_out, K)


def render_bank_pixels(img, bank, depth_maps, field_radii, inv_depths, lam_of_c,
                       pitch, pixels):
    """The bank-source definition evaluated only at the listed output pixels
    (n, y, x): returns [len(pixels), 2C]."""
    img = np.asarray(img, dtype=np.float64)
    bank = np.asarray(bank, dtype=np.float64)
    N, C, H, W = img.shape
    ks = bank.shape[-1]
    pad = (ks - 1) // 2
    out = np.zeros((len(pixels), 2 * C))
    looked = {}
    for k, (n, y, x) in enumerate(pixels):
        if n not in looked:
            looked[n] = bank_lookup(H, W, depth_maps[n], field_radii, inv_depths, pitch)
        fi, di, mx, my = looked[n]
        rows = np.clip(y + pad - np.arange(ks), 0, H - 1)
        cols = np.clip(x + pad - np.arange(ks), 0, W - 1)
        for c in range(C):
            kern = bank[fi[y, x], di[y, x], lam_of_c[c]]
            if mx[y, x]:
                kern = kern[::-1, :, ::-1]
            if my[y, x]:
                kern = kern[:, ::-1, :]
            patch = img[n, c][rows][:, cols]
            for s in range(2):
                out[k, s * C + c] = np.sum(kern[s] * patch)
    return out


def render_bank_adjoint_pixels(grad_out, bank, depth_maps, field_radii, inv_depths,
                               lam_of_c, pitch, pixels):
    """The image adjoint of the bank render (render_bank_adjoint) evaluated
    only at the listed image pixels (n, y, x): returns [len(pixels), C].
    Image pixel (y, x) collects K[s][i][j] * grad_out[s C + c] of every
    output pixel (y', x') and tap (i, j) with clamp(y' + pad - i) = y and
    clamp(x' + pad - j) = x; those outputs lie within pad of (y, x)."""
    g = np.asarray(grad_out, dtype=np.float64)
    bank = np.asarray(bank, dtype=np.float64)
    N, C2, H, W = g.shape
    C = C2 // 2
    ks = bank.shape[-1]
    pad = (ks - 1) // 2
    taps = np.arange(ks)
    out = np.zeros((len(pixels), C))
    looked = {}
    for k, (n, y, x) in enumerate(pixels):
        if n not in looked:
            looked[n] = bank_lookup(H, W, depth_maps[n], field_radii, inv_depths, pitch)
        fi, di, mx, my = looked[n]
        ys, ii, xs, jj = [], [], [], []
        for yo in range(max(0, y - pad), min(H - 1, y + pad) + 1):
            hit = np.nonzero(np.clip(yo + pad - taps, 0, H - 1) == y)[0]
            ys += [yo] * len(hit)
            ii += list(hit)
        for xo in range(max(0, x - pad), min(W - 1, x + pad) + 1):
            hit = np.nonzero(np.clip(xo + pad - taps, 0, W - 1) == x)[0]
            xs += [xo] * len(hit)
            jj += list(hit)
        yo = np.repeat(np.asarray(ys), len(xs))
        io = np.repeat(np.asarray(ii), len(xs))
        xo = np.tile(np.asarray(xs), len(ys))
        jo = np.tile(np.asarray(jj), len(ys))
        # tap (i, j) of side s of the output pixel's kernel, in the stored
        # entry: rows flipped below the centre, columns flipped and sides
        # swapped left of it
        fy, fx = my[yo, xo], mx[yo, xo]
        si = np.where(fy, ks - 1 - io, io)
        sj = np.where(fx, ks - 1 - jo, jo)
        for c in range(C):
            e = bank[fi[yo, xo], di[yo, xo], lam_of_c[c]]          # [m, 2, ks, ks]
            m = np.arange(len(yo))
            for s in range(2):
                ss = np.where(fx, 1 - s, s)
                out[k, c] += np.sum(e[m, ss, si, sj] * g[n, s * C + c, yo, xo])
    return out


# ---- 2-D (exact-azimuth) bank -------------------------------------------
# A bank traced on a first-quadrant grid (h_x = xs[fx] >= 0, h_y = ys[fy] >= 0)
# is reused in the other quadrants through the flip symmetry of DP PSFs
# about both axes (Sec. 5.1): a pixel takes the grid point nearest to
# (|h_x|, |h_y|), mirrored in columns with the sides swapped when h_x < 0
# and in rows when h_y < 0, and blends the two depth planes that bracket its
# inverse depth linearly.  Readings: h_x of pixel x is (x - (W-1)/2) * pitch;
# the nearest grid point is decided on the exact half-pixel integer
# |2x - (W-1)| against floor(2 * midpoint / pitch); the inverse depth and the
# blend weight are float32 computations (iv = 1/depth, planes as float32),
# d0 = the last plane k <= D-2 with iv_k <= iv (0 if none) and
# w = clamp((iv - iv_d0) / (iv_d0+1 - iv_d0), 0, 1), w = 0 for one plane.

def bank2d_lookup(H, W, depth, xs, ys, inv_depths, pitch):
    """Per pixel: fx, fy, d0, w (float32), mirror-x flag, mirror-y flag."""
    yy, xx = np.meshgrid(np.arange(H, dtype=np.int64), np.arange(W, dtype=np.int64),
                         indexing="ij")
    X2 = 2 * xx - (W - 1)
    Y2 = 2 * yy - (H - 1)
    xs, ys = np.asarray(xs, dtype=np.float64), np.asarray(ys, dtype=np.float64)
    tx = np.floor((xs[:-1] + xs[1:]) / pitch)
    ty = np.floor((ys[:-1] + ys[1:]) / pitch)
    fx = np.zeros((H, W), dtype=np.int64)
    fy = np.zeros((H, W), dtype=np.int64)
    for t in tx:
        fx += np.abs(X2) > t
    for t in ty:
        fy += np.abs(Y2) > t
    ivk = np.asarray(inv_depths, dtype=np.float32)
    D = len(ivk)
    iv = np.float32(1.0) / np.asarray(depth, dtype=np.float32)
    d0 = np.zeros((H, W), dtype=np.int64)
    for k in range(1, D - 1):
        d0 += iv >= ivk[k]
    if D > 1:
        with np.errstate(all="ignore"):
            w = (iv - ivk[d0]) / (ivk[d0 + 1] - ivk[d0])
        w = np.minimum(np.maximum(w, np.float32(0)), np.float32(1)).astype(np.float32)
    else:
        w = np.zeros((H, W), dtype=np.float32)
    return fx, fy, d0, w, X2 < 0, Y2 < 0


def dense_from_bank2d(bank, depth_maps, xs, ys, inv_depths, lam_of_c, pitch):
    """Expand a 2-D bank [Fy][Fx][D][L][2][ks][ks] to dense per-pixel kernels
    [N][H][W][C][2][ks][ks] by the rule above."""
    bank = np.asarray(bank, dtype=np.float64)
    N, H, W = depth_maps.shape
    C = len(lam_of_c)
    ks = bank.shape[-1]
    D = bank.shape[2]
    K = np.zeros((N, H, W, C, 2, ks, ks))
    for n in range(N):
        fx, fy, d0, w, mx, my = bank2d_lookup(H, W, depth_maps[n], xs, ys, inv_depths, pitch)
        for y in range(H):
            for x in range(W):
                wt = float(w[y, x])
                for c in range(C):
                    e = bank[fy[y, x], fx[y, x], :, lam_of_c[c]]
                    k = (1.0 - wt) * e[d0[y, x]]
                    if D > 1:
                        k = k + wt * e[d0[y, x] + 1]
                    if mx[y, x]:
                        k = k[::-1, :, ::-1]     # swap L/R, flip columns
                    if my[y, x]:
                        k = k[:, ::-1, :]        # flip rows
                    K[n, y, x, c] = k
    return K


def render_bank2d(img, bank, depth_maps, xs, ys, inv_depths, lam_of_c, pitch):
    return render_dense(img, dense_from_bank2d(bank, depth_maps, xs, ys, inv_depths,
                                               lam_of_c, pitch))


def render_bank2d_adjoint(grad_out, bank, depth_maps, xs, ys, inv_depths, lam_of_c, pitch):
    return render_dense_adjoint(grad_out, dense_from_bank2d(bank, depth_maps, xs, ys,
                                                            inv_depths, lam_of_c, pitch))


def _bank_scatter(gK, bank_shape, entries):
    """Adjoint of a bank expansion: gK [N][H][W][C][2][ks][ks] per-pixel
    kernel gradients summed back into the bank entries they were read from;
    entries(n) yields, per pixel and channel, (index tuple, weight, mx, my)."""
    out = np.zeros(bank_shape)
    N, H, W, C = gK.shape[:4]
    for n in range(N):
        for (y, x, c, idx, wt, mx, my) in entries(n):
            k = gK[n, y, x, c]
            if my:
                k = k[:, ::-1, :]
            if mx:
                k = k[::-1, :, ::-1]
            out[idx] += wt * k
    return out


def render_bank_psf_adjoint(img, grad_out, bank_shape, depth_maps, field_radii, inv_depths,
                            lam_of_c, pitch):
    """Transpose of render_bank with respect to the bank [F][Dn][L][2][ks][ks]."""
    N, C, H, W = np.asarray(img).shape
    gK = render_dense_psf_adjoint(img, grad_out, C, bank_shape[-1])

    def entries(n):
        fi, di, mx, my = bank_lookup(H, W, depth_maps[n], field_radii, inv_depths, pitch)
        for y in range(H):
            for x in range(W):
                for c in range(C):
                    yield (y, x, c, (fi[y, x], di[y, x], lam_of_c[c]), 1.0, mx[y, x], my[y, x])
    return _bank_scatter(gK, bank_shape, entries)


def render_bank2d_psf_adjoint(img, grad_out, bank_shape, depth_maps, xs, ys, inv_depths,
                              lam_of_c, pitch):
    """Transpose of render_bank2d with respect to the bank [Fy][Fx][D][L][2][ks][ks]."""
    N, C, H, W = np.asarray(img).shape
    D = bank_shape[2]
    gK = render_dense_psf_adjoint(img, grad_out, C, bank_shape[-1])

    def entries(n):
        fx, fy, d0, w, mx, my = bank2d_lookup(H, W, depth_maps[n], xs, ys, inv_depths, pitch)
        for y in range(H):
            for x in range(W):
                wt = float(w[y, x])
                for c in range(C):
                    yield (y, x, c, (fy[y, x], fx[y, x], d0[y, x], lam_of_c[c]), 1.0 - wt,
                           mx[y, x], my[y, x])
                    if D > 1:
                        yield (y, x, c, (fy[y, x], fx[y, x], d0[y, x] + 1, lam_of_c[c]), wt,
                               mx[y, x], my[y, x])
    return _bank_scatter(gK, bank_shape, entries)
