"""Oracle: dual-pixel split of a landed ray (float64).  Test infrastructure.

Microlens model, Sec. 3.1 with the Supplement S1.1 parameters (Eq. (S1):
h = 0.78 ps, f = 1.44 ps, w = 0.30 ps, r = 0.50 ps).  The ray k lands at
x_k inside DP pixel (i, j) with centre x_c and has tan(theta) = D_x / D_z.

  * inside the microlens (distance to the pixel centre <= r, a disk):
    Eq. (1)  x_L1 = x_c + w - (f tan - w) h / (f - h)
             x_M1 = x_c     -  f tan      h / (f - h)
             x_R1 = x_c - w - (f tan + w) h / (f - h)
  * outside it (no refraction), Eq. (2)
             x_L2 = x_c + w - h tan,  x_M2 = x_c - h tan,  x_R2 = x_c - w - h tan

Reading of the garbled interval sentence: the printed intervals are reversed
with respect to Eq. (1), where x_L > x_M > x_R.  The ray enters the left
sub-pixel iff x_M <= x_k < x_L and the right one iff x_R <= x_k < x_M
(half-open, so ties are assigned once), otherwise it is missed.  Tracing the
ray through an ideal thin microlens at the sensor surface down to the
sub-pixel plane at depth h shows this is exactly "lands in [x_c, x_c + w)"
for left and "[x_c - w, x_c)" for right.  Only x enters the sub-pixel test;
the sub-pixels span the pixel height.

Angular response (a smooth, differentiable alternative used by the
synthetic workloads, not in the paper): the left weight is the logistic
function of k_s sin(theta_x) with sin(theta_x) = D_x / sqrt(D_x^2 + D_z^2),
the same angle as tan(theta) above; the right weight is its complement.
Both rules favour the left sub-pixel for rays travelling toward +x.
"""

import numpy as np

LEFT, RIGHT, MISSED = 0, 1, 2


def microlens_side(xk, yk, xc, yc, tan_t, ps, h=0.78, f=1.44, w=0.30, r=0.50):
    """Sub-pixel (LEFT / RIGHT / MISSED) for rays landing at (xk, yk) in the
    pixel centred at (xc, yc); h, f, w, r in units of the pitch ps."""
    h, f, w, r = h * ps, f * ps, w * ps, r * ps
    inside = (xk - xc) ** 2 + (yk - yc) ** 2 <= r * r
    g = h / (f - h)
    xL1 = xc + w - (f * tan_t - w) * g
    xM1 = xc - (f * tan_t) * g
    xR1 = xc - w - (f * tan_t + w) * g
    xL2 = xc + w - h * tan_t
    xM2 = xc - h * tan_t
    xR2 = xc - w - h * tan_t
    xL = np.where(inside, xL1, xL2)
    xM = np.where(inside, xM1, xM2)
    xR = np.where(inside, xR1, xR2)
    side = np.full(np.shape(xk), MISSED, dtype=np.int32)
    side[(xM <= xk) & (xk < xL)] = LEFT
    side[(xR <= xk) & (xk < xM)] = RIGHT
    return side


def microlens_side_by_microtrace(xk, yk, xc, yc, tan_t, ps, h=0.78, f=1.44,
                                 w=0.30, r=0.50):
    """Independent derivation used as a pin: carry the ray through an ideal
    thin lens of focal f centred on the pixel (if it lands inside the
    radius-r disk) and on to the sub-pixel plane at depth h."""
    h, f, w, r = h * ps, f * ps, w * ps, r * ps
    inside = (xk - xc) ** 2 + (yk - yc) ** 2 <= r * r
    slope = np.where(inside, tan_t - (xk - xc) / f, tan_t)
    xs = xk + h * slope - xc
    side = np.full(np.shape(xk), MISSED, dtype=np.int32)
    side[(0.0 <= xs) & (xs < w)] = LEFT
    side[(-w <= xs) & (xs < 0.0)] = RIGHT
    return side


def sigmoid_weights(D, k):
    """Left / right weights of the angular response for directions D (n,3)."""
    sx = D[:, 0] / np.sqrt(D[:, 0] ** 2 + D[:, 2] ** 2)
    wl = 1.0 / (1.0 + np.exp(-k * sx))
    return wl, 1.0 - wl
