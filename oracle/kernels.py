"""Order-p B-spline mass-assignment kernels (Sec. 2.3) and their Fourier window.

Test infrastructure only (see ``oracle/__init__.py``).

The one-dimensional weights W^(p)(s), s = (x_grid - x)/H, are the
piecewise polynomials printed for NGP (p=1), CIC (p=2), TSC (p=3) and PCS
(p=4) in Sec. 2.3.  Orders p = 5, 6 (the higher-order B-splines Sec. 2.3
mentions) use the centred cardinal B-spline of order p, the p-fold
convolution of the unit box, written as its truncated-power sum

    W^(p)(s) = 1/(p-1)! sum_{k=0}^{p} (-1)^k C(p, k) (s + p/2 - k)_+^{p-1},

whose Fourier transform is sinc^p (eq. intkerFT).  Two readings:

* CIC: the printed support "|s| < 1/2" is a typo; the support is |s| < 1
  (partition of unity and the sinc^2 window of eq. intkerFT both require it).
* NGP: a particle belongs to the cell whose centre is nearest, cells being
  half-open [gH - H/2, gH + H/2); the weight of that cell is 1.  This equals
  W^(1)(s) = 1 on -1/2 < s <= 1/2, i.e. ties at |s| = 1/2 go to the upper
  cell so that no mass is dropped.
"""

from math import comb, factorial

import numpy as np

MAX_ORDER = 6


def _bspline(p, s, deriv=False):
    """Truncated-power sum of the centred order-p B-spline (or its derivative)."""
    s = np.asarray(s, dtype=np.float64)
    e = p - 2 if deriv else p - 1
    out = np.zeros_like(s)
    for k in range(p + 1):
        x = s + 0.5 * p - k
        out += (-1) ** k * comb(p, k) * np.where(x > 0, x, 0.0) ** e
    return out / factorial(e)


def weight(p, s):
    """W^(p)(s) of Sec. 2.3 for an array ``s`` (float64)."""
    s = np.asarray(s, dtype=np.float64)
    a = np.abs(s)
    if p == 1:
        # -1/2 < s <= 1/2 (tie rule above)
        return np.where((s > -0.5) & (s <= 0.5), 1.0, 0.0)
    if p == 2:
        return np.where(a < 1.0, 1.0 - a, 0.0)
    if p == 3:
        inner = 0.75 - s * s
        outer = 0.5 * (1.5 - a) ** 2
        return np.where(a < 0.5, inner, np.where(a < 1.5, outer, 0.0))
    if p == 4:
        inner = (4.0 - 6.0 * s * s + 3.0 * a ** 3) / 6.0
        outer = (2.0 - a) ** 3 / 6.0
        return np.where(a < 1.0, inner, np.where(a < 2.0, outer, 0.0))
    if p <= MAX_ORDER:
        return np.where(a < 0.5 * p, _bspline(p, s), 0.0)
    raise ValueError("order p must be 1..%d" % MAX_ORDER)


def dweight(p, s):
    """dW^(p)/ds, the derivative of the piecewise polynomials of Sec. 2.3.

    NGP is piecewise constant, so its derivative is 0 almost everywhere.
    """
    s = np.asarray(s, dtype=np.float64)
    a = np.abs(s)
    sg = np.sign(s)
    if p == 1:
        return np.zeros_like(s)
    if p == 2:
        return np.where(a < 1.0, -sg, 0.0)
    if p == 3:
        return np.where(a < 0.5, -2.0 * s, np.where(a < 1.5, -(1.5 - a) * sg, 0.0))
    if p == 4:
        inner = -2.0 * s + 1.5 * s * a
        outer = -0.5 * (2.0 - a) ** 2 * sg
        return np.where(a < 1.0, inner, np.where(a < 2.0, outer, 0.0))
    if p <= MAX_ORDER:
        return np.where(a < 0.5 * p, _bspline(p, s, deriv=True), 0.0)
    raise ValueError("order p must be 1..%d" % MAX_ORDER)


def window_1d(p, m, n_grid):
    """One axis of eq. intkerFT: [sin(k H/2)/(k H/2)]^p with k H/2 = pi m / N.

    ``m`` is the signed integer frequency on the grid.  sinc(0) = 1.
    """
    x = np.asarray(m, dtype=np.float64) / float(n_grid)
    return np.sinc(x) ** p  # numpy sinc(x) = sin(pi x)/(pi x)
