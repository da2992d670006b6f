"""FFT-shell bispectrum estimator (Sec. 4.1).

Test infrastructure only (see ``oracle/__init__.py``).

The shell-averaged bispectrum (eq. Best, normalised by eq. VBest) is
evaluated with the integral representation of the Dirac delta (eqs. Best2,
IntI): for every shell b

    I_b(x) = sum_{m in shell b} delta(m) exp(+2 pi i m.x/N)      (eq. IntI)
    J_b(x) = sum_{m in shell b} exp(+2 pi i m.x/N)                (V_B the same way)

and for a triangle (b1, b2, b3)

    sum_x I_b1 I_b2 I_b3 = N^3 * sum over closed triplets of delta delta delta,
    sum_x J_b1 J_b2 J_b3 = N^3 * number of closed triplets N_tri.

B = V^2 * sum_x I I I / sum_x J J J (standard normalisation; the paper's
(2 pi)^6 factor only rescales it).  Readings:

* Shells use the same lower-inclusive integer rule as P(k) with the width
  n_dk k_f (default 2 k_f).  Only shells below k_f N/3 are allowed (the
  triangle-aliasing limit of Sec. 4.1); they never touch a Nyquist plane, so
  delta is Hermitian inside every shell.
* "All closed triangles": b1 >= b2 >= b3 >= 1 and b1 <= b2 + b3 on bin
  centres.  A triangle with N_tri = 0 has B = NaN.
* Shot noise is not subtracted unless requested; when it is, the term
  (V/N_P)(P_b1 + P_b2 + P_b3) + (V/N_P)^2 uses bin-averaged raw P (an
  approximation of the per-triplet term).
"""

import numpy as np
import scipy.fft

from .spectrum import bin_index, delta_half, half_axes, bin_power


def closed_triangles(n_bins):
    """All (b1, b2, b3) with b1 >= b2 >= b3 >= 1 and b1 <= b2 + b3."""
    tri = [(b1, b2, b3)
           for b1 in range(1, n_bins + 1)
           for b2 in range(1, b1 + 1)
           for b3 in range(1, b2 + 1)
           if b1 <= b2 + b3]
    return np.array(tri, dtype=np.int32).reshape(-1, 3)


def max_bins(n, n_dk):
    """Largest n_bins with (n_bins + 1/2) n_dk < N/3 (triangle limit)."""
    b = 0
    while 3 * (2 * (b + 1) + 1) * n_dk < 2 * n:
        b += 1
    return b


def shell_masks(n, n_dk, n_bins):
    """Boolean half-spectrum masks S_b, b = 1..n_bins, shape (n_bins, N, N, N/2+1)."""
    mx, my, mz = half_axes(n)
    m2 = mx * mx + my * my + mz * mz
    b = bin_index(m2, n_dk)
    return np.stack([(b == i) & (m2 > 0) for i in range(1, n_bins + 1)])


def shell_fields(half, masks, n):
    """Real fields sum_{m in shell} half(m) exp(+2 pi i m.x/N) for every shell."""
    out = np.empty((masks.shape[0], n, n, n), dtype=np.float64)
    for i in range(masks.shape[0]):
        out[i] = scipy.fft.irfftn(np.where(masks[i], half, 0.0), s=(n, n, n),
                                  workers=-1) * float(n) ** 3
    return out


def triple_sums(fields, tri):
    """sum_x F[b1] F[b2] F[b3] for each triangle (1-based bins)."""
    nb = fields.shape[0]
    flat = fields.reshape(nb, -1)
    out = np.empty(len(tri), dtype=np.float64)
    # group by (b1, b2): (F_b1 * F_b2) . F_b3 for all b3 of the group
    for (b1, b2) in sorted({(int(t[0]), int(t[1])) for t in tri}):
        prod = flat[b1 - 1] * flat[b2 - 1]
        sel = np.nonzero((tri[:, 0] == b1) & (tri[:, 1] == b2))[0]
        out[sel] = flat[tri[sel, 2] - 1] @ prod
    return out


def bispectrum(pos, box, n_grid, order, interlace_on, n_dk=2, n_bins=None,
               triangles=None, subtract_shot=False):
    """FFT-shell bispectrum.  Returns (triangles, B, N_tri)."""
    if n_bins is None:
        n_bins = max_bins(n_grid, n_dk)
    if triangles is None:
        triangles = closed_triangles(n_bins)
    triangles = np.asarray(triangles, dtype=np.int32).reshape(-1, 3)
    delta, n_p = delta_half(np.asarray(pos), box, n_grid, order, interlace_on)
    masks = shell_masks(n_grid, n_dk, n_bins)
    i_fields = shell_fields(delta, masks, n_grid)
    s_iii = triple_sums(i_fields, triangles)
    del i_fields
    j_fields = shell_fields(np.ones_like(delta), masks, n_grid)
    s_jjj = triple_sums(j_fields, triangles)
    vol = float(box) ** 3
    with np.errstate(invalid="ignore", divide="ignore"):
        bk = vol * vol * s_iii / s_jjj
    bk = np.where(s_jjj > 0.5, bk, np.nan)
    n_tri = s_jjj / float(n_grid) ** 3
    if subtract_shot:
        _, pk, _ = bin_power(delta, box, n_grid, n_dk, n_bins)
        sn = vol / n_p
        bk = bk - sn * (pk[triangles[:, 0] - 1] + pk[triangles[:, 1] - 1]
                        + pk[triangles[:, 2] - 1]) - sn * sn
    return triangles, bk, n_tri
