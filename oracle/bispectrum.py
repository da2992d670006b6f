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


def shell_modes_band(band, n_dk, b):
    """Signed modes (k, 3) of shell b (same integer rule as P(k)) with every
    |m_a| <= band."""
    r = np.arange(-band, band + 1, dtype=np.int64)
    mx, my, mz = np.meshgrid(r, r, r, indexing="ij")
    q = np.stack([mx, my, mz], -1).reshape(-1, 3)
    m2 = (q * q).sum(1)
    sel = (m2 > 0) & (bin_index(m2, n_dk) == b)
    return q[sel]


def band_lookup(d_band, band, q):
    """delta at signed modes q from d_band[m_x + band, m_y + band, m_z]
    (m_z = 0 .. band), completed by delta(-m) = conj(delta(m))."""
    q = np.asarray(q, dtype=np.int64)
    neg = q[:, 2] < 0
    qq = np.where(neg[:, None], -q, q)
    v = d_band[qq[:, 0] + band, qq[:, 1] + band, qq[:, 2]]
    return np.where(neg, np.conj(v), v)


def brute_triplets(d_band, band, n_dk, tri):
    """For each triangle (b1, b2, b3): the number of closed triplets
    q1 + q2 + q3 = 0 with q_i in shell b_i, and sum delta(q1) delta(q2)
    delta(q3) and sum |delta delta delta| over them, by enumeration (eq. Best
    and the normalisation of eq. VBest by their definitions).  Every shell
    used must lie inside the band (|m| < (b + 1/2) n_dk <= band)."""
    counts, sums, abss = [], [], []
    for b1, b2, b3 in np.asarray(tri).reshape(-1, 3):
        if 2 * band < (2 * int(b1) + 1) * n_dk - 1:
            raise ValueError("shell %d reaches outside the band" % b1)
        q1 = shell_modes_band(band, n_dk, int(b1))
        q2 = shell_modes_band(band, n_dk, int(b2))
        d1 = band_lookup(d_band, band, q1)
        d2 = band_lookup(d_band, band, q2)
        c, s, a = 0, 0.0 + 0.0j, 0.0
        for i0 in range(0, len(q1), 512):
            q3 = -(q1[i0:i0 + 512, None, :] + q2[None, :, :])
            m2 = (q3 * q3).sum(-1)
            ok = (m2 > 0) & (bin_index(m2, n_dk) == b3)
            i1, i2 = np.nonzero(ok)
            if len(i1) == 0:
                continue
            d3 = band_lookup(d_band, band, q3[i1, i2])
            prod = d1[i0 + i1] * d2[i2] * d3
            c += len(i1)
            s += prod.sum()
            a += np.abs(prod).sum()
        counts.append(c)
        sums.append(s)
        abss.append(a)
    return np.array(counts), np.array(sums), np.array(abss)
