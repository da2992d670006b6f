"""FFT, interlace combination, window deconvolution and |k|-shell P(k).

Test infrastructure only (see ``oracle/__init__.py``).

Steps, in the paper's order:

1. F_a = unnormalised forward real-to-complex DFT of each grid, sign
   exp(-i k.x) as in the Fourier convention of Sec. 2.1 (library routine
   ``scipy.fft.rfftn``; half spectrum, last axis m_z = 0..N/2).
2. Interlacing (eq. intdelta and the shift theorem above it):
   C = (F_1 + exp(+i pi (m_x+m_y+m_z)/N) F_2) / 2; without interlacing C = F_1.
   More grids (Sec. 3.1 allows it without writing it out; reading): G grids
   sampled at u + s_j, s_j in {0, 1/2}^3 forming a group under addition mod 1,
   C = (1/G) sum_j F_j exp(+2 pi i m.s_j / N).  Image n then enters with
   theta_n = 1 if n.s_j is an integer for every j, else 0.  Codes: 0 one
   grid, 1 the paper's pair {0, (1,1,1)/2}, 2 the four face-centred shifts
   {0, (1,1,0)/2, (1,0,1)/2, (0,1,1)/2} (no image with components of mixed
   parity), 3 all eight shifts (no image with an odd component).
3. Window deconvolution (eqs. windowcorrection, intkerFT):
   delta = C / (N_P W(m)),  W = prod_i [sin(pi m_i/N)/(pi m_i/N)]^p.
4. Power in shells (eq. ps, the direct-summation estimator of Sec. 2.2, the
   shells of Sec. 4): P(m) = V |delta(m)|^2; a bin averages P over its modes.

Readings (the paper is silent or garbled here):

* Normalisation: the power is reported in the standard convention
  P = V |delta|^2 with delta -> 1 - like N_P^-1 sum_j exp(-i k.x_j); the
  paper's (2 pi)^3 factors only rescale it (P_paper = P / (2 pi)^3).  The shot
  noise is the constant V/N_P; it is subtracted only on request (the N-body
  test subtracts it, the Zel'dovich tests do not).
* Signed frequencies: index i maps to m = i for i <= N/2 and i - N above, so
  the Nyquist index N/2 is +N/2 on every axis (this only matters for the
  interlace phase on the Nyquist planes).
* Half-spectrum weights: w = 1 on the planes m_z = 0 and m_z = N/2, 2
  elsewhere; sum w over a bin equals the full-grid mode count.
* Bins: width dk = n_dk k_f, centred on b dk, lower-inclusive:
  (2b-1)^2 n_dk^2 <= 4 |m|^2 < (2b+1)^2 n_dk^2, decided in integers;
  the mode m = 0 is never used; b runs 1..n_bins.
"""

import numpy as np
import scipy.fft

from .assign import deposit, deposit_u, grid_coords
from .kernels import window_1d


def signed_index(n):
    """Signed frequency of each FFT index along a full axis (N/2 -> +N/2)."""
    i = np.arange(n, dtype=np.int64)
    return np.where(i <= n // 2, i, i - n)


def half_axes(n, x0=0, x1=None):
    """(m_x, m_y, m_z) broadcastable arrays for the rfftn half spectrum
    (m_x of the x planes x0 .. x1-1 only, all of them by default)."""
    mx = signed_index(n)[x0:(n if x1 is None else x1), None, None]
    my = signed_index(n)[None, :, None]
    mz = np.arange(n // 2 + 1, dtype=np.int64)[None, None, :]
    return mx, my, mz


def fft_grid(rho, workers=None):
    """Unnormalised forward r2c DFT, exp(-2 pi i m.g/N), in float64."""
    if workers is None:
        workers = -1
    return scipy.fft.rfftn(rho, workers=workers)


# shift sets: bit a of a mask shifts axis a by half a cell
SHIFT_SETS = {0: (0,), 1: (0, 7), 2: (0, 3, 5, 6), 3: tuple(range(8))}


def shift_masks(code):
    """Masks of the grids for an interlacing code (bool True = 1)."""
    return SHIFT_SETS[int(code)]


def mask_shift(mask):
    """Grid-coordinate shift (3,) of a mask: 1/2 on the axes whose bit is set."""
    return 0.5 * np.array([(mask >> a) & 1 for a in range(3)], dtype=np.float64)


def combine(fs, masks, n, x0=0):
    """C = (1/G) sum_j F_j exp(+i pi (sum of m_a over the shifted axes of j) / N).

    The F_j may hold only the x planes x0, x0 + 1, ... of the half spectrum."""
    mx, my, mz = half_axes(n, x0, x0 + fs[0].shape[0])
    m = (mx, my, mz)
    c = 0.0
    for f, mk in zip(fs, masks):
        s = sum((m[a] if (mk >> a) & 1 else 0) for a in range(3))
        c = c + np.exp(1j * np.pi * np.asarray(s, dtype=np.float64) / n) * f
    return c / len(fs)


def interlace(f1, f2, n, x0=0):
    """C = (F_1 + exp(i pi (m_x+m_y+m_z)/N) F_2) / 2  (eq. intdelta).

    f1, f2 may hold only the x planes x0, x0 + 1, ... of the half spectrum."""
    mx, my, mz = half_axes(n, x0, x0 + f1.shape[0])
    phase = np.exp(1j * np.pi * (mx + my + mz).astype(np.float64) / n)
    return 0.5 * (f1 + phase * f2)


def window(n, p, x0=0, x1=None):
    """W(m) on the half spectrum (eq. intkerFT, three axes multiplied), on
    the x planes x0 .. x1-1 (all by default)."""
    mx, my, mz = half_axes(n, x0, x1)
    return window_1d(p, mx, n) * window_1d(p, my, n) * window_1d(p, mz, n)


def half_weights(n):
    """w = 1 on m_z in {0, N/2}, 2 elsewhere (broadcastable over the half)."""
    w = np.full(n // 2 + 1, 2, dtype=np.int64)
    w[0] = 1
    w[n // 2] = 1
    return w[None, None, :]


def isqrt(x):
    """Exact integer square root of a non-negative int64 array."""
    x = np.asarray(x, dtype=np.int64)
    r = np.floor(np.sqrt(x.astype(np.float64))).astype(np.int64)
    r = np.where(r * r > x, r - 1, r)
    r = np.where((r + 1) * (r + 1) <= x, r + 1, r)
    return r


def bin_index(m2, n_dk):
    """Bin b with (2b-1)^2 n^2 <= 4 m2 < (2b+1)^2 n^2 (b = 0 if 4 m2 < n^2).

    (2b-1) n <= 2 sqrt(m2) holds for integer (2b-1) n iff it is <= isqrt(4 m2).
    """
    q = isqrt(4 * np.asarray(m2, dtype=np.int64)) // n_dk
    return (q + 1) // 2


def max_bins(n, n_dk):
    """Bins reaching the Nyquist frequency: b <= N / (2 n_dk)."""
    return n // (2 * n_dk)


def mode_table(n, n_dk, n_bins, planes=None):
    """(N_b int64, sum_b w|m| float64) per bin, from the half spectrum.

    ``planes`` processes that many x-planes at a time (memory bound for
    large N); the result does not depend on it.
    """
    planes = n if planes is None else planes
    mx_all, my, mz = half_axes(n)
    counts = np.zeros(n_bins + 1, dtype=np.int64)
    ksum = np.zeros(n_bins + 1, dtype=np.float64)
    for x0 in range(0, n, planes):
        mx = mx_all[x0:x0 + planes]
        m2 = mx * mx + my * my + mz * mz
        b = np.broadcast_to(bin_index(m2, n_dk), m2.shape)
        w = np.broadcast_to(half_weights(n), m2.shape)
        sel = (m2 > 0) & (b >= 1) & (b <= n_bins)
        counts += np.bincount(b[sel], weights=w[sel], minlength=n_bins + 1).astype(np.int64)
        ksum += np.bincount(b[sel], weights=(w * np.sqrt(m2.astype(np.float64)))[sel],
                            minlength=n_bins + 1)
    return counts[1:], ksum[1:]


def total_weight(pos, weights):
    """(W, sum w^2): N_P and N_P for equal masses."""
    if weights is None:
        return float(pos.shape[0]), float(pos.shape[0])
    w = np.asarray(weights, dtype=np.float64)
    return float(w.sum()), float((w * w).sum())


def shot_noise(pos, box, weights=None):
    """V sum w^2 / W^2 (V / N_P for equal masses): the self-pair term of
    V |delta(k)|^2 for the weighted density."""
    if weights is None:
        return float(box) ** 3 / pos.shape[0]
    wsum, w2sum = total_weight(pos, weights)
    return float(box) ** 3 * w2sum / (wsum * wsum)


def delta_half(pos, box, n, p, interlace_on, workers=None, weights=None):
    """delta(m) on the half spectrum (steps 1-3 above) and the total mass W
    (N_P for equal masses), which normalises it."""
    n_p, _ = total_weight(pos, weights)
    if int(interlace_on) >= 2:
        u = grid_coords(pos, box, n)
        masks = shift_masks(interlace_on)
        fs = [fft_grid(deposit_u(u + mask_shift(mk), p, n, weights), workers) for mk in masks]
        return combine(fs, masks, n) / (n_p * window(n, p)), n_p
    rho1, rho2 = deposit(pos, box, n, p, interlace_on, weights)
    f1 = fft_grid(rho1, workers)
    if interlace_on:
        f2 = fft_grid(rho2, workers)
        c = interlace(f1, f2, n)
    else:
        c = f1
    return c / (n_p * window(n, p)), n_p


def shell_sums(delta, box, n, n_dk, n_bins, x0=0):
    """Per shell, sum over its modes of w V |delta(m)|^2 (step 4 before the
    division by N_b), for a half spectrum ``delta`` that holds the x planes
    x0, x0 + 1, ... (all of them by default).  Shells are disjoint, so the sums
    of consecutive plane ranges add up to those of the whole half spectrum."""
    mx, my, mz = half_axes(n, x0, x0 + delta.shape[0])
    m2 = mx * mx + my * my + mz * mz
    b = np.broadcast_to(bin_index(m2, n_dk), m2.shape)
    w = np.broadcast_to(half_weights(n), m2.shape).astype(np.float64)
    sel = (m2 > 0) & (b >= 1) & (b <= n_bins)
    vol = float(box) ** 3
    pk_mode = vol * np.abs(delta) ** 2
    return np.bincount(b[sel], weights=(w * pk_mode)[sel], minlength=n_bins + 1)[1:]


def bin_power(delta, box, n, n_dk, n_bins):
    """(k_b, P_b raw, N_b) from a half-spectrum delta (step 4)."""
    s = shell_sums(delta, box, n, n_dk, n_bins)
    counts, ksum = mode_table(n, n_dk, n_bins)
    kf = 2.0 * np.pi / box
    with np.errstate(invalid="ignore", divide="ignore"):
        k = kf * ksum / counts
        pk = s / counts
    return k, pk, counts


def bin_cross(a, b, box, n, n_dk, n_bins, shot=0.0):
    """(k_b, P_b, N_b) with P_b = V sum_shell w Re(a b*) / N_b - shot.

    a and b are half spectra (``half_axes`` layout); b = a gives the auto
    spectrum of the direct-summation estimator (Sec. 2.2) or of the grid
    estimator, a = delta_G and b = delta_DS the cross spectrum P_{G-DS} used
    to measure aliasing in Sec. 3.2.  Shells, weights and mode counts as in
    ``bin_power``.
    """
    mx, my, mz = half_axes(n)
    m2 = mx * mx + my * my + mz * mz
    bi = np.broadcast_to(bin_index(m2, n_dk), m2.shape)
    w = np.broadcast_to(half_weights(n), m2.shape).astype(np.float64)
    sel = (m2 > 0) & (bi >= 1) & (bi <= n_bins)
    re = (np.asarray(a) * np.conj(np.asarray(b))).real
    s = np.bincount(bi[sel], weights=(w * re)[sel], minlength=n_bins + 1)[1:]
    counts, ksum = mode_table(n, n_dk, n_bins)
    kf = 2.0 * np.pi / box
    vol = float(box) ** 3
    with np.errstate(invalid="ignore", divide="ignore"):
        k = kf * ksum / counts
        pk = vol * s / counts - shot
    return k, pk, counts


def power(pos, box, n_grid, order, interlace_on, n_dk=1, n_bins=None,
          subtract_shot=False, workers=None, weights=None):
    """Binned power spectrum of a particle set (optionally with masses).

    Returns (k_b [h/Mpc units of 1/box], P_b, N_b); P is raw unless
    ``subtract_shot`` (then P_b - V sum w^2 / W^2, i.e. V/N_P for equal
    masses).
    """
    if n_bins is None:
        n_bins = max_bins(n_grid, n_dk)
    pos = np.asarray(pos)
    delta, _ = delta_half(pos, box, n_grid, order, interlace_on, workers, weights)
    k, pk, counts = bin_power(delta, box, n_grid, n_dk, n_bins)
    if subtract_shot:
        pk = pk - shot_noise(pos, box, weights)
    return k, pk, counts
