"""Pins of the oracle's interlacing with more than two grids (codes 2 and 3:
the four face-centred and all eight half-cell shifts; code 1 is the paper's
pair, eq. intdelta).

* Fine-grid identity: G grids at u + s, s in a group S of {0, 1/2}^3, tile a
  grid of spacing H/2.  With the phases exp(2 pi i m.s/N) the sum
  sum_j F_j(m) exp(...) is exactly the DFT of that fine grid at m (fine
  cells of the parity classes in S, each holding the kernel of width pH
  evaluated at its own position), summed here particle by particle with no
  FFT.
* The aliasing factor theta_n of the shift set: the closed-form white-noise
  expectation agrees with a brute-force sum over images in 3D, and Monte
  Carlo of the oracle's pipeline agrees with it.
"""

import cmath
import math

import numpy as np
import pytest

from oracle import kernels, spectrum, theory
import synth


def _fine_dft(pos, box, n, p, masks, modes):
    """sum over particles and fine cells g' (parity class in masks) of
    prod_a W(g'_a/2 - u_a) exp(-2 pi i m.g' / (2N))."""
    u = np.asarray(pos, dtype=np.float64) * (n / box)
    out = np.zeros(len(modes), dtype=np.complex128)
    for uj in u:
        per_axis = []
        for a in range(3):
            base = int(math.floor(2 * uj[a]))
            cells = [g for g in range(base - p - 2, base + p + 3)]
            per_axis.append([(g, float(kernels.weight(p, np.array(g / 2.0 - uj[a]))) if p > 1 else
                              (1.0 if abs(g / 2.0 - uj[a]) < 0.5 else 0.0)) for g in cells])
        for gx, wx in per_axis[0]:
            if wx == 0.0:
                continue
            for gy, wy in per_axis[1]:
                if wy == 0.0:
                    continue
                for gz, wz in per_axis[2]:
                    if wz == 0.0:
                        continue
                    cls = (gx & 1) | ((gy & 1) << 1) | ((gz & 1) << 2)
                    if cls not in masks:
                        continue
                    w = wx * wy * wz
                    for i, (mx, my, mz) in enumerate(modes):
                        out[i] += w * cmath.exp(-2j * math.pi * (mx * gx + my * gy + mz * gz) / (2 * n))
    return out


@pytest.mark.parametrize("code,p", [(1, 2), (2, 2), (3, 2), (2, 3), (3, 4), (1, 4)])
def test_combination_is_fine_grid_dft(code, p):
    n, box = 8, 40.0
    # positions away from half-cell ties so the brute-force support test is unambiguous
    pos = synth.uniform(6, box, 31 + code, np.float64)
    masks = spectrum.shift_masks(code)
    u = pos * (n / box)
    fs = [spectrum.fft_grid(spectrum.deposit_u(u + spectrum.mask_shift(mk), p, n)) for mk in masks]
    c = spectrum.combine(fs, masks, n) * len(masks)
    # index N/2 holds m = +N/2 (the fine grid tells +N/2 from -N/2)
    modes = [(0, 0, 1), (1, 2, 3), (-3, 4, 2), (4, 4, 4), (-1, -2, 0), (2, 4, 1)]
    ref = _fine_dft(pos, box, n, p, masks, modes)
    got = np.array([c[mx % n, my % n, mz] for mx, my, mz in modes])
    assert np.max(np.abs(got - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("code,p", [(2, 3), (3, 3), (2, 4), (3, 4), (1, 4)])
def test_theta_closed_form_matches_image_sum(code, p):
    n = 16
    masks = spectrum.shift_masks(code)
    nmax = 24
    rng = np.arange(-nmax, nmax + 1)
    for m in [(1, 2, 3), (8, 0, 5), (7, -7, 2), (8, 8, 8)]:
        x = np.array(m, dtype=np.float64) / n
        sx = np.sinc(x[0] - rng) ** (2 * p)
        sy = np.sinc(x[1] - rng) ** (2 * p)
        sz = np.sinc(x[2] - rng) ** (2 * p)
        tot = 0.0
        for mk in masks:
            # sum over images weighted by (-1)^(n_a) on the shifted axes
            f = [s * np.where((rng % 2 == 1) & bool((mk >> a) & 1), -1.0, 1.0)
                 for a, s in enumerate((sx, sy, sz))]
            tot += f[0].sum() * f[1].sum() * f[2].sum()
        brute = tot / len(masks)
        closed = theory.white_noise_power(np.array([m]), n, p, code, False, 1.0, 1.0)[0]
        assert closed == pytest.approx(brute, rel=1e-6, abs=1e-9), m


@pytest.mark.parametrize("code,p", [(2, 2), (3, 2), (3, 4)])
def test_white_noise_expectation_monte_carlo(code, p):
    n, box, n_p, reps = 16, 100.0, 2000, 60
    mx, my, mz = spectrum.half_axes(n)
    m = np.stack(np.broadcast_arrays(mx, my, mz), axis=-1)
    m2 = (m ** 2).sum(-1)
    w = np.broadcast_to(spectrum.half_weights(n), m2.shape)
    b = spectrum.bin_index(m2, 1)
    vol = box ** 3
    expect = theory.white_noise_power(m, n, p, code, True, vol, n_p)
    acc = np.zeros(m2.shape)
    for r in range(reps):
        pos = synth.uniform(n_p, box, 7000 + r, np.float64)
        delta, _ = spectrum.delta_half(pos, box, n, p, code)
        acc += vol * np.abs(delta) ** 2
    acc /= reps
    for bi in range(1, n // 2 + 1):
        sel = (b == bi) & (m2 > 0)
        nm = w[sel].sum()
        mc = (w[sel] * acc[sel]).sum() / nm
        th = (w[sel] * expect[sel]).sum() / nm
        assert abs(mc - th) < 4.0 * th / np.sqrt(reps * nm / 2.0), (bi, mc, th)


def test_eight_grids_reduce_aliasing_below_two():
    """At the Nyquist corner and along the axes, the residual aliased white
    noise of eight grids is below that of the paper's pair, which is below
    that of one grid (PCS, deconvolved)."""
    n = 64
    for m in [(32, 0, 0), (20, 20, 0), (32, 32, 32), (16, 16, 16)]:
        mm = np.array([m])
        r = [theory.white_noise_power(mm, n, 4, c, True, 1.0, 1.0)[0] - 1.0 for c in (0, 1, 3)]
        assert abs(r[2]) <= abs(r[1]) + 1e-12 and abs(r[1]) <= abs(r[0]) + 1e-12, (m, r)
