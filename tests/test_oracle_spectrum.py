"""Pins of the oracle's P(k): interlacing, deconvolution, normalisation, bins.

* Mode counts: brute force over the full N^3 grid of signed frequencies
  (no half-spectrum weights) must equal the weighted half-spectrum counts.
* Aliased white noise: for uniformly random particles the expected P(m) is a
  closed form of the aliasing sums (eq. Pknoint and the interlaced version
  with theta_n, Sec. 3.1); a Monte-Carlo average of the oracle must match it
  per bin within the sampling error, for every order, with and without
  interlacing and deconvolution.
* Direct summation (eq. deltaDS): on a smooth Zel'dovich field PCS +
  interlacing reproduces the alias-free direct-sum delta closely, much more
  closely than CIC without interlacing (the paper's central claim).
"""

import numpy as np
import pytest

from oracle import direct, spectrum, theory
import synth


def _full_grid_counts(n, n_dk, n_bins):
    m = spectrum.signed_index(n)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    m2 = (mx * mx + my * my + mz * mz).ravel()
    counts = np.zeros(n_bins, dtype=np.int64)
    # exact integer bins by direct comparison with the shell edges
    for b in range(1, n_bins + 1):
        lo = (2 * b - 1) ** 2 * n_dk ** 2
        hi = (2 * b + 1) ** 2 * n_dk ** 2
        counts[b - 1] = np.count_nonzero((4 * m2 >= lo) & (4 * m2 < hi))
    return counts


@pytest.mark.parametrize("n,n_dk", [(16, 1), (32, 1), (32, 2), (24, 3), (8, 1), (12, 1), (20, 2),
                                   (30, 1)])
def test_mode_counts_bruteforce(n, n_dk):
    nb = spectrum.max_bins(n, n_dk)
    counts, ksum = spectrum.mode_table(n, n_dk, nb)
    assert np.array_equal(counts, _full_grid_counts(n, n_dk, nb))
    assert np.all(ksum > 0)


def test_mode_counts_n32_table():
    counts, _ = spectrum.mode_table(32, 1, 16)
    expected = [18, 62, 98, 210, 350, 450, 602, 762, 1142, 1250, 1458, 1814,
                2178, 2498, 2622, 3191]
    assert counts.tolist() == expected


def test_bin_index_edges():
    # lower-inclusive centred bins: |m| = 0.5 goes to bin 1, 1.5 to bin 2, ...
    m2 = np.arange(0, 200)
    b = spectrum.bin_index(m2, 1)
    ref = np.floor(np.sqrt(m2) + 0.5).astype(int)
    assert np.array_equal(b, ref)
    b2 = spectrum.bin_index(np.array([0, 1, 8, 9, 10, 24, 25]), 2)
    # n_dk = 2: bin b covers 2b-1 <= |m| < 2b+1
    assert b2.tolist() == [0, 1, 1, 2, 2, 2, 3]


@pytest.mark.parametrize("p,il,n", [(1, False, 16), (1, True, 16), (2, False, 16), (2, True, 16),
                                    (3, False, 16), (3, True, 16), (4, False, 16), (4, True, 16),
                                    (4, True, 12), (2, False, 20), (3, True, 20)])
def test_white_noise_expectation_monte_carlo(p, il, n):
    """Also at N = 12 and 20 (factors 3 and 5): the oracle's FFT path has no
    power-of-two assumption."""
    box, n_p, reps = 100.0, 2000, 120
    mx, my, mz = spectrum.half_axes(n)
    m = np.stack(np.broadcast_arrays(mx, my, mz), axis=-1)
    m2 = (m ** 2).sum(-1)
    w = np.broadcast_to(spectrum.half_weights(n), m2.shape)
    b = spectrum.bin_index(m2, 1)
    vol = box ** 3
    expect = theory.white_noise_power(m, n, p, il, True, vol, n_p)
    acc = np.zeros(m2.shape)
    for r in range(reps):
        pos = synth.uniform(n_p, box, 1000 + r, np.float64)
        delta, _ = spectrum.delta_half(pos, box, n, p, il)
        acc += vol * np.abs(delta) ** 2
    acc /= reps
    for bi in range(1, n // 2 + 1):
        sel = (b == bi) & (m2 > 0)
        nmodes = w[sel].sum()
        mean_mc = (w[sel] * acc[sel]).sum() / nmodes
        mean_th = (w[sel] * expect[sel]).sum() / nmodes
        # each mode is exponentially distributed around its mean
        err = 4.0 * mean_th / np.sqrt(reps * nmodes / 2.0)
        assert abs(mean_mc - mean_th) < err, (bi, mean_mc, mean_th)


def test_white_noise_special_values():
    vol, n_p, n = 1.0, 1.0, 64
    nyq = np.array([[n // 2, 0, 0]])
    # PCS + interlacing at (k_N, 0, 0): 1.00016 V/N_P; without: 2.0003 V/N_P
    assert theory.white_noise_power(nyq, n, 4, True, True, vol, n_p)[0] == pytest.approx(1.00016, abs=1e-5)
    assert theory.white_noise_power(nyq, n, 4, False, True, vol, n_p)[0] == pytest.approx(2.0003, abs=1e-4)
    # NGP without interlacing or deconvolution is exactly flat
    m = np.array([[3, 5, 7], [32, 32, 32], [1, 0, 0]])
    assert np.allclose(theory.white_noise_power(m, n, 1, False, False, vol, n_p), 1.0)


def test_ngp_raw_power_is_flat_shot_noise():
    n, box, n_p, reps = 16, 100.0, 3000, 60
    acc = np.zeros(spectrum.max_bins(n, 1))
    for r in range(reps):
        pos = synth.uniform(n_p, box, 5000 + r, np.float64)
        delta, _ = spectrum.delta_half(pos, box, n, 1, False)
        # undo the deconvolution: raw grid power
        d_raw = delta * spectrum.window(n, 1)
        _, pk, counts = spectrum.bin_power(d_raw, box, n, 1, spectrum.max_bins(n, 1))
        acc += pk
    acc /= reps
    shot = box ** 3 / n_p
    _, _, counts = spectrum.bin_power(d_raw, box, n, 1, spectrum.max_bins(n, 1))
    assert np.all(np.abs(acc / shot - 1) < 4.0 / np.sqrt(reps * counts / 2.0))


def test_shot_noise_subtraction_constant():
    pos = synth.uniform(5000, 200.0, 3, np.float64)
    _, p_raw, _ = spectrum.power(pos, 200.0, 16, 2, True)
    _, p_sub, _ = spectrum.power(pos, 200.0, 16, 2, True, subtract_shot=True)
    assert np.allclose(p_raw - p_sub, 200.0 ** 3 / 5000)


def test_k_bin_centres():
    k, _, counts = spectrum.power(synth.uniform(1000, 100.0, 1, np.float64), 100.0, 16, 2, False)
    kf = 2 * np.pi / 100.0
    centres = kf * np.arange(1, 9)
    assert np.all(np.abs(k - centres) < 0.5 * kf)


def _za_direct_vs_grid(p, il, n=32):
    box = 1000.0
    pos = synth.zeldovich(16, box, 3, dtype=np.float64)
    delta, _ = spectrum.delta_half(pos, box, n, p, il)
    mx, my, mz = spectrum.half_axes(n)
    m = np.stack(np.broadcast_arrays(mx, my, mz), axis=-1)
    m2 = (m ** 2).sum(-1)
    sel = (m2 > 0) & (m2 <= (n // 4) ** 2)
    ds = direct.delta_direct(pos, box, m[sel])
    return np.abs(delta[sel] / ds - 1)


def test_direct_summation_pcs_interlaced_beats_cic():
    # smooth Zel'dovich field, modes up to k_N/2 of a 32^3 grid
    err_pcs = _za_direct_vs_grid(4, True)
    err_cic = _za_direct_vs_grid(2, False)
    assert np.median(err_pcs) < 1e-3
    assert np.median(err_cic) > 10 * np.median(err_pcs)
