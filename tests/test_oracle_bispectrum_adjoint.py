"""Pins of the FFT-shell bispectrum (Sec. 4.1) and of the P(k) adjoint.

* N_tri from the FFT-shell fields J_b equals a brute-force count of closed
  triplets q1 + q2 + q3 = 0 with q_i in shell b_i (the normalisation V_B of
  eq. VBest, up to k_f^6).
* sum_x I I I / N^3 equals the brute-force sum of delta delta delta over the
  same triplets (eq. Best evaluated by its definition).
* The closed-triangle list follows the ordering of Sec. 4.2.
* The adjoint equals central finite differences of the oracle's own forward
  loss in float64.
"""

import numpy as np
import pytest

from oracle import adjoint, bispectrum, spectrum
import synth


def _shell_modes(n, n_dk, b):
    m = spectrum.signed_index(n)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    q = np.stack([mx, my, mz], -1).reshape(-1, 3)
    m2 = (q * q).sum(1)
    sel = (m2 > 0) & (spectrum.bin_index(m2, n_dk) == b)
    return q[sel]


def _delta_full(delta_half, q, n):
    """delta at signed mode q from the half spectrum (Hermitian completion)."""
    out = np.empty(len(q), dtype=np.complex128)
    for i, (a, b, c) in enumerate(q):
        if c >= 0:
            out[i] = delta_half[a % n, b % n, c]
        else:
            out[i] = np.conj(delta_half[(-a) % n, (-b) % n, -c])
    return out


def _brute_triplets(n, n_dk, tri, delta_half=None):
    counts, sums = [], []
    for b1, b2, b3 in tri:
        q1 = _shell_modes(n, n_dk, b1)
        q2 = _shell_modes(n, n_dk, b2)
        q3 = -(q1[:, None, :] + q2[None, :, :])
        m2 = (q3 * q3).sum(-1)
        ok = (m2 > 0) & (spectrum.bin_index(m2, n_dk) == b3)
        counts.append(int(ok.sum()))
        if delta_half is not None:
            i1, i2 = np.nonzero(ok)
            d1 = _delta_full(delta_half, q1[i1], n)
            d2 = _delta_full(delta_half, q2[i2], n)
            d3 = _delta_full(delta_half, q3[i1, i2], n)
            sums.append((d1 * d2 * d3).sum())
    return np.array(counts), np.array(sums)


def test_triangle_counts_lists():
    assert len(bispectrum.closed_triangles(4)) == 17
    assert len(bispectrum.closed_triangles(32)) == 3384
    tri = bispectrum.closed_triangles(9)
    assert np.all(tri[:, 0] >= tri[:, 1]) and np.all(tri[:, 1] >= tri[:, 2])
    assert np.all(tri[:, 0] <= tri[:, 1] + tri[:, 2])
    assert bispectrum.max_bins(1024, 2) == 170 and bispectrum.max_bins(256, 2) == 42


def test_ntri_matches_bruteforce_16():
    n, n_dk = 16, 2
    tri = np.array([(1, 1, 1), (2, 1, 1), (2, 2, 1), (2, 2, 2)], dtype=np.int32)
    brute, _ = _brute_triplets(n, n_dk, tri)
    assert brute.tolist() == [3798, 4418, 17508, 39504]
    masks = bispectrum.shell_masks(n, n_dk, 2)
    j = bispectrum.shell_fields(np.ones(masks.shape[1:], dtype=np.complex128), masks, n)
    ntri = bispectrum.triple_sums(j, tri) / n ** 3
    assert np.allclose(ntri, brute, atol=1e-6)


@pytest.mark.parametrize("n,p,il", [(12, 4, True), (16, 2, False), (16, 3, True)])
def test_fft_shell_sum_matches_bruteforce_triplets(n, p, il):
    n_dk = 2
    box = 300.0
    pos = synth.zeldovich(8, box, 9, dtype=np.float64)
    delta, _ = spectrum.delta_half(pos, box, n, p, il)
    nb = bispectrum.max_bins(n, n_dk)
    tri = bispectrum.closed_triangles(nb)
    counts, sums = _brute_triplets(n, n_dk, tri, delta)
    masks = bispectrum.shell_masks(n, n_dk, nb)
    i_f = bispectrum.shell_fields(delta, masks, n)
    s_iii = bispectrum.triple_sums(i_f, tri) / n ** 3
    assert np.allclose(np.imag(sums), 0, atol=1e-12 * np.abs(sums).max())
    assert np.allclose(s_iii, np.real(sums), rtol=1e-9, atol=1e-12 * np.abs(sums).max())
    t, bk, ntri = bispectrum.bispectrum(pos, box, n, p, il, n_dk=n_dk)
    assert np.allclose(ntri, counts, atol=1e-6)
    assert np.allclose(bk, box ** 6 * np.real(sums) / counts, rtol=1e-9)


@pytest.mark.parametrize("p,il", [(4, True), (3, True), (2, False), (4, False), (4, 2), (2, 3)])
def test_adjoint_matches_finite_differences(p, il):
    n, box, n_dk, nb = 8, 100.0, 1, 4
    pos = synth.uniform(40, box, 77 + p, np.float64)
    tgt_pos = synth.uniform(40, box, 99, np.float64)
    _, target, counts = spectrum.power(tgt_pos, box, n, p, il, n_dk, nb)

    def loss(x):
        _, pk, _ = spectrum.power(x, box, n, p, il, n_dk, nb)
        return adjoint.chi2_loss(pk, target, counts)

    _, dldp = loss(pos)
    grad = adjoint.position_gradient(pos, box, n, p, il, n_dk, nb, dldp)
    h = 1e-5 * box / n
    rng = np.random.default_rng(1)
    for j in rng.choice(len(pos), 8, replace=False):
        for ax in range(3):
            xp = pos.copy()
            xm = pos.copy()
            xp[j, ax] += h
            xm[j, ax] -= h
            fd = (loss(xp)[0] - loss(xm)[0]) / (2 * h)
            scale = np.abs(grad).max()
            assert abs(fd - grad[j, ax]) < 1e-5 * scale + 1e-6 * abs(fd), (j, ax, fd, grad[j, ax])


def test_band_brute_triplets_match_fft_shell_sums():
    """oracle.bispectrum.brute_triplets (enumeration over a band of delta,
    the reference of the full-size bispectrum spot checks) equals the
    FFT-shell triple sums / N^3 and the counts of the J fields."""
    n, box, n_dk, band = 24, 300.0, 2, 7
    pos = synth.zeldovich(16, box, 9, dtype=np.float32)
    delta, _ = spectrum.delta_half(pos, box, n, 4, True)
    d_band = np.zeros((2 * band + 1, 2 * band + 1, band + 1), dtype=np.complex128)
    for mx in range(-band, band + 1):
        for my in range(-band, band + 1):
            d_band[mx + band, my + band] = delta[mx % n, my % n, :band + 1]
    tri = np.array([[1, 1, 1], [2, 1, 1], [2, 2, 1], [3, 2, 1], [3, 3, 2], [3, 3, 3]], dtype=np.int32)
    cnt, s, a = bispectrum.brute_triplets(d_band, band, n_dk, tri)
    masks = bispectrum.shell_masks(n, n_dk, 3)
    fi = bispectrum.shell_fields(delta, masks, n)
    fj = bispectrum.shell_fields(np.ones_like(delta), masks, n)
    assert np.allclose(cnt, bispectrum.triple_sums(fj, tri) / n ** 3, rtol=0, atol=1e-6)
    s_fft = bispectrum.triple_sums(fi, tri) / n ** 3
    assert np.all(np.abs(s.imag) <= 1e-12 * a)
    assert np.allclose(s.real, s_fft, rtol=1e-10, atol=1e-12 * np.max(a))
