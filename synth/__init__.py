"""Seeded synthetic particle sets shared by the tests, the bench and the oracle.

This module only draws inputs: it holds none of the estimator's arithmetic.
It stands in for the paper's missing data sets (the N-body test simulation and
the Zel'dovich-approximation realisations of Sec. 3.2-3.3) with inputs of the
same kind:

* ``uniform``: N_P positions uniform in the periodic box (shot-noise regime).
* ``lattice`` / ``half_lattice``: particles exactly on grid points / cell
  centres (exact test cases).
* ``zeldovich``: a cubic Lagrangian lattice displaced by a Gaussian
  displacement field Psi(k) = i k/k^2 delta_L(k), delta_L with power
  P(k) = A k^slope (slope -1.5 by default).  A is fixed so that the
  *expected* per-component rms displacement equals ``rms_frac`` times the
  lattice spacing (independent of the seed); k = 0 and every mode with a
  component at the lattice Nyquist index are zeroed.  Particles come in
  lattice order (i, j, l), l fastest.
* ``mocks``: a batch of mocks with Poisson counts drawn around log-uniform
  means in [n_min, n_max]; even mocks uniform, odd mocks Zel'dovich with
  n_i = round(N_i^(1/3)) per side (then N_i = n_i^3).

Every generator uses numpy's PCG64 ``default_rng(seed)`` in float64 and casts
once at the end.
"""

import numpy as np
import scipy.fft


def uniform(n_particles, box, seed, dtype=np.float32):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, box, size=(n_particles, 3)).astype(dtype)


def lattice(n_side, box, dtype=np.float64, offset=0.0):
    """Particles at (g + offset) * box / n_side, g on the n_side^3 lattice."""
    g = np.arange(n_side, dtype=np.float64) + offset
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    return (q * (box / n_side)).astype(dtype)


def half_lattice(n_side, box, dtype=np.float64):
    return lattice(n_side, box, dtype, offset=0.5)


def _lattice_freqs(n):
    k = np.fft.fftfreq(n, d=1.0 / n)  # integer frequencies, n/2 -> -n/2
    kz = np.arange(n // 2 + 1, dtype=np.float64)
    return k[:, None, None], k[None, :, None], kz[None, None, :]


def zeldovich(n_side, box, seed, slope=-1.5, rms_frac=0.3, dtype=np.float32):
    """Zel'dovich-displaced lattice of n_side^3 particles (see module doc)."""
    n = n_side
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    wk = scipy.fft.rfftn(white, workers=-1)
    del white
    kx, ky, kz = _lattice_freqs(n)
    k2 = kx * kx + ky * ky + kz * kz
    keep = (k2 > 0) & (np.abs(kx) != n // 2) & (np.abs(ky) != n // 2) & (kz != n // 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where(keep, np.sqrt(np.where(k2 > 0, k2, 1.0) ** (0.5 * slope)) / np.where(k2 > 0, k2, 1.0), 0.0)
    # expected per-component variance of Psi_x for unit A: E|w_k|^2 = n^3, and
    # the half spectrum counts each pair twice except the kz = 0 plane
    wz = np.full(n // 2 + 1, 2.0)
    wz[0] = 1.0
    var_x = float(np.sum((wz[None, None, :] * (amp * kx) ** 2))) / n ** 3
    spacing = box / n
    scale = rms_frac * spacing / np.sqrt(var_x)
    g = np.arange(n, dtype=np.float64) * spacing
    out = np.empty((n, n, n, 3), dtype=np.float64)
    comps = [kx, ky, kz]
    for ax in range(3):
        psi_k = 1j * comps[ax] * amp * wk * scale
        psi = scipy.fft.irfftn(psi_k, s=(n, n, n), workers=-1)
        del psi_k
        shape = [1, 1, 1]
        shape[ax] = n
        out[..., ax] = psi + g.reshape(shape)
    del wk
    out = np.mod(out, box)
    return out.reshape(-1, 3).astype(dtype)


def mock_counts(n_mocks, seed, n_min=100_000, n_max=4_000_000):
    """Poisson counts around log-uniform means, clipped; odd mocks cubed."""
    rng = np.random.default_rng(seed)
    lam = np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=n_mocks))
    counts = np.clip(rng.poisson(lam), n_min, n_max).astype(np.int64)
    for i in range(1, n_mocks, 2):
        side = int(round(counts[i] ** (1.0 / 3.0)))
        counts[i] = side ** 3
    return counts


def mocks(n_mocks, box, seed0, n_min=100_000, n_max=4_000_000, dtype=np.float32):
    """Concatenated positions of a batch of mocks and int64 offsets[n_mocks+1]."""
    counts = mock_counts(n_mocks, seed0, n_min, n_max)
    parts = []
    for i, c in enumerate(counts):
        if i % 2 == 0:
            parts.append(uniform(int(c), box, seed0 + 1 + i, dtype))
        else:
            side = int(round(c ** (1.0 / 3.0)))
            parts.append(zeldovich(side, box, seed0 + 1 + i, dtype=dtype))
    offsets = np.zeros(n_mocks + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    return np.concatenate(parts, axis=0), offsets
