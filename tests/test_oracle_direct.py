"""Pins of the oracle's direct-summation half spectrum and cross binning
(Sec. 2.2, eq. deltaDS; Sec. 3.2, P_{G-DS}).

Each check is fixed by something other than the function under test: a
closed form for lattices, a pure-Python sum over particles and modes, exact
identities of the binning, and the white-noise expectation.
"""

import cmath
import math

import numpy as np
import pytest

from oracle import direct, spectrum
import synth


@pytest.mark.parametrize("n,n_p,offset", [(8, 4, (0.0, 0.0, 0.0)), (16, 4, (0.25, 0.5, 0.125)),
                                          (16, 8, (0.5, 0.5, 0.5)), (12, 4, (0.25, 0.5, 0.125)),
                                          (20, 5, (0.5, 0.2, 0.0))])
def test_lattice_closed_form(n, n_p, offset):
    """n_p^3 particles at (i + o) L / n_p: delta(m) = exp(-2 pi i m.o / n_p) if
    every component of m is a multiple of n_p, else 0."""
    box = 300.0
    g = (np.arange(n_p)[:, None] + np.asarray(offset)[None, :]) * box / n_p
    pos = np.stack(np.meshgrid(g[:, 0], g[:, 1], g[:, 2], indexing="ij"), -1).reshape(-1, 3)
    d = direct.delta_half_direct(pos, box, n)
    mx, my, mz = spectrum.half_axes(n)
    mx, my, mz = np.broadcast_arrays(mx, my, mz)
    on = (mx % n_p == 0) & (my % n_p == 0) & (mz % n_p == 0)
    phase = np.exp(-2j * np.pi * (mx * offset[0] + my * offset[1] + mz * offset[2]) / n_p)
    expect = np.where(on, phase, 0.0)
    assert np.max(np.abs(d - expect)) < 1e-12


def test_brute_force_three_particles():
    """Pure-Python sum over particles and every half-spectrum mode."""
    n, box = 8, 50.0
    pos = np.array([[1.3, 47.9, 20.0], [49.99, 0.01, 33.3], [-3.0, 61.0, 12.5]])
    d = direct.delta_half_direct(pos, box, n)
    for ix in range(n):
        for iy in range(n):
            for mz in range(n // 2 + 1):
                mx = ix if ix <= n // 2 else ix - n
                my = iy if iy <= n // 2 else iy - n
                s = 0j
                for x, y, z in pos:
                    s += cmath.exp(-2j * math.pi * (mx * x + my * y + mz * z) / box)
                assert abs(d[ix, iy, mz] - s / 3) < 1e-12


def test_agrees_with_sampled_direct_sum():
    """The half spectrum at sampled modes equals the per-mode direct sum.
    Index N/2 holds m = +N/2: off the grid points exp(-i k x) differs
    between +N/2 and -N/2, so the convention is part of the output."""
    pos = synth.uniform(2000, 100.0, 3)
    d = direct.delta_half_direct(pos, 100.0, 16)
    modes = [(1, 2, 3), (-5, 8, 0), (8, 8, 8), (0, 0, 7), (-7, -1, 8)]
    ref = direct.delta_direct(pos, 100.0, modes)
    for (mx, my, mz), r in zip(modes, ref):
        assert abs(d[mx % 16, my % 16, mz] - r) < 1e-12


def test_cross_binning_single_mode():
    """A field with one non-zero mode puts V w |a|^2 / N_b in its shell only."""
    n, box, n_bins = 16, 200.0, 8
    a = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    a[3, 1, 2] = 0.3 - 0.4j  # m = (3, 1, 2), |m|^2 = 14, shell 4 (rule (2b-1)^2 <= 4|m|^2)
    k, p, cnt = spectrum.bin_cross(a, a, box, n, 1, n_bins)
    b = 4
    assert p[b - 1] == pytest.approx(box ** 3 * 2 * 0.25 / cnt[b - 1], rel=1e-14)
    assert np.all(np.delete(p, b - 1) == 0.0)
    assert cnt[b - 1] > 0


def test_cross_binning_phase_rotation_and_shot():
    """P_{a, a e^{i phi}} = cos(phi) P_{a a}, and shot shifts every shell."""
    n, box = 16, 200.0
    rng = np.random.default_rng(5)
    a = rng.standard_normal((n, n, n // 2 + 1)) + 1j * rng.standard_normal((n, n, n // 2 + 1))
    phi = 0.7
    _, paa, _ = spectrum.bin_cross(a, a, box, n, 1, 8)
    _, pab, _ = spectrum.bin_cross(a, a * np.exp(1j * phi), box, n, 1, 8)
    _, pshot, _ = spectrum.bin_cross(a, a, box, n, 1, 8, shot=3.5)
    assert np.allclose(pab, math.cos(phi) * paa, rtol=1e-12, atol=0)
    assert np.allclose(pshot, paa - 3.5, rtol=0, atol=1e-9 * np.max(np.abs(paa)))


def test_direct_power_of_uniform_particles_is_shot_noise():
    """Uniform random particles: <V |delta_DS|^2> = V / N_P in every shell
    (Sec. 2.2, the self-correlation term), within the scatter of N_b modes."""
    box, n, n_p = 100.0, 16, 3000
    pos = synth.uniform(n_p, box, 11)
    d = direct.delta_half_direct(pos, box, n)
    _, p, cnt = spectrum.bin_cross(d, d, box, n, 1, 8)
    shot = box ** 3 / n_p
    # |delta|^2 of independent modes is exponential: relative scatter 1/sqrt(N_b)
    sel = cnt > 200
    assert np.all(np.abs(p[sel] / shot - 1) < 5 / np.sqrt(cnt[sel] / 2))
