"""Pins of the oracle's assignment kernels (Sec. 2.3) and deposit (eq. delgrid).

Each check compares against something the paper or mathematics fixes, not
against the oracle itself: exact rational weights, partition of unity, the
Fourier transform of eq. intkerFT, finite differences, brute-force gather
sums with periodic images, and exact lattice identities.
"""

import numpy as np
import pytest
from scipy import integrate

from oracle import assign, direct, kernels, spectrum
import synth

ORDERS = [1, 2, 3, 4, 5, 6]


@pytest.mark.parametrize("p,u,expected", [
    # particle on a grid point: stencil cells and exact weights
    (2, 3.0, [1.0, 0.0]),
    (3, 3.0, [1 / 8, 3 / 4, 1 / 8]),
    (4, 3.0, [1 / 6, 2 / 3, 1 / 6, 0.0]),
    # particle at a cell centre (half-integer offset)
    (2, 3.5, [0.5, 0.5]),
    (3, 3.5, [0.5, 0.5, 0.0]),
    (4, 3.5, [1 / 48, 23 / 48, 23 / 48, 1 / 48]),
    (1, 3.49, [1.0]),
    # orders 5 and 6: centred quartic / quintic B-spline values at integers
    # and half-integers (p-fold convolution of the unit box)
    (5, 3.0, [1 / 384, 19 / 96, 115 / 192, 19 / 96, 1 / 384]),
    (6, 3.0, [1 / 120, 13 / 60, 11 / 20, 13 / 60, 1 / 120, 0.0]),
    (6, 3.5, [1 / 3840, 237 / 3840, 841 / 1920, 841 / 1920, 237 / 3840, 1 / 3840]),
])
def test_rational_weights(p, u, expected):
    cells, w = assign.stencil(np.array([u]), p, 16)
    nz = [x for x in expected]
    assert np.allclose(w[0], nz, rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", ORDERS)
def test_partition_of_unity(p):
    rng = np.random.default_rng(0)
    u = rng.uniform(0, 64, 5000)
    _, w = assign.stencil(u, p, 64)
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)
    # the stencil holds the whole kernel: W vanishes outside it
    for off in (-3, -2, p, p + 1):
        if p % 2 == 0:
            first = np.floor(u) - (p // 2 - 1)
        else:
            first = np.floor(u + 0.5) - (p - 1) // 2
        assert np.all(kernels.weight(p, first + off - u) == 0.0) or p == 1


@pytest.mark.parametrize("p", ORDERS)
def test_kernel_fourier_transform_is_sinc_power(p):
    """int W^(p)(s) exp(-i q s) ds = [sin(q/2)/(q/2)]^p  (eq. intkerFT, H = 1)."""
    for q in (0.3, 1.1, 2.5, np.pi, 5.0):
        def f(s):
            return kernels.weight(p, np.array([s]))[0] * np.cos(q * s)
        pts = [-3, -2.5, -2, -1.5, -1, -0.5, 0, 0.5, 1, 1.5, 2, 2.5, 3]
        val = integrate.quad(f, -3.5, 3.5, points=pts, limit=400, epsabs=1e-13)[0]
        assert val == pytest.approx(np.sinc(q / (2 * np.pi)) ** p, abs=1e-10)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_kernel_derivative_matches_finite_difference(p):
    s = np.linspace(-3.3, 3.3, 1501)
    knots = np.array([0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0])
    s = s[np.all(np.abs(np.abs(s)[:, None] - knots) > 1e-3, axis=1)]
    h = 1e-6
    fd = (kernels.weight(p, s + h) - kernels.weight(p, s - h)) / (2 * h)
    assert np.allclose(kernels.dweight(p, s), fd, atol=1e-6)


@pytest.mark.parametrize("p", ORDERS)
@pytest.mark.parametrize("il", [False, True])
def test_mass_conservation(p, il):
    pos = synth.uniform(3000, 500.0, 7, np.float64)
    r1, r2 = assign.deposit(pos, 500.0, 16, p, il)
    assert r1.sum() == pytest.approx(3000.0, rel=1e-13)
    if il:
        assert r2.sum() == pytest.approx(3000.0, rel=1e-13)


@pytest.mark.parametrize("p", ORDERS)
def test_deposit_equals_bruteforce_gather(p):
    """rho(g) = sum_j sum_images prod_i W(g_i - u_ji + n_i N), every cell x particle."""
    n, box = 8, 10.0
    rng = np.random.default_rng(p)
    pos = rng.uniform(-3.0, 13.0, size=(25, 3))  # also exercises the wrap
    r1, r2 = assign.deposit(pos, box, n, p, True)
    xw = np.mod(pos, box)
    u = xw * (n / box)
    g = np.arange(n, dtype=np.float64)
    for shift, rho in ((0.0, r1), (0.5, r2)):
        per_axis = []
        for ax in range(3):
            acc = np.zeros((len(pos), n))
            for img in (-1, 0, 1):
                s = g[None, :] + img * n - (u[:, ax, None] + shift)
                if p == 1:
                    # nearest cell, ties upward (a cell is [g - 1/2, g + 1/2))
                    acc += ((s > -0.5) & (s <= 0.5)).astype(float)
                else:
                    acc += kernels.weight(p, s)
            per_axis.append(acc)
        brute = np.einsum("jx,jy,jz->xyz", *per_axis)
        assert np.allclose(rho, brute, atol=1e-13)


def _lattice_factor(p, theta):
    # sum_n W(n) exp(-i n theta) over the integer points of the kernel
    return {1: np.ones_like(theta), 2: np.ones_like(theta),
            3: 0.75 + 0.25 * np.cos(theta), 4: 2 / 3 + np.cos(theta) / 3,
            5: 115 / 192 + 19 / 48 * np.cos(theta) + 1 / 192 * np.cos(2 * theta),
            6: 11 / 20 + 13 / 30 * np.cos(theta) + 1 / 60 * np.cos(2 * theta)}[p]


@pytest.mark.parametrize("p", ORDERS)
def test_lattice_particles_match_direct_sum(p):
    """Particles on grid points: FFT(rho1)(m) = sum_j exp(-i k.x_j) prod_i Lambda_p(2 pi m_i/N)."""
    n, box = 8, 100.0
    full = synth.lattice(n, box)
    rng = np.random.default_rng(11)
    pos = full[rng.choice(len(full), 150, replace=False)]
    r1, _ = assign.deposit(pos, box, n, p, False)
    f1 = spectrum.fft_grid(r1)
    mx, my, mz = spectrum.half_axes(n)
    modes = np.stack(np.broadcast_arrays(mx, my, mz), axis=-1).reshape(-1, 3)
    ds = direct.delta_direct(pos, box, modes) * len(pos)
    lam = np.prod(_lattice_factor(p, 2 * np.pi * modes / n), axis=1)
    assert np.allclose(f1.reshape(-1), ds * lam, atol=1e-10)


@pytest.mark.parametrize("p", ORDERS)
def test_half_lattice_interlaced_grid_matches_direct_sum(p):
    """Particles at cell centres: exp(+i pi sum m / N) FFT(rho2)(m) equals the
    direct sum at the same signed k (pins the interlace phase sign and the
    Nyquist index convention)."""
    n, box = 8, 100.0
    full = synth.half_lattice(n, box)
    rng = np.random.default_rng(12)
    pos = full[rng.choice(len(full), 150, replace=False)]
    _, r2 = assign.deposit(pos, box, n, p, True)
    f2 = spectrum.fft_grid(r2)
    mx, my, mz = spectrum.half_axes(n)
    phase = np.exp(1j * np.pi * (mx + my + mz) / n)
    modes = np.stack(np.broadcast_arrays(mx, my, mz), axis=-1).reshape(-1, 3)
    ds = direct.delta_direct(pos, box, modes) * len(pos)
    lam = np.prod(_lattice_factor(p, 2 * np.pi * modes / n), axis=1)
    assert np.allclose((phase * f2).reshape(-1), ds * lam, atol=1e-10)


@pytest.mark.parametrize("p", ORDERS)
@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_footprint_dft_matches_fft_of_deposit(p, shift):
    n, box = 12, 50.0
    pos = synth.uniform(200, box, 21 + p, np.float64)
    r1, r2 = assign.deposit(pos, box, n, p, True)
    rho = r1 if shift == 0.0 else r2
    f = spectrum.fft_grid(rho)
    rng = np.random.default_rng(5)
    idx = np.stack([rng.integers(0, n, 20), rng.integers(0, n, 20),
                    rng.integers(0, n // 2 + 1, 20)], axis=1)
    modes = np.where(idx <= n // 2, idx, idx - n)
    fp = direct.footprint_dft(pos, box, n, p, modes, shift=shift)
    assert np.allclose(f[idx[:, 0], idx[:, 1], idx[:, 2]], fp, atol=1e-10)


def test_wrap_edge_cases():
    box = 1000.0
    x = np.array([0.0, -0.0, 1000.0, -1e-300, 999.9999999999999, 2000.5, -0.25,
                  np.float32(999.99994)], dtype=np.float64)
    w = assign.wrap(x, box)
    assert np.all((w >= 0) & (w < box))
    assert w[2] == 0.0 and w[3] == 0.0
    assert w[5] == pytest.approx(0.5) and w[6] == pytest.approx(999.75)


@pytest.mark.parametrize("p", ORDERS)
@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_c_loops_match_numpy_oracle(p, shift):
    from oracle import native
    n, box = 16, 80.0
    pos = synth.uniform(3000, box, 31 + p, np.float32)
    ref = assign.deposit(pos, box, n, p, True)[0 if shift == 0.0 else 1]
    assert np.allclose(native.deposit(pos, box, n, p, shift), ref, rtol=0, atol=1e-12)
    modes = np.array([[0, 0, 0], [1, -3, 5], [8, 8, 8], [-7, 2, 0], [5, 8, 3]])
    assert np.allclose(native.footprint_dft(pos, box, n, p, modes, shift),
                       direct.footprint_dft(pos, box, n, p, modes, shift), atol=1e-9)


def test_c_delta_modes_and_power_match_numpy_oracle():
    from oracle import native
    n, box = 16, 200.0
    pos = synth.zeldovich(12, box, 4, dtype=np.float32)
    delta, _ = spectrum.delta_half(pos, box, n, 4, True)
    modes = np.array([[1, 0, 0], [8, 0, 0], [-3, 5, 7], [8, 8, 8], [0, 8, 2]])
    d = native.delta_modes(pos, box, n, 4, True, modes)
    assert np.allclose(d, delta[modes[:, 0] % n, modes[:, 1] % n, modes[:, 2]], rtol=1e-10, atol=1e-14)
    k0, p0, n0 = spectrum.power(pos, box, n, 4, True)
    k1, p1, n1 = native.power(pos, box, n, 4, True)
    assert np.array_equal(n0, n1) and np.allclose(p0, p1, rtol=1e-12)


def test_c_cell_values_and_mode_table_match_numpy_oracle():
    from oracle import native
    n, box = 16, 60.0
    pos = synth.uniform(2000, box, 8, np.float64)
    cells = np.array([[0, 0, 0], [15, 15, 15], [3, 9, 14], [8, 0, 1]])
    for shift in (0.0, 0.5):
        assert np.allclose(native.cell_values(pos, box, n, 4, cells, shift),
                           assign.cell_values(pos, box, n, 4, cells, shift), atol=1e-12)
    for nn, dk in ((32, 1), (24, 2), (16, 3)):
        nb = spectrum.max_bins(nn, dk)
        c0, k0 = spectrum.mode_table(nn, dk, nb)
        c1, k1 = native.mode_table(nn, dk, nb)
        assert np.array_equal(c0, c1) and np.allclose(k0, k1, rtol=1e-12)


# Every shift a grid of any interlacing code is sampled at (bit a of the
# mask: half a cell along axis a).
_ALL_SHIFTS = [spectrum.mask_shift(mk) for mk in range(8)]


@pytest.mark.parametrize("p", ORDERS)
def test_cell_values_match_deposit_every_order_and_shift(p):
    """assign.cell_values and the C cell_values loop, which the full-size GPU
    tests use as the reference grid values, equal the brute-force-pinned
    numpy deposit at every order and every half-cell shift."""
    from oracle import native
    n, box = 12, 60.0
    pos = synth.zeldovich(10, box, 40 + p, dtype=np.float32)
    rng = np.random.default_rng(p)
    cells = np.concatenate([np.array([[0, 0, 0], [11, 11, 11], [0, 11, 5], [6, 0, 11]]),
                            rng.integers(0, n, (12, 3))])
    every = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3)
    for sh in _ALL_SHIFTS:
        u = assign.grid_coords(pos, box, n) + sh
        ref = assign.deposit_u(u, p, n)
        assert np.allclose(native.cell_values(pos, box, n, p, every, sh),
                           ref.reshape(-1), rtol=0, atol=1e-12), sh
        assert np.allclose(assign.cell_values(pos, box, n, p, cells, sh),
                           ref[cells[:, 0], cells[:, 1], cells[:, 2]], rtol=0, atol=1e-12), sh


@pytest.mark.parametrize("p", ORDERS)
@pytest.mark.parametrize("code", [0, 1, 2, 3])
def test_delta_modes_match_delta_half_every_order_and_code(p, code):
    """native.delta_modes (footprint DFT per mode, combined and deconvolved),
    the reference of the sampled-mode GPU tests, equals the numpy oracle's
    delta on the half spectrum for every order and interlacing code."""
    from oracle import native
    n, box = 16, 150.0
    pos = synth.zeldovich(10, box, 50 + p, dtype=np.float32)
    delta, _ = spectrum.delta_half(pos, box, n, p, code)
    rng = np.random.default_rng(7 + p)
    idx = np.concatenate([np.array([[1, 0, 0], [8, 0, 0], [8, 8, 8], [0, 8, 2], [15, 9, 8]]),
                          np.stack([rng.integers(0, n, 10), rng.integers(0, n, 10),
                                    rng.integers(0, n // 2 + 1, 10)], axis=1)])
    modes = np.where(idx <= n // 2, idx, idx - n)
    got = native.delta_modes(pos, box, n, p, code, modes)
    ref = delta[idx[:, 0], idx[:, 1], idx[:, 2]]
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-13 * np.max(np.abs(ref)))


@pytest.mark.parametrize("n,p", [(12, 1), (16, 4), (20, 6), (17, 3)])
def test_deposit_slabs_equal_serial_loop(n, p):
    """The x-plane-parallel C deposit equals the serial C loop bit for bit
    (and so the numpy deposit it is pinned to)."""
    from oracle import native
    box = 70.0
    pos = synth.uniform(4000, box, 60 + p, np.float32)
    for sh in (0.0, 0.5):
        a = native.deposit(pos, box, n, p, sh)
        b = native.deposit_slabs(pos, box, n, p, sh)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("p,il", [(2, False), (4, True), (3, True)])
def test_power_large_matches_power(p, il):
    """The plane-chunked full-size oracle equals the all-at-once oracle, and
    its band of low modes equals delta on the half spectrum."""
    from oracle import native
    n, box, band = 24, 300.0, 5
    pos = synth.zeldovich(16, box, 70 + p, dtype=np.float32)
    k0, p0, n0 = spectrum.power(pos, box, n, p, il)
    k1, p1, n1, db = native.power_large(pos, box, n, p, il, planes=5, band=band)
    assert np.array_equal(n0, n1)
    assert np.allclose(p1, p0, rtol=1e-12) and np.allclose(k1, k0, rtol=1e-12)
    delta, _ = spectrum.delta_half(pos, box, n, p, il)
    for mx in range(-band, band + 1):
        for my in range(-band, band + 1):
            assert np.allclose(db[mx + band, my + band], delta[mx % n, my % n, :band + 1],
                               rtol=1e-12, atol=1e-15)
