"""GPU parity on grids whose size has factors 3 and 5 (N = 2^a 3^b 5^c, the
paper's N_G = 100 and 480), through the C ABI, against the FP64 oracle.

These sizes take the run-time-planned Stockham FFT (radix 16/8/4/2/3/5),
ragged deposit tiles (16 does not divide N) and super-buckets of a divisor of
N/4.  Tolerances as in the power-of-two parity tests: grids to 2e-6 of their
peak, mode counts bit-exact, P(k) to 1e-5 relative, delta(m) to 1e-5 (window
weighted), gradients to 1e-4 of their largest component.
"""

import numpy as np
import pytest

import oracle
from oracle import adjoint, assign, bispectrum, kernels, native, spectrum
import synth
from gpu_common import rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu

P_TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _est(n, box, p, il, batch=1, maxp=1 << 16, atomic_sort=False):
    from paper_1512_07295_amd.estimator import Estimator
    return Estimator(n, box, p, il, batch, maxp, atomic_sort=atomic_sort)


@pytest.mark.parametrize("n,p,il", [(12, 4, True), (12, 3, False), (20, 5, True), (20, 2, False),
                                    (24, 6, True), (36, 4, False), (40, 1, True), (60, 3, True),
                                    (100, 4, True), (100, 2, False), (100, 6, False)])
def test_grid_parity(torch, n, p, il):
    box = 500.0
    pos = synth.uniform(5000, box, 40 + n + p, np.float32)
    pos[:3] = [[0.0, 0.0, 0.0], [box - 1e-4, 0.5 * box, box], [-1.0, box + 2.0, 3.0]]
    est = _est(n, box, p, il, maxp=len(pos))
    est.deposit(to_dev(torch, pos))
    r1, r2 = assign.deposit(pos, box, n, p, il)
    g1 = est.copy_grid(1).cpu().numpy()
    assert np.max(np.abs(g1 - r1)) <= 2e-6 * max(1.0, r1.max())
    if il:
        g2 = est.copy_grid(2).cpu().numpy()
        assert np.max(np.abs(g2 - r2)) <= 2e-6 * max(1.0, r2.max())
    est.close()


@pytest.mark.parametrize("n,p,il", [(12, 2, True), (20, 4, False), (24, 4, True), (40, 3, False),
                                    (48, 6, True), (60, 2, True), (96, 4, True), (100, 4, True),
                                    (100, 2, False), (120, 5, False)])
def test_power_parity_uniform(torch, n, p, il):
    box = 1000.0
    pos = synth.uniform(30000, box, 200 + n + p, np.float32)
    est = _est(n, box, p, il, maxp=len(pos))
    k, pk, nm = est.power(to_dev(torch, pos))
    k0, p0, n0 = oracle.power(pos, box, n, p, il)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    assert rel_err(k.cpu().numpy()[0], k0) < 1e-12
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    est.close()


@pytest.mark.parametrize("p,il", [(4, True), (2, False), (3, True), (6, False)])
def test_power_parity_zeldovich_n100(torch, p, il):
    """The paper's grid N_G = 100 on a Zel'dovich set, plain and fused power."""
    box, n = 1000.0, 100
    pos = synth.zeldovich(40, box, 4, dtype=np.float32)
    est = _est(n, box, p, il, maxp=len(pos))
    k, pk, nm = est.power(to_dev(torch, pos))
    k0, p0, n0 = oracle.power(pos, box, n, p, il)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    # power again from the stored spectrum (run-time z pass, then binning)
    est.deposit(to_dev(torch, pos))
    est.transform()
    d = est.export_delta()
    k2, pk2, _ = est.power_only(1, n // 2)
    assert rel_err(pk2.cpu().numpy()[0], p0) < P_TOL
    ref, _ = spectrum.delta_half(pos, box, n, p, il)
    a = d.cpu().numpy()
    a = a[..., 0] + 1j * a[..., 1]
    ok = np.isfinite(ref)
    w = np.ones(ref.shape)
    mx, my, mz = spectrum.half_axes(n)
    w = (kernels.window_1d(p, mx, n) * kernels.window_1d(p, my, n) * kernels.window_1d(p, mz, n))
    w = np.broadcast_to(w, ref.shape)
    assert np.max(np.abs(a - ref)[ok] * w[ok]) <= 1e-5 * np.max(np.abs(ref[ok]) * w[ok])
    est.close()


@pytest.mark.parametrize("n,p,il", [(24, 4, True), (40, 2, False), (60, 4, True), (100, 3, False)])
def test_backward_matches_oracle_gradient(torch, n, p, il):
    box, n_bins = 1000.0, 10
    pos = synth.zeldovich(16, box, 5, dtype=np.float32)
    tgt = synth.zeldovich(16, box, 6, dtype=np.float32)
    _, target, counts = oracle.power(tgt, box, n, p, il, 1, n_bins)
    _, pk, _ = oracle.power(pos, box, n, p, il, 1, n_bins)
    _, dldp = adjoint.chi2_loss(pk, target, counts)
    est = _est(n, box, p, il, maxp=len(pos))
    g = est.backward(to_dev(torch, pos), to_dev(torch, dldp[None, :]), n_bins=n_bins).cpu().numpy()
    ref = adjoint.position_gradient(pos, box, n, p, il, 1, n_bins, dldp)
    assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))
    est.close()


@pytest.mark.parametrize("n,p,il", [(24, 4, True), (36, 2, False)])
def test_bispectrum_parity(torch, n, p, il):
    box, n_dk = 500.0, 2
    pos = synth.zeldovich(16, box, 21, dtype=np.float32)
    nb = bispectrum.max_bins(n, n_dk)
    tri = bispectrum.closed_triangles(nb)
    est = _est(n, box, p, il, maxp=len(pos))
    est.power(to_dev(torch, pos))
    bk, nt = est.bispectrum(tri, n_dk, nb)
    bk, nt = bk.cpu().numpy(), nt.cpu().numpy()
    _, b0, n0 = oracle.bispectrum_fn(pos, box, n, p, il, n_dk=n_dk, n_bins=nb, triangles=tri)
    delta, _ = spectrum.delta_half(pos, box, n, p, il)
    masks = bispectrum.shell_masks(n, n_dk, nb)
    s_abs = bispectrum.triple_sums(np.abs(bispectrum.shell_fields(delta, masks, n)), tri)
    s_jjj = bispectrum.triple_sums(bispectrum.shell_fields(np.ones_like(delta), masks, n), tri)
    scale = np.maximum(np.abs(b0), box ** 6 * s_abs / s_jjj)
    assert np.all(np.abs(nt - n0) <= 1e-5 * n0 + 1e-3)
    assert np.all(np.abs(bk - b0) <= 1e-5 * scale)
    est.close()


@pytest.mark.parametrize("n", [100, 480])
def test_two_level_and_atomic_sorts_agree(torch, n):
    """Super-bucket edges 5 (N = 100) and 15 (N = 480): same grid as the
    single-level sort, bit for bit."""
    box = 2400.0
    pos = synth.zeldovich(64, box, 9, dtype=np.float32)
    grids = []
    for atomic in (False, True):
        est = _est(n, box, 4, True, maxp=len(pos), atomic_sort=atomic)
        est.deposit(to_dev(torch, pos))
        grids.append(est.copy_grid(1).cpu().numpy())
        est.close()
    assert np.array_equal(grids[0], grids[1])


def test_direct_sum_on_mixed_grid(torch):
    """The direct-summation engine on the half spectrum of N = 20 (index
    N/2 = 10 is +N/2)."""
    from oracle import direct
    box, n = 300.0, 20
    pos = synth.uniform(3000, box, 17, np.float32)
    est = _est(n, box, 4, True, maxp=len(pos))
    d = est.direct_delta(to_dev(torch, pos)).cpu().numpy()
    d = d[..., 0] + 1j * d[..., 1]
    ref = direct.delta_half_direct(pos, box, n)
    assert np.max(np.abs(d - ref)) <= 1e-5 * np.max(np.abs(ref))
    est.close()


def test_paper_za_configuration_n480(torch):
    """The paper's Zel'dovich measurement shape: 360^3 particles, L = 2400,
    N_G = 480, PCS + interlacing.  Mode counts and mean k of all 240 shells
    (exact / 1e-10), both grids at sampled cells (tile edges, the periodic
    wrap), delta(m) at sampled modes (1e-5) and P(k) of all 240 shells
    against the full-size FP64 oracle (1e-5)."""
    box, n, p = 2400.0, 480, 4
    pos = synth.zeldovich(360, box, 11, dtype=np.float32)
    dpos = to_dev(torch, pos)
    est = _est(n, box, p, True, maxp=len(pos))
    k, pk, nm = est.power(dpos)
    counts, ksum = native.mode_table(n, 1, n // 2)
    assert np.array_equal(nm.cpu().numpy()[0], counts)
    assert rel_err(k.cpu().numpy()[0], 2 * np.pi / box * ksum / counts) < 1e-10
    _, p0, n0 = native.power_large(pos, box, n, p, True, 1, n // 2)
    assert np.array_equal(n0, counts)
    assert rel_err(pk.cpu().numpy()[0], p0) < 1e-5
    cells = np.array([[0, 0, 0], [479, 479, 479], [463, 464, 479], [464, 463, 0], [15, 16, 475],
                      [240, 239, 471], [476, 3, 468], [100, 200, 300]])
    est.deposit(dpos)
    for which, shift in ((1, 0.0), (2, 0.5)):
        g = est.copy_grid(which)
        got = g[cells[:, 0], cells[:, 1], cells[:, 2]].cpu().numpy().astype(np.float64)
        del g
        ref = native.cell_values(pos, box, n, p, cells, shift)
        assert np.all(np.abs(got - ref) <= 1e-6 + 1e-6 * np.abs(ref)), (which, got - ref)
    est.transform()
    modes = np.array([[1, 0, 0], [3, -2, 5], [240, 0, 0], [0, 240, 240], [-7, 100, 33],
                      [180, -180, 0]])
    got = est.sample_delta(modes).cpu().numpy()
    ref = native.delta_modes(pos, box, n, p, True, modes)
    # FP32 rounding is relative to the field's norm and amplified by 1/W(m)
    # (down to (2/pi)^8 at [0, 240, 240]): the bound is on |delta error| W(m)
    # against the largest |delta W| sampled
    w = np.prod([kernels.window_1d(p, modes[:, a], n) for a in range(3)], axis=0)
    assert np.max(np.abs(got - ref) * w) <= 1e-5 * np.max(np.abs(ref) * w), (got, ref)
    est.close()


def test_largest_mixed_grid_n1000(torch):
    """N = 1000 = 2^3 5^3: the longest run-time FFT plan (radix 8, 5, 5, 5 on
    63 threads per line, 1008-thread column workgroups) and ragged 8-cell last
    tiles.  P(k) and mode counts of all 500 shells against the full-size
    FP64 oracle, sampled cells of both grids and sampled delta(m) against the
    C oracle loops."""
    box, n, p = 1500.0, 1000, 4
    pos = synth.zeldovich(200, box, 13, dtype=np.float32)
    dpos = to_dev(torch, pos)
    est = _est(n, box, p, True, maxp=len(pos))
    k, pk, nm = est.power(dpos)
    counts, ksum = native.mode_table(n, 1, n // 2)
    assert np.array_equal(nm.cpu().numpy()[0], counts)
    assert rel_err(k.cpu().numpy()[0], 2 * np.pi / box * ksum / counts) < 1e-10
    _, p0, n0 = native.power_large(pos, box, n, p, True, 1, n // 2)
    assert np.array_equal(n0, counts)
    assert rel_err(pk.cpu().numpy()[0], p0) < 1e-5
    cells = np.array([[0, 0, 0], [999, 999, 999], [992, 991, 999], [991, 992, 0], [7, 8, 995],
                      [500, 499, 996], [996, 3, 992], [123, 456, 789]])
    est.deposit(dpos)
    for which, shift in ((1, 0.0), (2, 0.5)):
        g = est.copy_grid(which)
        got = g[cells[:, 0], cells[:, 1], cells[:, 2]].cpu().numpy().astype(np.float64)
        del g
        ref = native.cell_values(pos, box, n, p, cells, shift)
        assert np.all(np.abs(got - ref) <= 1e-6 + 1e-6 * np.abs(ref)), (which, got - ref)
    est.transform()
    modes = np.array([[1, 0, 0], [3, -2, 5], [500, 0, 0], [0, 500, 500], [-77, 321, 33],
                      [250, -250, 125]])
    got = est.sample_delta(modes).cpu().numpy()
    ref = native.delta_modes(pos, box, n, p, True, modes)
    w = np.prod([kernels.window_1d(p, modes[:, a], n) for a in range(3)], axis=0)
    assert np.max(np.abs(got - ref) * w) <= 1e-5 * np.max(np.abs(ref) * w), (got, ref)
    est.close()
