"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Same seeded inputs on both sides (the generators in ``synth``); the GPU reads
the float32 (or float64) positions the oracle promotes to float64.
Tolerances: mode counts bit-exact; k to 1e-12; P(k) (raw, float32 grids) to
1e-5 relative; grids to 2e-6 of their peak; delta(m) to 1e-5 of the largest
|delta| sampled.
"""

import numpy as np
import pytest

import oracle
from oracle import kernels, assign, spectrum
import synth
from gpu_common import rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu

P_TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _est(torch, n, box, p, il, batch=1, maxp=1 << 16):
    from paper_1512_07295_amd.estimator import Estimator
    return Estimator(n, box, p, il, batch, maxp)


@pytest.mark.parametrize("n", [8, 16, 32])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("il", [False, True])
def test_grid_parity(torch, n, p, il):
    box = 500.0
    pos = synth.uniform(3000, box, 10 + p, np.float32)
    est = _est(torch, n, box, p, il, maxp=len(pos))
    est.deposit(to_dev(torch, pos))
    r1, r2 = assign.deposit(pos, box, n, p, il)
    g1 = est.copy_grid(1).cpu().numpy()
    assert np.max(np.abs(g1 - r1)) <= 2e-6 * max(1.0, r1.max())
    assert abs(g1.astype(np.float64).sum() - len(pos)) < 1e-3
    if il:
        g2 = est.copy_grid(2).cpu().numpy()
        assert np.max(np.abs(g2 - r2)) <= 2e-6 * max(1.0, r2.max())
    est.close()


@pytest.mark.parametrize("n", [8, 16, 32, 64])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("il", [False, True])
def test_power_parity_uniform(torch, n, p, il):
    box = 1000.0
    pos = synth.uniform(20000, box, 100 + n + p, np.float32)
    est = _est(torch, n, box, p, il, maxp=len(pos))
    k, pk, nm = est.power(to_dev(torch, pos))
    k0, p0, n0 = oracle.power(pos, box, n, p, il)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    assert rel_err(k.cpu().numpy()[0], k0) < 1e-12
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    est.close()


@pytest.mark.parametrize("p,il", [(4, True), (2, False), (3, True), (1, False), (5, True),
                                  (6, True), (6, False)])
def test_power_parity_zeldovich_f32(torch, p, il):
    box = 1000.0
    pos = synth.zeldovich(32, box, 2, dtype=np.float32)
    n = 64
    est = _est(torch, n, box, p, il, maxp=len(pos))
    k, pk, nm = est.power(to_dev(torch, pos))
    k0, p0, n0 = oracle.power(pos, box, n, p, il)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    est.close()


@pytest.mark.parametrize("n,p,il", [(128, 4, True), (256, 4, True), (256, 3, False)])
def test_power_parity_staged_rows(torch, n, p, il):
    """Grids of 128^3 and 256^3: rows of 128 to 256 elements in the fused z
    + P(k) pass, several row groups per workgroup and a ragged last group."""
    box = 1000.0
    pos = synth.zeldovich(32, box, 9 + n, dtype=np.float32)
    est = _est(torch, n, box, p, il, maxp=len(pos))
    k0, p0, n0 = oracle.power(pos, box, n, p, il)
    for choice in (None, 0):  # default and 256 reduction workgroups
        if choice is not None:
            est.set_launch(choice)
        k, pk, nm = est.power(to_dev(torch, pos))
        assert np.array_equal(nm.cpu().numpy()[0], n0)
        assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    est.close()


@pytest.mark.parametrize("n,il,n_dk,n_bins", [(256, True, 2, 20), (256, False, 1, 100),
                                               (240, True, 3, 30)])
def test_power_few_shells_large_grid(torch, n, il, n_dk, n_bins):
    """Shells well below the Nyquist frequency on 240^3 and 256^3 grids: the
    fused pass enumerates only the row pairs inside the last shell (columns
    whose valid y wrap around in two pieces) and splits each row's modes
    below the last edge over its threads; counts exact, P within 1e-5."""
    box = 1000.0
    pos = synth.zeldovich(32, box, 19 + n, dtype=np.float32)
    est = _est(torch, n, box, 4, il, maxp=len(pos))
    k, pk, nm = est.power(to_dev(torch, pos), n_dk=n_dk, n_bins=n_bins)
    k0, p0, n0 = oracle.power(pos, box, n, 4, il, n_dk, n_bins)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    assert rel_err(k.cpu().numpy()[0], k0) < 1e-12
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    est.close()


def test_power_parity_f64_positions_cic(torch):
    """Config-1 shape: 32^3 uniform float64 particles, 32^3 grid, CIC, no interlacing."""
    box = 1000.0
    pos = synth.uniform(32 ** 3, box, 1, np.float64)
    est = _est(torch, 32, box, 2, False, maxp=len(pos))
    for sub in (False, True):
        est.deposit(to_dev(torch, pos))
        est.transform()
        k, pk, nm = est.power_only(1, 16, sub)
        k0, p0, n0 = oracle.power(pos, box, 32, 2, False, 1, 16, subtract_shot=sub)
        assert np.array_equal(nm.cpu().numpy()[0], n0)
        if sub:
            # compare raw power; the subtracted constant is exact on both sides
            assert np.allclose(pk.cpu().numpy()[0] - p0, 0, atol=P_TOL * (p0 + box ** 3 / len(pos)).max())
        else:
            assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    est.close()


@pytest.mark.parametrize("n_dk,n_bins", [(2, 8), (3, 5), (1, 7), (4, 4)])
def test_power_bins_options(torch, n_dk, n_bins):
    box = 300.0
    pos = synth.zeldovich(16, box, 5, dtype=np.float32)
    est = _est(torch, 32, box, 4, True, maxp=len(pos))
    k, pk, nm = est.power(to_dev(torch, pos), n_dk=n_dk, n_bins=n_bins)
    k0, p0, n0 = oracle.power(pos, box, 32, 4, True, n_dk, n_bins)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    assert rel_err(k.cpu().numpy()[0], k0) < 1e-12
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    # power can be called again on the same transform
    k2, pk2, _ = est.power_only(n_dk, n_bins)
    assert rel_err(pk2.cpu().numpy()[0], p0) < P_TOL
    est.close()


@pytest.mark.parametrize("p,il", [(4, True), (2, False), (3, False), (1, True), (5, True),
                                  (6, False)])
def test_sampled_delta(torch, p, il):
    box, n = 200.0, 32
    pos = synth.zeldovich(16, box, 8, dtype=np.float32)
    est = _est(torch, n, box, p, il, maxp=len(pos))
    est.deposit(to_dev(torch, pos))
    est.transform()
    rng = np.random.default_rng(3)
    modes = np.stack([rng.integers(-n // 2 + 1, n // 2 + 1, 200), rng.integers(-n // 2 + 1, n // 2 + 1, 200),
                      rng.integers(0, n // 2 + 1, 200)], axis=1)
    modes[:4] = [[n // 2, 0, 0], [0, n // 2, n // 2], [n // 2, n // 2, n // 2], [1, -1, 0]]
    d = est.sample_delta(modes).cpu().numpy()
    delta, _ = spectrum.delta_half(pos, box, n, p, il)
    ref = delta[modes[:, 0] % n, modes[:, 1] % n, modes[:, 2]]
    # FP32 grid and FFT rounding is relative to the field's norm; dividing by
    # the window W(m) (down to (2/pi)^(3p) at the Nyquist corner) scales it
    # by 1/W(m), so the bound is on |delta error| W(m)
    w = np.prod([kernels.window_1d(p, modes[:, a], n) for a in range(3)], axis=0)
    assert np.max(np.abs(d - ref) * w) <= 1e-5 * np.max(np.abs(ref) * w)
    est.close()


def test_edge_positions(torch):
    box, n = 100.0, 16
    h = box / n
    special = np.array([[0.0, 0.0, 0.0], [box, box, box], [-box / 2, 1.5 * box, 3 * box],
                        [h, 2 * h, 3 * h], [0.5 * h, 1.5 * h, 2.5 * h], [box - 1e-5, 1e-7, box / 2],
                        [-1e-6, -h, 7.0 * h]], dtype=np.float32)
    rng = np.random.default_rng(1)
    pos = np.concatenate([special, rng.uniform(-box, 2 * box, (500, 3)).astype(np.float32)])
    for p in (1, 2, 3, 4):
        est = _est(torch, n, box, p, True, maxp=len(pos))
        est.deposit(to_dev(torch, pos))
        r1, r2 = assign.deposit(pos, box, n, p, True)
        assert np.max(np.abs(est.copy_grid(1).cpu().numpy() - r1)) <= 2e-6 * r1.max()
        assert np.max(np.abs(est.copy_grid(2).cpu().numpy() - r2)) <= 2e-6 * r2.max()
        k, pk, nm = est.power(to_dev(torch, pos))
        assert rel_err(pk.cpu().numpy()[0], oracle.power(pos, box, n, p, True)[1]) < P_TOL
        est.close()


def test_single_particle_and_nonfinite(torch):
    box, n = 50.0, 8
    one = np.array([[3.3, 47.1, 0.2]], dtype=np.float32)
    est = _est(torch, n, box, 4, True, maxp=16)
    k, pk, nm = est.power(to_dev(torch, one))
    assert rel_err(pk.cpu().numpy()[0], oracle.power(one, box, n, 4, True)[1]) < P_TOL
    bad = np.array([[np.nan, 1.0, 2.0], [np.inf, -np.inf, 3.0], [1.0, 2.0, 3.0]], dtype=np.float32)
    est.deposit(to_dev(torch, bad))
    g = est.copy_grid(1).cpu().numpy()
    assert np.isfinite(g).all() and abs(g.sum() - 3.0) < 1e-5
    est.close()


def test_batched_sets_match_single(torch):
    box, n = 400.0, 32
    parts = [synth.uniform(5000, box, 40, np.float32), np.zeros((0, 3), np.float32),
             synth.uniform(777, box, 42, np.float32), synth.zeldovich(12, box, 43, dtype=np.float32),
             synth.uniform(1, box, 44, np.float32)]
    counts = [len(q) for q in parts]
    pos = np.concatenate(parts)
    offs = np.zeros(len(counts) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(counts)
    est = _est(torch, n, box, 4, True, batch=len(counts), maxp=len(pos))
    k, pk, nm = est.power(to_dev(torch, pos), offsets=to_dev(torch, offs))
    pk = pk.cpu().numpy()
    for i, part in enumerate(parts):
        if len(part) == 0:
            assert np.all(np.isnan(pk[i]))
            continue
        _, p0, n0 = oracle.power(part, box, n, 4, True)
        assert np.array_equal(nm.cpu().numpy()[i], n0)
        assert rel_err(pk[i], p0) < P_TOL
    est.close()


def test_graph_replay_matches_eager(torch):
    box, n = 400.0, 32
    pos, offs = synth.mocks(4, box, 7, n_min=2000, n_max=20000)
    est = _est(torch, n, box, 4, True, batch=4, maxp=len(pos))
    dpos, doffs = to_dev(torch, pos), to_dev(torch, offs)
    _, eager, _ = est.power(dpos, offsets=doffs)
    eager = eager.cpu().numpy()
    k, pk, nm = est.capture(dpos, offsets=doffs)
    for rep in range(3):
        est.replay()
        torch.cuda.synchronize()
        got = pk.cpu().numpy()
        assert rel_err(got, eager) < 1e-6, rep
        # unrelated eager work between replays
        est.power(dpos, offsets=doffs)
        torch.cuda.synchronize()
    for i in range(4):
        part = pos[offs[i]:offs[i + 1]]
        assert rel_err(eager[i], oracle.power(part, box, n, 4, True)[1]) < P_TOL
    est.close()


def test_autotune_keeps_results(torch):
    box, n = 400.0, 32
    pos = synth.zeldovich(16, box, 3, dtype=np.float32)
    est = _est(torch, n, box, 4, True, maxp=len(pos))
    dpos = to_dev(torch, pos)
    choice = est.autotune(dpos, iters=1)
    assert 0 <= choice < 48
    _, pk, _ = est.power(dpos)
    assert rel_err(pk.cpu().numpy()[0], oracle.power(pos, box, n, 4, True)[1]) < P_TOL
    est.close()


def test_call_order_errors(torch):
    import paper_1512_07295_amd as F
    est = _est(torch, 16, 100.0, 4, True, maxp=10)
    with pytest.raises(F.FsestError) as ei:
        est.transform()
    assert ei.value.status == F.EST_ESTATE
    with pytest.raises(F.FsestError) as ei:
        est.power_only()
    assert ei.value.status == F.EST_ESTATE
    pos = to_dev(torch, synth.uniform(10, 100.0, 1, np.float32))
    with pytest.raises(F.FsestError) as ei:
        F.estimator_deposit(est.h, pos, F.EST_F32, None, 11)
    assert ei.value.status == F.EST_EINVAL
    est.deposit(pos)
    est.transform()
    with pytest.raises(F.FsestError) as ei:
        est.power_only(1, 9)
    assert ei.value.status == F.EST_EINVAL
    with pytest.raises(F.FsestError):
        est.transform()
    est.close()


@pytest.mark.parametrize("choice", [0, 1, 2, 3, 4, 7, 13, 24, 47])
def test_every_launch_variant_matches_oracle(torch, choice):
    """Each autotuner candidate (FFT lines per workgroup, reduction blocks,
    deposit workgroup size, 32/64-bit fixed point, tiles grouped per XCD)."""
    box, n = 300.0, 32
    pos = synth.zeldovich(16, box, 11, dtype=np.float32)
    est = _est(torch, n, box, 4, True, maxp=len(pos))
    est.set_launch(choice)
    est.deposit(to_dev(torch, pos))
    r1, r2 = assign.deposit(pos, box, n, 4, True)
    assert np.max(np.abs(est.copy_grid(1).cpu().numpy() - r1)) <= 2e-6 * r1.max()
    assert np.max(np.abs(est.copy_grid(2).cpu().numpy() - r2)) <= 2e-6 * r2.max()
    _, pk, _ = est.power(to_dev(torch, pos))
    assert rel_err(pk.cpu().numpy()[0], oracle.power(pos, box, n, 4, True)[1]) < P_TOL
    est.close()


@pytest.mark.parametrize("p", [4, 6])
def test_clustered_input_uses_wide_fixed_point(torch, p):
    """A dense clump (thousands of particles in one bucket) exceeds the 32-bit
    fixed-point bound and must go through the 64-bit path (p = 6 also checks
    the 64-bit layout's margin for the widest stencil)."""
    box, n = 100.0, 32
    rng = np.random.default_rng(4)
    clump = (37.1 + 0.3 * rng.random((6000, 3))).astype(np.float32)
    pos = np.concatenate([clump, synth.uniform(4000, box, 5, np.float32)])
    for choice in (0, 2):
        est = _est(torch, n, box, p, True, maxp=len(pos))
        est.set_launch(choice)
        est.deposit(to_dev(torch, pos))
        r1, r2 = assign.deposit(pos, box, n, p, True)
        assert np.max(np.abs(est.copy_grid(1).cpu().numpy() - r1)) <= 2e-6 * r1.max()
        assert np.max(np.abs(est.copy_grid(2).cpu().numpy() - r2)) <= 2e-6 * r2.max()
        _, pk, _ = est.power(to_dev(torch, pos))
        assert rel_err(pk.cpu().numpy()[0], oracle.power(pos, box, n, p, True)[1]) < P_TOL
        est.close()


@pytest.mark.parametrize("choice", [2, 7, 4, None])
def test_dense_tiles_deposit_their_item_list_several_times(torch, choice):
    """About 2 x 6300 work items per 16^3 tile, several times the item list:
    the list is deposited whenever a round of candidates would overflow it and
    after the last round.  Choices: 512-thread workgroups (2), 1024-thread
    workgroups with registers capped for two per CU (7), the 64-bit kernel
    (4), the default shapes (None); the 32-bit format holds here (F = 24)."""
    box, n = 100.0, 32
    pos = synth.uniform(30000, box, 12, np.float32)
    est = _est(torch, n, box, 4, True, maxp=len(pos))
    if choice is not None:
        est.set_launch(choice)
    est.deposit(to_dev(torch, pos))
    r1, r2 = assign.deposit(pos, box, n, 4, True)
    assert np.max(np.abs(est.copy_grid(1).cpu().numpy() - r1)) <= 2e-6 * r1.max()
    assert np.max(np.abs(est.copy_grid(2).cpu().numpy() - r2)) <= 2e-6 * r2.max()
    est.close()


@pytest.mark.parametrize("choice", [7, 4])
def test_dense_buckets_keep_the_32_bit_format_down_to_22_bits(torch, choice):
    """80000 particles on 32^3 (about 160 per 4^3 bucket, at most ~200): the
    bound 8 M (w_max^3 2^F + 1/2) < 2^32 gives F = 23 for PCS, below 24 but
    above the 22-bit minimum, so the 32-bit kernel deposits (choice 7); the
    64-bit kernel (choice 4) gives the same grids within the same tolerance."""
    box, n = 100.0, 32
    pos = synth.uniform(80000, box, 14, np.float32)
    est = _est(torch, n, box, 4, True, maxp=len(pos))
    est.set_launch(choice)
    est.deposit(to_dev(torch, pos))
    r1, r2 = assign.deposit(pos, box, n, 4, True)
    assert np.max(np.abs(est.copy_grid(1).cpu().numpy() - r1)) <= 2e-6 * r1.max()
    assert np.max(np.abs(est.copy_grid(2).cpu().numpy() - r2)) <= 2e-6 * r2.max()
    _, pk, _ = est.power(to_dev(torch, pos))
    assert rel_err(pk.cpu().numpy()[0], oracle.power(pos, box, n, 4, True)[1]) < P_TOL
    est.close()


@pytest.mark.parametrize("n,p", [(16, 1), (16, 2), (32, 1), (32, 2), (32, 4), (24, 1), (24, 2),
                                 (40, 4)])
@pytest.mark.parametrize("choice", [None, 42])
def test_register_capped_deposit_kernels(torch, n, p, choice):
    """The interlaced-pair kernels built for two 1024-thread workgroups per CU
    (orders 1, 2 and 4; the grid as one tile, a power-of-two grid, any other
    N) at their default shapes and with 512-thread workgroups (42), which runs
    the uncapped build of the same kernel.  14 particles per 4^3-cell bucket
    on average keep the 32-bit format (F >= 24 for these seeds)."""
    box = 400.0
    pos = synth.uniform(14 * (n // 4) ** 3, box, 200 + n + p, np.float32)
    est = _est(torch, n, box, p, True, maxp=len(pos))
    if choice is not None:
        est.set_launch(choice)
    est.deposit(to_dev(torch, pos))
    r1, r2 = assign.deposit(pos, box, n, p, True)
    assert np.max(np.abs(est.copy_grid(1).cpu().numpy() - r1)) <= 2e-6 * r1.max()
    assert np.max(np.abs(est.copy_grid(2).cpu().numpy() - r2)) <= 2e-6 * r2.max()
    est.close()


def test_deposit_is_bitwise_reproducible(torch):
    box, n = 200.0, 32
    pos = to_dev(torch, synth.uniform(50000, box, 6, np.float32))
    est = _est(torch, n, box, 4, True, maxp=50000)
    est.deposit(pos)
    a = est.copy_grid(1).cpu().numpy().copy()
    b = est.copy_grid(2).cpu().numpy().copy()
    for _ in range(3):
        est.deposit(pos)
        assert np.array_equal(est.copy_grid(1).cpu().numpy(), a)
        assert np.array_equal(est.copy_grid(2).cpu().numpy(), b)
    est.close()


@pytest.mark.parametrize("n,batch", [(16, 1), (64, 1), (128, 1), (128, 3)])
def test_two_level_and_atomic_sorts_give_identical_grids(torch, n, batch):
    """The default two-level bucket sort (super-buckets of 16^3 buckets) and
    the counting sort with device-scope atomics order particles differently
    inside buckets, but integer fixed-point sums make the grids bitwise
    equal; both match the oracle."""
    from paper_1512_07295_amd.estimator import Estimator
    box = 500.0
    if batch == 1:
        pos = synth.zeldovich(32, box, 13, dtype=np.float32)
        offs = None
    else:
        pos, offs = synth.mocks(batch, box, 31, n_min=2000, n_max=40000)
    grids = []
    for atomic in (False, True):
        est = Estimator(n, box, 4, True, batch, len(pos), atomic_sort=atomic)
        est.deposit(to_dev(torch, pos), offsets=None if offs is None else to_dev(torch, offs))
        grids.append([est.copy_grid(w, m).cpu().numpy().copy()
                      for m in range(batch) for w in (1, 2)])
        est.close()
    for a, b in zip(*grids):
        assert np.array_equal(a, b)
    s0 = 0 if offs is None else int(offs[0])
    s1 = len(pos) if offs is None else int(offs[1])
    r1, r2 = assign.deposit(pos[s0:s1], box, n, 4, True)
    assert np.max(np.abs(grids[0][0] - r1)) <= 2e-6 * r1.max()
    assert np.max(np.abs(grids[0][1] - r2)) <= 2e-6 * r2.max()
