"""Parity at the full workload sizes, in the launch configuration the bench
times (autotuned the same way), on outputs the oracle can reach:

* headline (512^3 Zel'dovich particles, L = 2000, 1024^3 grid, PCS +
  interlacing): P(k), mode counts and mean k of all 512 shells from the fused
  pass the bench times, against the FP64 oracle run at full size (1e-5 /
  exact / 1e-10), both grids at sampled cells (tile corners, faces, the periodic wrap), and
  delta(m) at sampled modes including Bragg peaks of the particle lattice on
  the Nyquist planes (1e-5 relative); the same particles and grid with
  NGP, CIC and TSC, with and without interlacing (sampled cells and modes);
  P(k) and the adjoint with both strided-FFT workgroup shapes; a batch of
  two sets on 1024^3 grids against each set alone;
* 256^3 particles on a 256^3 grid: all 128 P(k) shells (1e-5) and every
  one of the 3,384 closed bispectrum triangles of 2 k_f shells up to k_N/2
  (tolerance relative to the L1 scale of the summands);
* 64 uneven mocks on 128^3 grids replayed as one graph: every mock;
* adjoint: 128^3 particles on a 256^3 grid.

The oracle uses its C loops (oracle/native.py) for the large deposits and
sampled sums; at 1024^3 it deposits with the x-plane-parallel loop, keeps
FFT(rho_1) while rho_2 is transformed and bins x-plane chunks
(``native.power_large``), about 40 GB of host memory.
"""

import numpy as np
import pytest

from oracle import adjoint, bispectrum, native, spectrum
import synth
from gpu_common import rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu

P_TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def headline(torch):
    from paper_1512_07295_amd.estimator import Estimator
    pos = synth.zeldovich(512, 2000.0, 3, dtype=np.float32)
    dpos = to_dev(torch, pos)
    est = Estimator(1024, 2000.0, 4, True, 1, len(pos))
    est.autotune(dpos, n_bins=512, iters=1)
    yield pos, dpos, est
    est.close()


@pytest.fixture(scope="module")
def headline_oracle(headline):
    """The FP64 oracle's P(k) of the headline workload at full size, and its
    delta on the modes with every |m_a| <= 17 (shells up to 8 of width 2 k_f)."""
    pos, _, _ = headline
    return native.power_large(pos, 2000.0, 1024, 4, True, 1, 512, band=17)


def test_headline_power_all_shells(torch, headline, headline_oracle):
    """P(k) of all 512 shells from the fused z-FFT + interlace + deconvolve +
    bin pass (k_pairs<1024, true, 0>, launch shapes autotuned as the bench
    does) against the full-size FP64 oracle: counts exact, P within 1e-5."""
    pos, dpos, est = headline
    k, pk, nm = est.power(dpos, n_bins=512)
    k0, p0, n0, _ = headline_oracle
    counts, ksum = native.mode_table(1024, 1, 512)
    assert np.array_equal(nm.cpu().numpy()[0], counts)
    assert np.array_equal(n0, counts)
    # FP64 sums of up to 3.3M terms in different orders: |error| <= n eps ~ 4e-10
    assert rel_err(k.cpu().numpy()[0], 2 * np.pi / 2000.0 * ksum / counts) < 1e-10
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL


def test_headline_bispectrum_every_triangle(torch, headline, headline_oracle):
    """The bispectrum of the headline workload: 128 shells of 2 k_f (up to
    k_N/2 of the 1024^3 grid), all 185,056 closed triangles
    in one call (fields on the alias-free 800^3 grid).  Spot triangles with
    every shell inside |m| < 17 against a brute-force enumeration of the
    closed triplets with the full-size oracle's delta (N_tri exact, B within
    1e-5 of max(|B|, V^2 sum |delta delta delta| / N_tri)); a second call,
    which reuses the handle's count sums, gives the same values."""
    pos, dpos, est = headline
    box, nb, n_dk = 2000.0, 128, 2
    est.deposit(dpos)
    est.transform()
    tri = bispectrum.closed_triangles(nb)
    assert len(tri) == 185056
    bk, nt = est.bispectrum(tri, n_dk, nb)
    bk, nt = bk.cpu().numpy(), nt.cpu().numpy()
    assert np.all(nt >= 0.5) and np.all(np.isfinite(bk))
    spot = np.array([[1, 1, 1], [2, 1, 1], [2, 2, 2], [3, 2, 1], [3, 3, 3], [4, 2, 2], [5, 3, 2],
                     [6, 6, 1], [7, 4, 3], [8, 4, 4], [8, 5, 4], [8, 8, 1], [8, 8, 8]], dtype=np.int32)
    where = {tuple(t): i for i, t in enumerate(tri.tolist())}
    idx = np.array([where[tuple(t)] for t in spot.tolist()])
    cnt, s3, a3 = bispectrum.brute_triplets(headline_oracle[3], 17, n_dk, spot)
    v2 = box ** 6
    b0 = v2 * s3.real / cnt
    scale = np.maximum(np.abs(b0), v2 * a3 / cnt)
    assert np.all(np.abs(nt[idx] - cnt) <= 1e-5 * cnt + 1e-3), (nt[idx], cnt)
    assert np.all(np.abs(bk[idx] - b0) <= 1e-5 * scale), (bk[idx], b0)
    bk2, nt2 = est.bispectrum(tri, n_dk, nb)
    assert np.array_equal(bk2.cpu().numpy(), bk) and np.array_equal(nt2.cpu().numpy(), nt)


def test_headline_sampled_cells(torch, headline):
    pos, dpos, est = headline
    rng = np.random.default_rng(0)
    cells = np.concatenate([
        np.array([[0, 0, 0], [1023, 1023, 1023], [15, 16, 31], [16, 15, 0], [512, 511, 1023],
                  [0, 1023, 16], [31, 32, 47], [1008, 15, 16]]),
        rng.integers(0, 1024, (8, 3))])
    est.deposit(dpos)
    for which, shift in ((1, 0.0), (2, 0.5)):
        g = est.copy_grid(which)
        got = g[cells[:, 0], cells[:, 1], cells[:, 2]].cpu().numpy().astype(np.float64)
        del g
        ref = native.cell_values(pos, 2000.0, 1024, 4, cells, shift)
        assert np.all(np.abs(got - ref) <= 1e-6 + 1e-6 * np.abs(ref)), (which, got - ref)


def test_headline_sampled_modes(torch, headline):
    pos, dpos, est = headline
    est.deposit(dpos)
    est.transform()
    modes = np.array([[1, 0, 0], [3, -2, 5], [512, 0, 0], [0, 512, 512], [-7, 100, 33],
                      [512, 512, 512]])
    got = est.sample_delta(modes).cpu().numpy()
    ref = native.delta_modes(pos, 2000.0, 1024, 4, True, modes)
    assert np.all(np.abs(got - ref) <= 1e-5 * np.abs(ref) + 1e-10), (got, ref)


@pytest.mark.parametrize("p,il", [(1, False), (2, False), (2, True), (3, True)])
def test_headline_other_orders_sampled(torch, headline, p, il):
    """The headline particles and grid with the other assignment orders, with
    and without interlacing: sampled cells of every grid and sampled delta(m)
    (window-weighted bound) against the C oracle loops."""
    from paper_1512_07295_amd.estimator import Estimator
    pos, dpos, _ = headline
    est = Estimator(1024, 2000.0, p, il, 1, len(pos))
    cells = np.array([[0, 0, 0], [1023, 1023, 1023], [15, 16, 31], [512, 511, 1023],
                      [1008, 15, 16], [300, 700, 900]])
    est.deposit(dpos)
    for which, shift in ((1, 0.0), (2, 0.5))[: 2 if il else 1]:
        g = est.copy_grid(which)
        got = g[cells[:, 0], cells[:, 1], cells[:, 2]].cpu().numpy().astype(np.float64)
        del g
        ref = native.cell_values(pos, 2000.0, 1024, p, cells, shift)
        assert np.all(np.abs(got - ref) <= 1e-6 + 1e-6 * np.abs(ref)), (which, got - ref)
    est.transform()
    modes = np.array([[1, 0, 0], [3, -2, 5], [512, 0, 0], [0, 512, 512], [-7, 100, 33]])
    got = est.sample_delta(modes).cpu().numpy()
    ref = native.delta_modes(pos, 2000.0, 1024, p, il, modes)
    from oracle import kernels
    w = np.prod([kernels.window_1d(p, modes[:, a], 1024) for a in range(3)], axis=0)
    assert np.max(np.abs(got - ref) * w) <= 1e-5 * np.max(np.abs(ref) * w), (got, ref)
    est.close()


def test_headline_strided_pass_shapes_agree(torch, headline, headline_oracle):
    """The headline P(k) and its adjoint with 16 lines per strided-FFT
    workgroup (the persistent kernel that prefetches the next chunk and runs
    forward and inverse 1024-point lines as 32 x 32) and with 8 (one chunk
    per workgroup, 16 x 16 x 4): P(k) of both against the FP64 oracle
    (1e-5), and the position gradients of both within 1e-4 of the largest
    component (the adjoint's tolerance against the oracle; the two plans
    round differently in FP32)."""
    pos, dpos, est = headline
    k0, p0, n0, _ = headline_oracle
    dldp = np.random.default_rng(11).standard_normal(512)
    ddldp = to_dev(torch, dldp[None, :])
    grads = []
    for choice in (46, 22):  # 16 and 8 lines per workgroup, the rest equal
        est.set_launch(choice)
        _, pk, nm = est.power(dpos, n_bins=512)
        assert np.array_equal(nm.cpu().numpy()[0], n0)
        assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL, choice
        grads.append(est.backward(dpos, ddldp, n_bins=512))
    assert bool(torch.isfinite(grads[0]).all())
    scale = float(grads[0].abs().max())
    assert scale > 0 and float((grads[0] - grads[1]).abs().max()) <= 1e-4 * scale
    est.autotune(dpos, n_bins=512, iters=1)


def test_batch_of_two_sets_at_1024_matches_single_sets(torch):
    """Two particle sets on 1024^3 grids in one batch (the strided passes'
    prefetching kernel with two outer blocks, the fused pass with one grid
    row of workgroups per set) give each set's P(k) and mode counts as a
    handle of its own does: counts exactly, P(k) to 1e-6 (the transforms
    and sums take the same arithmetic; the deposit's fixed-point step
    follows the fullest bucket of the whole batch, so the grids round
    differently at about 1e-7)."""
    from paper_1512_07295_amd.estimator import Estimator
    box, n = 2000.0, 1024
    parts = [synth.zeldovich(128, box, 21, dtype=np.float32),
             synth.uniform(1 << 20, box, 22, np.float32)]
    pos = np.concatenate(parts)
    offs = np.array([0, len(parts[0]), len(pos)], dtype=np.int64)
    est = Estimator(n, box, 4, True, 2, len(pos))
    _, pk, nm = est.power(to_dev(torch, pos), offsets=to_dev(torch, offs), n_bins=512)
    pk, nm = pk.cpu().numpy(), nm.cpu().numpy()
    est.close()
    for i, part in enumerate(parts):
        one = Estimator(n, box, 4, True, 1, len(part))
        _, p1, n1 = one.power(to_dev(torch, part), n_bins=512)
        one.close()
        assert np.array_equal(nm[i], n1.cpu().numpy()[0])
        assert rel_err(pk[i], p1.cpu().numpy()[0]) < 1e-6, i


def test_c2_power_all_shells_and_every_triangle(torch):
    from paper_1512_07295_amd.estimator import Estimator
    box, n = 1000.0, 256
    pos = synth.zeldovich(256, box, 2, dtype=np.float32)
    est = Estimator(n, box, 4, True, 1, len(pos))
    dpos = to_dev(torch, pos)
    est.autotune(dpos, iters=1)
    k, pk, nm = est.power(dpos)
    delta, _ = native.delta_half(pos, box, n, 4, True)
    k0, p0, n0 = spectrum.bin_power(delta, box, n, 1, n // 2)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    # bispectrum: every shell up to k_N/2 (32 shells of 2 k_f), all 3,384
    # closed triangles
    nb, n_dk = 32, 2
    tri = bispectrum.closed_triangles(nb)
    assert len(tri) == 3384
    bk, nt = est.bispectrum(tri, n_dk, nb)
    bk, nt = bk.cpu().numpy(), nt.cpu().numpy()
    masks = bispectrum.shell_masks(n, n_dk, nb)
    fi = bispectrum.shell_fields(delta, masks, n)
    s_iii = bispectrum.triple_sums(fi, tri)
    s_abs = bispectrum.triple_sums(np.abs(fi), tri)
    del fi
    fj = bispectrum.shell_fields(np.ones_like(delta), masks, n)
    s_jjj = bispectrum.triple_sums(fj, tri)
    del fj
    b0 = box ** 6 * s_iii / s_jjj
    scale = np.maximum(np.abs(b0), box ** 6 * s_abs / s_jjj)
    assert np.all(np.abs(nt - s_jjj / n ** 3) <= 1e-5 * s_jjj / n ** 3 + 1e-3)
    assert np.all(np.abs(bk - b0) <= 1e-5 * scale)
    est.close()


def test_c4_batched_graph_every_mock(torch):
    from paper_1512_07295_amd.estimator import Estimator
    box, n, nm_ = 500.0, 128, 64
    pos, offs = synth.mocks(nm_, box, 100)
    est = Estimator(n, box, 4, True, nm_, len(pos))
    dpos, doffs = to_dev(torch, pos), to_dev(torch, offs)
    est.autotune(dpos, offsets=doffs, iters=1)
    k, pk, nmodes = est.capture(dpos, offsets=doffs)
    est.replay()
    est.replay()
    torch.cuda.synchronize()
    pk = pk.cpu().numpy()
    for i in range(nm_):
        part = pos[offs[i]:offs[i + 1]]
        _, p0, n0 = native.power(part, box, n, 4, True)
        assert np.array_equal(nmodes.cpu().numpy()[i], n0)
        assert rel_err(pk[i], p0) < P_TOL, i
    est.close()


def test_c5_adjoint_full(torch):
    from paper_1512_07295_amd.estimator import Estimator
    box, n, nb = 1000.0, 256, 128
    pos = synth.zeldovich(128, box, 5, dtype=np.float32)
    tgt = synth.zeldovich(128, box, 6, dtype=np.float32)
    _, target, counts = native.power(tgt, box, n, 4, True, 1, nb)
    _, p_now, _ = native.power(pos, box, n, 4, True, 1, nb)
    _, dldp = adjoint.chi2_loss(p_now, target, counts)
    est = Estimator(n, box, 4, True, 1, len(pos))
    g = est.backward(to_dev(torch, pos), to_dev(torch, dldp[None, :]), n_bins=nb).cpu().numpy()
    ref = adjoint.position_gradient(pos, box, n, 4, True, 1, nb, dldp)
    assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))
    est.close()
