"""GPU parity of weighted particles (per-particle masses, EST_FLAG_WEIGHTS)
through the C ABI against the FP64 oracle.

Tolerances as for equal masses: grids to 2e-6 of their peak, P(k) to 1e-5
relative, gradients to 1e-4 of their largest component, delta_DS to 1e-5 of
its largest modulus.  Unit masses must reproduce the equal-mass grid bit for
bit (the mass factor is exactly 1).
"""

import numpy as np
import pytest

from oracle import adjoint, assign, direct, spectrum
import oracle
import synth
from gpu_common import rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu

P_TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _est(n, box, p, il, batch=1, maxp=1 << 16, atomic_sort=False, weighted=True):
    from paper_1512_07295_amd.estimator import Estimator
    return Estimator(n, box, p, il, batch, maxp, atomic_sort=atomic_sort, weighted=weighted)


def _masses(n, seed):
    return np.random.default_rng(seed).exponential(1.0, n).astype(np.float32)


@pytest.mark.parametrize("n,p,il,dtype,atomic", [
    (32, 4, True, np.float32, False), (32, 2, False, np.float32, False),
    (32, 1, True, np.float64, False), (64, 6, True, np.float32, False),
    (32, 3, False, np.float32, True), (100, 4, True, np.float32, False),
    (16, 5, True, np.float32, False)])
def test_weighted_grid_parity(torch, n, p, il, dtype, atomic):
    box = 500.0
    pos = synth.uniform(6000, box, 30 + p, dtype)
    w = _masses(len(pos), 1 + p)
    est = _est(n, box, p, il, maxp=len(pos), atomic_sort=atomic)
    wd = to_dev(torch, w)
    est.set_weights(wd)
    est.deposit(to_dev(torch, pos))
    r1, r2 = assign.deposit(pos, box, n, p, il, weights=w)
    g1 = est.copy_grid(1).cpu().numpy()
    assert np.max(np.abs(g1 - r1)) <= 2e-6 * r1.max()
    if il:
        g2 = est.copy_grid(2).cpu().numpy()
        assert np.max(np.abs(g2 - r2)) <= 2e-6 * r2.max()
    est.close()


def test_unit_masses_reproduce_equal_mass_grid_bitwise(torch):
    box, n = 400.0, 64
    pos = to_dev(torch, synth.zeldovich(32, box, 3, dtype=np.float32))
    grids = []
    for weighted in (False, True):
        est = _est(n, box, 4, True, maxp=pos.shape[0], weighted=weighted)
        if weighted:
            est.set_weights(torch.ones(pos.shape[0], dtype=torch.float32, device="cuda"))
        est.deposit(pos)
        grids.append((est.copy_grid(1).cpu().numpy(), est.copy_grid(2).cpu().numpy()))
        est.close()
    assert np.array_equal(grids[0][0], grids[1][0]) and np.array_equal(grids[0][1], grids[1][1])


@pytest.mark.parametrize("p,il,sub", [(4, True, False), (4, True, True), (2, False, True),
                                      (3, True, False)])
def test_weighted_power_parity(torch, p, il, sub):
    box, n = 1000.0, 64
    pos = synth.zeldovich(32, box, 2, dtype=np.float32)
    w = _masses(len(pos), 5)
    est = _est(n, box, p, il, maxp=len(pos))
    est.set_weights(to_dev(torch, w))
    k, pk, nm = est.power(to_dev(torch, pos), subtract_shot=sub)
    k0, p0, n0 = oracle.power(pos, box, n, p, il, weights=w, subtract_shot=sub)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    got = pk.cpu().numpy()[0]
    if sub:
        raw0 = p0 + spectrum.shot_noise(pos, box, w)
        assert np.max(np.abs(got - p0)) <= P_TOL * np.max(np.abs(raw0))
    else:
        assert rel_err(got, p0) < P_TOL
    est.close()


def test_weighted_batch_uses_per_set_totals(torch):
    box, n = 500.0, 32
    a = synth.zeldovich(16, box, 1, dtype=np.float32)
    b = synth.uniform(5000, box, 2, np.float32)
    pos = np.concatenate([a, b])
    offs = np.array([0, len(a), len(pos)], dtype=np.int64)
    w = np.concatenate([_masses(len(a), 3) * 10.0, _masses(len(b), 4)]).astype(np.float32)
    est = _est(n, box, 4, True, batch=2, maxp=len(pos))
    est.set_weights(to_dev(torch, w))
    k, pk, nm = est.power(to_dev(torch, pos), offsets=to_dev(torch, offs), subtract_shot=True)
    for i in range(2):
        s = slice(offs[i], offs[i + 1])
        _, p0, _ = oracle.power(pos[s], box, n, 4, True, weights=w[s], subtract_shot=True)
        raw0 = p0 + spectrum.shot_noise(pos[s], box, w[s])
        assert np.max(np.abs(pk.cpu().numpy()[i] - p0)) <= P_TOL * np.max(np.abs(raw0)), i
    est.close()


@pytest.mark.parametrize("p,il", [(4, True), (2, False)])
def test_weighted_backward(torch, p, il):
    n, box, nb = 32, 1000.0, 12
    pos = synth.zeldovich(16, box, 5, dtype=np.float32)
    w = _masses(len(pos), 8)
    dldp = np.random.default_rng(0).normal(size=nb)
    est = _est(n, box, p, il, maxp=len(pos))
    est.set_weights(to_dev(torch, w))
    g = est.backward(to_dev(torch, pos), to_dev(torch, dldp[None, :]), n_bins=nb).cpu().numpy()
    ref = adjoint.position_gradient(pos, box, n, p, il, 1, nb, dldp, weights=w)
    assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))
    est.close()


def test_weighted_direct_sum(torch):
    box, n = 300.0, 16
    pos = synth.uniform(3000, box, 6, np.float32)
    w = _masses(len(pos), 9)
    est = _est(n, box, 4, True, maxp=len(pos))
    est.set_weights(to_dev(torch, w))
    d = est.direct_delta(to_dev(torch, pos)).cpu().numpy()
    d = d[..., 0] + 1j * d[..., 1]
    ref = direct.delta_half_direct(pos, box, n, weights=w)
    assert np.max(np.abs(d - ref)) <= 1e-5 * np.max(np.abs(ref))
    est.close()


def test_weighted_graph_replay_matches_eager(torch):
    box, n = 500.0, 32
    pos = to_dev(torch, synth.zeldovich(16, box, 7, dtype=np.float32))
    w = to_dev(torch, _masses(pos.shape[0], 10))
    est = _est(n, box, 4, True, maxp=pos.shape[0])
    est.set_weights(w)
    _, p_eager, _ = est.power(pos)
    p_eager = p_eager.cpu().numpy()
    k, p, nm = est.capture(pos)
    for _ in range(3):
        est.replay()
        torch.cuda.synchronize()
        assert np.array_equal(p.cpu().numpy(), p_eager)
        _ = (pos * 1.0).sum().item()  # eager work between replays
    est.close()


def test_invalid_and_zero_masses_give_nan(torch):
    box, n = 300.0, 16
    pos = to_dev(torch, synth.uniform(500, box, 11, np.float32))
    est = _est(n, box, 2, True, maxp=500)
    for bad in (-1.0, float("nan"), float("inf")):
        w = torch.ones(500, dtype=torch.float32, device="cuda")
        w[17] = bad
        est.set_weights(w)
        _, pk, _ = est.power(pos)
        assert torch.isnan(pk).all(), bad
    est.set_weights(torch.zeros(500, dtype=torch.float32, device="cuda"))
    _, pk, _ = est.power(pos)
    assert torch.isnan(pk).all()
    # NULL restores equal masses
    est.set_weights(None)
    _, pk, _ = est.power(pos)
    _, p0, _ = oracle.power(pos.cpu().numpy(), box, n, 2, True)
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    est.close()


def test_set_weights_needs_flag(torch):
    import paper_1512_07295_amd as F
    est = _est(16, 100.0, 2, True, maxp=10, weighted=False)
    with pytest.raises(F.FsestError) as ei:
        est.set_weights(torch.ones(10, dtype=torch.float32, device="cuda"))
    assert ei.value.status == F.EST_EINVAL
    est.close()


def test_weighted_batch_with_empty_and_massless_sets(torch):
    """An empty set and a set whose masses are all zero give NaN P(k) for that
    set only; the others match the oracle."""
    box, n = 400.0, 32
    parts = [synth.uniform(3000, box, 50, np.float32), np.zeros((0, 3), np.float32),
             synth.uniform(500, box, 51, np.float32), synth.zeldovich(12, box, 52, dtype=np.float32)]
    masses = [_masses(3000, 53), np.zeros(0, np.float32), np.zeros(500, np.float32),
              _masses(12 ** 3, 54)]
    pos = np.concatenate(parts)
    w = np.concatenate(masses).astype(np.float32)
    offs = np.zeros(len(parts) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(q) for q in parts])
    est = _est(n, box, 4, True, batch=len(parts), maxp=len(pos))
    est.set_weights(to_dev(torch, w))
    _, pk, _ = est.power(to_dev(torch, pos), offsets=to_dev(torch, offs))
    pk = pk.cpu().numpy()
    for i in (1, 2):
        assert np.all(np.isnan(pk[i])), i
    for i in (0, 3):
        _, p0, _ = oracle.power(parts[i], box, n, 4, True, weights=masses[i])
        assert rel_err(pk[i], p0) < P_TOL, i
    est.close()
