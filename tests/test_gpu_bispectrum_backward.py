"""GPU parity of the FFT-shell bispectrum and of the P(k) adjoint.

Bispectrum: B within 1e-5 of max(|B|, V^2 sum|I I I| / sum J J J) (the L1
scale of the summands, since B can cross zero); N_tri within 1e-5 relative.
Adjoint: dL/dx within 1e-4 of max |dL/dx| of the FP64 oracle gradient, which
is itself pinned to finite differences of the oracle forward.
"""

import numpy as np
import pytest

import oracle
from oracle import adjoint, bispectrum, spectrum
import synth
from gpu_common import rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _oracle_l1_scale(pos, box, n, p, il, n_dk, n_bins, tri):
    delta, _ = spectrum.delta_half(pos, box, n, p, il)
    masks = bispectrum.shell_masks(n, n_dk, n_bins)
    fi = np.abs(bispectrum.shell_fields(delta, masks, n))
    s_abs = bispectrum.triple_sums(fi, tri)
    fj = bispectrum.shell_fields(np.ones_like(delta), masks, n)
    s_jjj = bispectrum.triple_sums(fj, tri)
    return box ** 6 * s_abs / s_jjj


@pytest.mark.parametrize("n,p,il", [(32, 4, True), (32, 2, False), (64, 4, True), (32, 3, True)])
def test_bispectrum_parity(torch, n, p, il):
    from paper_1512_07295_amd.estimator import Estimator
    box, n_dk = 500.0, 2
    pos = synth.zeldovich(16, box, 21, dtype=np.float32)
    nb = bispectrum.max_bins(n, n_dk)
    tri = bispectrum.closed_triangles(nb)
    est = Estimator(n, box, p, il, 1, len(pos))
    est.power(to_dev(torch, pos))
    bk, nt = est.bispectrum(tri, n_dk, nb)
    bk, nt = bk.cpu().numpy(), nt.cpu().numpy()
    _, b0, n0 = oracle.bispectrum_fn(pos, box, n, p, il, n_dk=n_dk, n_bins=nb, triangles=tri)
    scale = np.maximum(np.abs(b0), _oracle_l1_scale(pos, box, n, p, il, n_dk, nb, tri))
    assert np.all(np.abs(nt - n0) <= 1e-5 * n0 + 1e-3)
    assert np.all(np.abs(bk - b0) <= 1e-5 * scale)
    est.close()


def test_bispectrum_rejects_beyond_triangle_limit(torch):
    import paper_1512_07295_amd as F
    from paper_1512_07295_amd.estimator import Estimator
    est = Estimator(32, 100.0, 4, True, 1, 100)
    est.power(to_dev(torch, synth.uniform(100, 100.0, 1, np.float32)))
    with pytest.raises(F.FsestError) as ei:
        est.bispectrum(bispectrum.closed_triangles(5), 2, 5)
    assert ei.value.status == F.EST_EINVAL
    est.close()


def _setup_loss(n, box, p, il, n_bins):
    pos = synth.zeldovich(16, box, 5, dtype=np.float32)
    tgt = synth.zeldovich(16, box, 6, dtype=np.float32)
    _, target, counts = oracle.power(tgt, box, n, p, il, 1, n_bins)
    _, pk, _ = oracle.power(pos, box, n, p, il, 1, n_bins)
    _, dldp = adjoint.chi2_loss(pk, target, counts)
    return pos, target, counts, dldp


@pytest.mark.parametrize("p,il", [(4, True), (4, False), (2, False), (3, True), (2, True),
                                  (5, True), (6, True), (6, False)])
def test_backward_matches_oracle_gradient(torch, p, il):
    from paper_1512_07295_amd.estimator import Estimator
    n, box, n_bins = 32, 1000.0, 16
    pos, target, counts, dldp = _setup_loss(n, box, p, il, n_bins)
    est = Estimator(n, box, p, il, 1, len(pos))
    g = est.backward(to_dev(torch, pos), to_dev(torch, dldp[None, :]), n_bins=n_bins).cpu().numpy()
    ref = adjoint.position_gradient(pos, box, n, p, il, 1, n_bins, dldp)
    assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))
    est.close()


def test_backward_batched_and_f64(torch):
    from paper_1512_07295_amd.estimator import Estimator
    n, box, n_bins = 32, 800.0, 12
    a = synth.zeldovich(12, box, 1, dtype=np.float64)
    b = synth.uniform(3000, box, 2, np.float64)
    pos = np.concatenate([a, b])
    offs = np.array([0, len(a), len(a) + len(b)], dtype=np.int64)
    rng = np.random.default_rng(0)
    dldp = rng.normal(size=(2, n_bins))
    est = Estimator(n, box, 4, True, 2, len(pos))
    g = est.backward(to_dev(torch, pos), to_dev(torch, dldp), offsets=to_dev(torch, offs),
                     n_bins=n_bins).cpu().numpy()
    for i, part in enumerate((a, b)):
        ref = adjoint.position_gradient(part, box, n, 4, True, 1, n_bins, dldp[i])
        assert np.max(np.abs(g[offs[i]:offs[i + 1]] - ref)) <= 1e-4 * np.max(np.abs(ref))
    est.close()


def test_autograd_function(torch):
    from paper_1512_07295_amd.estimator import Estimator, PowerSpectrumFn
    n, box, n_bins = 32, 1000.0, 16
    pos, target, counts, dldp = _setup_loss(n, box, 4, True, n_bins)
    est = Estimator(n, box, 4, True, 1, len(pos))
    x = to_dev(torch, pos).requires_grad_(True)
    pk = PowerSpectrumFn.apply(x, est, 1, n_bins, None)[0]
    t = to_dev(torch, target)
    sigma2 = 2 * t ** 2 / to_dev(torch, counts.astype(np.float64))
    loss = ((pk - t) ** 2 / sigma2).sum()
    loss.backward()
    ref = adjoint.position_gradient(pos, box, n, 4, True, 1, n_bins,
                                    adjoint.chi2_loss(pk.detach().cpu().numpy(), target, counts)[1])
    g = x.grad.cpu().numpy()
    assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))
    est.close()
