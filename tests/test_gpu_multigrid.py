"""GPU parity of interlacing with more than two grids (codes 2: four
face-centred half-cell shifts, 3: all eight) through the C ABI against the
FP64 oracle.  Tolerances as for the pair: grids to 2e-6 of their peak, mode
counts bit-exact, P(k) to 1e-5 relative, delta(m) to 1e-5 (window weighted).
"""

import numpy as np
import pytest

import oracle
from oracle import assign, bispectrum, kernels, native, spectrum
import synth
from gpu_common import rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu

P_TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _est(n, box, p, code, batch=1, maxp=1 << 16, **kw):
    from paper_1512_07295_amd.estimator import Estimator
    return Estimator(n, box, p, code, batch, maxp, **kw)


@pytest.mark.parametrize("n,p,code", [(32, 4, 2), (32, 2, 3), (16, 3, 3), (100, 4, 3), (64, 6, 2)])
def test_every_grid_matches_oracle(torch, n, p, code):
    box = 500.0
    pos = synth.uniform(4000, box, 60 + p + code, np.float32)
    est = _est(n, box, p, code, maxp=len(pos))
    est.deposit(to_dev(torch, pos))
    u = assign.grid_coords(pos, box, n)
    for j, mk in enumerate(spectrum.shift_masks(code)):
        ref = assign.deposit_u(u + spectrum.mask_shift(mk), p, n)
        got = est.copy_grid(j + 1).cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 2e-6 * ref.max(), (j, mk)
    est.close()


@pytest.mark.parametrize("n,p,code", [(32, 4, 2), (32, 4, 3), (64, 2, 3), (48, 3, 2), (100, 4, 3)])
def test_power_parity(torch, n, p, code):
    box = 1000.0
    pos = synth.zeldovich(32, box, 2, dtype=np.float32)
    est = _est(n, box, p, code, maxp=len(pos))
    k, pk, nm = est.power(to_dev(torch, pos))
    k0, p0, n0 = oracle.power(pos, box, n, p, code)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    assert rel_err(k.cpu().numpy()[0], k0) < 1e-12
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    # again from the stored spectra
    k2, pk2, _ = est.power_only()
    assert rel_err(pk2.cpu().numpy()[0], p0) < P_TOL
    est.close()


@pytest.mark.parametrize("n,code,n_dk,n_bins", [(32, 3, 3, 4), (64, 2, 2, 6), (48, 3, 1, 9)])
def test_power_few_shells(torch, n, code, n_dk, n_bins):
    """Shells well below the Nyquist frequency: the fused pass skips the row
    pairs with no mode inside the last shell; counts exact, P within 1e-5."""
    box = 1000.0
    pos = synth.zeldovich(32, box, 4, dtype=np.float32)
    est = _est(n, box, 4, code, maxp=len(pos))
    k, pk, nm = est.power(to_dev(torch, pos), n_dk=n_dk, n_bins=n_bins)
    k0, p0, n0 = oracle.power(pos, box, n, 4, code, n_dk, n_bins)
    assert np.array_equal(nm.cpu().numpy()[0], n0)
    assert rel_err(k.cpu().numpy()[0], k0) < 1e-12
    assert rel_err(pk.cpu().numpy()[0], p0) < P_TOL
    est.close()


@pytest.mark.parametrize("code", [2, 3])
def test_export_and_sampled_delta(torch, code):
    box, n, p = 300.0, 32, 4
    pos = synth.zeldovich(16, box, 8, dtype=np.float32)
    est = _est(n, box, p, code, maxp=len(pos))
    est.deposit(to_dev(torch, pos))
    est.transform()
    d = est.export_delta().cpu().numpy()
    d = d[..., 0] + 1j * d[..., 1]
    ref, _ = spectrum.delta_half(pos, box, n, p, code)
    mx, my, mz = spectrum.half_axes(n)
    w = np.broadcast_to(kernels.window_1d(p, mx, n) * kernels.window_1d(p, my, n)
                        * kernels.window_1d(p, mz, n), ref.shape)
    ok = np.isfinite(ref)
    assert np.max(np.abs(d - ref)[ok] * w[ok]) <= 1e-5 * np.max(np.abs(ref[ok]) * w[ok])
    modes = np.array([[1, 0, 0], [16, 16, 16], [-5, 7, 3], [16, 0, 16], [3, -15, 9]])
    s = est.sample_delta(modes).cpu().numpy()
    r = native.delta_modes(pos, box, n, p, code, modes)
    wm = np.prod([kernels.window_1d(p, modes[:, a], n) for a in range(3)], axis=0)
    assert np.all(np.abs(s - r) * wm <= 1e-5 * np.max(np.abs(r) * wm)), (s, r)
    est.close()


def test_bispectrum_with_eight_grids(torch):
    box, n, n_dk, p, code = 500.0, 32, 2, 4, 3
    pos = synth.zeldovich(16, box, 21, dtype=np.float32)
    nb = bispectrum.max_bins(n, n_dk)
    tri = bispectrum.closed_triangles(nb)
    est = _est(n, box, p, code, maxp=len(pos))
    est.power(to_dev(torch, pos))
    bk, nt = est.bispectrum(tri, n_dk, nb)
    bk, nt = bk.cpu().numpy(), nt.cpu().numpy()
    _, b0, n0 = oracle.bispectrum_fn(pos, box, n, p, code, n_dk=n_dk, n_bins=nb, triangles=tri)
    delta, _ = spectrum.delta_half(pos, box, n, p, code)
    masks = bispectrum.shell_masks(n, n_dk, nb)
    s_abs = bispectrum.triple_sums(np.abs(bispectrum.shell_fields(delta, masks, n)), tri)
    s_jjj = bispectrum.triple_sums(bispectrum.shell_fields(np.ones_like(delta), masks, n), tri)
    scale = np.maximum(np.abs(b0), box ** 6 * s_abs / s_jjj)
    assert np.all(np.abs(nt - n0) <= 1e-5 * n0 + 1e-3)
    assert np.all(np.abs(bk - b0) <= 1e-5 * scale)
    est.close()


def test_batched_weighted_graph_with_four_grids(torch):
    box, n, code = 500.0, 32, 2
    a = synth.zeldovich(16, box, 1, dtype=np.float32)
    b = synth.uniform(5000, box, 2, np.float32)
    pos = np.concatenate([a, b])
    offs = np.array([0, len(a), len(pos)], dtype=np.int64)
    w = np.random.default_rng(3).exponential(1.0, len(pos)).astype(np.float32)
    est = _est(n, box, 4, code, batch=2, maxp=len(pos), weighted=True)
    est.set_weights(to_dev(torch, w))
    dpos, doffs = to_dev(torch, pos), to_dev(torch, offs)
    _, p_eager, _ = est.power(dpos, offsets=doffs)
    p_eager = p_eager.cpu().numpy()
    for i in range(2):
        s = slice(offs[i], offs[i + 1])
        _, p0, _ = oracle.power(pos[s], box, n, 4, code, weights=w[s])
        assert rel_err(p_eager[i], p0) < P_TOL, i
    k, p, nm = est.capture(dpos, offsets=doffs)
    for _ in range(3):
        est.replay()
        torch.cuda.synchronize()
        assert np.array_equal(p.cpu().numpy(), p_eager)
        _ = (dpos * 2.0).sum().item()
    est.close()


@pytest.mark.parametrize("n,p,code,dtype", [(32, 4, 2, np.float32), (32, 2, 3, np.float32),
                                            (24, 3, 3, np.float64), (16, 4, 3, np.float32)])
def test_backward_matches_oracle_gradient(torch, n, p, code, dtype):
    from oracle import adjoint
    box, nb = 1000.0, 8
    pos = synth.zeldovich(16, box, 5, dtype=dtype)
    tgt = synth.zeldovich(16, box, 6, dtype=dtype)
    _, target, counts = oracle.power(tgt, box, n, p, code, 1, nb)
    _, pk, _ = oracle.power(pos, box, n, p, code, 1, nb)
    _, dldp = adjoint.chi2_loss(pk, target, counts)
    est = _est(n, box, p, code, maxp=len(pos))
    g = est.backward(to_dev(torch, pos), to_dev(torch, dldp[None, :]), n_bins=nb).cpu().numpy()
    ref = adjoint.position_gradient(pos, box, n, p, code, 1, nb, dldp)
    assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))
    # the handle computes the forward again afterwards
    k, pk2, _ = est.power(to_dev(torch, pos), n_bins=nb)
    assert rel_err(pk2.cpu().numpy()[0], pk) < P_TOL
    est.close()


def test_backward_batched_weighted_four_grids(torch):
    from oracle import adjoint
    n, box, nb, code = 32, 800.0, 10, 2
    a = synth.zeldovich(12, box, 1, dtype=np.float32)
    b = synth.uniform(3000, box, 2, np.float32)
    pos = np.concatenate([a, b])
    offs = np.array([0, len(a), len(pos)], dtype=np.int64)
    w = np.random.default_rng(4).exponential(1.0, len(pos)).astype(np.float32)
    dldp = np.random.default_rng(0).normal(size=(2, nb))
    est = _est(n, box, 4, code, batch=2, maxp=len(pos), weighted=True)
    est.set_weights(to_dev(torch, w))
    g = est.backward(to_dev(torch, pos), to_dev(torch, dldp), offsets=to_dev(torch, offs),
                     n_bins=nb).cpu().numpy()
    for i in range(2):
        s = slice(offs[i], offs[i + 1])
        ref = adjoint.position_gradient(pos[s], box, n, 4, code, 1, nb, dldp[i], weights=w[s])
        assert np.max(np.abs(g[s] - ref)) <= 1e-4 * np.max(np.abs(ref)), i
    est.close()


def test_eight_grids_reduce_aliasing_against_direct_sum(torch):
    """Against the alias-free direct sum (Sec. 3.2 at reduced size): eight
    grids leave less aliasing than the pair up to 3/4 of the Nyquist
    frequency (PCS)."""
    box, n = 500.0, 32
    pos = to_dev(torch, synth.zeldovich(32, box, 8, dtype=np.float32))
    est = _est(n, box, 4, 1, maxp=pos.shape[0])
    dds = est.direct_delta(pos)
    _, p_ds, _ = est.spectrum_power(dds)
    p_ds = p_ds.cpu().numpy()
    est.close()
    errs = {}
    for code in (1, 3):
        e = _est(n, box, 4, code, maxp=pos.shape[0])
        e.deposit(pos)
        e.transform()
        dg = e.export_delta()
        _, p_g, _ = e.spectrum_power(dg)
        errs[code] = np.abs(p_g.cpu().numpy() / p_ds - 1)
        e.close()
    sel = np.arange(1, n // 2 + 1) <= 3 * n // 8
    assert np.max(errs[3][sel]) < np.max(errs[1][sel])
