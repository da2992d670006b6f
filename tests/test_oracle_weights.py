"""Pins of the oracle's weighted-particle path (masses w_j >= 0; the paper
takes equal masses for simplicity, Sec. 2.1).

Each check is fixed by the unweighted path or by a closed form, not by the
weighted code itself: integer masses equal coincident copies of a particle;
constant masses leave delta unchanged; the white-noise expectation with
masses is V sum w^2 / W^2 times the aliasing sum of the unit-mass case.
"""

import numpy as np
import pytest

from oracle import adjoint, assign, direct, spectrum, theory
import synth


def _replicated(pos, iw):
    return np.repeat(pos, iw, axis=0)


@pytest.mark.parametrize("p,il,n", [(1, False, 16), (2, True, 16), (4, True, 12), (6, False, 16)])
def test_integer_masses_equal_coincident_copies(p, il, n):
    box = 200.0
    pos = synth.uniform(400, box, 7, np.float64)
    iw = np.random.default_rng(1).integers(0, 4, len(pos))
    rep = _replicated(pos, iw)
    r1, r2 = assign.deposit(pos, box, n, p, il, weights=iw)
    q1, q2 = assign.deposit(rep, box, n, p, il)
    assert np.allclose(r1, q1, rtol=0, atol=1e-12 * q1.max())
    if il:
        assert np.allclose(r2, q2, rtol=0, atol=1e-12 * q2.max())
    _, pw, _ = spectrum.power(pos, box, n, p, il, weights=iw)
    _, pr, _ = spectrum.power(rep, box, n, p, il)
    assert np.allclose(pw, pr, rtol=1e-12, atol=1e-9 * np.abs(pr).max())
    # coincident copies are not independent particles: the self-pair term
    # of the weighted set is V sum w^2 / W^2, not V / sum w
    _, ps, _ = spectrum.power(pos, box, n, p, il, weights=iw, subtract_shot=True)
    assert np.allclose(pw - ps, box ** 3 * np.sum(iw ** 2) / np.sum(iw) ** 2, rtol=1e-12)
    dw = direct.delta_half_direct(pos, box, 8, weights=iw)
    dr = direct.delta_half_direct(rep, box, 8)
    assert np.max(np.abs(dw - dr)) < 1e-12


def test_integer_masses_gradient_is_sum_over_copies():
    box, n, p, il, nb = 500.0, 16, 4, True, 6
    pos = synth.uniform(60, box, 3, np.float64)
    iw = np.random.default_rng(2).integers(1, 4, len(pos))
    rep = _replicated(pos, iw)
    dldp = np.random.default_rng(4).normal(size=nb)
    gw = adjoint.position_gradient(pos, box, n, p, il, 1, nb, dldp, weights=iw)
    gr = adjoint.position_gradient(rep, box, n, p, il, 1, nb, dldp)
    # the copies of particle j sit at the same place: their gradients add up
    owner = np.repeat(np.arange(len(pos)), iw)
    summed = np.zeros_like(gw)
    np.add.at(summed, owner, gr)
    assert np.allclose(gw, summed, rtol=1e-10, atol=1e-12 * np.abs(summed).max())


def test_constant_masses_leave_delta_unchanged():
    box, n = 300.0, 16
    pos = synth.zeldovich(8, box, 5, dtype=np.float64)
    d0, w0 = spectrum.delta_half(pos, box, n, 3, True)
    d1, w1 = spectrum.delta_half(pos, box, n, 3, True, weights=np.full(len(pos), 2.75))
    assert w0 == len(pos) and w1 == pytest.approx(2.75 * len(pos))
    assert np.allclose(d0, d1, rtol=1e-12, atol=1e-15)
    assert spectrum.shot_noise(pos, box, np.full(len(pos), 2.75)) == pytest.approx(box ** 3 / len(pos))


def test_weighted_white_noise_expectation():
    """Uniform random positions with fixed unequal masses: each mode's
    <V |delta|^2> is the unit-mass aliased white-noise spectrum at the
    effective number W^2 / sum w^2."""
    n, box, n_p, reps, p, il = 16, 100.0, 1500, 100, 2, True
    w = np.random.default_rng(9).exponential(1.0, n_p)
    n_eff = w.sum() ** 2 / (w * w).sum()
    mx, my, mz = spectrum.half_axes(n)
    m = np.stack(np.broadcast_arrays(mx, my, mz), axis=-1)
    m2 = (m ** 2).sum(-1)
    hw = np.broadcast_to(spectrum.half_weights(n), m2.shape)
    b = spectrum.bin_index(m2, 1)
    expect = theory.white_noise_power(m, n, p, il, True, box ** 3, n_eff)
    acc = np.zeros(m2.shape)
    for r in range(reps):
        pos = synth.uniform(n_p, box, 3000 + r, np.float64)
        d, _ = spectrum.delta_half(pos, box, n, p, il, weights=w)
        acc += box ** 3 * np.abs(d) ** 2
    acc /= reps
    for bi in range(1, n // 2 + 1):
        sel = (b == bi) & (m2 > 0)
        nm = hw[sel].sum()
        mc = (hw[sel] * acc[sel]).sum() / nm
        th = (hw[sel] * expect[sel]).sum() / nm
        assert abs(mc - th) < 4.0 * th / np.sqrt(reps * nm / 2.0), (bi, mc, th)
    assert spectrum.shot_noise(pos, box, w) == pytest.approx(box ** 3 / n_eff)
