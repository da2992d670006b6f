"""Pins of the closed forms the oracle is checked against (Sec. 3.1).

The per-axis aliasing sums are checked against brute-force image sums; the
Hurwitz-zeta forms of F_res (eqs. res1Dnoi, res1Di) against their image sums
with mpmath; and F^int(x) = F^no-int(x/2) (eq. res_comp).
"""

import numpy as np
import pytest

from oracle import theory


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("alt", [False, True])
def test_image_sum_closed_forms(p, alt):
    x = np.linspace(-0.5, 0.5, 41)
    brute = theory.image_sum(x, p, alternate=alt, nmax=4000 if p == 1 else 400)
    tol = 2e-4 if p == 1 else 1e-9
    assert np.allclose(theory.image_sum_closed(x, p, alternate=alt), brute, atol=tol)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_fres_hurwitz_equals_image_sum(p):
    x = np.array([0.05, 0.17, 0.3, 0.41, 0.5])
    for il in (False, True):
        hz = theory.fres_1d_hurwitz(x, p, interlace=il)
        nmax = 20000 if p == 1 else 2000
        im = theory.fres_1d_images(x, p, interlace=il, nmax=nmax)
        # truncated image sums miss a tail of about 2 x^2p / ((2p-1) nmax^(2p-1))
        tail = 4 * x ** (2 * p) / ((2 * p - 1) * float(nmax) ** (2 * p - 1))
        assert np.all(np.abs(hz - im) <= tail + 1e-13 * np.abs(hz))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_fres_interlaced_is_half_argument(p):
    x = np.linspace(0.01, 0.5, 25)
    assert np.allclose(theory.fres_1d_hurwitz(x, p, True),
                       theory.fres_1d_hurwitz(x / 2, p, False), rtol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_deconvolved_white_noise_is_one_plus_fres(p):
    """1 + F_res,1D^no-int(x) = sum_n sinc^2p(pi(x-n)) / sinc^2p(pi x) (eqs. this, Fres)."""
    x = np.array([0.1, 0.25, 0.4, 0.5])
    lhs = 1 + theory.fres_1d_hurwitz(x, p, False)
    rhs = theory.image_sum_closed(x, p) / np.sinc(x) ** (2 * p)
    assert np.allclose(lhs, rhs, rtol=1e-12)
