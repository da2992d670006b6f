"""Closed forms that pin the estimator: aliased white noise and F_res.

Test infrastructure only (see ``oracle/__init__.py``).

For particles placed uniformly at random (P = 0, P_tot = shot noise V/N_P),
the aliasing sum of eq. Pknoint and its interlaced version (Sec. 3.1,
theta_n = [1 + (-1)^(n_x+n_y+n_z)]/2) factorise per axis.  With
x_i = m_i/N and S(y) = sinc^(2p)(pi y):

    <P(m)> (no interlacing, no deconvolution) = V/N_P prod_i sum_n S(x_i - n)
    <P(m)> (deconvolved)     = V/N_P prod_i A_i,  A_i = 1 + F_res,1D^no-int(x_i)
    <P(m)> (interlaced, deconvolved) = V/N_P (prod_i A_i + prod_i B_i) / 2,
                               B_i = sum_n (-1)^n (x_i/(x_i-n))^(2p)

The residual factor of eq. Fres is F_res = sum_{n != 0} theta_n
prod_i (x_i/(x_i-n_i))^(2p); in one dimension eqs. res1Dnoi and res1Di give it
through Hurwitz zeta functions and F^int(x) = F^no-int(x/2) (eq. res_comp).

The per-axis image sums are evaluated by brute force (``image_sum``) and by
their trigonometric closed forms (``image_sum_closed``), which are
Hockney-Eastwood / Jing sums of the B-spline windows.
"""

import numpy as np


def image_sum(x, p, alternate=False, nmax=2000):
    """sum_n (+/-1)^n sinc^(2p)(pi (x - n)), brute force with |n| <= nmax."""
    x = np.asarray(x, dtype=np.float64)
    n = np.arange(-nmax, nmax + 1, dtype=np.float64)
    y = x[..., None] - n
    terms = np.sinc(y) ** (2 * p)
    if alternate:
        terms = terms * np.where(n.astype(np.int64) % 2 == 0, 1.0, -1.0)
    return terms.sum(axis=-1)


def image_sum_closed(x, p, alternate=False):
    """Closed forms of ``image_sum`` for p = 1..4."""
    x = np.asarray(x, dtype=np.float64)
    if not alternate:
        s2 = np.sin(np.pi * x) ** 2
        return {
            1: np.ones_like(x),
            2: 1.0 - 2.0 / 3.0 * s2,
            3: 1.0 - s2 + 2.0 / 15.0 * s2 ** 2,
            4: 1.0 - 4.0 / 3.0 * s2 + 2.0 / 5.0 * s2 ** 2 - 4.0 / 315.0 * s2 ** 3,
        }[p]
    c = [np.cos((2 * j + 1) * np.pi * x) for j in range(4)]
    coef = {
        1: [1.0],
        2: [23.0 / 24.0, 1.0 / 24.0],
        3: [841.0 / 960.0, 79.0 / 640.0, 1.0 / 1920.0],
        4: [259723.0 / 322560.0, 20219.0 / 107520.0, 2179.0 / 322560.0,
            1.0 / 322560.0],
    }[p]
    return sum(a * cj for a, cj in zip(coef, c))


def fres_1d_images(x, p, interlace=False, nmax=20000):
    """F_res,1D by its image sum: sum_{n != 0} (x/(x - s n))^(2p), s = 2 if
    interlaced (eq. res1Di) else 1 (eq. res1Dnoi)."""
    x = np.asarray(x, dtype=np.float64)
    step = 2.0 if interlace else 1.0
    n = np.arange(1, nmax + 1, dtype=np.float64)
    t = (x[..., None] / (x[..., None] - step * n)) ** (2 * p) \
        + (x[..., None] / (x[..., None] + step * n)) ** (2 * p)
    return t.sum(axis=-1)


def fres_1d_hurwitz(x, p, interlace=False):
    """F_res,1D through the Hurwitz zeta forms of eqs. res1Dnoi / res1Di."""
    import mpmath
    xs = np.atleast_1d(np.asarray(x, dtype=np.float64))
    out = []
    mpmath.mp.dps = 40
    for xv in xs:
        y = xv / 2.0 if interlace else xv
        v = mpmath.mpf(y) ** (2 * p) * (mpmath.zeta(2 * p, mpmath.mpf(y))
                                         + mpmath.zeta(2 * p, -mpmath.mpf(y))) - 2
        out.append(float(v))
    return np.array(out).reshape(np.shape(x))


def white_noise_power(m, n_grid, p, interlace, deconvolve, vol, n_p):
    """Expected P(m) of uniformly random particles (see module docstring).

    ``m`` has shape (..., 3) of signed integer frequencies.  ``interlace`` is
    the interlacing code (False/0, True/1, 2 face-centred, 3 all eight
    shifts): for a shift set S, theta_n = (1/G) sum_{s in S} (-1)^(2 n.s), so
    the expectation is V/N_P (1/G) sum_{s in S} prod_i (B_i if s_i = 1/2
    else A_i), which gives the pair formula above for S = {0, (1,1,1)/2}.
    """
    if int(interlace) >= 2:
        from .spectrum import shift_masks
        x = np.asarray(m, dtype=np.float64) / n_grid
        a = image_sum_closed(x, p)
        b = image_sum_closed(x, p, alternate=True)
        if deconvolve:
            win2 = np.sinc(x) ** (2 * p)
            a, b = a / win2, b / win2
        masks = shift_masks(interlace)
        tot = 0.0
        for mk in masks:
            tot = tot + np.prod([b[..., i] if (mk >> i) & 1 else a[..., i] for i in range(3)], axis=0)
        return vol / n_p * tot / len(masks)
    x = np.asarray(m, dtype=np.float64) / n_grid
    s = image_sum_closed(x, p)
    if deconvolve:
        win2 = np.sinc(x) ** (2 * p)
        a = np.prod(s / win2, axis=-1)
        if interlace:
            b = np.prod(image_sum_closed(x, p, alternate=True) / win2, axis=-1)
            return vol / n_p * 0.5 * (a + b)
        return vol / n_p * a
    if interlace:
        d = image_sum_closed(x, p, alternate=True)
        return vol / n_p * 0.5 * (np.prod(s, axis=-1) + np.prod(d, axis=-1))
    return vol / n_p * np.prod(s, axis=-1)
