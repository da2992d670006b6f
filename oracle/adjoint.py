"""Exact gradient of the binned P(k) with respect to the particle positions.

Test infrastructure only (see ``oracle/__init__.py``).

Not in the paper: this is the derivative of the forward computed in
``spectrum`` (deposit -> FFT -> interlace -> deconvolve -> bin), taken
literally on the weighted half spectrum

    P_b = V / N_b * sum_{m stored, m in b} w_m |C(m)|^2 / (N_P W(m))^2.

With g_b = dL/dP_b and Gamma(m) = dL/dRe C + i dL/dIm C
= 2 g_b V C(m) / (N_b N_P^2 W(m)^2):

    dL/drho_a(g) = sum_{m stored} w_m Re[G_a(m) exp(+2 pi i m.g/N)],
    G_1 = Gamma / 2,  G_2 = Gamma exp(-i pi (m_x+m_y+m_z)/N) / 2
    (without interlacing C = F_1 and G_1 = Gamma),

evaluated here as the real part of an unnormalised inverse DFT of a full
N^3 array that holds w_m G_a(m) at the stored half-spectrum indices and zero
elsewhere.  The chain rule through the deposit (u = x N/L, s = g - u) gives

    dL/dx_{j,alpha} = -(N/L) sum_a sum_{g in stencil} dL/drho_a(g)
                      W'(g_alpha - u_alpha) prod_{beta != alpha} W(g_beta - u_beta).

The example loss is L = sum_b (P_b - T_b)^2 / sigma_b^2 with the Gaussian
variance sigma_b^2 = 2 T_b^2 / N_b (reading: the paper defines no loss).
"""

import numpy as np
import scipy.fft

from .assign import deposit_u, grid_coords, stencil
from .kernels import dweight
from .spectrum import (bin_index, combine, fft_grid, half_axes, half_weights, mask_shift,
                       mode_table, shift_masks, window)


def chi2_loss(pk, target, counts):
    """L = sum_b (P_b - T_b)^2 / sigma_b^2 and dL/dP_b, sigma_b^2 = 2 T_b^2/N_b."""
    sigma2 = 2.0 * target ** 2 / counts
    r = pk - target
    return float(np.sum(r * r / sigma2)), 2.0 * r / sigma2


def grid_gradient(pos, box, n, p, interlace_on, n_dk, n_bins, dldp, weights=None):
    """dL/drho_a on the grids, for a given dL/dP_b.  Returns (u, [g1, g2]).
    With masses, N_P above is the total mass W (the masses are constants)."""
    n_p = pos.shape[0] if weights is None else float(np.sum(np.asarray(weights, dtype=np.float64)))
    u = grid_coords(pos, box, n)
    masks = shift_masks(interlace_on)
    fs = [fft_grid(deposit_u(u + mask_shift(mk), p, n, weights)) for mk in masks]
    c = combine(fs, masks, n) if len(masks) > 1 else fs[0]
    win = window(n, p)
    mx, my, mz = half_axes(n)
    m2 = mx * mx + my * my + mz * mz
    b = np.broadcast_to(bin_index(m2, n_dk), m2.shape)
    sel = (m2 > 0) & (b >= 1) & (b <= n_bins)
    counts, _ = mode_table(n, n_dk, n_bins)
    vol = float(box) ** 3
    bb = np.where(sel, b, 1) - 1
    coef = np.where(sel, 2.0 * np.asarray(dldp)[bb] * vol
                    / (counts[bb] * float(n_p) ** 2), 0.0)
    gamma = coef * c / (win * win)
    w = np.broadcast_to(half_weights(n), m2.shape)
    m = (mx, my, mz)
    phases = [np.broadcast_to(np.pi * sum((m[a] if (mk >> a) & 1 else 0) for a in range(3)) / n,
                              m2.shape).astype(np.float64) for mk in masks]
    grads = []
    frac = 1.0 / len(masks)  # dC/dF_j = exp(+i phi_j) / G
    for ph in phases:
        ga = frac * gamma * np.exp(-1j * ph)
        full = np.zeros((n, n, n), dtype=np.complex128)
        full[:, :, : n // 2 + 1] = w * ga
        grads.append(np.real(scipy.fft.ifftn(full, workers=-1)) * float(n) ** 3)
    return u, grads, masks


def position_gradient(pos, box, n, p, interlace_on, n_dk, n_bins, dldp, weights=None):
    """dL/dx_j (N_P, 3) for a given dL/dP_b (n_bins,); a particle of mass
    w_j deposits w_j times the kernel, so its gradient carries the factor w_j."""
    pos = np.asarray(pos)
    u, grads, masks = grid_gradient(pos, box, n, p, interlace_on, n_dk, n_bins, dldp, weights)
    out = np.zeros((pos.shape[0], 3), dtype=np.float64)
    for mk, gam in zip(masks, grads):
        ua = u + mask_shift(mk)
        sten = []
        for ax in range(3):
            cells, w = stencil(ua[:, ax], p, n)
            # offsets s = cell - u use the unwrapped first cell; recompute them
            if p % 2 == 0:
                first = np.floor(ua[:, ax]) - (p // 2 - 1)
            else:
                first = np.floor(ua[:, ax] + 0.5) - (p - 1) // 2
            s = first[:, None] + np.arange(p) - ua[:, ax][:, None]
            sten.append((cells, w, dweight(p, s)))
        (cx, wx, dx), (cy, wy, dy), (cz, wz, dz) = sten
        for a in range(p):
            for bq in range(p):
                for cq in range(p):
                    gv = gam[cx[:, a], cy[:, bq], cz[:, cq]]
                    out[:, 0] += gv * dx[:, a] * wy[:, bq] * wz[:, cq]
                    out[:, 1] += gv * wx[:, a] * dy[:, bq] * wz[:, cq]
                    out[:, 2] += gv * wx[:, a] * wy[:, bq] * dz[:, cq]
    if weights is not None:
        out *= np.asarray(weights, dtype=np.float64)[:, None]
    return out * (-float(n) / float(box))
