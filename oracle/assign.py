"""Wrap, locate and deposit particles on the primary and interlaced grids.

Test infrastructure only (see ``oracle/__init__.py``).

Follows Sec. 2.3 (eq. delgrid: each grid point receives the cell-integrated
kernel weight of every particle, W(x) = W^(p)(x/H) W^(p)(y/H) W^(p)(z/H)) and
Sec. 3.1 (a second grid shifted by H/2 along every axis).  Readings:

* Grid origin: grid-1 points sit at x = g H, g = 0..N-1, H = L/N.
* Periodic box (Sec. 2.1): positions are wrapped into [0, L) with the fixed
  float64 sequence of ``wrap``; a value that rounds to L maps to 0.
* Index arithmetic: u = fl64(x_wrapped * fl64(N / L)) in float64, so that the
  cell choice is the same wherever the same float64 sequence is used.
* Interlaced grid: sampling at x + H/2, i.e. u2 = fl64(u + 1/2) on the same
  index lattice; its Fourier transform is later multiplied by
  exp(+i pi (m_x + m_y + m_z)/N) (eq. intdelta, shift theorem).
* Stencil: even p -> first cell floor(u) - (p/2 - 1); odd p -> first cell
  floor(u + 1/2) - (p - 1)/2; p consecutive cells, indices mod N; the
  weights are W^(p)(cell - u) (NGP: 1 for its single cell).

The density grid is rho[g] = sum_j prod_axes W^(p)(g_i - u_{j,i}); it sums to
N_P.  The overdensity of eq. delgrid is rho / (N_P / N^3) - 1; the constant
only affects the k = 0 mode, which no estimator uses.

Weighted particles (the paper takes equal masses for simplicity, Sec. 2.1):
particle j carries a mass w_j >= 0, rho[g] = sum_j w_j prod_axes W^(p)(...),
which sums to W = sum_j w_j; unit weights give the equal-mass grid.
"""

import numpy as np

from .kernels import weight


def wrap(x, box):
    """Periodic wrap into [0, L) in float64 (fixed operation sequence).

    x - L floor(x/L), +L if negative, -L if >= L, 0 if still outside [0, L).
    For x already in [0, L) the sequence returns x itself, so only the other
    entries are evaluated.
    """
    x = np.array(x, dtype=np.float64)
    bad = ~((x >= 0.0) & (x < box))
    if bad.any():
        xb = x[bad]
        q = np.floor(xb / box)
        xw = xb - q * box
        xw = np.where(xw < 0.0, xw + box, xw)
        xw = np.where(xw >= box, xw - box, xw)
        ok = (xw >= 0.0) & (xw < box)
        x[bad] = np.where(ok, xw, 0.0)
    return x


def grid_coords(pos, box, n_grid):
    """u = fl64(wrap(x) * fl64(N/L)) for every particle and axis, shape (n, 3)."""
    inv = np.float64(n_grid) / np.float64(box)
    return wrap(pos, box) * inv


def stencil(u, p, n_grid):
    """Cells (mod N) and weights of the p-point stencil along one axis.

    Returns (cells, weights), each of shape u.shape + (p,).
    """
    u = np.asarray(u, dtype=np.float64)
    if p % 2 == 0:
        first = np.floor(u) - (p // 2 - 1)
    else:
        first = np.floor(u + 0.5) - (p - 1) // 2
    cells = first[..., None] + np.arange(p, dtype=np.float64)
    if p == 1:
        # the nearest cell gets the whole particle (evaluating W^(1) at the
        # rounded offset could drop it when fl64(u + 1/2) rounds up)
        w = np.ones_like(cells)
    else:
        w = weight(p, cells - u[..., None])
    cells_i = np.mod(cells.astype(np.int64), n_grid)
    return cells_i, w


def deposit_u(u, p, n_grid, weights=None):
    """Deposit particles given their float64 grid coordinates u (n, 3) and
    optional masses (n,)."""
    n = n_grid
    cx, wx = stencil(u[:, 0], p, n)
    cy, wy = stencil(u[:, 1], p, n)
    cz, wz = stencil(u[:, 2], p, n)
    rho = np.zeros(n * n * n, dtype=np.float64)
    if weights is not None:
        wx = wx * np.asarray(weights, dtype=np.float64)[:, None]
    for a in range(p):
        for b in range(p):
            wab = wx[:, a] * wy[:, b]
            base = (cx[:, a] * n + cy[:, b]) * n
            for c in range(p):
                rho += np.bincount(base + cz[:, c], weights=wab * wz[:, c],
                                   minlength=n * n * n)
    return rho.reshape(n, n, n)


def deposit(pos, box, n_grid, p, interlace, weights=None):
    """Primary grid rho1 and (if ``interlace``) the H/2-shifted grid rho2.

    ``pos`` is (N_P, 3) in any float dtype; it is promoted to float64, as
    are the optional masses ``weights`` (N_P,).  Returns (rho1, rho2 or
    None), float64 arrays of shape (N, N, N) indexed [x, y, z] with z fastest.
    """
    u = grid_coords(pos, box, n_grid)
    rho1 = deposit_u(u, p, n_grid, weights)
    rho2 = deposit_u(u + 0.5, p, n_grid, weights) if interlace else None
    return rho1, rho2


def cell_values(pos, box, n_grid, p, cells, shift=0.0):
    """rho at the given integer cells (k, 3) of the grid sampled at u + shift,
    summing the stencil weights of every particle whose stencil holds the
    cell (the same sum as ``deposit_u`` restricted to those cells)."""
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    u = grid_coords(pos, box, n_grid) + shift
    out = np.zeros(len(cells), dtype=np.float64)
    base = np.floor(u).astype(np.int64)
    for i, g in enumerate(cells):
        # stencils reach at most 3 cells from floor(u) on either side
        d = np.mod(base - g, n_grid)
        near = np.all((d <= 3) | (d >= n_grid - 3), axis=1)
        un = u[near]
        wsum = np.ones(len(un))
        for ax in range(3):
            c, w = stencil(un[:, ax], p, n_grid)
            wsum *= np.where(c == g[ax], w, 0.0).sum(axis=1)
        out[i] = wsum.sum()
    return out
