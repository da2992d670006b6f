"""Direct summation (Sec. 2.2) and the footprint DFT of the deposit.

Test infrastructure only (see ``oracle/__init__.py``).

* ``delta_direct``: delta_DS(k) = N_P^-1 sum_j exp(-i k.x_j) for k != 0, the
  alias-free Fourier density of eq. deltaDS in the standard normalisation.
* ``footprint_dft``: the DFT of a deposited grid evaluated particle by
  particle, F(m) = sum_j prod_i sum_t w_{j,i,t} exp(-2 pi i m_i c_{j,i,t}/N),
  with no grid and no FFT (separability of the kernel, Sec. 2.3).
* ``delta_half_direct``: delta_DS at every mode of the half spectrum (the
  layout of ``spectrum.half_axes``), the alias-free reference of Sec. 3.2.
"""

import numpy as np

from .assign import grid_coords, stencil, wrap
from .spectrum import signed_index


def delta_direct(pos, box, modes, chunk=1 << 16):
    """N_P^-1 sum_j exp(-2 pi i m.x_j / L) for integer modes (n_modes, 3)."""
    pos = np.asarray(pos, dtype=np.float64)
    modes = np.asarray(modes, dtype=np.float64).reshape(-1, 3)
    kvec = 2.0 * np.pi / box * modes
    acc = np.zeros(len(modes), dtype=np.complex128)
    for s in range(0, len(pos), chunk):
        ph = pos[s:s + chunk] @ kvec.T
        acc += np.exp(-1j * ph).sum(axis=0)
    return acc / len(pos)


def footprint_dft(pos, box, n_grid, p, modes, shift=0.0, chunk=1 << 21):
    """DFT of the (shifted) deposit at integer modes, without a grid.

    ``shift`` = 0 for the primary grid and 0.5 for the interlaced one.  The
    phase exp(-2 pi i m c / N) of an integer cell c is looked up in a table
    of its N values.
    """
    modes = np.asarray(modes, dtype=np.int64).reshape(-1, 3)
    out = np.zeros(len(modes), dtype=np.complex128)
    pos = np.asarray(pos)
    c_all = np.arange(n_grid)
    tables = [[np.exp(-2j * np.pi * ((m[ax] * c_all) % n_grid) / n_grid) for ax in range(3)]
              for m in modes]
    for s in range(0, len(pos), chunk):
        u = grid_coords(pos[s:s + chunk], box, n_grid) + shift
        per_axis = [stencil(u[:, ax], p, n_grid) for ax in range(3)]
        for i in range(len(modes)):
            f = np.ones(len(u), dtype=np.complex128)
            for ax in range(3):
                cells, w = per_axis[ax]
                f *= (w * tables[i][ax][cells]).sum(axis=1)
            out[i] += f.sum()
    return out


def delta_half_direct(pos, box, n, chunk=4096, weights=None):
    """N_P^-1 sum_j exp(-2 pi i m.x_j / L) on the half spectrum [n][n][n/2+1]
    (with masses: W^-1 sum_j w_j exp(...), W = sum_j w_j).

    Entry (ix, iy, mz) is the mode (signed_index(n)[ix], signed_index(n)[iy],
    mz).  The exponential factorises over the axes, so for a chunk of
    particles the sum is the contraction of three per-axis phase matrices
    exp(-2 pi i m_a x_a / L) over the particle index.
    """
    pos = wrap(np.asarray(pos, dtype=np.float64), box)
    m_full = signed_index(n).astype(np.float64)
    m_half = np.arange(n // 2 + 1, dtype=np.float64)
    out = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    w = None if weights is None else np.asarray(weights, dtype=np.float64)
    for s in range(0, len(pos), chunk):
        t = pos[s:s + chunk] / box
        ex = np.exp(-2j * np.pi * np.outer(m_full, t[:, 0]))
        if w is not None:
            ex = ex * w[s:s + chunk][None, :]
        ey = np.exp(-2j * np.pi * np.outer(m_full, t[:, 1]))
        ez = np.exp(-2j * np.pi * np.outer(m_half, t[:, 2]))
        exy = ex[:, None, :] * ey[None, :, :]
        out += np.matmul(exy.reshape(n * n, -1), ez.T).reshape(n, n, n // 2 + 1)
    return out / (len(pos) if w is None else w.sum())
