"""ctypes access to the plain-C loops of the oracle (oracle/csrc/oracle_loops.c).

Test infrastructure only (see ``oracle/__init__.py``).  Same arithmetic as
``assign.deposit``, ``assign.cell_values``, ``direct.footprint_dft`` and
``spectrum.mode_table`` for inputs too large for the numpy forms; pinned
against them by the CPU tests.  The library is built with
gcc on first use (or by ``__graft_entry__.build()``).
"""

import ctypes
import os
import subprocess

import numpy as np

from .assign import grid_coords

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "csrc", "oracle_loops.c")
LIB = os.path.join(_HERE, "_oracle_loops.so")
_lib = None


def build():
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-shared", "-fPIC", "-o",
                    tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        d, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.oracle_deposit.argtypes = [d, i64, i64, i32, d]
        lib.oracle_deposit.restype = None
        lib.oracle_deposit_slabs.argtypes = [d, i64, i64, i32, d]
        lib.oracle_deposit_slabs.restype = None
        lib.oracle_footprint_dft.argtypes = [d, i64, i64, i32, d, i64, d, d]
        lib.oracle_footprint_dft.restype = None
        lib.oracle_cell_values.argtypes = [d, i64, i64, i32, d, i64, d]
        lib.oracle_cell_values.restype = None
        lib.oracle_mode_table.argtypes = [i64, i64, i64, d, d]
        lib.oracle_mode_table.restype = None
        _lib = lib
    return _lib


def _u(pos, box, n, shift):
    return np.ascontiguousarray(grid_coords(np.asarray(pos), box, n) + shift, dtype=np.float64)


def deposit(pos, box, n, p, shift=0.0):
    """Grid (N, N, N) float64 of the particles sampled at u + shift."""
    u = _u(pos, box, n, shift)
    rho = np.zeros(n * n * n, dtype=np.float64)
    _load().oracle_deposit(u.ctypes.data, len(u), n, p, rho.ctypes.data)
    return rho.reshape(n, n, n)


def deposit_u_slabs(u, n, p):
    """Grid (N, N, N) float64 of particles at grid coordinates u (n_p, 3),
    deposited by the x-plane-parallel C loop (equal to ``deposit`` bit for
    bit)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    rho = np.zeros(n * n * n, dtype=np.float64)
    _load().oracle_deposit_slabs(u.ctypes.data, len(u), n, p, rho.ctypes.data)
    return rho.reshape(n, n, n)


def deposit_slabs(pos, box, n, p, shift=0.0):
    """Same as ``deposit`` through the x-plane-parallel C loop."""
    return deposit_u_slabs(_u(pos, box, n, shift), n, p)


def footprint_dft(pos, box, n, p, modes, shift=0.0):
    """Same as ``direct.footprint_dft``."""
    u = _u(pos, box, n, shift)
    modes = np.ascontiguousarray(np.asarray(modes, dtype=np.int64).reshape(-1, 3))
    re = np.zeros(len(modes))
    im = np.zeros(len(modes))
    _load().oracle_footprint_dft(u.ctypes.data, len(u), n, p, modes.ctypes.data, len(modes),
                                 re.ctypes.data, im.ctypes.data)
    return re + 1j * im


def cell_values(pos, box, n, p, cells, shift=0.0):
    """Same as ``assign.cell_values``."""
    u = _u(pos, box, n, shift)
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).reshape(-1, 3))
    out = np.zeros(len(cells))
    _load().oracle_cell_values(u.ctypes.data, len(u), n, p, cells.ctypes.data, len(cells),
                               out.ctypes.data)
    return out


def mode_table(n, n_dk, n_bins):
    """Same as ``spectrum.mode_table``."""
    counts = np.zeros(n_bins, dtype=np.int64)
    ksum = np.zeros(n_bins)
    _load().oracle_mode_table(n, n_dk, n_bins, counts.ctypes.data, ksum.ctypes.data)
    return counts, ksum


def delta_modes(pos, box, n, p, interlace_on, modes):
    """delta(m) = C(m) / (N_P W(m)) at signed modes (the oracle's steps 1-3
    evaluated mode by mode through the footprint DFT)."""
    from .kernels import window_1d
    from .spectrum import mask_shift, shift_masks
    modes = np.asarray(modes, dtype=np.int64).reshape(-1, 3)
    masks = shift_masks(interlace_on)
    if len(masks) == 1:
        c = footprint_dft(pos, box, n, p, modes, 0.0)
    elif len(masks) == 2:
        f1 = footprint_dft(pos, box, n, p, modes, 0.0)
        f2 = footprint_dft(pos, box, n, p, modes, 0.5)
        c = 0.5 * (f1 + np.exp(1j * np.pi * modes.sum(axis=1) / n) * f2)
    else:
        c = 0.0
        for mk in masks:
            sel = np.array([(mk >> a) & 1 for a in range(3)])
            c = c + np.exp(1j * np.pi * (modes * sel).sum(axis=1) / n) \
                * footprint_dft(pos, box, n, p, modes, mask_shift(mk))
        c = c / len(masks)
    w = np.prod(window_1d(p, modes, n), axis=1)
    return c / (len(pos) * w)


def delta_half(pos, box, n, p, interlace_on):
    """Same as ``spectrum.delta_half`` with the deposit done by the C loops."""
    from . import spectrum
    pos = np.asarray(pos)
    masks = spectrum.shift_masks(interlace_on)
    if len(masks) > 2:
        fs = [spectrum.fft_grid(deposit(pos, box, n, p, spectrum.mask_shift(mk))) for mk in masks]
        return spectrum.combine(fs, masks, n) / (len(pos) * spectrum.window(n, p)), len(pos)
    f1 = spectrum.fft_grid(deposit(pos, box, n, p, 0.0))
    if interlace_on:
        f2 = spectrum.fft_grid(deposit(pos, box, n, p, 0.5))
        c = spectrum.interlace(f1, f2, n)
    else:
        c = f1
    return c / (len(pos) * spectrum.window(n, p)), len(pos)


def power(pos, box, n, p, interlace_on, n_dk=1, n_bins=None):
    """The oracle P(k) with the deposit done by the C loops."""
    from . import spectrum
    if n_bins is None:
        n_bins = spectrum.max_bins(n, n_dk)
    delta, _ = delta_half(pos, box, n, p, interlace_on)
    return spectrum.bin_power(delta, box, n, n_dk, n_bins)


def power_large(pos, box, n, p, interlace_on, n_dk=1, n_bins=None, planes=16, band=0):
    """The oracle P(k) (``spectrum.power``: equal masses, raw P) for grids too
    large for the all-at-once numpy form: both deposits by the x-plane
    parallel C loop, one grid at a time (F_1 = FFT(rho_1) is kept while
    rho_2 is deposited and transformed), then delta = C / (N_P W) formed and
    binned ``planes`` x planes at a time with the same spectrum functions.

    Returns (k_b, P_b, N_b) and, when ``band`` > 0, delta at every mode with
    all |m_a| <= band as a dense complex array d[m_x + band, m_y + band, m_z]
    (m_z = 0 .. band) for brute-force checks on the low shells."""
    from . import spectrum
    if int(interlace_on) not in (0, 1):
        raise ValueError("power_large handles one grid or the interlaced pair")
    if n_bins is None:
        n_bins = spectrum.max_bins(n, n_dk)
    pos = np.asarray(pos)
    n_p = float(len(pos))
    u = _u(pos, box, n, 0.0)
    f1 = spectrum.fft_grid(deposit_u_slabs(u, n, p))
    f2 = None
    if interlace_on:
        u += 0.5  # the grid sampled at u + 1/2
        f2 = spectrum.fft_grid(deposit_u_slabs(u, n, p))
    del u
    sums = np.zeros(n_bins)
    d_band = np.zeros((2 * band + 1, 2 * band + 1, band + 1), dtype=np.complex128) if band else None
    for x0 in range(0, n, planes):
        x1 = min(n, x0 + planes)
        c = spectrum.interlace(f1[x0:x1], f2[x0:x1], n, x0) if interlace_on else f1[x0:x1]
        delta = c / (n_p * spectrum.window(n, p, x0, x1))
        sums += spectrum.shell_sums(delta, box, n, n_dk, n_bins, x0)
        if band:
            for ix in range(x0, x1):
                mx = ix if ix <= n // 2 else ix - n
                if abs(mx) > band:
                    continue
                for my in range(-band, band + 1):
                    d_band[mx + band, my + band, :] = delta[ix - x0, my % n, :band + 1]
    counts, ksum = mode_table(n, n_dk, n_bins)
    kf = 2.0 * np.pi / box
    with np.errstate(invalid="ignore", divide="ignore"):
        k = kf * ksum / counts
        pk = sums / counts
    if band:
        return k, pk, counts, d_band
    return k, pk, counts
