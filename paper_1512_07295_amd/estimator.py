"""Torch-facing helpers over the C ABI: workspace allocation, tensor outputs,
graph replay and the autograd function of P(k).

PyTorch only provides device memory and the stream; every step of the
estimator runs in the HIP kernels of ``libfsest.so``.
"""

import numpy as np
import torch

from . import (EST_F32, EST_F64, EST_FLAG_ATOMIC_SORT, EST_FLAG_WEIGHTS, estimator_autotune, estimator_backward, estimator_bispectrum,
               estimator_bispectrum_workspace_bytes, estimator_copy_grid, estimator_create,
               estimator_deposit, estimator_destroy, estimator_direct_delta,
               estimator_direct_workspace_bytes, estimator_export_delta, estimator_graph_capture,
               estimator_graph_launch, estimator_power, estimator_sample_delta, estimator_set_launch,
               estimator_set_weights,
               estimator_spectrum_power, estimator_transform, estimator_workspace_bytes,
               make_config)


def _dtype_code(t):
    if t.dtype == torch.float32:
        return EST_F32
    if t.dtype == torch.float64:
        return EST_F64
    raise TypeError("positions must be float32 or float64")


def _check_pos(pos):
    if not pos.is_cuda:
        raise ValueError("positions must be a device tensor")
    if pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_contiguous():
        raise ValueError("positions must be a contiguous (n, 3) tensor")


def _aligned_workspace(nbytes, device):
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


class Estimator:
    """One handle: grid size N, box L, order p, interlacing, batch of sets."""

    def __init__(self, n_grid, box, order=4, interlace=True, batch=1, max_particles=1 << 20,
                 device="cuda", stream=None, atomic_sort=False, weighted=False):
        self.n_grid = int(n_grid)
        self.box = float(box)
        self.order = int(order)
        self.interlace = int(interlace)  # 0..3 (grids: 1, 2, 4, 8)
        self.batch = int(batch)
        self.device = torch.device(device)
        flags = (EST_FLAG_ATOMIC_SORT if atomic_sort else 0) | (EST_FLAG_WEIGHTS if weighted else 0)
        self.cfg = make_config(n_grid, box, order, int(interlace), batch, max_particles, flags)
        self.ws_bytes = estimator_workspace_bytes(self.cfg)
        self._ws, self._ws_ptr = _aligned_workspace(self.ws_bytes, self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = estimator_create(self.cfg, self._ws_ptr, self.ws_bytes, self.stream.cuda_stream)
        self._graph_bufs = None
        self._weights = None

    def set_weights(self, weights):
        """Per-particle masses (float32 device tensor of n entries, in the
        order of the positions of the following calls) or None for equal
        masses.  The tensor is kept alive by the handle."""
        if weights is not None:
            if not weights.is_cuda or weights.dtype != torch.float32 or weights.dim() != 1 \
                    or not weights.is_contiguous():
                raise ValueError("weights must be a contiguous float32 device vector")
        estimator_set_weights(self.h, weights)
        self._weights = weights

    def _check_weights(self, n):
        if self._weights is not None and self._weights.shape[0] < n:
            raise ValueError("weights hold %d entries, %d particles given" % (self._weights.shape[0], n))

    def close(self):
        if getattr(self, "h", None) is not None:
            estimator_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _outputs(self, n_bins):
        k = torch.empty((self.batch, n_bins), dtype=torch.float64, device=self.device)
        p = torch.empty_like(k)
        nm = torch.empty((self.batch, n_bins), dtype=torch.int64, device=self.device)
        return k, p, nm

    def default_bins(self, n_dk):
        return self.n_grid // (2 * n_dk)

    # ---- forward
    def deposit(self, pos, offsets=None):
        _check_pos(pos)
        self._check_weights(pos.shape[0])
        estimator_deposit(self.h, pos, _dtype_code(pos), offsets, pos.shape[0])

    def transform(self):
        estimator_transform(self.h)

    def power_only(self, n_dk=1, n_bins=None, subtract_shot=False):
        n_bins = n_bins or self.default_bins(n_dk)
        k, p, nm = self._outputs(n_bins)
        estimator_power(self.h, n_dk, n_bins, int(subtract_shot), k, p, nm)
        return k, p, nm

    def power(self, pos, offsets=None, n_dk=1, n_bins=None, subtract_shot=False):
        """(k, P, N_modes), each [batch, n_bins], for the particle set(s) ``pos``."""
        self.deposit(pos, offsets)
        self.transform()
        return self.power_only(n_dk, n_bins, subtract_shot)

    def bispectrum(self, triangles, n_dk=2, n_bins=None, mock=0):
        """FFT-shell bispectrum of set ``mock`` after ``power``/``transform``.

        ``triangles``: int array (n_tri, 3), 1 <= b3 <= b2 <= b1 <= n_bins.
        Returns (B, N_tri) as float64 device tensors.
        """
        tri = np.ascontiguousarray(np.asarray(triangles, dtype=np.int32).reshape(-1, 3))
        if n_bins is None:
            n_bins = int(tri.max())
        nbytes = estimator_bispectrum_workspace_bytes(self.h, n_dk, n_bins, len(tri))
        buf, ptr = _aligned_workspace(nbytes, self.device)
        bk = torch.empty(len(tri), dtype=torch.float64, device=self.device)
        nt = torch.empty_like(bk)
        estimator_bispectrum(self.h, mock, n_dk, n_bins, tri, len(tri), ptr, nbytes, bk, nt)
        del buf
        return bk, nt

    # ---- adjoint
    def backward(self, pos, dldp, offsets=None, n_dk=1, n_bins=None):
        _check_pos(pos)
        n_bins = n_bins or self.default_bins(n_dk)
        dldp = dldp.to(device=self.device, dtype=torch.float64).contiguous()
        if dldp.numel() != self.batch * n_bins:
            raise ValueError("dL/dP must have batch * n_bins entries")
        self._check_weights(pos.shape[0])
        grad = torch.empty_like(pos)
        estimator_backward(self.h, pos, _dtype_code(pos), offsets, pos.shape[0], dldp, n_dk,
                           n_bins, grad)
        return grad

    # ---- graph replay
    def capture(self, pos, offsets=None, n_dk=1, n_bins=None, subtract_shot=False):
        _check_pos(pos)
        n_bins = n_bins or self.default_bins(n_dk)
        self._check_weights(pos.shape[0])
        k, p, nm = self._outputs(n_bins)
        estimator_graph_capture(self.h, pos, _dtype_code(pos), offsets, pos.shape[0], n_dk,
                                n_bins, int(subtract_shot), k, p, nm)
        self._graph_bufs = (pos, offsets, k, p, nm)
        return k, p, nm

    def replay(self):
        estimator_graph_launch(self.h)
        return self._graph_bufs[2:]

    def autotune(self, pos, offsets=None, n_dk=1, n_bins=None, iters=3):
        _check_pos(pos)
        n_bins = n_bins or self.default_bins(n_dk)
        self._check_weights(pos.shape[0])
        return estimator_autotune(self.h, pos, _dtype_code(pos), offsets, pos.shape[0], n_dk,
                                  n_bins, iters)

    def set_launch(self, choice):
        estimator_set_launch(self.h, choice)

    # ---- test hooks
    def copy_grid(self, which=1, mock=0):
        out = torch.empty((self.n_grid,) * 3, dtype=torch.float32, device=self.device)
        estimator_copy_grid(self.h, which, mock, out)
        return out

    def sample_delta(self, modes, mock=0):
        m = torch.as_tensor(np.asarray(modes, dtype=np.int32).reshape(-1, 3), device=self.device)
        out = torch.empty((m.shape[0], 2), dtype=torch.float64, device=self.device)
        estimator_sample_delta(self.h, mock, m, m.shape[0], out)
        return torch.complex(out[:, 0], out[:, 1])

    # ---- direct summation and half-spectrum statistics
    def _half(self):
        n = self.n_grid
        return torch.empty((n, n, n // 2 + 1, 2), dtype=torch.float64, device=self.device)

    def direct_delta(self, pos):
        """delta_DS on the half spectrum ([N, N, N/2+1, 2] float64) by direct summation."""
        _check_pos(pos)
        n = pos.shape[0]
        self._check_weights(n)
        nbytes = estimator_direct_workspace_bytes(self.h, n)
        ws, ws_ptr = _aligned_workspace(nbytes, self.device)
        out = self._half()
        estimator_direct_delta(self.h, pos, _dtype_code(pos), n, ws_ptr, nbytes, out)
        self.stream.synchronize()  # the workspace is released on return
        del ws
        return out

    def export_delta(self, mock=0):
        """The estimator's delta(m) on the half spectrum ([N, N, N/2+1, 2] float64)."""
        out = self._half()
        estimator_export_delta(self.h, mock, out)
        return out

    def spectrum_power(self, a, b=None, n_dk=1, n_bins=None, shot=0.0):
        """(k, P, N) with P = V <Re(a b*)> per shell - shot (b = a if None)."""
        if n_bins is None:
            n_bins = self.n_grid // (2 * n_dk)
        k = torch.empty(n_bins, dtype=torch.float64, device=self.device)
        p = torch.empty_like(k)
        nm = torch.empty(n_bins, dtype=torch.int64, device=self.device)
        estimator_spectrum_power(self.h, a, b, n_dk, n_bins, shot, k, p, nm)
        return k, p, nm


class PowerSpectrumFn(torch.autograd.Function):
    """P(k) of particle positions with a hand-written adjoint.

    forward(pos, est, n_dk, n_bins, offsets) -> P [batch, n_bins] (raw);
    backward recomputes the grids and returns dL/dpos.
    """

    @staticmethod
    def forward(ctx, pos, est, n_dk=1, n_bins=None, offsets=None):
        n_bins = n_bins or est.default_bins(n_dk)
        _, p, _ = est.power(pos.detach(), offsets, n_dk, n_bins)
        ctx.est = est
        ctx.cfg = (n_dk, n_bins, offsets)
        ctx.save_for_backward(pos)
        return p

    @staticmethod
    def backward(ctx, dldp):
        (pos,) = ctx.saved_tensors
        n_dk, n_bins, offsets = ctx.cfg
        grad = ctx.est.backward(pos.detach(), dldp, offsets, n_dk, n_bins)
        return grad, None, None, None, None
