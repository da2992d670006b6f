"""Interlaced order-p Fourier-space estimators on AMD MI355X (gfx950).

Thin ctypes binding of ``libfsest.so`` (declared in ``include/fsest.h``).
The functions ``estimator_*`` below carry the C names and only marshal
arguments: device pointers may be given as integers or as torch tensors
(their ``data_ptr()`` is used).  Every non-zero status raises
:class:`FsestError` with the library's message.  There is no CPU fallback:
importing this package fails loudly when the HIP library is missing.

Higher-level helpers (workspace allocation with torch, outputs as tensors,
autograd) live in :mod:`paper_1512_07295_amd.estimator`.
"""

import ctypes
import os

# torch ships its own HIP runtime.  It must be loaded before libfsest.so so
# that the library's libamdhip64 dependency resolves to that same runtime:
# loaded first, the library would bring in a second HIP runtime, which then
# sees no device, and stream handles would not be shared.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsest.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libfsest.so is not built (%s); run `python paper_1512_07295_amd/build.py`" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

EST_OK, EST_EINVAL, EST_ENOMEM, EST_ESTATE, EST_EDEVICE, EST_EUNSUPPORTED = range(6)
EST_F32, EST_F64 = 0, 1
EST_FLAG_ATOMIC_SORT = 1
EST_FLAG_WEIGHTS = 2
STATUS_NAMES = {0: "EST_OK", 1: "EST_EINVAL", 2: "EST_ENOMEM", 3: "EST_ESTATE",
                4: "EST_EDEVICE", 5: "EST_EUNSUPPORTED"}

# every symbol declared in include/fsest.h
EXPORTS = [
    "estimator_workspace_bytes", "estimator_create", "estimator_destroy",
    "estimator_deposit", "estimator_transform", "estimator_power",
    "estimator_bispectrum_workspace_bytes", "estimator_bispectrum",
    "estimator_backward", "estimator_graph_capture", "estimator_graph_launch",
    "estimator_autotune", "estimator_set_launch", "estimator_set_weights", "estimator_copy_grid",
    "estimator_sample_delta",
    "estimator_direct_workspace_bytes", "estimator_direct_delta", "estimator_direct_delta_noalloc",
    "estimator_export_delta",
    "estimator_spectrum_power",
    "estimator_profile", "estimator_profile_read", "estimator_last_error",
]


class est_config(ctypes.Structure):
    _fields_ = [
        ("n_grid", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("interlace", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("box", ctypes.c_double),
        ("max_particles", ctypes.c_int64),
        ("flags", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class FsestError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t

_SIGS = {
    "estimator_workspace_bytes": [ctypes.POINTER(est_config), ctypes.POINTER(_SZ)],
    "estimator_create": [ctypes.POINTER(est_config), _P, _SZ, _P, ctypes.POINTER(_P)],
    "estimator_destroy": [_P],
    "estimator_deposit": [_P, _P, _I32, _P, _I64],
    "estimator_transform": [_P],
    "estimator_power": [_P, _I32, _I32, _I32, _P, _P, _P],
    "estimator_bispectrum_workspace_bytes": [_P, _I32, _I32, _I64, ctypes.POINTER(_SZ)],
    "estimator_bispectrum": [_P, _I32, _I32, _I32, _P, _I64, _P, _SZ, _P, _P],
    "estimator_backward": [_P, _P, _I32, _P, _I64, _P, _I32, _I32, _P],
    "estimator_graph_capture": [_P, _P, _I32, _P, _I64, _I32, _I32, _I32, _P, _P, _P],
    "estimator_graph_launch": [_P],
    "estimator_autotune": [_P, _P, _I32, _P, _I64, _I32, _I32, _I32, ctypes.POINTER(_I32)],
    "estimator_set_launch": [_P, _I32],
    "estimator_set_weights": [_P, _P],
    "estimator_copy_grid": [_P, _I32, _I32, _P],
    "estimator_sample_delta": [_P, _I32, _P, _I64, _P],
    "estimator_direct_workspace_bytes": [_P, _I64, ctypes.POINTER(_SZ)],
    "estimator_direct_delta": [_P, _P, _I32, _I64, _P, _SZ, _P],
    "estimator_direct_delta_noalloc": [_P, _P, _I32, _I64, _P],
    "estimator_export_delta": [_P, _I32, _P],
    "estimator_spectrum_power": [_P, _P, _P, _I32, _I32, ctypes.c_double, _P, _P, _P],
    "estimator_profile": [_P, _I32],
    "estimator_profile_read": [_P, _I32, ctypes.c_char_p, _SZ, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(_I64), ctypes.POINTER(_I32)],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.estimator_last_error.argtypes = []
_lib.estimator_last_error.restype = ctypes.c_char_p


def _ptr(x):
    """Device/host address of a torch tensor, an int, or None."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(int(x))


def _check(status):
    if status != EST_OK:
        raise FsestError(status, estimator_last_error())


def make_config(n_grid, box, order=4, interlace=1, batch=1, max_particles=1, flags=0):
    return est_config(int(n_grid), int(order), int(interlace), int(batch), float(box),
                      int(max_particles), int(flags), 0)


def estimator_last_error():
    return _lib.estimator_last_error().decode(errors="replace")


def estimator_workspace_bytes(cfg):
    out = _SZ(0)
    _check(_lib.estimator_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)))
    return int(out.value)


def estimator_create(cfg, workspace, workspace_bytes, stream=None):
    h = _P()
    _check(_lib.estimator_create(ctypes.byref(cfg), _ptr(workspace), _SZ(int(workspace_bytes)),
                                 _ptr(stream), ctypes.byref(h)))
    return h


def estimator_destroy(h):
    _check(_lib.estimator_destroy(h))


def estimator_deposit(h, pos, dtype, offsets, n_total):
    _check(_lib.estimator_deposit(h, _ptr(pos), int(dtype), _ptr(offsets), int(n_total)))


def estimator_transform(h):
    _check(_lib.estimator_transform(h))


def estimator_power(h, n_dk, n_bins, subtract_shot, k, p, nmodes):
    _check(_lib.estimator_power(h, int(n_dk), int(n_bins), int(subtract_shot), _ptr(k), _ptr(p),
                                _ptr(nmodes)))


def estimator_bispectrum_workspace_bytes(h, n_dk, n_bins, n_tri):
    out = _SZ(0)
    _check(_lib.estimator_bispectrum_workspace_bytes(h, int(n_dk), int(n_bins), int(n_tri),
                                                     ctypes.byref(out)))
    return int(out.value)


def estimator_bispectrum(h, mock, n_dk, n_bins, tri_host, n_tri, bws, bws_bytes, b, ntri):
    """``tri_host``: a C-contiguous int32 numpy array (n_tri, 3) in host memory."""
    tri_ptr = ctypes.c_void_p(tri_host.ctypes.data) if hasattr(tri_host, "ctypes") else _ptr(tri_host)
    _check(_lib.estimator_bispectrum(h, int(mock), int(n_dk), int(n_bins), tri_ptr, int(n_tri),
                                     _ptr(bws), _SZ(int(bws_bytes)), _ptr(b), _ptr(ntri)))


def estimator_backward(h, pos, dtype, offsets, n_total, dldp, n_dk, n_bins, grad):
    _check(_lib.estimator_backward(h, _ptr(pos), int(dtype), _ptr(offsets), int(n_total),
                                   _ptr(dldp), int(n_dk), int(n_bins), _ptr(grad)))


def estimator_graph_capture(h, pos, dtype, offsets, n_total, n_dk, n_bins, subtract_shot, k, p,
                            nmodes):
    _check(_lib.estimator_graph_capture(h, _ptr(pos), int(dtype), _ptr(offsets), int(n_total),
                                        int(n_dk), int(n_bins), int(subtract_shot), _ptr(k),
                                        _ptr(p), _ptr(nmodes)))


def estimator_graph_launch(h):
    _check(_lib.estimator_graph_launch(h))


def estimator_autotune(h, pos, dtype, offsets, n_total, n_dk, n_bins, iters):
    choice = _I32(-1)
    _check(_lib.estimator_autotune(h, _ptr(pos), int(dtype), _ptr(offsets), int(n_total),
                                   int(n_dk), int(n_bins), int(iters), ctypes.byref(choice)))
    return int(choice.value)


def estimator_set_launch(h, choice):
    _check(_lib.estimator_set_launch(h, int(choice)))


def estimator_set_weights(h, weights):
    _check(_lib.estimator_set_weights(h, _ptr(weights)))


def estimator_copy_grid(h, which, mock, dst):
    _check(_lib.estimator_copy_grid(h, int(which), int(mock), _ptr(dst)))


def estimator_sample_delta(h, mock, modes, n, out):
    _check(_lib.estimator_sample_delta(h, int(mock), _ptr(modes), int(n), _ptr(out)))


def estimator_direct_workspace_bytes(h, n):
    out = _SZ(0)
    _check(_lib.estimator_direct_workspace_bytes(h, int(n), ctypes.byref(out)))
    return int(out.value)


def estimator_direct_delta(h, pos, dtype, n, dws, dws_bytes, out):
    _check(_lib.estimator_direct_delta(h, _ptr(pos), int(dtype), int(n), _ptr(dws),
                                       _SZ(int(dws_bytes)), _ptr(out)))


def estimator_direct_delta_noalloc(h, pos, dtype, n, out):
    _check(_lib.estimator_direct_delta_noalloc(h, _ptr(pos), int(dtype), int(n), _ptr(out)))


def estimator_export_delta(h, mock, out):
    _check(_lib.estimator_export_delta(h, int(mock), _ptr(out)))


def estimator_spectrum_power(h, a, b, n_dk, n_bins, shot, k, p, nmodes):
    _check(_lib.estimator_spectrum_power(h, _ptr(a), _ptr(b), int(n_dk), int(n_bins),
                                         ctypes.c_double(float(shot)), _ptr(k), _ptr(p),
                                         _ptr(nmodes)))


def estimator_profile(h, enable):
    _check(_lib.estimator_profile(h, int(enable)))


def estimator_profile_read(h, idx):
    """(name, total_ms, launches, n_labels) of profiling label ``idx``."""
    name = ctypes.create_string_buffer(64)
    ms = ctypes.c_double(0.0)
    cnt = _I64(0)
    nl = _I32(0)
    _check(_lib.estimator_profile_read(h, int(idx), name, 64, ctypes.byref(ms), ctypes.byref(cnt),
                                       ctypes.byref(nl)))
    return name.value.decode(), float(ms.value), int(cnt.value), int(nl.value)


def profile_table(h):
    """{label: (total_ms, launches)} for every label with at least one launch."""
    first = estimator_profile_read(h, 0)
    out = {}
    for i in range(first[3]):
        name, ms, cnt, _ = estimator_profile_read(h, i)
        if cnt:
            out[name] = (ms, cnt)
    return out
