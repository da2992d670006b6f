"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every symbol declared in include/fsest.h, and
reject invalid arguments on the host before touching the device.
"""

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsest.h")

fsest = pytest.importorskip("paper_1512_07295_amd", reason="libfsest.so not built")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(estimator_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert _declared() == sorted(fsest.EXPORTS)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", fsest.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = set(re.findall(r"\s[TW]\s+(\S+)$", out, flags=re.M))
    for name in _declared():
        assert name in syms, name
        assert getattr(fsest._lib, name) is not None


def _cfg(**kw):
    base = dict(n_grid=32, box=1000.0, order=4, interlace=1, batch=1, max_particles=1000)
    base.update(kw)
    return fsest.make_config(**base)


def test_workspace_bytes_valid_and_monotone():
    a = fsest.estimator_workspace_bytes(_cfg(n_grid=16))
    b = fsest.estimator_workspace_bytes(_cfg(n_grid=32))
    c = fsest.estimator_workspace_bytes(_cfg(n_grid=32, interlace=0))
    d = fsest.estimator_workspace_bytes(_cfg(n_grid=32, batch=4))
    assert 0 < a < b and c < b < d
    big = fsest.estimator_workspace_bytes(_cfg(n_grid=1024, max_particles=512 ** 3))
    # two float32 grids of 1024^3 dominate
    assert big > 2 * 4 * 1024 ** 3


@pytest.mark.parametrize("kw,status", [
    (dict(order=0), fsest.EST_EINVAL),
    (dict(order=7), fsest.EST_EINVAL),
    (dict(interlace=4), fsest.EST_EINVAL),
    (dict(interlace=3, batch=20000), fsest.EST_EINVAL),  # 4 complex grids per set
    (dict(interlace=-1), fsest.EST_EINVAL),
    (dict(batch=0), fsest.EST_EINVAL),
    (dict(box=0.0), fsest.EST_EINVAL),
    (dict(box=-1.0), fsest.EST_EINVAL),
    (dict(box=float("inf")), fsest.EST_EINVAL),
    (dict(box=float("nan")), fsest.EST_EINVAL),
    (dict(max_particles=0), fsest.EST_EINVAL),
    (dict(max_particles=1 << 31), fsest.EST_EINVAL),
    (dict(flags=4), fsest.EST_EINVAL),
    (dict(flags=-1), fsest.EST_EINVAL),
    (dict(n_grid=28), fsest.EST_EUNSUPPORTED),   # prime factor 7
    (dict(n_grid=90), fsest.EST_EUNSUPPORTED),   # not a multiple of the 4-cell bucket
    (dict(n_grid=1020), fsest.EST_EUNSUPPORTED),  # prime factor 17
    (dict(n_grid=20, order=6), fsest.EST_EUNSUPPORTED),  # N < 16 + p - 1 with 16-cell tiles
    (dict(n_grid=4), fsest.EST_EUNSUPPORTED),
    (dict(n_grid=2048), fsest.EST_EUNSUPPORTED),
    (dict(n_grid=1024, batch=300), fsest.EST_EINVAL),
])
def test_invalid_config_rejected_on_host(kw, status):
    with pytest.raises(fsest.FsestError) as ei:
        fsest.estimator_workspace_bytes(_cfg(**kw))
    assert ei.value.status == status
    assert fsest.estimator_last_error() != ""


def test_create_rejects_bad_workspace_without_gpu():
    cfg = _cfg()
    need = fsest.estimator_workspace_bytes(cfg)
    with pytest.raises(fsest.FsestError) as ei:
        fsest.estimator_create(cfg, None, need)
    assert ei.value.status == fsest.EST_EINVAL
    with pytest.raises(fsest.FsestError) as ei:
        fsest.estimator_create(cfg, 4096 * 1024, need - 1)
    assert ei.value.status == fsest.EST_ENOMEM
    with pytest.raises(fsest.FsestError) as ei:
        fsest.estimator_create(cfg, 4096 * 1024 + 8, need)
    assert ei.value.status == fsest.EST_EINVAL
    assert "aligned" in fsest.estimator_last_error()


def test_null_handle_calls_fail_cleanly():
    fsest.estimator_destroy(None)  # always safe
    for call in (lambda: fsest.estimator_transform(None),
                 lambda: fsest.estimator_graph_launch(None),
                 lambda: fsest.estimator_deposit(None, 1, 0, None, 1),
                 lambda: fsest.estimator_power(None, 1, 1, 0, 1, 1, 1)):
        with pytest.raises(fsest.FsestError) as ei:
            call()
        assert ei.value.status == fsest.EST_EINVAL


def test_product_path_has_no_oracle_dependency():
    pkg = os.path.join(ROOT, "paper_1512_07295_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_package_binds_to_one_hip_runtime():
    """Importing the package in a fresh interpreter (before anything else
    loads torch) maps exactly one HIP runtime: the library resolves its
    libamdhip64 dependency to the copy torch ships, instead of loading a
    second runtime that would see no device."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1512_07295_amd\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n" % root)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


@pytest.mark.parametrize("n", [12, 20, 24, 100, 480, 800, 960, 1000])
def test_mixed_radix_grid_sizes_accepted(n):
    """N = 2^a 3^b 5^c, a multiple of 4 (the paper's N_G = 100 and 480)."""
    assert fsest.estimator_workspace_bytes(_cfg(n_grid=n)) > 2 * 4 * n ** 3


def test_weights_flag_reserves_mass_buffers():
    """EST_FLAG_WEIGHTS adds the bucket-order and staging copies of the
    masses (4 + 4 bytes per particle) and the per-set mass partial sums."""
    base = fsest.estimator_workspace_bytes(_cfg(n_grid=64, max_particles=1 << 16))
    wtd = fsest.estimator_workspace_bytes(_cfg(n_grid=64, max_particles=1 << 16,
                                               flags=fsest.EST_FLAG_WEIGHTS))
    both = fsest.estimator_workspace_bytes(_cfg(n_grid=64, max_particles=1 << 16,
                                                flags=fsest.EST_FLAG_WEIGHTS | fsest.EST_FLAG_ATOMIC_SORT))
    assert wtd >= base + 8 * (1 << 16)
    assert both > 0


def test_set_weights_null_handle():
    with pytest.raises(fsest.FsestError) as ei:
        fsest.estimator_set_weights(None, None)
    assert ei.value.status == fsest.EST_EINVAL


@pytest.mark.parametrize("code,slabs", [(0, 1), (1, 1), (2, 2), (3, 4)])
def test_interlace_codes_reserve_one_complex_grid_per_pair(code, slabs):
    """Codes 2 and 3 hold 4 and 8 real grids as 2 and 4 complex grids, plus a
    half-spectrum buffer of the combined C(m)."""
    base = fsest.estimator_workspace_bytes(_cfg(n_grid=64, interlace=1))
    ws = fsest.estimator_workspace_bytes(_cfg(n_grid=64, interlace=code))
    grid = 64 * (64 * 64) * 8  # one complex grid: 64 planes of 4096 elements (no pad)
    cbuf = 64 * 64 * 33 * 8 if code >= 2 else 0  # combined C(m) for the adjoint
    if code >= 1:
        assert ws - base == (slabs - 1) * grid + cbuf


def test_atomic_sort_flag_accepted_and_drops_two_level_buffers():
    """EST_FLAG_ATOMIC_SORT is a valid flag; the atomic sort needs no
    super-bucket staging buffers, so its workspace is smaller."""
    two = fsest.estimator_workspace_bytes(_cfg(n_grid=64, max_particles=1 << 16))
    one = fsest.estimator_workspace_bytes(_cfg(n_grid=64, max_particles=1 << 16,
                                               flags=fsest.EST_FLAG_ATOMIC_SORT))
    assert one < two
