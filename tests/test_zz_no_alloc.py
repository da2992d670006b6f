"""estimator_direct_delta_noalloc (static device workspace, allocates
nothing) against estimator_direct_delta (caller workspace) through the C ABI:
the same kernels on the same inputs give the same half spectrum, on two calls
in a row (the second with fewer particles, so stale contents of the shared
static workspace would show), and a request above the static workspace's
64 MiB is refused before any launch."""

import numpy as np
import pytest

import synth
from gpu_common import require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _both(torch, lib, est, pos):
    n = pos.shape[0]
    nbytes = lib.estimator_direct_workspace_bytes(est.h, n)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    half = (est.n_grid, est.n_grid, est.n_grid // 2 + 1, 2)
    ref = torch.empty(half, dtype=torch.float64, device="cuda")
    got = torch.full(half, np.nan, dtype=torch.float64, device="cuda")
    lib.estimator_direct_delta(est.h, pos, lib.EST_F32, n, ws_ptr, nbytes, ref)
    lib.estimator_direct_delta_noalloc(est.h, pos, lib.EST_F32, n, got)
    est.stream.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_direct_sum_matches_workspace_entry_point():
    torch = require_gpu()
    import paper_1512_07295_amd as lib
    from paper_1512_07295_amd.estimator import Estimator
    box, n = 400.0, 32
    est = Estimator(n, box, 4, True, 1, 6000)
    for count, seed in ((6000, 3), (1500, 4)):  # the second call is smaller
        pos = to_dev(torch, synth.uniform(count, box, seed, np.float32))
        ref, got = _both(torch, lib, est, pos)
        assert np.all(np.isfinite(got))
        assert np.array_equal(ref, got), np.max(np.abs(ref - got))
    # a workspace above the static 64 MiB is refused before anything runs
    big = 6_000_000
    assert lib.estimator_direct_workspace_bytes(est.h, big) > (64 << 20)
    pos = torch.zeros((big, 3), dtype=torch.float32, device="cuda")
    out = torch.empty((n, n, n // 2 + 1, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.FsestError) as exc:
        lib.estimator_direct_delta_noalloc(est.h, pos, lib.EST_F32, big, out)
    assert exc.value.status == lib.EST_ENOMEM
    est.close()
