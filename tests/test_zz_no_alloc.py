"""The allocation-free assembly entry point (bcsr_assemble_noalloc, static
device scratch) against bcsr_assemble (caller workspace) through the C ABI:
pattern and values bitwise equal, on two calls in a row, the second with a
smaller list, and the size limit rejected before any launch."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2411_06224_amd as mp

    mp.load()
    return torch.device("cuda:0")


def _list(n, m, seed, dev):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, n, m)
    cols = rng.integers(0, n, m)
    blocks = rng.standard_normal((m, 3, 3)) * 10.0 ** rng.integers(-6, 6, (m, 1, 1))
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dtype=dt), device=dev)
    return t(rows, np.int32), t(cols, np.int32), t(blocks, np.float64)


def _noalloc(n, rows, cols, blocks, cap, dev):
    from paper_2411_06224_amd import bcsr_assemble_noalloc

    # outputs poisoned, so entries the call should write but does not show up
    row_ptr = torch.full((n + 1,), -7, dtype=torch.int32, device=dev)
    col_idx = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    val = torch.full((cap, 3, 3), float("nan"), dtype=torch.float64, device=dev)
    nb = bcsr_assemble_noalloc(n, rows, cols, blocks, row_ptr, col_idx, val)
    torch.cuda.synchronize()
    return row_ptr.cpu().numpy(), col_idx[:nb].cpu().numpy(), val[:nb].cpu().numpy()


def test_noalloc_matches_workspace_entry_point_twice(dev):
    from paper_2411_06224_amd import bcsr_assemble

    for n, m, seed in ((3000, 200000, 11), (500, 9000, 12)):  # the second call smaller
        _say("assemble no-alloc", n, m)
        rows, cols, blocks = _list(n, m, seed, dev)
        ref = bcsr_assemble(n, rows, cols, blocks)
        got = _noalloc(n, rows, cols, blocks, m, dev)
        assert np.array_equal(got[0], ref.row_ptr.cpu().numpy())
        assert np.array_equal(got[1], ref.col_idx.cpu().numpy())
        assert np.array_equal(got[2].view(np.int64), ref.val.cpu().numpy().view(np.int64))


def test_noalloc_limits(dev):
    import ctypes

    from paper_2411_06224_amd import _lib

    L = _lib.load()
    _say("assemble no-alloc limits")
    # a list whose scratch exceeds the static array is refused before any launch
    big = (_lib.MAS_NOALLOC_SCRATCH_BYTES // 8) + 1
    assert L.bcsr_assemble_workspace_size(1000, big) > _lib.MAS_NOALLOC_SCRATCH_BYTES
    nb = ctypes.c_int64(0)
    dummy = torch.zeros(16, dtype=torch.int32, device=dev)
    p = ctypes.c_void_p(dummy.data_ptr())
    rc = L.bcsr_assemble_noalloc(1000, big, p, p, p, p, p, p, 0, ctypes.byref(nb), None)
    assert rc == _lib.MAS_WORKSPACE_TOO_SMALL
    # an empty list: every row empty
    rows, cols, blocks = _list(5, 0, 0, dev)
    got = _noalloc(5, rows, cols, blocks, 1, dev)
    assert np.array_equal(got[0], np.zeros(6, np.int32)) and got[1].size == 0
