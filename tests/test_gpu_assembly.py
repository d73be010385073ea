"""GPU block-list assembly (bcsr_assemble) against the oracle's assembly:
pattern and values bit-exact (equal blocks are summed in list order on both
sides), including the full 48^3 cube's element, mass and contact blocks."""

import sys

import numpy as np
import pytest

import oracle
import synth

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


def _gpu(n, rows, cols, blocks, dev, capacity=None):
    from paper_2411_06224_amd import bcsr_assemble

    r = torch.as_tensor(np.asarray(rows, dtype=np.int32), device=dev)
    c = torch.as_tensor(np.asarray(cols, dtype=np.int32), device=dev)
    b = torch.as_tensor(np.ascontiguousarray(blocks, dtype=np.float64).reshape(-1, 3, 3), device=dev)
    H = bcsr_assemble(n, r, c, b, capacity=capacity)
    return H.row_ptr.cpu().numpy(), H.col_idx.cpu().numpy(), H.val.cpu().numpy()


def _same(a, b):
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2].shape == b[2].shape
    assert np.array_equal(a[2].view(np.int64), b[2].view(np.int64))  # bitwise


def test_assemble_head_segmented_reduce_example(dev):
    """The paper's warp-segmented reduction example (Sec. 6.2; the values and
    sums in tests/golden), in list order and shuffled."""
    import json
    import os

    _say("assemble segmented-reduce example")
    with open(os.path.join(os.path.dirname(__file__), "golden", "head_segmented_reduce_example.json")) as fh:
        g = json.load(fh)
    seg = np.cumsum(g["tags"]) - 1
    blocks = np.asarray(g["values"], dtype=np.float64)[:, None, None] * np.ones((1, 3, 3))
    n = len(g["segment_sums"])
    for perm in (np.arange(seg.size), np.random.default_rng(3).permutation(seg.size)):
        got = _gpu(n, seg[perm], np.zeros(seg.size, np.int64), blocks[perm], dev)
        assert list(got[2][:, 0, 0]) == g["segment_sums"]
        _same(got, oracle.assemble(n, seg[perm], np.zeros(seg.size, np.int64), blocks[perm]))


@pytest.mark.parametrize("n,m,seed", [(1, 20, 3), (2, 40, 4), (7, 50, 0), (300, 20000, 1), (2000, 150000, 2),
                                      (65536, 30000, 5), (3_000_000, 60000, 6)])
def test_assemble_random_lists(dev, n, m, seed):
    _say("assemble random", n, m)
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, n, m)
    cols = rng.integers(0, n, m)
    blocks = rng.standard_normal((m, 3, 3)) * 10.0 ** rng.integers(-8, 8, (m, 1, 1))
    _same(_gpu(n, rows, cols, blocks, dev), oracle.assemble(n, rows, cols, blocks))


def test_assemble_list_order_and_edges(dev):
    from paper_2411_06224_amd import MasError

    _say("assemble order and edge cases")
    big, one = np.full((3, 3), 1e16), np.ones((3, 3))
    _, _, v = _gpu(2, [1, 1, 1], [0, 0, 0], np.stack([big, one, -big]), dev)
    assert np.all(v[0] == 0.0)
    _, _, v = _gpu(2, [1, 1, 1], [0, 0, 0], np.stack([big, -big, one]), dev)
    assert np.all(v[0] == 1.0)
    rp, ci, v = _gpu(5, [], [], np.zeros((0, 3, 3)), dev)
    assert list(rp) == [0] * 6 and ci.size == 0
    _same(_gpu(5, [4, 0], [1, 2], np.stack([one, 2 * one]), dev), oracle.assemble(5, [4, 0], [1, 2], np.stack([one, 2 * one])))
    with pytest.raises(MasError):
        _gpu(3, [0, 3], [0, 0], np.stack([one, one]), dev)
    with pytest.raises(MasError):
        _gpu(3, [0, 1], [0, -1], np.stack([one, one]), dev)
    # output capacity too small: the binding learns the size and assembles again
    rows = np.arange(40) % 10
    cols = np.arange(40) // 10
    blocks = np.random.default_rng(3).standard_normal((40, 3, 3))
    _same(_gpu(10, rows, cols, blocks, dev, capacity=3), oracle.assemble(10, rows, cols, blocks))
    # one long row (no per-row limit): 20,000 listed blocks over four columns
    many = 20000
    rows, cols = np.zeros(many, dtype=np.int64), np.arange(many) % 4
    blocks = np.random.default_rng(5).standard_normal((many, 3, 3))
    _same(_gpu(4, rows, cols, blocks, dev), oracle.assemble(4, rows, cols, blocks))
    # rows before, between and after the listed ones stay empty
    _same(_gpu(9, [7, 2, 7], [3, 8, 3], np.stack([one, 2 * one, 3 * one]), dev),
          oracle.assemble(9, [7, 2, 7], [3, 8, 3], np.stack([one, 2 * one, 3 * one])))


def test_assemble_cube_blocks(dev):
    _say("assemble 8^3 cube blocks")
    s = synth.cube_system(8, 1e5, 0.4, seed=1000, n_contacts=30, keep_blocks=True)
    rows, cols, blocks = s.meta["blocks"]
    got = _gpu(s.n, rows, cols, blocks, dev)
    _same(got, oracle.assemble(s.n, rows, cols, blocks))
    assert np.array_equal(got[0], s.row_ptr) and np.array_equal(got[1], s.col_idx)


@pytest.mark.slow
def test_assemble_large_cube_blocks(dev):
    _say("assemble 48^3 cube blocks")
    s = synth.config_large(E=1e6, keep_blocks=True)
    rows, cols, blocks = s.meta["blocks"]
    got = _gpu(s.n, rows, cols, blocks, dev)
    _same(got, oracle.assemble(s.n, rows, cols, blocks))
    assert np.array_equal(got[1], s.col_idx)
