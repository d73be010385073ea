"""Supernode hierarchy rebuilt on the device (mas_hierarchy_device) against
the oracle's hierarchy (Sec. 4.1, Supp. Alg. 2-5): level count, units per
level and the unit of every node at every level, bit-exact."""

import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import cube, large_cube, small_cube

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


def _check(S, P, dev):
    units, sn = S.hierarchy_device(dev)
    torch.cuda.synchronize()
    assert len(units) == P.levels
    for l in range(P.levels):
        assert units[l] == P.units(l), l
        assert np.array_equal(sn[l], P.sn(l)), l
    # the host analysis that builds the solver's plans agrees as well
    inf = S.info()
    _, _, sn_host = S.ordering()
    assert inf["levels"] == len(units) and np.array_equal(sn_host, sn)
    return units


CASES = {
    "cube1": lambda: cube(1),
    "cube2": lambda: cube(2),
    "cube8": small_cube,
    "rand300_local": lambda: synth.random_spd_system(300, 700, seed=2, local=12),
    "contact6": lambda: cube(6, E=1e6, nu=0.49, seed=21, n_contacts=60),
    "wide4000": lambda: synth.random_spd_system(4000, 60000, seed=4),
    "dense_local": lambda: synth.random_spd_system(2000, 90000, seed=6, local=60),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("N", [8, 16, 32, 40])
def test_hierarchy_device(dev, name, N):
    from paper_2411_06224_amd import MasPcg

    _say("hierarchy", name, N)
    s = CASES[name]()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, gptr=s.gptr, gadj=s.gadj)
    S = MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=N)
    _check(S, P, dev)


@pytest.mark.parametrize("max_levels", [1, 2, 3])
def test_hierarchy_device_level_cap(dev, max_levels):
    from paper_2411_06224_amd import MasPcg

    _say("hierarchy cap", max_levels)
    s = CASES["contact6"]()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, max_levels=max_levels, gptr=s.gptr, gadj=s.gadj)
    S = MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16, max_levels=max_levels)
    units = _check(S, P, dev)
    assert len(units) <= max_levels


def test_hierarchy_device_given_partition(dev):
    """Morton-ordered level-0 domains: padded slots and disconnected pieces
    inside a domain."""
    from paper_2411_06224_amd import MasPcg, morton_partition

    _say("hierarchy morton")
    s = CASES["contact6"]()
    part = morton_partition(s.meta["positions"], 16)
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, part=part, M=int(part.max()) + 1)
    S = MasPcg(s.row_ptr, s.col_idx, domain_size=16, partition=part)
    _check(S, P, dev)


def test_morton_partition_matches_reference(dev):
    """The device Morton partition (mas_morton_partition) against the numpy
    definition in tests/morton_reference.py, bit for bit: lattice and noisy
    cube positions, random points, a flat set (zero extent in z), duplicate
    positions (ties broken by node id), one node, and domain sizes that do
    not divide the node count."""
    from paper_2411_06224_amd import morton_partition
    from morton_reference import morton_partition as reference

    _say("morton partition")
    rng = np.random.default_rng(17)
    flat = rng.uniform(-1.0, 1.0, (997, 3))
    flat[:, 2] = 0.25
    dup = np.repeat(rng.uniform(0.0, 1.0, (50, 3)), 7, axis=0)[rng.permutation(350)]
    cases = [
        (small_cube().meta["positions"], 16),
        (large_cube().meta["positions"], 16),
        (rng.uniform(-3.0, 7.0, (10007, 3)), 16),
        (flat, 7),
        (dup, 5),
        (np.array([[0.5, -1.0, 2.0]]), 16),
        (rng.standard_normal((4099, 3)) * 1e-9, 40),
    ]
    for pos, N in cases:
        got = morton_partition(pos, N, device=dev)
        ref = reference(pos, N)
        assert got.dtype == np.int32 and np.array_equal(got, ref), (len(pos), N)


def test_hierarchy_device_repeated_calls(dev):
    """The scratch is reused: a second call (and one after a solver build on
    another workspace) gives the same hierarchy."""
    from paper_2411_06224_amd import BlockMatrix, MasPcg

    _say("hierarchy repeated")
    s = small_cube()
    S = MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16)
    u1, sn1 = S.hierarchy_device(dev)
    S.build(BlockMatrix.from_numpy(s.row_ptr, s.col_idx, s.val, device=dev))
    u2, sn2 = S.hierarchy_device(dev)
    assert np.array_equal(u1, u2) and np.array_equal(sn1, sn2)


@pytest.mark.slow
def test_hierarchy_device_large_cube(dev):
    """48^3 nodes, domain size 16 (the full-size workload)."""
    from paper_2411_06224_amd import MasPcg

    _say("hierarchy 48^3")
    s = large_cube()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, gptr=s.gptr, gadj=s.gadj)
    S = MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16)
    units = _check(S, P, dev)
    print("units per level:", list(units))


def _graph_pattern(s):
    """Block pattern of the mesh graph alone (diagonal plus graph edges):
    the pattern before any contact."""
    n = s.n
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    deg = np.diff(s.gptr)
    rows.append(np.repeat(np.arange(n), deg))
    cols.append(s.gadj)
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    key = np.unique(r * n + c)
    r, c = key // n, key % n
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp).astype(np.int32), c.astype(np.int32)


def _upper(rp, ci):
    n = rp.size - 1
    r = np.repeat(np.arange(n), np.diff(rp))
    keep = ci >= r
    rp2 = np.zeros(n + 1, np.int32)
    np.add.at(rp2, r[keep] + 1, 1)
    return np.cumsum(rp2).astype(np.int32), ci[keep].astype(np.int32)


def _check_rebuild(units_d, sn_d, P):
    units = units_d.cpu().numpy()
    sn = sn_d.cpu().numpy()
    L = int(units[0])
    assert L == P.levels
    for l in range(L):
        assert units[1 + l] == P.units(l), l
        assert np.array_equal(sn[l], P.sn(l)), l
    assert np.all(sn[L:] == -1) and np.all(units[1 + L:] == 0)


def _add_pairs(rp, ci, n_pairs, seed):
    """The pattern with n_pairs random node pairs added in both directions
    (contacts appearing between Newton steps), and diagonally dominant
    values on it (10 I on the diagonal, 0.01 I elsewhere: the hierarchy
    depends on the pattern only)."""
    n = rp.size - 1
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n, n_pairs)
    b = rng.integers(0, n, n_pairs)
    r = np.concatenate([np.repeat(np.arange(n), np.diff(rp)), a, b]).astype(np.int64)
    c = np.concatenate([ci, b, a]).astype(np.int64)
    key = np.unique(r * n + c)
    r, c = key // n, key % n
    rp2 = np.zeros(n + 1, np.int32)
    np.add.at(rp2, r + 1, 1)
    val = np.where((r == c)[:, None, None], 10.0, 0.01) * np.eye(3)[None]
    return np.cumsum(rp2).astype(np.int32), c.astype(np.int32), val


REBUILD_CASES = {
    "cube8_200": lambda: (small_cube(), 200),
    "cube8_800": lambda: (small_cube(), 800),
    "contact6_300": lambda: (cube(6, E=1e6, nu=0.49, seed=21, n_contacts=60), 300),
    "local2000_500": lambda: (synth.random_spd_system(2000, 6000, seed=6, local=30), 500),
}


@pytest.mark.parametrize("name", list(REBUILD_CASES))
@pytest.mark.parametrize("N", [16, 40])
def test_hierarchy_rebuild_after_contact_change(dev, name, N):
    """Analysed on the contact-free pattern; the hierarchy of the pattern
    with new contacts, rebuilt on the device under the same partition,
    equals the oracle's hierarchy of that pattern (whole or one triangle)."""
    from paper_2411_06224_amd import MasPcg

    _say("hierarchy rebuild", name, N)
    s, n_pairs = REBUILD_CASES[name]()
    rp1, ci1 = _graph_pattern(s)
    rp2, ci2, val2 = _add_pairs(rp1, ci1, n_pairs, seed=N)
    S = MasPcg(rp1, ci1, graph=(s.gptr, s.gadj), domain_size=N)
    P = oracle.MAS(rp2, ci2, val2, N=N, gptr=s.gptr, gadj=s.gadj)
    P1 = oracle.MAS(rp1, ci1, np.tile(np.eye(3), (ci1.size, 1, 1)) * 4.0, N=N, gptr=s.gptr, gadj=s.gadj)
    if N == 16:  # there the new contacts change the hierarchy in every case
        assert P.levels != P1.levels or any(not np.array_equal(P.sn(l), P1.sn(l)) for l in range(P.levels))
    for rp, ci in ((rp2, ci2), _upper(rp2, ci2)):
        units, sn = S.hierarchy_rebuild(torch.as_tensor(rp, device=dev), torch.as_tensor(ci, device=dev))
        _check_rebuild(units, sn, P)
    # the contact-free pattern gives the analysed hierarchy back
    units, sn = S.hierarchy_rebuild(torch.as_tensor(rp1, device=dev), torch.as_tensor(ci1, device=dev))
    _check_rebuild(units, sn, P1)
    assert int(units[0]) == S.info()["levels"]


@pytest.mark.parametrize("max_levels", [1, 2, 3])
def test_hierarchy_rebuild_level_cap(dev, max_levels):
    from paper_2411_06224_amd import MasPcg

    _say("hierarchy rebuild cap", max_levels)
    s, n_pairs = REBUILD_CASES["cube8_200"]()
    rp1, ci1 = _graph_pattern(s)
    rp2, ci2, val2 = _add_pairs(rp1, ci1, n_pairs, seed=3)
    S = MasPcg(rp1, ci1, graph=(s.gptr, s.gadj), domain_size=16, max_levels=max_levels)
    P = oracle.MAS(rp2, ci2, val2, N=16, max_levels=max_levels, gptr=s.gptr, gadj=s.gadj)
    units, sn = S.hierarchy_rebuild(torch.as_tensor(rp2, device=dev), torch.as_tensor(ci2, device=dev))
    _check_rebuild(units, sn, P)


def test_hierarchy_rebuild_after_build(dev):
    """After mas_build the rebuild reads the partition's map from the
    solver's workspace; the result is the same, and a solve on the analysed
    pattern still works afterwards."""
    from paper_2411_06224_amd import BlockMatrix, MasPcg

    _say("hierarchy rebuild after build")
    s, n_pairs = REBUILD_CASES["contact6_300"]()
    rp1, ci1 = _graph_pattern(s)
    rp2, ci2, val2 = _add_pairs(rp1, ci1, n_pairs, seed=16)
    val1 = np.where((np.repeat(np.arange(s.n), np.diff(rp1)) == ci1)[:, None, None], 10.0, 0.01) * np.eye(3)[None]
    S = MasPcg(rp1, ci1, graph=(s.gptr, s.gadj), domain_size=16)
    H1 = BlockMatrix.from_numpy(rp1, ci1, val1, device=dev)
    S.build(H1)
    P = oracle.MAS(rp2, ci2, val2, N=16, gptr=s.gptr, gadj=s.gadj)
    units, sn = S.hierarchy_rebuild(torch.as_tensor(rp2, device=dev), torch.as_tensor(ci2, device=dev))
    _check_rebuild(units, sn, P)
    b = torch.ones(3 * s.n, dtype=torch.float64, device=dev)
    x, res = S.solve(H1, b, tol=1e-10)
    assert res["status"] == 0 and res["true_rel_residual"] <= 1e-10


def test_hierarchy_rebuild_deep(dev):
    """A pattern whose hierarchy reaches the level limit (16 levels)."""
    from paper_2411_06224_amd import MasPcg

    _say("hierarchy rebuild deep")
    s = synth.random_spd_system(4000, 60000, seed=4)
    S = MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16)
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, gptr=s.gptr, gadj=s.gadj)
    assert P.levels == 16
    units, sn = S.hierarchy_rebuild(torch.as_tensor(s.row_ptr, device=dev), torch.as_tensor(s.col_idx, device=dev))
    _check_rebuild(units, sn, P)


def test_hierarchy_rebuild_rejects_out_of_range_columns(dev):
    from paper_2411_06224_amd import MasPcg

    _say("hierarchy rebuild bad pattern")
    s = cube(6, E=1e6, nu=0.49, seed=21, n_contacts=60)
    S = MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16)
    ci = s.col_idx.copy()
    ci[5] = s.n  # one column past the last node
    units, _ = S.hierarchy_rebuild(torch.as_tensor(s.row_ptr, device=dev), torch.as_tensor(ci, device=dev))
    assert int(units[0]) == -1
    rp = s.row_ptr.copy()
    rp[-1] = rp[-1] + 7  # row range past the column list
    units, _ = S.hierarchy_rebuild(torch.as_tensor(rp, device=dev), torch.as_tensor(s.col_idx, device=dev))
    assert int(units[0]) == -1


def test_hierarchy_rebuild_diagonal_only_pattern(dev):
    """A pattern without off-diagonal blocks merges nothing: one level, every
    node its own level-0 unit (its slot)."""
    from paper_2411_06224_amd import MasPcg

    _say("hierarchy rebuild diagonal-only pattern")
    s = cube(4, E=1e6, nu=0.49, seed=3, n_contacts=0)
    S = MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16)
    n = s.n
    rp = torch.arange(n + 1, dtype=torch.int32, device=dev)
    ci = torch.arange(n, dtype=torch.int32, device=dev)
    units, sn = S.hierarchy_rebuild(rp, ci)
    u = units.cpu().numpy()
    mp_, _, _ = S.ordering()
    assert u[0] == 1 and u[1] == S.info()["units"][0] and np.all(u[2:] == 0)
    assert np.array_equal(sn.cpu().numpy()[0], mp_) and np.all(sn.cpu().numpy()[1:] == -1)
    # no blocks at all (row_ptr of zeros): the same
    units, sn = S.hierarchy_rebuild(torch.zeros(n + 1, dtype=torch.int32, device=dev),
                                    torch.zeros(0, dtype=torch.int32, device=dev))
    assert int(units[0]) == 1 and np.array_equal(sn.cpu().numpy()[0], mp_)
