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
