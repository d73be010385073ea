"""Host-side checks of libmaspcg: it loads, exports every symbol the header
declares, validates arguments, and its symbolic analysis (partition, slots,
supernode hierarchy) matches the oracle bit for bit.  No GPU work is run."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from conftest import cube, small_cube

from paper_2411_06224_amd import _lib
from paper_2411_06224_amd.solver import MasPcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "mas_pcg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"sizeof"})


def test_library_exports_every_header_function():
    L = _lib.load()
    names = _header_functions()
    assert set(names) == set(_lib.SYMBOLS)
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert _lib.status_string(code) and _lib.status_string(code) != "unknown status"
    assert _lib.status_string(42) == "unknown status"


def test_create_rejects_bad_options():
    L = _lib.load()
    h = ctypes.c_void_p()
    for opts in ((0, 0, 0, 0), (41, 0, 0, 0), (16, 0, 7, 0), (16, 0, 0, 1), (16, 17, 0, 0)):
        o = _lib.MasOptions(*opts)
        assert L.mas_create(ctypes.byref(o), ctypes.byref(h)) == _lib.MAS_INVALID_ARG
    assert L.mas_create(None, ctypes.byref(h)) == _lib.MAS_OK
    assert L.mas_workspace_size(h) == 0
    L.mas_destroy(h)


def _analyze_rc(rp, ci, graph=None, N=16):
    L = _lib.load()
    h = ctypes.c_void_p()
    o = _lib.MasOptions(N, 0, 0, 0)
    assert L.mas_create(ctypes.byref(o), ctypes.byref(h)) == 0
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci, np.int32)
    rc = L.mas_analyze(h, rp.size - 1, ci.size, rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p), None, None)
    L.mas_destroy(h)
    return rc


def test_analyze_rejects_invalid_patterns():
    s = cube(1)
    rp, ci = s.row_ptr.copy(), s.col_idx.copy()
    assert _analyze_rc(rp, ci) == _lib.MAS_OK
    bad = ci.copy()
    bad[1], bad[2] = bad[2], bad[1]  # unsorted row
    assert _analyze_rc(rp, bad) == _lib.MAS_INVALID_ARG
    bad = ci.copy()
    bad[0] = s.n  # out of range
    assert _analyze_rc(rp, bad) == _lib.MAS_INVALID_ARG
    # drop the (0,1) block only: pattern becomes asymmetric
    k = int(np.nonzero(ci[rp[0] : rp[1]] == 1)[0][0])
    ci2 = np.delete(ci, k)
    rp2 = rp.copy()
    rp2[1:] -= 1
    assert _analyze_rc(rp2, ci2) == _lib.MAS_INVALID_ARG
    # drop a diagonal block
    k = int(np.nonzero(ci[rp[3] : rp[4]] == 3)[0][0]) + rp[3]
    ci3 = np.delete(ci, k)
    rp3 = rp.copy()
    rp3[4:] -= 1
    assert _analyze_rc(rp3, ci3) == _lib.MAS_INVALID_ARG
    assert _analyze_rc(np.zeros(1, np.int32), np.zeros(0, np.int32)) == _lib.MAS_INVALID_ARG


def _compare_with_oracle(s, N, max_levels=0, use_graph=True):
    graph = (s.gptr, s.gadj) if use_graph else None
    lib = MasPcg(s.row_ptr, s.col_idx, graph=graph, domain_size=N, max_levels=max_levels)
    inf = lib.info()
    mp, rm, sn = lib.ordering()
    if use_graph:
        P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, max_levels=max_levels, gptr=s.gptr, gadj=s.gadj)
    else:
        P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, max_levels=max_levels)
    omp, orm = P.maps()
    assert inf["parts"] == P.parts and inf["slack"] == P.slack
    assert np.array_equal(mp, omp)
    assert np.array_equal(rm, orm)
    assert inf["levels"] == P.levels
    for l in range(P.levels):
        assert inf["units"][l] == P.units(l)
        assert inf["domains"][l] == P.domains(l)
        assert np.array_equal(sn[l], P.sn(l))
    lib.close()
    return inf


@pytest.mark.parametrize("N", [1, 2, 4, 7, 16, 21, 32, 40])
def test_ordering_bit_exact_small_cube(N):
    _compare_with_oracle(small_cube(), N)


@pytest.mark.parametrize("ml", [1, 2, 3])
def test_ordering_bit_exact_level_cap(ml):
    inf = _compare_with_oracle(small_cube(), 16, max_levels=ml)
    assert inf["levels"] <= ml


def test_ordering_bit_exact_default_graph_and_random_systems():
    _compare_with_oracle(cube(3), 4, use_graph=False)
    for seed in range(4):
        s = synth.random_spd_system(300, 700, seed=seed, local=12)
        _compare_with_oracle(s, 8)
        _compare_with_oracle(s, 16, use_graph=False)


def test_ordering_bit_exact_contact_cube():
    s = cube(6, E=1e6, nu=0.49, seed=21, n_contacts=60)
    inf = _compare_with_oracle(s, 16)
    assert inf["levels"] >= 2


@pytest.mark.slow
def test_ordering_bit_exact_large_cube():
    from conftest import large_cube

    inf = _compare_with_oracle(large_cube(), 16)
    assert inf["n_rows"] == 117649 and inf["nnzb"] == 1526513


def _morton_bruteforce(q):
    """Bit-by-bit interleave of three 21-bit integers (x highest of each triple)."""
    code = 0
    for bit in range(21):
        code |= ((int(q[0]) >> bit) & 1) << (3 * bit + 2)
        code |= ((int(q[1]) >> bit) & 1) << (3 * bit + 1)
        code |= ((int(q[2]) >> bit) & 1) << (3 * bit)
    return code


def test_morton_codes_match_bitwise_interleave():
    from morton_reference import morton_codes

    rng = np.random.default_rng(3)
    pts = rng.uniform(-2.0, 5.0, size=(200, 3))
    pts[0] = pts.min(axis=0)
    pts[1] = pts.max(axis=0)
    codes = morton_codes(pts)
    lo, hi = pts.min(axis=0), pts.max(axis=0)
    q = np.clip(np.floor((pts - lo) / (hi - lo) * ((1 << 21) - 1)).astype(np.int64), 0, (1 << 21) - 1)
    for i in range(len(pts)):
        assert int(codes[i]) == _morton_bruteforce(q[i])
    # a 2x2x2 lattice orders as the Z-curve: x is the most significant bit of each triple
    lat = np.array([[x, y, z] for x in (0.0, 1.0) for y in (0.0, 1.0) for z in (0.0, 1.0)])
    assert list(np.argsort(morton_codes(lat))) == list(range(8))


def test_given_partition_bit_exact_with_oracle():
    """Morton-ordered level-0 domains (the earlier MAS ordering, Sec. 4.1)
    through mas_analyze_partition: slots, supernodes and levels as the oracle
    builds them from the same partition."""
    from morton_reference import morton_partition

    for s, N in ((small_cube(), 16), (cube(6, E=1e6, nu=0.49, seed=21, n_contacts=60), 16), (small_cube(), 4)):
        part = morton_partition(s.meta["positions"], N)
        M = int(part.max()) + 1
        lib = MasPcg(s.row_ptr, s.col_idx, domain_size=N, partition=part)
        inf = lib.info()
        mp, rm, sn = lib.ordering()
        P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, part=part, M=M)
        omp, orm = P.maps()
        assert inf["parts"] == M == P.parts
        assert np.array_equal(mp, omp) and np.array_equal(rm, orm)
        assert inf["levels"] == P.levels
        for l in range(P.levels):
            assert inf["units"][l] == P.units(l)
            assert np.array_equal(sn[l], P.sn(l))
        lib.close()


def test_given_partition_rejects_invalid():
    s = cube(2)
    n = s.n
    L = _lib.load()
    opts = _lib.MasOptions(4, 0, 0, 0)

    def rc(part, n_parts):
        h = ctypes.c_void_p()
        assert L.mas_create(ctypes.byref(opts), ctypes.byref(h)) == 0
        p = np.ascontiguousarray(part, dtype=np.int32)
        r = L.mas_analyze_partition(h, n, s.col_idx.size, s.row_ptr.ctypes.data_as(ctypes.c_void_p),
                                    s.col_idx.ctypes.data_as(ctypes.c_void_p), p.ctypes.data_as(ctypes.c_void_p),
                                    n_parts)
        L.mas_destroy(h)
        return r

    ok = np.arange(n) // 4
    assert rc(ok, int(ok.max()) + 1) == 0
    assert rc(ok, int(ok.max())) == _lib.MAS_INVALID_ARG  # id out of range
    assert rc(ok, int(ok.max()) + 2) == _lib.MAS_INVALID_ARG  # an empty part
    big = np.arange(n) // 5  # parts of 5 > domain size 4
    assert rc(big, int(big.max()) + 1) == _lib.MAS_INVALID_ARG
    neg = ok.copy()
    neg[0] = -1
    assert rc(neg, int(ok.max()) + 1) == _lib.MAS_INVALID_ARG


def test_hierarchy_device_argument_checks():
    """mas_hierarchy_device validates its arguments on the host before any
    device work: not analysed, missing or misaligned workspace, too small."""
    L = _lib.load()
    h = ctypes.c_void_p()
    assert L.mas_create(None, ctypes.byref(h)) == _lib.MAS_OK
    assert L.mas_hierarchy_workspace_size(h) == 0
    assert L.mas_hierarchy_device(h, None, None, None, ctypes.c_void_p(256), 1 << 20, None) == _lib.MAS_NOT_READY
    L.mas_destroy(h)
    s = small_cube()
    S = MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16)
    need = S._L.mas_hierarchy_workspace_size(S._h)
    assert need > 0
    call = lambda ws, n: S._L.mas_hierarchy_device(S._h, None, None, None, ws, n, None)
    assert call(None, need) == _lib.MAS_INVALID_ARG
    assert call(ctypes.c_void_p(4096 + 8), need) == _lib.MAS_INVALID_ARG  # not 256-byte aligned
    assert call(ctypes.c_void_p(4096), need - 1) == _lib.MAS_WORKSPACE_TOO_SMALL
    assert S._L.mas_hierarchy_device(None, None, None, None, ctypes.c_void_p(4096), need, None) == _lib.MAS_INVALID_ARG


def test_new_entry_points_argument_checks():
    """mas_hierarchy_rebuild, mas_replan, abd_contact_blocks, bcsr_assemble
    and mas_morton_partition reject bad arguments on the host, before any
    device work."""
    L = _lib.load()
    vp = ctypes.c_void_p
    s = small_cube()
    S = MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16)
    need = S._L.mas_hierarchy_workspace_size(S._h)
    ws = vp(4096)
    rb = lambda h, nnzb, rp, ci, u, sn, w, n: L.mas_hierarchy_rebuild(h, nnzb, rp, ci, u, sn, w, n, None)
    assert rb(None, 10, ws, ws, ws, ws, ws, need) == _lib.MAS_INVALID_ARG
    assert rb(S._h, -1, ws, ws, ws, ws, ws, need) == _lib.MAS_INVALID_ARG
    assert rb(S._h, 10, None, ws, ws, ws, ws, need) == _lib.MAS_INVALID_ARG  # no row_ptr
    assert rb(S._h, 10, ws, None, ws, ws, ws, need) == _lib.MAS_INVALID_ARG  # blocks but no col_idx
    assert rb(S._h, 10, ws, ws, None, ws, ws, need) == _lib.MAS_INVALID_ARG  # no outputs
    assert rb(S._h, 10, ws, ws, ws, ws, vp(4096 + 8), need) == _lib.MAS_INVALID_ARG  # misaligned workspace
    assert rb(S._h, 10, ws, ws, ws, ws, ws, need - 1) == _lib.MAS_WORKSPACE_TOO_SMALL
    h = ctypes.c_void_p()
    assert L.mas_create(None, ctypes.byref(h)) == _lib.MAS_OK
    assert rb(h, 10, ws, ws, ws, ws, ws, 1 << 20) == _lib.MAS_NOT_READY
    L.mas_destroy(h)

    n_out = ctypes.c_int64(0)
    wsz = int(L.abd_contact_workspace_size(10, 4))
    assert wsz > 0
    ab = lambda n, m, levels, w, nb: L.abd_contact_blocks(n, ws, ws, ws, m, ws, ws, ws, levels, ws, ws, ws, 64,
                                                         ctypes.byref(n_out), w, nb, None)
    assert ab(0, 4, 2, ws, wsz) == _lib.MAS_INVALID_ARG  # no nodes
    assert ab(10, -1, 2, ws, wsz) == _lib.MAS_INVALID_ARG
    assert ab(10, 4, 3, ws, wsz) == _lib.MAS_INVALID_ARG  # levels must be 1 or 2
    assert ab(10, 4, 2, vp(4096 + 8), wsz) == _lib.MAS_INVALID_ARG
    assert ab(10, 4, 2, ws, wsz - 1) == _lib.MAS_WORKSPACE_TOO_SMALL

    nb = ctypes.c_int64(0)
    asm = lambda n_rows, n_in: L.bcsr_assemble(n_rows, n_in, ws, ws, ws, ws, ws, ws, 16, ctypes.byref(nb), ws,
                                               1 << 30, None)
    assert asm(0, 4) == _lib.MAS_INVALID_ARG
    assert asm(0x7fffffff, 4) == _lib.MAS_INVALID_ARG  # n_rows + 1 must fit an int32 row_ptr
    assert asm(10, -1) == _lib.MAS_INVALID_ARG
    assert int(L.bcsr_assemble_workspace_size(3_000_000, 1000)) > 0  # beyond 2^20 rows

    rw = int(L.mas_replan_workspace_size(S._h, s.col_idx.size))
    assert rw > 0 and int(L.mas_replan_workspace_size(S._h, 0)) == 0
    assert int(L.mas_replan_workspace_size(None, 10)) == 0
    rpl = lambda h, nnzb, rp, ci, w, n: L.mas_replan(h, nnzb, rp, ci, w, n, None)
    nz = int(s.col_idx.size)
    assert rpl(None, nz, ws, ws, ws, rw) == _lib.MAS_INVALID_ARG
    assert rpl(S._h, s.n - 1, ws, ws, ws, rw) == _lib.MAS_INVALID_ARG  # fewer blocks than diagonal blocks
    assert rpl(S._h, 1 << 31, ws, ws, ws, rw) == _lib.MAS_INVALID_ARG
    assert rpl(S._h, nz, None, ws, ws, rw) == _lib.MAS_INVALID_ARG
    assert rpl(S._h, nz, ws, None, ws, rw) == _lib.MAS_INVALID_ARG
    assert rpl(S._h, nz, ws, ws, vp(4096 + 8), rw) == _lib.MAS_INVALID_ARG  # misaligned workspace
    assert rpl(S._h, nz, ws, ws, ws, rw - 1) == _lib.MAS_WORKSPACE_TOO_SMALL
    h = ctypes.c_void_p()
    assert L.mas_create(None, ctypes.byref(h)) == _lib.MAS_OK
    assert rpl(h, nz, ws, ws, ws, rw) == _lib.MAS_NOT_READY
    L.mas_destroy(h)
    assert S.info()["nnzb"] == nz  # the refused calls left the handle as it was

    mw = int(L.mas_morton_workspace_size(100))
    assert mw > 0
    assert L.mas_morton_partition(0, ws, 16, ws, ws, mw, None) == _lib.MAS_INVALID_ARG
    assert L.mas_morton_partition(100, ws, 0, ws, ws, mw, None) == _lib.MAS_INVALID_ARG
    assert L.mas_morton_partition(100, ws, 16, ws, vp(4096 + 8), mw, None) == _lib.MAS_INVALID_ARG
    assert L.mas_morton_partition(100, ws, 16, ws, ws, mw - 1, None) == _lib.MAS_WORKSPACE_TOO_SMALL
