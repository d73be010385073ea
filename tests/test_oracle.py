"""Pins of the CPU oracle against things other than itself.

Each check compares the oracle with an independent source: dense numpy /
scipy linear algebra, networkx connected components, the paper's worked
examples (``tests/golden``), closed forms and CG invariants.  Nothing here
touches the GPU.
"""

import json
import os

import networkx as nx
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth
from conftest import cube, small_cube

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- helpers ---


def coarsener(sn, units, V):
    """Dense C_l (3*units x 3V) with 3x3 identity blocks at (sn(i), i)."""
    C = np.zeros((3 * units, 3 * V))
    for i, s in enumerate(sn):
        C[3 * s : 3 * s + 3, 3 * i : 3 * i + 3] = np.eye(3)
    return C


def dense_mas(P, H):
    """sum_l C_l^T blockdiag_d(inv(S_d C_l H C_l^T S_d^T)|occupied) C_l with numpy."""
    V, N = P.V, P.N
    _, remap = P.maps()
    out = np.zeros((3 * V, 3 * V))
    for l in range(P.levels):
        nd = P.domains(l)
        C = coarsener(P.sn(l), nd * N, V)
        A = C @ H @ C.T
        BD = np.zeros_like(A)
        for d in range(nd):
            lanes = range(d * N, d * N + N)
            occ = [u for u in lanes if (remap[u] >= 0 if l == 0 else u < P.units(l))]
            idx = np.array([3 * u + c for u in occ for c in range(3)], dtype=np.int64)
            if idx.size:
                BD[np.ix_(idx, idx)] = np.linalg.inv(A[np.ix_(idx, idx)])
        out += C.T @ BD @ C
    return out


def systems_small():
    return [
        cube(1),
        cube(2),
        cube(3, E=1e7, nu=0.45, seed=5),
        synth.random_spd_system(40, 90, seed=3, local=6),
        synth.random_spd_system(23, 30, seed=4),
    ]


# -------------------------------------------------------------- SpMV (O8) ---


@pytest.mark.parametrize("k", range(5))
def test_spmv_matches_scipy_bsr(k):
    s = systems_small()[k]
    x = np.random.default_rng(k).standard_normal(3 * s.n)
    y = oracle.spmv(s.row_ptr, s.col_idx, s.val, x)
    ref = s.scipy_bsr() @ x
    assert np.allclose(y, ref, rtol=1e-14, atol=1e-14 * np.abs(ref).max())


# ------------------------------------------------- partition and slots ------


def test_partition_hand_trace_ladder():
    g = _golden("bfs_bisection_ladder.json")
    gp, ga = synth.graph_from_edges(8, np.array(g["edges"]))
    part, M, No = oracle.partition(8, gp, ga, g["domain_size"])
    assert (M, No) == (g["parts"], g["slack"])
    assert part.tolist() == g["part"]
    mp, _ = oracle.slots(part, M, g["domain_size"])
    assert mp.tolist() == g["map"]


def test_partition_path_graph_gives_contiguous_runs():
    V, N = 37, 4
    gp, ga = synth.graph_from_edges(V, np.stack([np.arange(V - 1), np.arange(1, V)], 1))
    part, M, No = oracle.partition(V, gp, ga, N)
    assert M == -(-V // (N - No))
    # every part is a run of consecutive ids
    for p in range(M):
        ids = np.nonzero(part == p)[0]
        assert ids.size and ids.max() - ids.min() + 1 == ids.size


def test_partition_keeps_disconnected_cliques_apart():
    # two 8-cliques with interleaved ids; N = 8 -> each part is one clique
    a = np.arange(0, 16, 2)
    b = np.arange(1, 16, 2)
    edges = [(u, v) for grp in (a, b) for i, u in enumerate(grp) for v in grp[i + 1 :]]
    gp, ga = synth.graph_from_edges(16, np.array(edges))
    part, M, No = oracle.partition(16, gp, ga, 8)
    assert (M, No) == (2, 0)
    assert len(set(part[a])) == 1 and len(set(part[b])) == 1 and part[a[0]] != part[b[0]]


@pytest.mark.parametrize("N", [1, 3, 4, 16, 21])
def test_partition_and_slot_invariants(N):
    s = cube(3)
    V = s.n
    part, M, No = oracle.partition(V, s.gptr, s.gadj, N)
    # Eq. num_subdomains with the smallest slack
    assert M == -(-V // (N - No))
    sizes = np.bincount(part, minlength=M)
    assert sizes.max() <= N and sizes.sum() == V and sizes.size == M
    mp, rm = oracle.slots(part, M, N)
    assert np.array_equal(rm[mp], np.arange(V))  # remap inverts map
    assert (rm == -1).sum() == M * N - V  # -1 padding fills the rest
    assert np.array_equal(mp // N, part)  # one part per domain
    for p in range(M):  # ascending ids inside a domain, packed from lane 0
        lanes = rm[p * N : (p + 1) * N]
        occ = lanes[lanes >= 0]
        assert np.all(np.diff(occ) > 0) and np.all(lanes[: occ.size] >= 0)


# ------------------------------------------------------- hierarchy (O4) ----


def _components_reference(s, sn_l, units_l, N, occupied):
    """Next-level supernode ids from networkx components, numbered per domain by
    lowest lane."""
    nd = -(-units_l // N)
    G = nx.Graph()
    G.add_nodes_from([u for u in range(units_l) if occupied(u)])
    for i in range(s.n):
        for p in range(s.row_ptr[i], s.row_ptr[i + 1]):
            j = s.col_idx[p]
            a, b = sn_l[i], sn_l[j]
            if i != j and a != b and a // N == b // N:
                G.add_edge(a, b)
    comp_of = {}
    nxt = 0
    for d in range(nd):
        for u in range(d * N, min(d * N + N, units_l)):
            if not occupied(u) or u in comp_of:
                continue
            for v in nx.node_connected_component(G, u):
                comp_of[v] = nxt
            nxt += 1
    return np.array([comp_of[sn_l[i]] for i in range(s.n)]), nxt


@pytest.mark.parametrize("k,N", [(0, 2), (1, 4), (2, 4), (2, 8), (3, 4), (4, 3)])
def test_hierarchy_matches_networkx_components(k, N):
    s = systems_small()[k]
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, gptr=s.gptr, gadj=s.gadj)
    _, remap = P.maps()
    for l in range(P.levels - 1):
        occ = (lambda u: remap[u] >= 0) if l == 0 else (lambda u, S=P.units(l): u < S)
        ref, S_next = _components_reference(s, P.sn(l), P.units(l), N, occ)
        assert np.array_equal(P.sn(l + 1), ref)
        assert P.units(l + 1) == S_next
        assert P.domains(l + 1) == -(-S_next // N)
    # stopping rule: top level is a single domain, or nothing would merge
    L = P.levels
    if P.domains(L - 1) > 1:
        occ = (lambda u: remap[u] >= 0) if L == 1 else (lambda u, S=P.units(L - 1): u < S)
        _, S_next = _components_reference(s, P.sn(L - 1), P.units(L - 1), N, occ)
        occupied = s.n if L == 1 else P.units(L - 1)
        assert S_next == occupied


def test_hierarchy_supernodes_are_connected_subgraphs():
    s = cube(3)
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=8, gptr=s.gptr, gadj=s.gadj)
    G = nx.Graph()
    G.add_nodes_from(range(s.n))
    for i in range(s.n):
        for p in range(s.row_ptr[i], s.row_ptr[i + 1]):
            if s.col_idx[p] != i:
                G.add_edge(i, int(s.col_idx[p]))
    for l in range(1, P.levels):
        sn = P.sn(l)
        assert np.array_equal(np.unique(sn), np.arange(P.units(l)))  # every id used
        for sid in range(P.units(l)):
            assert nx.is_connected(G.subgraph(np.nonzero(sn == sid)[0].tolist()))
        # sn_{l} is a function of sn_{l-1}
        prev = P.sn(l - 1)
        for u in np.unique(prev):
            assert np.unique(sn[prev == u]).size == 1


def _case_study_system():
    g = _golden("case_study_16_nodes.json")
    idx = {c: i for i, c in enumerate(g["nodes"])}
    edges = np.array([(idx[a], idx[b]) for a, b in g["edges"]])
    return g, idx, synth.spd_system_from_edges(16, edges, seed=7)


def test_case_study_index_order_aggregation():
    g, idx, s = _case_study_system()
    N = g["domain_size"]
    part = np.arange(16) // N  # Morton order == node order in the example
    P = oracle.MAS.from_parts(s.row_ptr, s.col_idx, s.val, part, 4, N)
    sn1 = P.sn(1)
    groups = sorted(sorted(c for c in g["nodes"] if sn1[idx[c]] == u) for u in range(P.units(1)))
    assert groups == sorted(sorted(x) for x in g["index_order"]["level1_groups"])
    for c, u in g["index_order"]["level1_supernode_of"].items():
        assert sn1[idx[c]] == u  # merged b,d placed before c (lowest member)
    # first level-1 domain has no internal coupling
    K = P.domain_matrix(1, 0)
    off = K.copy()
    for a in range(N):
        off[3 * a : 3 * a + 3, 3 * a : 3 * a + 3] = 0
    assert np.count_nonzero(off) == 0
    assert P.levels == g["index_order"]["levels"]


def test_case_study_connectivity_order_is_two_level():
    g, idx, s = _case_study_system()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=g["domain_size"], gptr=s.gptr, gadj=s.gadj)
    co = g["connectivity_order"]
    assert P.units(1) == co["level1_supernodes"]
    assert P.domains(1) == co["level1_domains"]
    assert P.levels == co["levels"]


def test_alg2_same_domain_neighbour_mask():
    g = _golden("alg2_hash_example.json")
    N, lane = g["domain_size"], g["lane"]
    V = 4 * N  # identity placement: node i sits in slot i
    edges = [(lane, v) for v in g["neighbour_slots"]]
    s = synth.spd_system_from_edges(V, np.array(edges), seed=11)
    P = oracle.MAS.from_parts(s.row_ptr, s.col_idx, s.val, np.arange(V) // N, 4, N, max_levels=1)
    K = P.domain_matrix(0, 0)
    row = K[3 * lane : 3 * lane + 3]
    mask = 0
    for b in range(N):
        if np.any(row[:, 3 * b : 3 * b + 3] != 0):
            mask |= 1 << b
    assert format(mask, "08b") == g["mask_binary"]


# ------------------------------------- domain matrices, inverses (O5, O6) ---


@pytest.mark.parametrize("k,N", [(1, 4), (2, 4), (3, 5)])
def test_domain_matrices_and_inverses_match_dense_coarsening(k, N):
    s = systems_small()[k]
    H = s.dense()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, gptr=s.gptr, gadj=s.gadj)
    _, remap = P.maps()
    assert P.levels >= 2
    for l in range(P.levels):
        nd = P.domains(l)
        C = coarsener(P.sn(l), nd * N, s.n)
        A = C @ H @ C.T
        for d in range(nd):
            sl = slice(3 * N * d, 3 * N * (d + 1))
            K = P.domain_matrix(l, d)
            assert np.array_equal(K, K.T)
            assert np.allclose(K, A[sl, sl], rtol=1e-13, atol=1e-13 * np.abs(A).max())
            Inv = P.inverse(l, d)
            occ = np.array(
                [u - d * N for u in range(d * N, d * N + N) if (remap[u] >= 0 if l == 0 else u < P.units(l))]
            )
            idx = (3 * occ[:, None] + np.arange(3)[None]).ravel()
            kap = np.linalg.cond(K[np.ix_(idx, idx)])
            assert np.allclose(Inv[np.ix_(idx, idx)] @ K[np.ix_(idx, idx)], np.eye(idx.size), atol=1e-12 * kap)
            mask = np.ones(3 * N, bool)
            mask[idx] = False
            assert not Inv[mask].any() and not Inv[:, mask].any()


# ------------------------------------------------------ MAS apply (O7) ----


@pytest.mark.parametrize("k,N,ml", [(1, 4, 0), (2, 4, 0), (2, 8, 2), (3, 5, 0), (4, 3, 0)])
def test_mas_apply_matches_dense_operator(k, N, ml):
    s = systems_small()[k]
    H = s.dense()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, max_levels=ml, gptr=s.gptr, gadj=s.gadj)
    D = dense_mas(P, H)
    R = np.random.default_rng(k).standard_normal((3 * s.n, 4))
    for c in range(R.shape[1]):
        z = P.apply(R[:, c])
        ref = D @ R[:, c]
        assert np.linalg.norm(z - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("k", range(5))
def test_mas_operator_symmetric_positive_definite(k):
    s = systems_small()[k]
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=4, gptr=s.gptr, gadj=s.gadj)
    n = 3 * s.n
    Z = np.stack([P.apply(e) for e in np.eye(n)], axis=1)
    assert np.abs(Z - Z.T).max() <= 1e-14 * np.abs(Z).max() * 10
    assert np.linalg.eigvalsh(0.5 * (Z + Z.T)).min() > 0
    rng = np.random.default_rng(k)
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    assert abs(u @ P.apply(v) - v @ P.apply(u)) <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(Z @ v)


def test_single_domain_is_exact_inverse_and_one_iteration():
    s = cube(1)  # 8 nodes, N = 16 -> one domain holds everything
    H = s.dense()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, gptr=s.gptr, gadj=s.gadj)
    assert P.levels == 1 and P.domains(0) == 1
    r = np.random.default_rng(0).standard_normal(3 * s.n)
    assert np.linalg.norm(P.apply(r) - np.linalg.solve(H, r)) <= 1e-12 * np.linalg.norm(np.linalg.solve(H, r))
    x, st, it, rr, tr = P.pcg(s.b, tol=1e-12)
    assert st == oracle.OK and it == 1
    xs = np.linalg.solve(H, s.b)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_one_level_is_domain_block_jacobi_and_n1_is_3x3_jacobi():
    s = cube(2)
    H = s.dense()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=4, max_levels=1, gptr=s.gptr, gadj=s.gadj)
    mp, _ = P.maps()
    r = np.random.default_rng(1).standard_normal(3 * s.n)
    z = P.apply(r)
    ref = np.zeros_like(r)
    for d in range(P.parts):
        nodes = np.nonzero(mp // 4 == d)[0]
        idx = (3 * nodes[:, None] + np.arange(3)[None]).ravel()
        ref[idx] = np.linalg.solve(H[np.ix_(idx, idx)], r[idx])
    assert np.linalg.norm(z - ref) <= 1e-13 * np.linalg.norm(ref)
    P1 = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=1, max_levels=1, gptr=s.gptr, gadj=s.gadj)
    z1 = P1.apply(r)
    ref1 = np.concatenate([np.linalg.solve(H[3 * i : 3 * i + 3, 3 * i : 3 * i + 3], r[3 * i : 3 * i + 3]) for i in range(s.n)])
    assert np.linalg.norm(z1 - ref1) <= 1e-13 * np.linalg.norm(ref1)


# ------------------------------------------------------------ PCG (O9) ----


@pytest.mark.parametrize("k", range(5))
def test_pcg_matches_dense_cholesky(k):
    s = systems_small()[k]
    H = s.dense()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=4, gptr=s.gptr, gadj=s.gadj)
    x, st, it, rr, tr = P.pcg(s.b, tol=1e-13, max_iter=2000)
    assert st == oracle.OK and rr <= 1e-13
    xs = sla.cho_solve(sla.cho_factor(H), s.b)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert abs(tr - np.linalg.norm(s.b - H @ x) / np.linalg.norm(s.b)) <= 1e-14


def test_pcg_energy_norm_error_is_monotone():
    s = cube(3, E=1e7, nu=0.45, seed=5)
    H = s.dense()
    xs = np.linalg.solve(H, s.b)
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=4, gptr=s.gptr, gadj=s.gadj)
    errs = []
    for k in range(1, 25):
        x, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=k)
        assert it == k and st == oracle.NOT_CONVERGED
        e = x - xs
        errs.append(np.sqrt(e @ H @ e))
    assert all(b <= a * (1 + 1e-10) for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.05 * errs[0]


def test_pcg_edge_cases():
    s = cube(2)
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=4, gptr=s.gptr, gadj=s.gadj)
    x, st, it, rr, tr = P.pcg(np.zeros(3 * s.n))
    assert st == oracle.OK and it == 0 and not x.any()
    x, st, it, rr, tr = P.pcg(s.b, tol=1e-12, max_iter=1)
    assert st == oracle.NOT_CONVERGED and it == 1 and rr > 1e-12
    # indefinite H: flip a diagonal block -> a domain pivot fails
    val = s.val.copy()
    dpos = [p for p in range(s.row_ptr[5], s.row_ptr[6]) if s.col_idx[p] == 5][0]
    val[dpos] = -val[dpos] - np.eye(3)
    Pb = oracle.MAS(s.row_ptr, s.col_idx, val, N=4, gptr=s.gptr, gadj=s.gadj)
    assert Pb.status == oracle.NOT_SPD


def test_pcg_breakdown_on_indefinite_coupling():
    """sigma = p^T H p <= 0 stops PCG with NOT_SPD (O9) while every domain
    matrix is SPD: two nodes, H = [[I, 2I], [2I, I]] (eigenvalues 3 and -1),
    domains of one node (3x3 block Jacobi, M^-1 = I).  With b = (e1, -e1):
    z = p = b and H p = (-e1, e1), so p^T H p = -2 at the first iteration;
    with b = (e1, e1) the first direction is an eigenvector of eigenvalue 3
    and the solve ends in one iteration with x = b / 3."""
    I3 = np.eye(3)
    row_ptr = np.array([0, 2, 4], dtype=np.int32)
    col_idx = np.array([0, 1, 0, 1], dtype=np.int32)
    val = np.stack([I3, 2 * I3, 2 * I3, I3])
    P = oracle.MAS(row_ptr, col_idx, val, N=1)
    assert P.status == oracle.OK
    b = np.array([1.0, 0, 0, -1.0, 0, 0])
    x, st, it, *_ = P.pcg(b, tol=1e-10)
    assert st == oracle.NOT_SPD and it == 0 and not x.any()
    b = np.array([1.0, 0, 0, 1.0, 0, 0])
    x, st, it, *_ = P.pcg(b, tol=1e-10)
    assert st == oracle.OK and it == 1
    assert np.allclose(x, b / 3.0, rtol=0, atol=1e-15)


# -------------------------------------------------------- adjoint (O11) ---


def test_adjoint_gradient_matches_central_differences():
    s = cube(2, E=1e6, nu=0.45, seed=3)
    H = s.dense()
    rng = np.random.default_rng(0)
    xt = rng.standard_normal(3 * s.n)

    def loss(Hm):
        x = np.linalg.solve(Hm, s.b)
        return 0.5 * np.sum((x - xt) ** 2)

    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=4, gptr=s.gptr, gadj=s.gadj)
    x, *_ = P.pcg(s.b, tol=1e-14)
    lam, *_ = P.pcg(x - xt, tol=1e-14)
    G = oracle.adjoint_scatter(s.row_ptr, s.col_idx, lam, x)
    # dL/db = lambda
    eb = rng.standard_normal(3 * s.n)
    hb = 1e-6
    fd_b = (0.5 * np.sum((np.linalg.solve(H, s.b + hb * eb) - xt) ** 2) - 0.5 * np.sum((np.linalg.solve(H, s.b - hb * eb) - xt) ** 2)) / (2 * hb)
    assert abs(fd_b - lam @ eb) <= 1e-6 * abs(fd_b)
    # symmetric block perturbations: H_ij += eps D, H_ji += eps D^T
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    pos = {(int(r), int(c)): p for p, (r, c) in enumerate(zip(rows, s.col_idx))}
    eps = 1e-6 * np.abs(H).max()
    for p in rng.choice(s.nnzb, size=12, replace=False):
        i, j = int(rows[p]), int(s.col_idx[p])
        D = rng.standard_normal((3, 3))
        if i == j:
            D = D + D.T
        dH = np.zeros_like(H)
        dH[3 * i : 3 * i + 3, 3 * j : 3 * j + 3] += D
        if i != j:
            dH[3 * j : 3 * j + 3, 3 * i : 3 * i + 3] += D.T
        fd = (loss(H + eps * dH) - loss(H - eps * dH)) / (2 * eps)
        pred = np.sum(G[p] * D) + (np.sum(G[pos[(j, i)]] * D.T) if i != j else 0.0)
        assert abs(fd - pred) <= 1e-5 * max(abs(fd), 1e-12)


# ------------------------------------------------------------- assembly ---


def test_assemble_integer_blocks_match_dense_accumulation():
    """Integer-valued blocks sum exactly in any order: the assembled matrix
    equals a dense np.add.at accumulation, the pattern is the set of keys."""
    rng = np.random.default_rng(8)
    n, m = 40, 3000
    rows = rng.integers(0, n, m)
    cols = rng.integers(0, n, m)
    rows[:5] = 7  # a row with many duplicates
    cols[:5] = 3
    blocks = rng.integers(-50, 50, (m, 3, 3)).astype(np.float64)
    rp, ci, val = oracle.assemble(n, rows, cols, blocks)
    dense = np.zeros((3 * n, 3 * n))
    for k in range(m):
        dense[3 * rows[k]:3 * rows[k] + 3, 3 * cols[k]:3 * cols[k] + 3] += blocks[k]
    keys = sorted(set(zip(rows.tolist(), cols.tolist())))
    assert rp[-1] == len(keys) == ci.size
    got = np.zeros_like(dense)
    for i in range(n):
        assert list(ci[rp[i]:rp[i + 1]]) == sorted(c for (r, c) in keys if r == i)
        for p in range(rp[i], rp[i + 1]):
            got[3 * i:3 * i + 3, 3 * ci[p]:3 * ci[p] + 3] = val[p]
    assert np.array_equal(got, dense)


def test_assemble_head_segmented_reduce_example():
    """The paper's warp-segmented reduction example (tests/golden): listed
    blocks whose keys start a new segment where the tag is 1 reduce to the
    printed segment sums, and the same list shuffled gives the same."""
    g = _golden("head_segmented_reduce_example.json")
    seg = np.cumsum(g["tags"]) - 1
    blocks = np.asarray(g["values"], dtype=np.float64)[:, None, None] * np.ones((1, 3, 3))
    rp, ci, val = oracle.assemble(len(g["segment_sums"]), seg, np.zeros_like(seg), blocks)
    assert list(val[:, 0, 0]) == g["segment_sums"] and np.all(val == val[:, :1, :1])
    perm = np.random.default_rng(3).permutation(seg.size)
    _, _, val2 = oracle.assemble(len(g["segment_sums"]), seg[perm], np.zeros_like(seg), blocks[perm])
    assert np.array_equal(val2, val)


def test_assemble_sums_in_list_order_and_edge_cases():
    big = np.full((3, 3), 1e16)
    one = np.ones((3, 3))
    # (1e16 + 1) - 1e16 = 0 in FP64; (1e16 - 1e16) + 1 = 1
    _, _, v = oracle.assemble(2, [1, 1, 1], [0, 0, 0], np.stack([big, one, -big]))
    assert np.all(v[0] == 0.0)
    _, _, v = oracle.assemble(2, [1, 1, 1], [0, 0, 0], np.stack([big, -big, one]))
    assert np.all(v[0] == 1.0)
    rp, ci, v = oracle.assemble(5, [], [], np.zeros((0, 3, 3)))
    assert list(rp) == [0] * 6 and ci.size == 0
    rp, ci, v = oracle.assemble(5, [4, 0], [1, 2], np.stack([one, 2 * one]))
    assert list(rp) == [0, 1, 1, 1, 1, 2] and list(ci) == [2, 1]
    with pytest.raises(ValueError):
        oracle.assemble(3, [0, 3], [0, 0], np.stack([one, one]))


def test_assemble_reproduces_generated_cube():
    """The tet cube's element, mass and contact blocks reassembled: same
    pattern as the generator's (independent numpy) assembly, values equal to
    rounding (the generator adds with a different summation order and
    mirrors its upper triangle)."""
    s = synth.cube_system(4, 1e5, 0.45, seed=3, n_contacts=20, keep_blocks=True)
    rows, cols, blocks = s.meta["blocks"]
    rp, ci, val = oracle.assemble(s.n, rows, cols, blocks)
    assert np.array_equal(rp, s.row_ptr) and np.array_equal(ci, s.col_idx)
    assert np.allclose(val, s.val, rtol=1e-12, atol=1e-12 * np.abs(s.val).max())


# ------------------------------------------ dot modes and perturbation ---
# Used only to derive the iteration-count contract (tests/golden/
# count_ensemble_cube48.json); pinned here against exact arithmetic.


def _exact_dot(a, b):
    from fractions import Fraction

    return sum((Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b)), Fraction(0))


def test_compensated_dot_recovers_cancelled_terms():
    # 1e16 + 1 - 1e16: the plain sum loses the 1, the compensated one keeps it
    a = np.array([1e16, 1.0, -1e16])
    b = np.ones(3)
    assert oracle.dot(a, b, oracle.DOT_SEQUENTIAL) == 0.0
    assert oracle.dot(a, b, oracle.DOT_COMPENSATED) == 1.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_compensated_dot_error_bound(seed):
    # Dot2 (Ogita, Rump, Oishi 2005, Prop. 5.5 / Thm 5.3): |res - a.b| <= u |a.b| + gamma_n^2 sum |a_i b_i|
    rng = np.random.default_rng(seed)
    n = 2000
    a = rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))
    b = rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))
    # ill-conditioned: append the negated sum of a few large products
    a = np.concatenate([a, -a[:50]])
    b = np.concatenate([b, b[:50]])
    exact = _exact_dot(a, b)
    u = 2.0 ** -53
    n2 = a.size
    gamma = n2 * u / (1 - n2 * u)
    absum = float(np.sum(np.abs(a * b)))
    comp = oracle.dot(a, b, oracle.DOT_COMPENSATED)
    seq = oracle.dot(a, b, oracle.DOT_SEQUENTIAL)
    err_c = abs(float(exact - type(exact)(comp)))
    assert err_c <= u * abs(float(exact)) + gamma ** 2 * absum
    # the plain sum meets only the classical bound gamma_n sum |a_i b_i|
    assert abs(float(exact - type(exact)(seq))) <= gamma * absum


def test_pcg_dot_modes():
    s = small_cube()
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, max_levels=2, gptr=s.gptr, gadj=s.gadj)
    x0, st0, it0, *_ = P.pcg(s.b, tol=1e-10)
    lib = oracle.lib()
    # the default PCG is the sequential mode, bit for bit
    import ctypes

    xr = np.empty(3 * s.n)
    it, rr, tr = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    rp = np.ascontiguousarray(s.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(s.col_idx, dtype=np.int32)
    vv = np.ascontiguousarray(s.val, dtype=np.float64).reshape(-1)
    bb = np.ascontiguousarray(s.b, dtype=np.float64)
    st = lib.orc_pcg(s.n, rp.ctypes.data_as(oracle._pi), ci.ctypes.data_as(oracle._pi),
                     vv.ctypes.data_as(oracle._pd), P._h, bb.ctypes.data_as(oracle._pd),
                     xr.ctypes.data_as(oracle._pd), 1e-10, 10000, ctypes.byref(it), ctypes.byref(rr), ctypes.byref(tr))
    assert st == st0 == oracle.OK and it.value == it0
    assert np.array_equal(xr.view(np.uint64), x0.view(np.uint64))
    # compensated dots: same solution up to the tolerance, Cholesky as the reference
    x1, st1, it1, *_ = P.pcg(s.b, tol=1e-10, dots=oracle.DOT_COMPENSATED)
    H = sparse_dense(s)
    xs = sla.cho_solve(sla.cho_factor(H), s.b)
    assert st1 == oracle.OK and abs(it1 - it0) <= 2
    assert np.linalg.norm(x1 - xs) <= 1e-7 * np.linalg.norm(xs)


def sparse_dense(s):
    import scipy.sparse as sp

    return sp.bsr_matrix((s.val.reshape(-1, 3, 3), s.col_idx, s.row_ptr), shape=(3 * s.n, 3 * s.n)).toarray()


def test_perturbation_of_inverses():
    s = cube(4, 1e6, 0.45, seed=3, n_contacts=10)
    args = (s.row_ptr, s.col_idx, s.val)
    kw = dict(N=8, gptr=s.gptr, gadj=s.gadj)
    P0 = oracle.MAS(*args, **kw)
    L = P0.levels
    ref = [[P0.inverse(l, d) for d in range(P0.domains(l))] for l in range(L)]
    P0.perturb(0.0, 7)  # eps = 0 changes nothing
    for l in range(L):
        for d in range(P0.domains(l)):
            assert np.array_equal(P0.inverse(l, d), ref[l][d])
    eps = 1e-6
    Pa, Pb, Pc = oracle.MAS(*args, **kw), oracle.MAS(*args, **kw), oracle.MAS(*args, **kw)
    Pa.perturb(eps, 7)
    Pb.perturb(eps, 7)
    Pc.perturb(eps, 8)
    ratios = []
    for l in range(L):
        for d in range(P0.domains(l)):
            A, B, C, R = Pa.inverse(l, d), Pb.inverse(l, d), Pc.inverse(l, d), ref[l][d]
            assert np.array_equal(A, A.T)  # stays exactly symmetric
            assert np.array_equal(A, B)  # same seed, same perturbation
            nz = R != 0
            assert np.array_equal(A != 0, nz)  # zero lanes stay zero
            q = (A[nz] - R[nz]) / R[nz] / eps
            ratios.append(q)
            assert not np.array_equal(A[nz], C[nz])  # another seed, another perturbation
    q = np.concatenate(ratios)
    # u ~ U[-1, 1): bounded by one, centred, spread as a uniform variable (variance 1/3)
    assert np.all(np.abs(q) <= 1.0 + 1e-6)
    assert abs(q.mean()) < 0.05 and abs(q.var() - 1.0 / 3.0) < 0.05
