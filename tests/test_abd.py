"""Two-level reduction of contact Hessians on affine bodies (Sec. 6.1).

CPU: the oracle's expansion against the Jacobian of the affine map itself
(finite differences of x = t + A xbar, Sec. 3) and a dense sum of
J_r^T C J_c over the contact list.  GPU: the device's first level (node-pair
reduction), its per-pair mapping and the single-level variant against the
oracle, bit for bit, and the two variants' assembled DOF matrices against
each other.
"""

import numpy as np
import pytest

import oracle
from synth.abd import body_contacts


def small_contacts(seed=7):
    return body_contacts(cells=8, n_bodies=5, n_vf=40, n_ee=12, seed=seed)


def affine_jacobian(xbar, n_dof_rows, row, is_body):
    """3 x 3 n_dof_rows Jacobian of a node's position with respect to the
    system's DOFs, by central differences of the motion map: a body node at
    rest position xbar moves as t + A xbar, with q = [t, A[:, 0], A[:, 1],
    A[:, 2]] in block rows row .. row + 3; a mesh node is its own DOF block."""
    n = 3 * n_dof_rows
    J = np.zeros((3, n))
    h = 0.5

    def pos(q):
        if not is_body:
            return q[3 * row:3 * row + 3].copy()
        t = q[3 * row:3 * row + 3]
        A = np.stack([q[3 * row + 3 * (k + 1):3 * row + 3 * (k + 2)] for k in range(3)], axis=1)
        return t + A @ xbar

    q0 = np.zeros(n)
    for j in range(3 * row, 3 * row + (12 if is_body else 3)):
        e = np.zeros(n)
        e[j] = h
        J[:, j] = (pos(q0 + e) - pos(q0 - e)) / (2 * h)
    return J


def dense_from_list(n_rows, rows, cols, blocks):
    D = np.zeros((3 * n_rows, 3 * n_rows))
    for r, c, b in zip(rows, cols, blocks):
        D[3 * r:3 * r + 3, 3 * c:3 * c + 3] += b
    return D


def test_abd_expand_matches_jacobian_products():
    d = small_contacts()
    nd = d["n_dof_rows"]
    J = [affine_jacobian(d["node_xbar"][i], nd, int(d["node_row"][i]), bool(d["node_is_body"][i]))
         for i in range(d["n_nodes"])]
    ref = np.zeros((3 * nd, 3 * nd))
    for r, c, C in zip(d["rows"], d["cols"], d["blocks"]):
        ref += J[r].T @ C @ J[c]
    er, ec, eb = oracle.abd_expand(d["node_row"], d["node_is_body"], d["node_xbar"], d["rows"], d["cols"],
                                   d["blocks"])
    got = dense_from_list(nd, er, ec, eb)
    scale = np.abs(d["blocks"]).max()
    assert np.abs(got - ref).max() <= 1e-12 * scale
    # sub-block counts: 16 body-body, 4 body-mesh / mesh-body, 1 mesh-mesh
    ib = d["node_is_body"]
    want = int(np.sum(np.where(ib[d["rows"]] == 1, 4, 1) * np.where(ib[d["cols"]] == 1, 4, 1)))
    assert er.size == want


def test_abd_two_level_equals_single_level_on_dense_sums():
    """Reducing equal node pairs first (then mapping each pair once) gives
    the same DOF matrix as mapping every listed block."""
    d = small_contacts(seed=11)
    nd = d["n_dof_rows"]
    one = oracle.abd_expand(d["node_row"], d["node_is_body"], d["node_xbar"], d["rows"], d["cols"], d["blocks"])
    rp, ci, val = oracle.assemble(d["n_nodes"], d["rows"], d["cols"], d["blocks"])
    pr = np.repeat(np.arange(d["n_nodes"], dtype=np.int32), np.diff(rp))
    two = oracle.abd_expand(d["node_row"], d["node_is_body"], d["node_xbar"], pr, ci, val)
    assert two[0].size < one[0].size
    D1 = dense_from_list(nd, *one)
    D2 = dense_from_list(nd, *two)
    assert np.abs(D1 - D2).max() <= 1e-12 * np.abs(D1).max()


def test_abd_expand_worked_example_and_edges():
    # one body node (row 5, xbar = (0.1, 0.2, 0.3)) against one mesh node
    # (row 2): 4 sub-blocks (5 + a, 2) = w_a C, w = (1, xbar)
    node_row = np.array([5, 2], dtype=np.int32)
    is_body = np.array([1, 0], dtype=np.int32)
    xbar = np.array([[0.1, 0.2, 0.3], [0.0, 0.0, 0.0]])
    C = np.arange(9, dtype=np.float64).reshape(1, 3, 3) + 1
    r, c, b = oracle.abd_expand(node_row, is_body, xbar, np.array([0], np.int32), np.array([1], np.int32), C)
    assert r.tolist() == [5, 6, 7, 8] and c.tolist() == [2, 2, 2, 2]
    for a, w in enumerate((1.0, 0.1, 0.2, 0.3)):
        assert np.array_equal(b[a], w * C[0])
    # empty list, and a node index out of range
    r, c, b = oracle.abd_expand(node_row, is_body, xbar, np.zeros(0, np.int32), np.zeros(0, np.int32),
                                np.zeros((0, 3, 3)))
    assert r.size == 0
    with pytest.raises(ValueError):
        oracle.abd_expand(node_row, is_body, xbar, np.array([2], np.int32), np.array([0], np.int32), C)


# ---------------------------------------------------------------- GPU parity


def _device_inputs(d, torch):
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev)
         for k in ("node_row", "node_is_body", "node_xbar", "rows", "cols", "blocks")}
    return t


def _oracle_two_level(d):
    rp, ci, val = oracle.assemble(d["n_nodes"], d["rows"], d["cols"], d["blocks"])
    pr = np.repeat(np.arange(d["n_nodes"], dtype=np.int32), np.diff(rp))
    return oracle.abd_expand(d["node_row"], d["node_is_body"], d["node_xbar"], pr, ci, val)


@pytest.mark.gpu
@pytest.mark.parametrize("kw", [dict(cells=8, n_bodies=5, n_vf=40, n_ee=12, seed=3),
                                dict(cells=64, n_bodies=60, n_vf=20000, n_ee=3000, seed=5)])
def test_abd_contact_blocks_match_oracle(kw):
    import torch
    import paper_2411_06224_amd as mp

    d = body_contacts(**kw)
    t = _device_inputs(d, torch)
    args = (d["n_nodes"], t["node_row"], t["node_is_body"], t["node_xbar"], t["rows"], t["cols"], t["blocks"])
    # single level: every listed block mapped, list order
    r1, c1, b1 = mp.abd_contact_blocks(*args, levels=1)
    o1 = oracle.abd_expand(d["node_row"], d["node_is_body"], d["node_xbar"], d["rows"], d["cols"], d["blocks"])
    assert np.array_equal(r1.cpu().numpy(), o1[0]) and np.array_equal(c1.cpu().numpy(), o1[1])
    assert np.array_equal(b1.cpu().numpy(), o1[2])
    # two levels: node pairs summed in list order, each pair mapped once
    r2, c2, b2 = mp.abd_contact_blocks(*args, levels=2)
    o2 = _oracle_two_level(d)
    assert np.array_equal(r2.cpu().numpy(), o2[0]) and np.array_equal(c2.cpu().numpy(), o2[1])
    assert np.array_equal(b2.cpu().numpy(), o2[2])
    # both assemble to one DOF matrix, up to the order of the sums: each
    # entry is a sum of K products w C, so both sides lie within
    # gamma_(K+2) = (K + 2) u of the exact sum, relative to the sum of the
    # magnitudes of its terms
    nd = d["n_dof_rows"]
    A1 = mp.bcsr_assemble(nd, r1, c1, b1)
    A2 = mp.bcsr_assemble(nd, r2, c2, b2)
    assert torch.equal(A1.row_ptr, A2.row_ptr) and torch.equal(A1.col_idx, A2.col_idx)
    _, _, mag = oracle.assemble(nd, o1[0], o1[1], np.abs(o1[2]))
    _, _, cnt = oracle.assemble(nd, o1[0], o1[1], np.ones_like(o1[2]))
    diff = (A1.val - A2.val).abs().cpu().numpy()
    assert np.all(diff <= 2 * (cnt + 2) * 2.0 ** -53 * mag)


@pytest.mark.gpu
def test_abd_contact_blocks_edges():
    import torch
    import paper_2411_06224_amd as mp

    dev = torch.device("cuda:0")
    node_row = torch.tensor([5, 2], dtype=torch.int32, device=dev)
    is_body = torch.tensor([1, 0], dtype=torch.int32, device=dev)
    xbar = torch.tensor([[0.1, 0.2, 0.3], [0.0, 0.0, 0.0]], dtype=torch.float64, device=dev)
    e_i = torch.zeros(0, dtype=torch.int32, device=dev)
    e_b = torch.zeros((0, 3, 3), dtype=torch.float64, device=dev)
    for levels in (1, 2):
        r, c, b = mp.abd_contact_blocks(2, node_row, is_body, xbar, e_i, e_i, e_b, levels=levels)
        assert r.numel() == 0 and b.shape[0] == 0
        bad = torch.tensor([2], dtype=torch.int32, device=dev)
        ok = torch.tensor([0], dtype=torch.int32, device=dev)
        C = torch.ones((1, 3, 3), dtype=torch.float64, device=dev)
        with pytest.raises(RuntimeError):
            mp.abd_contact_blocks(2, node_row, is_body, xbar, bad, ok, C, levels=levels)
        with pytest.raises(RuntimeError):
            mp.abd_contact_blocks(2, node_row, is_body, xbar, ok, bad, C, levels=levels)
    # a pair listed twice: summed once, then mapped (body-body: 16 blocks)
    rr = torch.tensor([0, 0], dtype=torch.int32, device=dev)
    C = torch.stack([torch.full((3, 3), 1.0), torch.full((3, 3), 2.0)]).to(torch.float64).to(dev)
    r, c, b = mp.abd_contact_blocks(2, node_row, is_body, xbar, rr, rr, C, levels=2)
    assert r.numel() == 16
    w = torch.tensor([1.0, 0.1, 0.2, 0.3], dtype=torch.float64)
    want = (w[:, None] * w[None, :]).reshape(16, 1, 1) * torch.full((1, 3, 3), 3.0, dtype=torch.float64)
    assert torch.equal(b.cpu(), want)
    assert r.cpu().tolist() == [5 + a for a in range(4) for _ in range(4)]
    assert c.cpu().tolist() == [5 + bb for _ in range(4) for bb in range(4)]


@pytest.mark.gpu
def test_contact_system_assembled_and_solved():
    """The step before the solve, end to end on a small membrane with bodies:
    the system's own blocks plus the two-level-reduced contact blocks,
    assembled on the GPU (bit-exact with the oracle's assembly of the same
    lists), then analysed and solved with the MAS-PCG; the solution agrees
    with the oracle's PCG on the same matrix."""
    import torch
    import paper_2411_06224_amd as mp
    from synth import membrane_system

    s = membrane_system(16, 6, seed=5)
    d = body_contacts(cells=16, n_bodies=6, n_vf=300, n_ee=60, seed=6)
    assert d["n_dof_rows"] == s.n
    dev = torch.device("cuda:0")
    t = _device_inputs(d, torch)
    r2, c2, b2 = mp.abd_contact_blocks(d["n_nodes"], t["node_row"], t["node_is_body"], t["node_xbar"], t["rows"],
                                       t["cols"], t["blocks"], levels=2)
    mr = np.repeat(np.arange(s.n, dtype=np.int32), np.diff(s.row_ptr))
    mc = s.col_idx.astype(np.int32)
    rows = torch.cat([torch.as_tensor(mr, device=dev), r2])
    cols = torch.cat([torch.as_tensor(mc, device=dev), c2])
    blocks = torch.cat([torch.as_tensor(s.val.reshape(-1, 3, 3), device=dev), b2])
    Hg = mp.bcsr_assemble(s.n, rows, cols, blocks)
    o2 = _oracle_two_level(d)
    rp, ci, val = oracle.assemble(s.n, np.concatenate([mr, o2[0]]), np.concatenate([mc, o2[1]]),
                                  np.concatenate([s.val.reshape(-1, 3, 3), o2[2]]))
    assert np.array_equal(Hg.row_ptr.cpu().numpy(), rp) and np.array_equal(Hg.col_idx.cpu().numpy(), ci)
    assert np.array_equal(Hg.val.cpu().numpy().view(np.int64), val.view(np.int64))
    assert ci.size > s.col_idx.size  # the contacts added blocks
    S = mp.MasPcg(rp, ci, graph=(s.gptr, s.gadj), domain_size=16)
    b = torch.as_tensor(s.b, device=dev)
    S.build(Hg)
    P = oracle.MAS(rp, ci, val, N=16, gptr=s.gptr, gadj=s.gadj)
    # ten iterations against the oracle's ten (the parity contract of the
    # fixed-iteration tests), then a converged solve
    xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
    x, res = S.solve(Hg, b, tol=0.0, max_iter=10)
    assert res["iterations"] == it == 10
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)
    # converged: the count contract of the other converged tests (the
    # oracle's spread under rounding-level changes, +-2) and x against it
    from count_contract import oracle_ensemble

    lo, hi, x_tol, x_ref, _ = oracle_ensemble(lambda: oracle.MAS(rp, ci, val, N=16, gptr=s.gptr, gadj=s.gadj),
                                              s.b, 1e-10)
    x, res = S.solve(Hg, b, tol=1e-10)
    assert res["status"] == 0 and res["true_rel_residual"] <= 1e-10
    assert lo <= res["iterations"] <= hi
    assert np.linalg.norm(x.cpu().numpy() - x_ref) <= x_tol * np.linalg.norm(x_ref)
