"""Solver plans of a changed pattern derived on the device (mas_replan;
Sec. 4.2, Supp. Alg. 2-5, Supp. Eq. 5).

A handle analysed on the contact-free pattern is re-planned on the device
for the pattern with contacts.  Its plans must be the host analysis's for
the same pattern and partition, bit for bit: after build, and again after a
fixed number of PCG iterations, the whole solver workspace (plans, matrix
copies, coarse matrices, inverses, vectors) equals byte for byte that of a
handle analysed on the host with that partition, and converged solutions
are identical.  The solve is also checked
against the oracle on the same partition, and bad patterns are rejected
with the previous plans left working."""

import sys
import time

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


def _csr(n, r, c):
    key = np.unique(r.astype(np.int64) * n + c.astype(np.int64))
    r, c = key // n, key % n
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp).astype(np.int32), c.astype(np.int32), r


def _graph_pattern(s):
    """Diagonal plus the mesh graph's edges: the pattern before contacts."""
    n = s.n
    deg = np.diff(s.gptr)
    r = np.concatenate([np.arange(n), np.repeat(np.arange(n), deg)])
    c = np.concatenate([np.arange(n), s.gadj])
    rp, ci, _ = _csr(n, r, c)
    return rp, ci


def _add_pairs(rp, ci, n_pairs, seed):
    """The pattern with n_pairs random node pairs in both directions, and
    diagonally dominant values on it (10 I diagonal, 0.01 I elsewhere)."""
    n = rp.size - 1
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n, n_pairs)
    b = rng.integers(0, n, n_pairs)
    r = np.concatenate([np.repeat(np.arange(n), np.diff(rp)), a, b])
    c = np.concatenate([ci, b, a])
    rp2, ci2, r2 = _csr(n, r, c)
    val = np.where((r2 == ci2)[:, None, None], 10.0, 0.01) * np.eye(3)[None]
    return rp2, ci2, val


def _slice(S):
    off = S._ws_ptr - S._ws.data_ptr()
    return S._ws[off:off + S.workspace_size()]


def _same_bytes(A, B, when):
    wa, wb = _slice(A), _slice(B)
    assert wa.numel() == wb.numel()
    diff = torch.nonzero(wa != wb).flatten().cpu().numpy()
    if diff.size:
        runs = np.split(diff, np.nonzero(np.diff(diff) > 8)[0] + 1)
        spans = [(int(r[0]), int(r[-1]) + 1) for r in runs[:8]]
        o = int(diff[0]) // 8 * 8
        va = wa[o:o + 32].cpu().numpy().view(np.float64)
        vb = wb[o:o + 32].cpu().numpy().view(np.float64)
        raise AssertionError(f"{when}: {diff.size} differing bytes of {wa.numel()}, spans {spans}; "
                             f"doubles at {o}: {va} vs {vb}")


def _compare(A, B, rp, ci, val, dev, tol=1e-8, b=None):
    """A (device plans) against B (host plans, same partition): description,
    ordering, the solution and the whole workspace after build and solve."""
    from paper_2411_06224_amd import BlockMatrix

    ia, ib = A.info(), B.info()
    for k in ("levels", "units", "domains", "coarse_nnzb", "workspace_bytes", "inverse_bytes", "stored_blocks",
              "nnzb", "parts"):
        assert ia[k] == ib[k], (k, ia[k], ib[k])
    ma, ra, sa = A.ordering()
    mb, rb, sb = B.ordering()
    assert np.array_equal(ma, mb) and np.array_equal(ra, rb) and np.array_equal(sa, sb)
    H = BlockMatrix.from_numpy(rp, ci, val, device=dev)
    if b is None:
        b = np.random.default_rng(7).standard_normal(3 * (rp.size - 1))
    bt = torch.as_tensor(b, device=dev)
    A.build(H)
    B.build(H)
    torch.cuda.synchronize()
    _same_bytes(A, B, "after build")
    xa, resa = A.solve(H, bt, tol=tol)
    xb, resb = B.solve(H, bt, tol=tol)
    torch.cuda.synchronize()
    assert resa == resb
    assert torch.equal(xa, xb)
    # a converged solve may leave launches queued past its stop (they return
    # early, but the coarse vectors they touch depend on how far the host had
    # queued); a fixed number of iterations leaves the whole workspace equal
    xa, _ = A.solve(H, bt, tol=0.0, max_iter=12)
    xb, _ = B.solve(H, bt, tol=0.0, max_iter=12)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)
    _same_bytes(A, B, "after 12 iterations")
    return ia, resa


def _pair(s, rp2, ci2, N, precision="f64", max_levels=0):
    """A: analysed on the contact-free pattern, re-planned on the device for
    (rp2, ci2); B: the host analysis of (rp2, ci2) on A's partition."""
    from paper_2411_06224_amd import MasPcg

    rp1, ci1 = _graph_pattern(s)
    A = MasPcg(rp1, ci1, graph=(s.gptr, s.gadj), domain_size=N, precision=precision, max_levels=max_levels,
               poison=True)
    dev = torch.device("cuda:0")
    A.replan(torch.as_tensor(rp2, device=dev), torch.as_tensor(ci2, device=dev))
    mp_, _, _ = A.ordering()
    B = MasPcg(rp2, ci2, domain_size=N, precision=precision, max_levels=max_levels, partition=mp_ // N,
               poison=True)
    return A, B


CASES = {
    "cube8_200": lambda: (small_cube(), 200),
    "cube8_800": lambda: (small_cube(), 800),
    "contact6_300": lambda: (cube(6, E=1e6, nu=0.49, seed=21, n_contacts=60), 300),
    "local2000_500": lambda: (synth.random_spd_system(2000, 6000, seed=6, local=30), 500),
    # dense local rows: groups with more transposed entries than the
    # symmetric storage holds, so the SpMV keeps the full storage
    "dense_local_100": lambda: (synth.random_spd_system(2000, 90000, seed=6, local=60), 100),
}


@pytest.mark.parametrize("precision", ["f64", "mixed"])
@pytest.mark.parametrize("N", [16, 40, 7])
@pytest.mark.parametrize("name", list(CASES))
def test_replan_matches_host_plans(dev, name, N, precision):
    _say("replan", name, N, precision)
    s, n_pairs = CASES[name]()
    rp1, ci1 = _graph_pattern(s)
    rp2, ci2, val2 = _add_pairs(rp1, ci1, n_pairs, seed=N)
    A, B = _pair(s, rp2, ci2, N, precision)
    inf, res = _compare(A, B, rp2, ci2, val2, dev, tol=1e-8)
    assert res["status"] == 0
    if name == "dense_local_100" and N == 16:
        assert inf["stored_blocks"] == inf["nnzb"]  # the full-storage case is covered
    print("levels", inf["levels"], "units", inf["units"], "iterations", res["iterations"])


TINY = {
    "cube1": lambda: cube(1),
    "cube2": lambda: cube(2),
    "rand300_local": lambda: synth.random_spd_system(300, 700, seed=2, local=12),
}


@pytest.mark.parametrize("N", [1, 4, 16])
@pytest.mark.parametrize("name", list(TINY))
def test_replan_tiny_systems(dev, name, N):
    """Small systems and domain sizes (a single domain, one node per
    domain, padded slots), with contacts added and with the pattern
    reduced to its diagonal (nothing merges: one level)."""
    _say("replan tiny", name, N)
    s = TINY[name]()
    rp1, ci1 = _graph_pattern(s)
    n = s.n
    rp2, ci2, val2 = _add_pairs(rp1, ci1, max(2, n // 4), seed=N)
    A, B = _pair(s, rp2, ci2, N)
    _compare(A, B, rp2, ci2, val2, dev)
    rpd = np.arange(n + 1, dtype=np.int32)
    cid = np.arange(n, dtype=np.int32)
    vald = np.tile(np.eye(3) * 4.0, (n, 1, 1))
    A, B = _pair(s, rpd, cid, N)
    inf, _ = _compare(A, B, rpd, cid, vald, dev)
    assert inf["levels"] == 1


def test_replan_deep_hierarchy(dev):
    """A pattern whose hierarchy reaches the 16-level limit."""
    _say("replan deep")
    s = synth.random_spd_system(4000, 60000, seed=4)
    A, B = _pair(s, s.row_ptr, s.col_idx, 16)
    inf, _ = _compare(A, B, s.row_ptr, s.col_idx, s.val, dev, tol=1e-8, b=s.b)
    assert inf["levels"] == 16


@pytest.mark.parametrize("max_levels", [1, 2, 3])
def test_replan_level_cap(dev, max_levels):
    _say("replan cap", max_levels)
    s, n_pairs = CASES["contact6_300"]()
    rp1, ci1 = _graph_pattern(s)
    rp2, ci2, val2 = _add_pairs(rp1, ci1, n_pairs, seed=5)
    A, B = _pair(s, rp2, ci2, 16, max_levels=max_levels)
    inf, _ = _compare(A, B, rp2, ci2, val2, dev)
    assert inf["levels"] <= max_levels


def test_replan_contact_system_against_oracle(dev):
    """The cube with contacts (its own values), re-planned from the
    contact-free pattern: the MAS apply and ten PCG iterations against the
    oracle on the same partition (1e-10, as for host-planned handles)."""
    _say("replan contact6 oracle")
    s = cube(6, E=1e6, nu=0.49, seed=21, n_contacts=60)
    A, B = _pair(s, s.row_ptr, s.col_idx, 16)
    _compare(A, B, s.row_ptr, s.col_idx, s.val, dev, tol=1e-8, b=s.b)
    mp_, _, _ = A.ordering()
    part = mp_ // 16
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, part=part, M=int(part.max()) + 1)
    assert P.levels == A.info()["levels"]
    from paper_2411_06224_amd import BlockMatrix

    H = BlockMatrix.from_numpy(s.row_ptr, s.col_idx, s.val, device=dev)
    A.build(H)
    rng = np.random.default_rng(3)
    for _ in range(3):
        r = rng.standard_normal(3 * s.n)
        z = A.apply(torch.as_tensor(r, device=dev)).cpu().numpy()
        ref = P.apply(r)
        assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
    x, res = A.solve(H, torch.as_tensor(s.b, device=dev), tol=0.0, max_iter=10)
    assert res["iterations"] == it == 10
    x = x.cpu().numpy()
    assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_replan_adjoint(dev, precision):
    """The adjoint solve and the dL/dH scatter of a re-planned handle equal
    those of the host-planned handle, bit for bit."""
    from paper_2411_06224_amd import BlockMatrix

    _say("replan adjoint", precision)
    s, n_pairs = CASES["contact6_300"]()
    rp1, ci1 = _graph_pattern(s)
    rp2, ci2, val2 = _add_pairs(rp1, ci1, n_pairs, seed=2)
    A, B = _pair(s, rp2, ci2, 16, precision)
    H = BlockMatrix.from_numpy(rp2, ci2, val2, device=dev)
    rng = np.random.default_rng(4)
    b = torch.as_tensor(rng.standard_normal(3 * s.n), device=dev)
    g = torch.as_tensor(rng.standard_normal(3 * s.n), device=dev)
    out = []
    for S in (A, B):
        S.build(H)
        x, _ = S.solve(H, b, tol=1e-10)
        lam, dH, res = S.adjoint(H, x, g, tol=1e-10)
        out.append((x, lam, dH, res))
    torch.cuda.synchronize()
    (xa, la, da, ra), (xb, lb, db, rb) = out
    assert ra == rb and ra["status"] == 0
    assert torch.equal(xa, xb) and torch.equal(la, lb) and torch.equal(da, db)


def test_replan_back_and_forth(dev):
    """Contacts appear, change and disappear: three re-plans in a row on one
    handle, each checked against the host analysis of its pattern."""
    from paper_2411_06224_amd import MasPcg

    _say("replan back and forth")
    s = small_cube()
    rp1, ci1 = _graph_pattern(s)
    A = MasPcg(rp1, ci1, graph=(s.gptr, s.gadj), domain_size=16, poison=True)
    mp_, _, _ = A.ordering()
    part = mp_ // 16
    val1 = np.where((np.repeat(np.arange(s.n), np.diff(rp1)) == ci1)[:, None, None], 10.0, 0.01) * np.eye(3)[None]
    steps = [_add_pairs(rp1, ci1, 300, seed=1), _add_pairs(rp1, ci1, 900, seed=2), (rp1, ci1, val1)]
    for rp, ci, val in steps:
        A.replan(torch.as_tensor(rp, device=dev), torch.as_tensor(ci, device=dev))
        B = MasPcg(rp, ci, domain_size=16, partition=part, poison=True)
        A._ws = None  # a fresh poisoned workspace, so that the byte comparison sees only this step's writes
        _compare(A, B, rp, ci, val, dev)
        # the device hierarchy of a re-planned handle is built from the re-planned pattern
        units, sn = A.hierarchy_device(dev)
        inf = B.info()
        assert list(units) == inf["units"] and np.array_equal(sn, B.ordering()[2])


def test_replan_rejects_bad_patterns(dev):
    """Patterns that break the analysis rules are refused, and the handle
    keeps solving with its previous plans."""
    from paper_2411_06224_amd import BlockMatrix, MasError, MasPcg
    from paper_2411_06224_amd._lib import MAS_INVALID_ARG

    _say("replan bad patterns")
    s = cube(6, E=1e6, nu=0.49, seed=21, n_contacts=60)
    rp1, ci1 = _graph_pattern(s)
    rp2, ci2, val2 = _add_pairs(rp1, ci1, 200, seed=9)
    A = MasPcg(rp1, ci1, graph=(s.gptr, s.gadj), domain_size=16)
    A.replan(torch.as_tensor(rp2, device=dev), torch.as_tensor(ci2, device=dev))
    H = BlockMatrix.from_numpy(rp2, ci2, val2, device=dev)
    b = torch.as_tensor(np.random.default_rng(1).standard_normal(3 * s.n), device=dev)
    A.build(H)
    x0, r0 = A.solve(H, b, tol=1e-10)
    n = s.n
    rows = np.repeat(np.arange(n), np.diff(rp2))
    bad = []
    ci = ci2.copy()
    ci[3] = n  # column past the last node
    bad.append((rp2, ci, "column range"))
    k = int(np.nonzero(rows != ci2)[0][0])
    keep = np.ones(ci2.size, bool)
    keep[k] = False  # drop one off-diagonal block: the pattern is no longer symmetric
    rpd = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=n))]).astype(np.int32)
    bad.append((rpd, ci2[keep], "symmetry"))
    d = int(np.nonzero(rows == ci2)[0][5])
    keep = np.ones(ci2.size, bool)
    keep[d] = False  # drop a diagonal block
    rpd = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=n))]).astype(np.int32)
    bad.append((rpd, ci2[keep], "diagonal"))
    ci = ci2.copy()
    r0_ = int(np.nonzero(np.diff(rp2) >= 3)[0][0])
    p = rp2[r0_]
    ci[p], ci[p + 1] = ci[p + 1], ci[p]  # two columns out of order
    bad.append((rp2, ci, "order"))
    rp = rp2.copy()
    rp[-1] -= 1  # row_ptr does not end at nnzb (one column left over)
    bad.append((rp, ci2, "row_ptr end"))
    rp = rp2.copy()
    rp[n // 2] = rp[n // 2 + 1] + 1  # a row range that runs backwards
    bad.append((rp, ci2, "row_ptr order"))
    for rp, ci, what in bad:
        with pytest.raises(MasError) as e:
            A.replan(torch.as_tensor(rp, device=dev), torch.as_tensor(ci, device=dev))
        assert e.value.code == MAS_INVALID_ARG, what
        A.build(H)
        x, r = A.solve(H, b, tol=1e-10)
        assert r == r0 and torch.equal(x, x0), what


@pytest.mark.parametrize("case", [(64, 60, 8), (512, 2000, 1003)])
def test_replan_membrane(dev, case):
    """The membrane with affine bodies (groups with hundreds of coarse
    writers, 16 levels at full size), re-planned for its pattern plus
    random couplings, in both precisions."""
    _say("replan membrane", case)
    s = synth.membrane_system(case[0], case[1], seed=case[2])
    rp2, ci2, val2 = _add_pairs(s.row_ptr, s.col_idx, 500, seed=11)
    for precision in ("f64", "mixed"):
        A, B = _pair(s, rp2, ci2, 16, precision)
        inf, res = _compare(A, B, rp2, ci2, val2, dev, tol=1e-6)
        assert res["status"] == 0
        print(precision, "levels", inf["levels"], "iterations", res["iterations"])


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_newton_steps_on_device(dev, precision):
    """The per-Newton path with no host analysis, for two contact sets in
    turn on a small membrane with bodies: contact Hessians reduced in two
    levels and assembled with the system's own blocks on the GPU, the
    solver re-planned from the assembled device pattern, built and solved.
    Each step equals the host analysis of its pattern on the same partition
    byte for byte, and ten iterations agree with the oracle (1e-10)."""
    import paper_2411_06224_amd as mp
    from synth.abd import body_contacts

    _say("newton steps on device", precision)
    s = synth.membrane_system(16, 6, seed=5)
    S = mp.MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16, precision=precision, poison=True)
    part = S.ordering()[0] // 16
    own_r = torch.as_tensor(np.repeat(np.arange(s.n, dtype=np.int32), np.diff(s.row_ptr)), device=dev)
    own_c = torch.as_tensor(s.col_idx, device=dev)
    own_v = torch.as_tensor(s.val.reshape(-1, 3, 3), device=dev)
    for seed in (6, 8):
        d = body_contacts(cells=16, n_bodies=6, n_vf=300, n_ee=60, seed=seed)
        assert d["n_dof_rows"] == s.n
        t = {k: torch.as_tensor(np.ascontiguousarray(d[k]), device=dev)
             for k in ("node_row", "node_is_body", "node_xbar", "rows", "cols", "blocks")}
        r2, c2, b2 = mp.abd_contact_blocks(d["n_nodes"], t["node_row"], t["node_is_body"], t["node_xbar"],
                                           t["rows"], t["cols"], t["blocks"], levels=2)
        Hg = mp.bcsr_assemble(s.n, torch.cat([own_r, r2]), torch.cat([own_c, c2]), torch.cat([own_v, b2]))
        S.replan(Hg.row_ptr, Hg.col_idx)
        rp, ci, val = Hg.row_ptr.cpu().numpy(), Hg.col_idx.cpu().numpy(), Hg.val.cpu().numpy()
        assert ci.size > s.col_idx.size  # the contacts added blocks
        B = mp.MasPcg(rp, ci, domain_size=16, partition=part, precision=precision, poison=True)
        S._ws = None  # a fresh poisoned workspace for the byte comparison
        _compare(S, B, rp, ci, val, dev, tol=1e-8, b=s.b)
        if precision != "f64":
            continue  # the oracle comparison below is the FP64 one
        P = oracle.MAS(rp, ci, val, N=16, part=part, M=int(part.max()) + 1)
        xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
        x, res = S.solve(Hg, torch.as_tensor(s.b, device=dev), tol=0.0, max_iter=10)
        assert res["iterations"] == it == 10
        assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_replan_large_cube(dev, precision):
    """48^3 nodes with 20,000 contacts, re-planned from the contact-free
    pattern; the time of the device re-plan is printed beside the host
    analysis of the same pattern and partition."""
    from paper_2411_06224_amd import MasPcg

    _say("replan 48^3", precision)
    s = large_cube()
    rp1, ci1 = _graph_pattern(s)
    A = MasPcg(rp1, ci1, graph=(s.gptr, s.gadj), domain_size=16, precision=precision, poison=True)
    rp_d = torch.as_tensor(s.row_ptr, device=dev)
    ci_d = torch.as_tensor(s.col_idx, device=dev)
    A.replan(rp_d, ci_d)  # warm-up (code objects, allocator)
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A.replan(rp_d, ci_d)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    mp_, _, _ = A.ordering()
    t0 = time.perf_counter()
    B = MasPcg(s.row_ptr, s.col_idx, domain_size=16, partition=mp_ // 16, precision=precision, poison=True)
    t_host = time.perf_counter() - t0
    inf, res = _compare(A, B, s.row_ptr, s.col_idx, s.val, dev, tol=1e-4, b=s.b)
    print(f"replan on the device {1e3 * min(times):.2f} ms; host analysis {1e3 * t_host:.1f} ms; "
          f"levels {inf['levels']}, iterations {res['iterations']}")
