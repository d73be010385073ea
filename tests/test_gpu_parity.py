"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances:
  SpMV (FP64)             |y - y_ref|_i <= 1e-14 (|H||x|)_i + tiny
  MAS apply (FP64)        ||z - z_ref|| <= 1e-10 ||z_ref||
  PCG, fixed iterations   ||x_k - x_k,ref|| <= 1e-10 ||x_k,ref||
  PCG, converged          both meet tol on the true residual; the iteration count within
                          2 of the range the oracle spans under rounding-level changes
                          (count_contract.py); x within twice the oracle's own spread
  tight solve             ||x - x_ref|| <= 1e-10 ||x_ref|| at tol 1e-13
  mixed precision         true FP64 residual <= tol; error vs the FP64 oracle printed
  gradients               vs dense FP64 gradient <= 1e-8 relative
"""

import sys

import numpy as np
import pytest

import oracle
import synth
from conftest import cube, large_cube, small_cube
from count_contract import oracle_ensemble

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

    mp.load()  # fail loudly if the library is missing
    return torch.device("cuda:0")


def _H(s, dev, dtype=torch.float64):
    from paper_2411_06224_amd import BlockMatrix

    return BlockMatrix.from_numpy(s.row_ptr, s.col_idx, s.val, device=dev, dtype=dtype)


def _t(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)


def _solver(s, N=16, max_levels=0, precision="f64", graph=True, poison=True):
    """Workspaces start as NaN bit patterns: reading memory the library did
    not write turns into a failure."""
    from paper_2411_06224_amd import MasPcg

    return MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj) if graph else None, domain_size=N,
                  max_levels=max_levels, precision=precision, poison=poison)


def _oracle(s, N=16, max_levels=0, graph=True):
    if graph:
        return oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, max_levels=max_levels, gptr=s.gptr, gadj=s.gadj)
    return oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, max_levels=max_levels)


def _count_contract(s, tol, N=16, graph=True):
    """(lo, hi, x_tol, x_ref) of count_contract.oracle_ensemble for system s."""
    lo, hi, xt, x0, _ = oracle_ensemble(lambda: _oracle(s, N, graph=graph), s.b, tol)
    return lo, hi, xt, x0


def _absH_absx(s, x):
    return oracle.spmv(s.row_ptr, s.col_idx, np.abs(s.val), np.abs(x))


SYSTEMS = {
    "cube1": lambda: cube(1),
    "cube2": lambda: cube(2),
    "cube3_stiff": lambda: cube(3, E=1e7, nu=0.45, seed=5),
    "cube8": small_cube,
    "rand300": lambda: synth.random_spd_system(300, 700, seed=2, local=12),
    "contact6": lambda: cube(6, E=1e6, nu=0.49, seed=21, n_contacts=60),
}


# ------------------------------------------------------------------ SpMV ---


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_spmv(dev, name, dtype):
    from paper_2411_06224_amd import bcsr_spmv

    _say("spmv", name, dtype)
    s = SYSTEMS[name]()
    x = np.random.default_rng(1).standard_normal(3 * s.n)
    vals = s.val if dtype == "f64" else s.val.astype(np.float32).astype(np.float64)
    H = _H(s, dev, torch.float64 if dtype == "f64" else torch.float32)
    y = bcsr_spmv(H, _t(x, dev)).cpu().numpy()
    ref = oracle.spmv(s.row_ptr, s.col_idx, vals, x)
    bound = 1e-14 * oracle.spmv(s.row_ptr, s.col_idx, np.abs(vals), np.abs(x)) + 1e-300
    assert np.all(np.abs(y - ref) <= bound)


def test_spmv_empty_rows_and_zero_sizes(dev):
    from paper_2411_06224_amd import BlockMatrix, bcsr_spmv

    _say("spmv empty rows")
    rp = np.array([0, 0, 1, 1, 3, 3], np.int32)  # rows 0, 2, 4 empty
    ci = np.array([1, 1, 3], np.int32)
    val = np.random.default_rng(0).standard_normal((3, 3, 3))
    H = BlockMatrix.from_numpy(rp, ci, val, device=dev)
    x = np.random.default_rng(1).standard_normal(15)
    y = bcsr_spmv(H, _t(x, dev)).cpu().numpy()
    assert np.allclose(y, oracle.spmv(rp, ci, val, x), rtol=1e-14, atol=1e-14)
    assert np.all(y[0:3] == 0) and np.all(y[6:9] == 0) and np.all(y[12:15] == 0)


# ------------------------------------------------------------- MAS apply ---

APPLY_CASES = [
    ("cube1", 16, 0),
    ("cube2", 4, 0),
    ("cube3_stiff", 4, 0),
    ("cube3_stiff", 1, 0),
    ("cube8", 16, 2),
    ("cube8", 16, 0),
    ("cube8", 21, 0),
    ("cube8", 32, 0),
    ("cube8", 40, 0),
    ("cube8", 7, 1),
    ("rand300", 8, 0),
    ("contact6", 16, 0),
]


@pytest.mark.parametrize("name,N,ml", APPLY_CASES)
def test_mas_apply(dev, name, N, ml):
    _say("mas_apply", name, N, ml)
    s = SYSTEMS[name]()
    P = _oracle(s, N, ml)
    S = _solver(s, N, ml)
    S.build(_H(s, dev))
    rng = np.random.default_rng(3)
    for _ in range(3):
        r = rng.standard_normal(3 * s.n)
        z = S.apply(_t(r, dev)).cpu().numpy()
        ref = P.apply(r)
        assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


def test_mas_apply_dense_operator_tiny(dev):
    _say("mas_apply dense operator cube2 N=4")
    s = cube(2)
    P = _oracle(s, 4)
    S = _solver(s, 4)
    S.build(_H(s, dev))
    n = 3 * s.n
    E = torch.eye(n, dtype=torch.float64, device=dev)
    Z = torch.stack([S.apply(E[:, k].contiguous()) for k in range(n)], 1).cpu().numpy()
    Zr = np.stack([P.apply(np.eye(n)[:, k]) for k in range(n)], 1)
    assert np.linalg.norm(Z - Zr) <= 1e-10 * np.linalg.norm(Zr)
    assert np.abs(Z - Z.T).max() <= 1e-12 * np.abs(Z).max()


# ------------------------------------------------------------------- PCG ---


# every: period of the iterations that restrict r_k directly (50: all ten by
# the coarse recurrence, 1: none, 3: the two kinds interleaved)
@pytest.mark.parametrize("every", [50, 3, 1])
@pytest.mark.parametrize("name,N", [("cube2", 4), ("cube3_stiff", 4), ("cube8", 16), ("rand300", 8), ("contact6", 16)])
def test_pcg_fixed_iterations(dev, name, N, every):
    _say("pcg fixed 10", name, N, every)
    s = SYSTEMS[name]()
    P = _oracle(s, N)
    xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
    S = _solver(s, N)
    H = _H(s, dev)
    S.build(H)
    x, res = S.solve(H, _t(s.b, dev), tol=0.0, max_iter=10, replace_every=every)
    assert res["iterations"] == it == 10 and res["status"] == 1
    x = x.cpu().numpy()
    assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.parametrize("name,N,tol", [("cube8", 16, 1e-8), ("contact6", 16, 1e-6), ("rand300", 8, 1e-8), ("cube3_stiff", 4, 1e-10)])
def test_pcg_converged(dev, name, N, tol):
    _say("pcg converged", name, N, tol)
    s = SYSTEMS[name]()
    P = _oracle(s, N)
    xr, st, it, rr, tr = P.pcg(s.b, tol=tol)
    S = _solver(s, N)
    H = _H(s, dev)
    S.build(H)
    x, res = S.solve(H, _t(s.b, dev), tol=tol)
    assert res["status"] == 0 and st == 0
    lo, hi, xt, _ = _count_contract(s, tol, N)
    assert lo <= res["iterations"] <= hi, (res["iterations"], it, lo, hi)
    assert res["true_rel_residual"] <= tol * 1.01
    xv = x.cpu().numpy()
    assert np.linalg.norm(xv - xr) <= xt * np.linalg.norm(xr), (np.linalg.norm(xv - xr) / np.linalg.norm(xr), xt)
    true = np.linalg.norm(s.b - oracle.spmv(s.row_ptr, s.col_idx, s.val, xv)) / np.linalg.norm(s.b)
    assert true <= tol * 1.01


@pytest.mark.parametrize("name,N,ml", [("cube8", 16, 2), ("cube8", 16, 0), ("contact6", 16, 0), ("rand300", 8, 0),
                                        ("cube3_stiff", 4, 0), ("cube2", 5, 0)])
def test_inverses(dev, name, N, ml):
    """P3: every domain inverse of every level against the oracle's,
    relative Frobenius <= 1e-10 (FP64); the FP32 copy of a mixed handle
    within FP32 rounding of the FP64 one."""
    _say("inverses", name, N, ml)
    s = SYSTEMS[name]()
    P = _oracle(s, N, ml)
    H = _H(s, dev)
    for prec in ("f64", "mixed"):
        S = _solver(s, N, ml, precision=prec)
        S.build(H)
        assert S.info()["levels"] == P.levels
        for l in range(P.levels):
            G = S.inverses(l)
            for d in range(G.shape[0]):
                R = P.inverse(l, d)
                e = np.linalg.norm(G[d] - R) / np.linalg.norm(R)
                assert e <= 1e-10, (prec, l, d, e)
            if prec == "mixed":  # the FP32 copy: each entry the FP64 one rounded (up to the
                # kappa u asymmetry of the unsymmetrised inverse the FP32 copy is cast from)
                G32 = S.inverses(l, "mixed")
                assert np.all(np.abs(G32 - G) <= 2.0 ** -24 * np.abs(G) + 1e-10 * np.abs(G).max())
        S.close()


def test_pcg_small_cube_tight(dev):
    _say("pcg cube8 tol 1e-13")
    s = small_cube()
    P = _oracle(s, 16, 2)
    xr, st, it, rr, tr = P.pcg(s.b, tol=1e-13)
    S = _solver(s, 16, 2)
    H = _H(s, dev)
    S.build(H)
    x, res = S.solve(H, _t(s.b, dev), tol=1e-13)
    x = x.cpu().numpy()
    assert res["status"] == 0
    assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)


def test_pcg_edge_cases(dev):
    from paper_2411_06224_amd import MasError

    _say("pcg edge cases")
    s = cube(2)
    S = _solver(s, 4)
    H = _H(s, dev)
    S.build(H)
    # b = 0 -> x = 0 after 0 iterations, also with a nonzero x0
    x, res = S.solve(H, torch.zeros(3 * s.n, dtype=torch.float64, device=dev), x0=_t(np.ones(3 * s.n), dev))
    assert res["status"] == 0 and res["iterations"] == 0 and not x.cpu().numpy().any()
    # max_iter = 1 -> not converged with the first iterate
    x, res = S.solve(H, _t(s.b, dev), tol=1e-12, max_iter=1)
    xr, st, it, *_ = _oracle(s, 4).pcg(s.b, tol=1e-12, max_iter=1)
    assert res["status"] == 1 and res["iterations"] == 1 and st == 1
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-12 * np.linalg.norm(xr)
    # max_iter = 0 -> x = x0 = 0
    x, res = S.solve(H, _t(s.b, dev), max_iter=0)
    assert res["status"] == 1 and res["iterations"] == 0 and not x.cpu().numpy().any()
    # warm start from the converged solution: 0 iterations
    xs, _ = S.solve(H, _t(s.b, dev), tol=1e-10)
    x, res = S.solve(H, _t(s.b, dev), tol=1e-8, x0=xs)
    assert res["status"] == 0 and res["iterations"] == 0
    # indefinite H: a flipped diagonal block fails the domain factorisation
    val = s.val.copy()
    dpos = [p for p in range(s.row_ptr[5], s.row_ptr[6]) if s.col_idx[p] == 5][0]
    val[dpos] = -val[dpos] - np.eye(3)
    Hb = _H(synth.BlockSystem(s.n, s.row_ptr, s.col_idx, val, s.b, s.gptr, s.gadj), dev)
    with pytest.raises(MasError) as e:
        S.build(Hb)
    assert e.value.code == -2


def test_pcg_breakdown_on_indefinite_coupling(dev):
    """p^T H p <= 0 inside PCG (every domain matrix SPD): the solve stops
    with NOT_SPD after 0 iterations and x untouched, as the oracle does; the
    eigenvector right-hand side converges in one iteration to b / 3."""
    from paper_2411_06224_amd import BlockMatrix, MasError, MasPcg

    _say("pcg breakdown on indefinite coupling")
    I3 = np.eye(3)
    row_ptr = np.array([0, 2, 4], dtype=np.int32)
    col_idx = np.array([0, 1, 0, 1], dtype=np.int32)
    val = np.stack([I3, 2 * I3, 2 * I3, I3])
    H = BlockMatrix.from_numpy(row_ptr, col_idx, val, device=dev)
    for every in (50, 1):  # the recurrence iteration and the direct one
        S = MasPcg(row_ptr, col_idx, domain_size=1, poison=True)
        S.build(H)
        b = np.array([1.0, 0, 0, -1.0, 0, 0])
        xr, st, it, *_ = oracle.MAS(row_ptr, col_idx, val, N=1).pcg(b, tol=1e-10)
        assert st == oracle.NOT_SPD and it == 0
        with pytest.raises(MasError) as e:
            S.solve(H, _t(b, dev), tol=1e-10, replace_every=every, allow_not_converged=False)
        assert e.value.code == -2
        x, res = S.solve(H, _t(np.array([1.0, 0, 0, 1.0, 0, 0]), dev), tol=1e-10, replace_every=every)
        assert res["status"] == 0 and res["iterations"] == 1
        assert np.allclose(x.cpu().numpy(), np.array([1.0, 0, 0, 1.0, 0, 0]) / 3.0, rtol=0, atol=1e-15)
        S.close()


def test_pcg_single_domain_one_iteration(dev):
    _say("pcg single domain")
    s = cube(1)
    S = _solver(s, 16)
    H = _H(s, dev)
    S.build(H)
    x, res = S.solve(H, _t(s.b, dev), tol=1e-12)
    assert res["iterations"] == 1 and res["status"] == 0
    xs = np.linalg.solve(s.dense(), s.b)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-12 * np.linalg.norm(xs)


def test_pcg_deterministic(dev):
    _say("pcg bitwise reproducible")
    s = SYSTEMS["contact6"]()
    S = _solver(s, 16)
    H = _H(s, dev)
    S.build(H)
    x1, r1 = S.solve(H, _t(s.b, dev), tol=1e-8)
    S.build(H)
    x2, r2 = S.solve(H, _t(s.b, dev), tol=1e-8)
    assert torch.equal(x1, x2) and r1 == r2


@pytest.mark.parametrize("max_iter", [1, 2, 7, 9, 17])
def test_pcg_stop_at_every_iteration_count(dev, max_iter):
    """Fixed iteration counts around the host check period (8): the iterate
    after exactly max_iter iterations, whatever batch the stop falls in."""
    _say("pcg max_iter", max_iter)
    s = SYSTEMS["contact6"]()
    xr, st, it, *_ = _oracle(s, 16).pcg(s.b, tol=0.0, max_iter=max_iter)
    S = _solver(s, 16)
    H = _H(s, dev)
    S.build(H)
    x, res = S.solve(H, _t(s.b, dev), tol=0.0, max_iter=max_iter)
    assert res["iterations"] == it == max_iter
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.parametrize("case", ["cube", "dense_local"])
def test_pcg_storage_paths(dev, case):
    """Group-symmetric storage of H (cube: each internal block pair kept once)
    and the full storage it falls back to when a group's transposed entries
    exceed the LDS list (dense local couplings): both against the oracle."""
    _say("pcg storage path", case)
    if case == "cube":
        s = SYSTEMS["contact6"]()
    else:
        s = synth.random_spd_system(2000, 90000, seed=6, local=60)
    P = _oracle(s, 16)
    S = _solver(s, 16)
    inf = S.info()
    if case == "cube":
        assert inf["stored_blocks"] < inf["nnzb"]
    else:
        assert inf["stored_blocks"] == inf["nnzb"]
    H = _H(s, dev)
    S.build(H)
    xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
    x, res = S.solve(H, _t(s.b, dev), tol=0.0, max_iter=10)
    assert res["iterations"] == it == 10
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)
    # the final FP64 residual b - H x is computed from the stored H as well
    true = np.linalg.norm(s.b - oracle.spmv(s.row_ptr, s.col_idx, s.val, x.cpu().numpy())) / np.linalg.norm(s.b)
    assert abs(res["true_rel_residual"] - true) <= 1e-12 * max(true, 1e-300) + 1e-15


def test_pcg_morton_partition(dev):
    """Level-0 domains in Morton order of the node positions (the earlier MAS
    ordering, Sec. 4.1) through mas_analyze_partition, against the oracle
    built from the same partition; iteration counts of both orderings are
    printed (the ablation of Sec. 4.1)."""
    from paper_2411_06224_amd import MasPcg, morton_partition

    _say("pcg morton partition")
    s = SYSTEMS["contact6"]()
    part = morton_partition(s.meta["positions"], 16)
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, part=part, M=int(part.max()) + 1)
    S = MasPcg(s.row_ptr, s.col_idx, domain_size=16, partition=part, poison=True)
    H = _H(s, dev)
    S.build(H)
    xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
    x, res = S.solve(H, _t(s.b, dev), tol=0.0, max_iter=10)
    assert res["iterations"] == it == 10
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)
    _, res_m = S.solve(H, _t(s.b, dev), tol=1e-6)
    C = _solver(s, 16)
    C.build(H)
    _, res_c = C.solve(H, _t(s.b, dev), tol=1e-6)
    print(f"iterations to 1e-6: connectivity ordering {res_c['iterations']}, Morton ordering {res_m['iterations']}")
    assert res_m["status"] == 0 and res_c["status"] == 0


def test_pcg_long_range_couplings(dev):
    """Random long-range couplings: every group touches thousands of columns
    and the hierarchy runs to the level cap."""
    _say("pcg wide random")
    s = synth.random_spd_system(4000, 60000, seed=4)
    P = _oracle(s, 16)
    S = _solver(s, 16)
    H = _H(s, dev)
    S.build(H)
    xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
    x, res = S.solve(H, _t(s.b, dev), tol=0.0, max_iter=10)
    assert res["iterations"] == it == 10 and res["status"] == 1
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)
    xr, st, it, *_ = P.pcg(s.b, tol=1e-8)
    x, res = S.solve(H, _t(s.b, dev), tol=1e-8)
    lo, hi, xt, _ = _count_contract(s, 1e-8)
    assert res["status"] == 0 and st == 0 and lo <= res["iterations"] <= hi
    xv = x.cpu().numpy()
    assert np.linalg.norm(xv - xr) <= xt * np.linalg.norm(xr)
    assert np.linalg.norm(s.b - oracle.spmv(s.row_ptr, s.col_idx, s.val, xv)) <= 1.01e-8 * np.linalg.norm(s.b)


# ----------------------------------------------------------------- mixed ---


@pytest.mark.parametrize("tol,replace_every", [(1e-4, 50), (1e-6, 50), (1e-6, 3), (1e-8, 7)])
def test_mixed_precision_small(dev, tol, replace_every):
    _say("mixed", tol, replace_every)
    s = small_cube()
    xr, *_ = _oracle(s, 16).pcg(s.b, tol=1e-12)
    S = _solver(s, 16, precision="mixed")
    H = _H(s, dev)
    S.build(H)
    x, res = S.solve(H, _t(s.b, dev), tol=tol, replace_every=replace_every)
    assert res["status"] == 0
    xv = x.cpu().numpy()
    true = np.linalg.norm(s.b - oracle.spmv(s.row_ptr, s.col_idx, s.val, xv)) / np.linalg.norm(s.b)
    assert true <= tol
    print(f"mixed tol={tol}: its={res['iterations']} true_res={true:.3e} err_vs_fp64={np.linalg.norm(xv - xr) / np.linalg.norm(xr):.3e}")


# ------------------------------------------------------------- gradients ---


def test_adjoint_dense_gradient_small_cube(dev):
    from paper_2411_06224_amd import mas_pcg_solve

    _say("adjoint dense gradient cube8")
    s = small_cube()
    A = s.dense()
    xt = np.random.default_rng(5).standard_normal(3 * s.n)
    S = _solver(s, 16)
    H = _H(s, dev)
    val = H.val.clone().requires_grad_(True)
    b = _t(s.b, dev).requires_grad_(True)
    from paper_2411_06224_amd import BlockMatrix

    Hg = BlockMatrix(H.row_ptr, H.col_idx, val)
    x = mas_pcg_solve(S, Hg, b, tol=1e-12)
    loss = 0.5 * ((x - _t(xt, dev)) ** 2).sum()
    loss.backward()
    xs = np.linalg.solve(A, s.b)
    lam = np.linalg.solve(A, xs - xt)
    gb = b.grad.cpu().numpy()
    assert np.linalg.norm(gb - lam) <= 1e-8 * np.linalg.norm(lam)
    G = val.grad.cpu().numpy()
    Gr = oracle.adjoint_scatter(s.row_ptr, s.col_idx, lam, xs)
    assert np.linalg.norm(G - Gr) <= 1e-8 * np.linalg.norm(Gr)


def test_autograd_raises_when_a_solve_does_not_converge(dev):
    """The differentiable solve refuses a forward (or adjoint) solve that stops
    at max_iter: its x, dL/db and dL/dH would not be the gradient."""
    from paper_2411_06224_amd import BlockMatrix, MasError, mas_pcg_solve

    _say("autograd max_iter too low")
    s = small_cube()
    S = _solver(s, 16, 2)
    H = _H(s, dev)
    val = H.val.clone().requires_grad_(True)
    b = _t(s.b, dev).requires_grad_(True)
    with pytest.raises(MasError):
        mas_pcg_solve(S, BlockMatrix(H.row_ptr, H.col_idx, val), b, tol=1e-12, max_iter=3)
    # forward converges, adjoint may not: it raises as well
    x = mas_pcg_solve(S, BlockMatrix(H.row_ptr, H.col_idx, val), b, tol=1e-8, max_iter=10000)
    S2 = _solver(s, 16, 2)
    S2.build(H)
    with pytest.raises(MasError):
        S2.adjoint(H, x.detach(), x.detach().clone(), tol=1e-12, max_iter=3, allow_not_converged=False)
    loss = 0.5 * (x ** 2).sum()
    loss.backward()  # the adjoint converges at the forward's max_iter
    assert torch.isfinite(b.grad).all()


def test_adjoint_matches_oracle_scatter_f32(dev):
    _say("adjoint scatter f32")
    s = SYSTEMS["contact6"]()
    S = _solver(s, 16)
    H = _H(s, dev)
    S.build(H)
    x, _ = S.solve(H, _t(s.b, dev), tol=1e-12)
    g = np.random.default_rng(2).standard_normal(3 * s.n)
    lam, dH, res = S.adjoint(H, x, _t(g, dev), dLdH_dtype=torch.float32, tol=1e-12)
    lr, *_ = _oracle(s, 16).pcg(g, tol=1e-12)
    assert np.linalg.norm(lam.cpu().numpy() - lr) <= 1e-9 * np.linalg.norm(lr)
    Gr = oracle.adjoint_scatter(s.row_ptr, s.col_idx, lam.cpu().numpy(), x.cpu().numpy())
    assert np.allclose(dH.cpu().numpy(), Gr, rtol=1e-6, atol=1e-6 * np.abs(Gr).max())


# --------------------------------------------------------- full-size case ---


@pytest.mark.slow
def test_large_cube_parity(dev):
    from paper_2411_06224_amd import bcsr_spmv

    _say("large cube 48^3 parity")
    s = large_cube()
    H = _H(s, dev)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(3 * s.n)
    y = bcsr_spmv(H, _t(x, dev)).cpu().numpy()
    ref = oracle.spmv(s.row_ptr, s.col_idx, s.val, x)
    assert np.all(np.abs(y - ref) <= 1e-14 * _absH_absx(s, x) + 1e-300)
    P = _oracle(s, 16)
    S = _solver(s, 16)
    S.build(H)
    r = rng.standard_normal(3 * s.n)
    z = S.apply(_t(r, dev)).cpu().numpy()
    zr = P.apply(r)
    assert np.linalg.norm(z - zr) <= 1e-10 * np.linalg.norm(zr)
    xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
    xg, res = S.solve(H, _t(s.b, dev), tol=0.0, max_iter=10)
    assert np.linalg.norm(xg.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)
