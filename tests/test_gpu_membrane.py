"""Parity on the stiff membrane + affine-body system (triangle sheet with
the cubic strain-limiting Hessians and bending, affine bodies of four block
rows coupled to random sheet nodes): FP64 and mixed precision against the
oracle, on small sheets and at full size (512^2 cells, 2,000 bodies,
271,169 block rows, 3.70 M blocks)."""

import functools
import sys
import time

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


@functools.lru_cache(maxsize=None)
def _system(cells, bodies, seed):
    return synth.membrane_system(cells, bodies, seed=seed)


@functools.lru_cache(maxsize=None)
def _oracle(cells, bodies, seed):
    s = _system(cells, bodies, seed)
    return oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, gptr=s.gptr, gadj=s.gadj)


def _solver(s, precision="f64"):
    from paper_2411_06224_amd import MasPcg

    return MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=16, precision=precision, poison=True)


def _H(s, dev):
    from paper_2411_06224_amd import BlockMatrix

    return BlockMatrix.from_numpy(s.row_ptr, s.col_idx, s.val, device=dev)


def _t(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)


def _true_rel(s, x):
    return np.linalg.norm(s.b - oracle.spmv(s.row_ptr, s.col_idx, s.val, x)) / np.linalg.norm(s.b)


def _count_range(P, b, tol, n=6):
    """Oracle iteration counts for b and b perturbed at the rounding level
    (relative 1e-15), widened by 2: the arithmetic fixes PCG's count only up
    to this spread."""
    rng = np.random.default_rng(321)
    its = [P.pcg(b, tol=tol)[2]]
    for _ in range(n - 1):
        its.append(P.pcg(b * (1.0 + 1e-15 * rng.standard_normal(b.shape)), tol=tol)[2])
    return min(its) - 2, max(its) + 2


SMALL = [(24, 12, 7), (64, 60, 8)]


@pytest.mark.parametrize("case", SMALL)
def test_membrane_apply_and_fixed_iterations(dev, case):
    _say("membrane fixed iterations", case)
    s, P = _system(*case), _oracle(*case)
    S = _solver(s)
    H = _H(s, dev)
    S.build(H)
    r = np.random.default_rng(5).standard_normal(3 * s.n)
    z = S.apply(_t(r, dev)).cpu().numpy()
    zr = P.apply(r)
    assert np.linalg.norm(z - zr) <= 1e-10 * np.linalg.norm(zr)
    xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
    x, res = S.solve(H, _t(s.b, dev), tol=0.0, max_iter=10)
    assert res["iterations"] == it == 10
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.parametrize("case", SMALL)
@pytest.mark.parametrize("tol", [1e-4, 1e-8])
def test_membrane_converged_f64(dev, case, tol):
    _say("membrane f64", case, tol)
    s, P = _system(*case), _oracle(*case)
    S = _solver(s)
    H = _H(s, dev)
    S.build(H)
    x, res = S.solve(H, _t(s.b, dev), tol=tol)
    lo, hi = _count_range(P, s.b, tol)
    assert res["status"] == 0 and lo <= res["iterations"] <= hi, (res, lo, hi)
    assert _true_rel(s, x.cpu().numpy()) <= 1.01 * tol


@pytest.mark.parametrize("case", SMALL)
@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_membrane_mixed(dev, case, tol):
    """FP32 values and inverses, FP64 dots and x / r with residual
    replacement: converged on the FP64 residual; the error against the
    oracle's FP64 solution is printed."""
    _say("membrane mixed", case, tol)
    s, P = _system(*case), _oracle(*case)
    S = _solver(s, "mixed")
    H = _H(s, dev)
    S.build(H)
    x, res = S.solve(H, _t(s.b, dev), tol=tol)
    xv = x.cpu().numpy()
    true = _true_rel(s, xv)
    xr = P.pcg(s.b, tol=1e-12, max_iter=100000)[0]
    err = np.linalg.norm(xv - xr) / np.linalg.norm(xr)
    print(f"mixed {case} tol {tol}: {res['iterations']} its, true residual {true:.3e}, error vs oracle {err:.3e}")
    assert res["status"] == 0 and true <= 1.01 * tol


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_membrane_full_size(dev):
    """512^2 cells + 2,000 bodies: the hierarchy equals the oracle's, ten
    fixed FP64 iterations match it, and the FP64 and mixed solves to 1e-4
    reach the tolerance on the true residual (checked with the oracle's
    SpMV)."""
    _say("membrane full size")
    t0 = time.time()
    s = synth.config_membrane()
    print(f"generated in {time.time() - t0:.1f} s: {s.n} block rows, {s.nnzb} blocks", flush=True)
    P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=16, gptr=s.gptr, gadj=s.gadj)
    S = _solver(s)
    inf = S.info()
    assert inf["levels"] == P.levels
    for l in range(P.levels):
        assert inf["units"][l] == P.units(l)
    H = _H(s, dev)
    S.build(H)
    xr, st, it, *_ = P.pcg(s.b, tol=0.0, max_iter=10)
    x, res = S.solve(H, _t(s.b, dev), tol=0.0, max_iter=10)
    assert res["iterations"] == it == 10
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-10 * np.linalg.norm(xr)
    b = _t(s.b, dev)
    for prec in ("f64", "mixed"):
        Sp = S if prec == "f64" else _solver(s, "mixed")
        Sp.build(H)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, res = Sp.solve(H, b, tol=1e-4)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        true = _true_rel(s, x.cpu().numpy())
        print(f"{prec}: {res['iterations']} its, {ms:.1f} ms, true residual {true:.3e}, levels {inf['levels']}")
        assert res["status"] == 0 and true <= 1.01e-4
