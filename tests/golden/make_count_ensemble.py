"""Writes count_ensemble_cube48.json: how far the PCG iteration count and the
solution of the 48^3 benchmark system move when the MAS preconditioner is
changed at the rounding level.  Calls only the oracle (and the seeded input
generator).

Why this is needed.  Two correct FP64 implementations of the same MAS-PCG
(same partition, same hierarchy, same definition of every domain matrix,
Supp. Eq. 5, and of the operator, Supp. Eq. 6) differ in summation order
(coarse matrices level by level or straight from H, restriction through
per-group partials, SpMV and dot products in another order) and in the
inversion method (Cholesky against Gauss-Jordan: both give the inverse up
to about kappa * u).  CG in finite precision is sensitive to such
differences over hundreds of iterations, so the iteration count at which the
relative residual first drops below the tolerance is defined only up to a
spread.  The oracle's own count is one sample of that spread.  This script
measures it with the oracle alone, over two kinds of change that leave the
definition untouched:
  * how the dot products are summed: plainly in ascending order (the
    oracle's default) or compensated (Dot2 of Ogita, Rump and Oishi, as
    accurate as twice the working precision).  Any other order, e.g. the
    GPU's per-group partials added in a fixed tree, lies between the two in
    accuracy.  At 48^3 this alone moves the count by about 3;
  * the preconditioner at the rounding level: every inverse entry scaled by
    (1 + eps u), u uniform in [-1, 1) (symmetric, so the operator stays SPD),
    for eps from 1e-14 (about 100 u) to 1e-10 (kappa * u for the worst
    domain matrices at this size), with several seeds.

Usage: python tests/golden/make_count_ensemble.py [--jobs 6]
"""

import argparse
import json
import os
import sys
import tempfile
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "count_ensemble_cube48.json")
EPS = (1e-14, 1e-12, 1e-10)
SEEDS = (1, 2, 3, 4)
CASES = ((1e6, 1e-4), (1e6, 1e-8), (1e4, 1e-4), (1e8, 1e-4))


def _run(args):
    path, tol, dots, eps, seed = args
    import oracle

    z = np.load(path)
    P = oracle.MAS(z["rp"], z["ci"], z["val"], N=16, gptr=z["gptr"], gadj=z["gadj"])
    if eps > 0:
        P.perturb(eps, seed)
    x, st, it, rr, tr = P.pcg(z["b"], tol=tol, dots=dots)
    return {"dots": dots, "eps": eps, "seed": seed, "status": st, "iterations": it, "true_rel_residual": tr, "x": x}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    args = ap.parse_args()
    import synth

    out = {
        "citation": "PCG as stated in Sec. 3.2 (P d = -grad E solved by PCG to a relative tolerance, Sec. 7 setup: "
        "1e-4); MAS operator of Supp. Eq. 4-6 with domain matrices of Supp. Eq. 5 and their inverses "
        "(algorithm 'Compute MAS preconditioner', Sec. 4.3).  Values written by this script from the oracle only.",
        "workload": "48^3 tet cube, nu = 0.49, 20,000 contact couplings, seed 1001, N = 16, full hierarchy",
        "perturbation": "every inverse entry (p <= q, mirrored) scaled by 1 + eps*u, u ~ U[-1,1) (SplitMix64)",
        "dots": "0: sequential (the oracle's default), 1: compensated (Dot2)",
        "eps": list(EPS),
        "seeds": list(SEEDS),
        "cases": [],
    }
    with tempfile.TemporaryDirectory() as tmp:
        for E, tol in CASES:
            path = os.path.join(tmp, f"cube48_E{E:g}.npz")
            if not os.path.exists(path):
                s = synth.config_large(E=E)
                np.savez(path, rp=s.row_ptr, ci=s.col_idx, val=s.val, b=s.b, gptr=s.gptr, gadj=s.gadj)
            jobs = [(path, tol, 0, 0.0, 0)] + [(path, tol, dm, e, sd) for dm in (0, 1)
                                                for e in (0.0,) + EPS for sd in (SEEDS if e > 0 else (0,))
                                                if (dm, e) != (0, 0.0)]
            with ProcessPoolExecutor(max_workers=args.jobs) as ex:
                res = list(ex.map(_run, jobs))
            x0 = res[0]["x"]
            nx0 = float(np.linalg.norm(x0))
            samples = []
            for r in res[1:]:
                assert r["status"] == 0, r["status"]
                samples.append({
                    "dots": r["dots"],
                    "eps": r["eps"],
                    "seed": r["seed"],
                    "iterations": r["iterations"],
                    "true_rel_residual": r["true_rel_residual"],
                    "x_rel_diff": float(np.linalg.norm(r["x"] - x0) / nx0),
                })
            its = [res[0]["iterations"]] + [s_["iterations"] for s_ in samples]
            case = {
                "E": E,
                "tol": tol,
                "oracle_iterations": res[0]["iterations"],
                "oracle_true_rel_residual": res[0]["true_rel_residual"],
                "ensemble_min": int(min(its)),
                "ensemble_max": int(max(its)),
                "x_rel_diff_max": float(max(s_["x_rel_diff"] for s_ in samples)),
                "samples": samples,
            }
            out["cases"].append(case)
            print(f"E={E:g} tol={tol:g}: oracle {case['oracle_iterations']}, ensemble "
                  f"[{case['ensemble_min']}, {case['ensemble_max']}], x diff max {case['x_rel_diff_max']:.2e}",
                  flush=True)
            with open(OUT, "w") as fh:
                json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
