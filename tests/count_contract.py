"""Iteration-count contract of a converged PCG solve (GPU against oracle).

PCG (Sec. 3.2) with the MAS operator (Supp. Eq. 4-6) fixes what is computed,
not the order of the sums nor the inversion method.  Over hundreds of
iterations CG in finite precision turns rounding-level differences between
two correct FP64 evaluations of the same definition into a spread of the
iteration count at which ||r|| first drops below tol ||b||.  The oracle
measures that spread itself, with changes that leave the definition intact:

  * dot products summed in ascending order (its default) or compensated
    (Dot2, as accurate as twice the working precision); any other order,
    e.g. per-group partials added in a fixed tree, lies between the two;
  * every inverse entry scaled by (1 + eps u), u uniform in [-1, 1), for eps
    from 1e-14 (about 100 u) to 1e-10 (kappa u of the worst domain matrices
    of the full-size system), several seeds;
  * for small systems also b perturbed by 1e-15 relative.

Reading of "iteration counts within +-2": the GPU count lies within 2 of the
range the oracle spans under these changes.  The solution is compared with
the oracle's own within twice the largest difference between the oracle's
solution and those of the perturbed runs (floor 1e-12 relative), since a
count one higher or lower moves x by about the last step.
"""

import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = (1e-14, 1e-12, 1e-10)


def oracle_ensemble(make_P, b, tol, seeds=(1, 2), n_rhs=3):
    """(lo, hi, x_tol, x_ref, its): the contract for a small system.
    make_P() returns a fresh oracle.MAS (perturb() changes it in place)."""
    P = make_P()
    x0, st, it0, *_ = P.pcg(b, tol=tol)
    nx = np.linalg.norm(x0)
    its, dx = [it0], []

    def add(x, it):
        its.append(it)
        dx.append(np.linalg.norm(x - x0) / nx if nx > 0 else 0.0)

    x, _, it, *_ = P.pcg(b, tol=tol, dots=oracle.DOT_COMPENSATED)
    add(x, it)
    rng = np.random.default_rng(123)
    for _ in range(n_rhs):
        x, _, it, *_ = P.pcg(b * (1.0 + 1e-15 * rng.standard_normal(b.shape)), tol=tol)
        add(x, it)
    for eps in EPS:
        for sd in seeds:
            Q = make_P()
            Q.perturb(eps, sd)
            for dots in (oracle.DOT_SEQUENTIAL, oracle.DOT_COMPENSATED):
                x, _, it, *_ = Q.pcg(b, tol=tol, dots=dots)
                add(x, it)
    return min(its) - 2, max(its) + 2, max(2.0 * max(dx), 1e-12), x0, its


def golden_cube48(E, tol):
    """(lo, hi, x_tol, oracle_iterations) for the 48^3 benchmark system from
    tests/golden/count_ensemble_cube48.json (written by the oracle only)."""
    with open(os.path.join(HERE, "golden", "count_ensemble_cube48.json")) as fh:
        d = json.load(fh)
    for c in d["cases"]:
        if c["E"] == E and c["tol"] == tol:
            return c["ensemble_min"] - 2, c["ensemble_max"] + 2, max(2.0 * c["x_rel_diff_max"], 1e-12), c["oracle_iterations"]
    raise KeyError((E, tol))
