"""Benchmark: MAS-PCG ms per Newton solve to 1e-4 relative residual on the
48^3 tet cube (117,649 nodes, 352,947 DOF, 552,960 tets, 20,000 contact-like
couplings, E = 1e6 Pa, nu = 0.49), one MI355X.

A step is one full linear solve of the Newton system: the numeric MAS build
(coarse sums + batched domain inversion) followed by PCG to ||r|| <= 1e-4 ||b||
in FP64, inputs resident in HBM.  The symbolic analysis (partition, hierarchy,
plans) runs once per sparsity pattern before the timed region, as the paper's
METIS reordering runs once at load.

Printed: one JSON line with the headline value plus the mixed-precision and
forward+adjoint measurements, the roofline of the dominant kernel (per-launch
HIP-event timing of one extra instrumented solve) and the CPU oracle baseline.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 256 << 20  # calibration copy: bytes read (and written) per copy

# Sources that define each hot kernel; HBM traffic measured with rocprofv3
# counters (profiles/pmc_traffic.json) is used only while they are unchanged.
KERNEL_SOURCES = {
    "spmv": ["spmv.hip", "common.hpp", "launch.hpp", "restrict.hpp"],
    "apply_level0": ["mas.hip", "common.hpp", "launch.hpp"],
    "level0_update": ["mas.hip", "common.hpp", "launch.hpp"],
}


def kernel_source_hash(kernel):
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(ROOT, "paper_2411_06224_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch (fetch + write) from the committed counter runs,
    or None when there is none for this kernel or its sources changed since."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(kernel)
    if not rec or rec.get("source_sha256") != kernel_source_hash(kernel):
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(info, mixed):
    """Bytes each hot kernel must move once per launch (no re-reads)."""
    V, N, L = info["n_rows"], info["domain_size"], info["levels"]
    nnzb = info["nnzb"]
    nsb = info["stored_blocks"]
    NS = info["parts"] * N
    n = 3 * N
    vb = 8 * 3 * NS  # one slot-ordered FP64 vector
    val = 36 if mixed else 72
    inv = 4 if mixed else 8
    coarse_y = sum(8 * 3 * info["domains"][l] * N for l in range(1, L))
    # level-0 inverses: FP64 symmetric-packed for N = 16 (n (n + 1) / 2 entries), else full
    inv0 = info["domains"][0] * (n * (n + 1) // 2 if (N == 16 and not mixed) else n * n) * inv
    r1b = 8 * 3 * info["units"][1] if L > 1 else 0  # one level-1 vector
    if mixed:  # the FP32 copy keeps every block: values, column index, row pointers
        stored = nnzb * (val + 4) + 4 * (NS + 1)
    else:  # symmetric FP64 storage: values, column index and local row of each stored block,
        # row pointers and transposed-entry lists
        stored = nsb * (val + 4 + 1) + 8 * (NS + 1) + 4 * (nnzb - nsb)
    out = {
        # the stored matrix; z and the previous direction read once (the
        # direction update is fused in), new direction and q written; the
        # restriction of q: per-slot plan (16 B) read, q_1 written
        "spmv": stored + 4 * vb + 16 * NS + r1b,
        # level-0 inverses, r read, z written, per-slot coarse ids, coarse corrections
        "apply_level0": inv0 + 2 * vb + 4 * (L - 1) * NS + coarse_y,
        # coarse inverses, restricted residual read (and, by recurrence, q_1
        # read and r_1 written), y written
        "apply_coarse": sum(info["domains"][l] * n * n * inv for l in range(1, L)) + 3 * r1b + coarse_y,
        # x, r read+write, p, q read, per-slot plan ints, r_1 written
        "update": 6 * vb + 8 * NS + (8 * 3 * info["units"][1] if L > 1 else 0),
    }
    # level-0 apply fused with the x/r update: also x read and written, r
    # written, p and q read
    out["level0_update"] = out["apply_level0"] + 5 * vb
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--E", type=float, default=1e6)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--domain-size", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip mixed / adjoint / instrumented runs")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (8^3 cube, E / tol sweep, mixed, membrane, adjoint at E = 1e7)")
    ap.add_argument(
        "--calibrate-copy",
        action="store_true",
        help="first copy a 256 MiB buffer three times (a plain copy of known size for counter calibration)",
    )
    args = ap.parse_args()

    if args.gpus != 1:
        print(
            "bench.py runs on one GPU only: this build has no multi-GPU path "
            f"(asked for --gpus {args.gpus}); run with --gpus 1.",
            file=sys.stderr,
        )
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2411_06224_amd as mp

    mp.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    t0 = time.time()
    s = synth.config_large(E=args.E, keep_blocks=not args.no_extras)
    log(f"workload generated in {time.time() - t0:.1f}s: {s.n} nodes, {s.nnzb} blocks")
    H = mp.BlockMatrix.from_numpy(s.row_ptr, s.col_idx, s.val, device=dev)
    b = torch.as_tensor(s.b, device=dev)

    t0 = time.time()
    solver = mp.MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=args.domain_size)
    t_symbolic = time.time() - t0
    info = solver.info()
    log(f"symbolic analysis {t_symbolic * 1e3:.0f} ms: levels {info['levels']} units {info['units']}")

    x = torch.empty_like(b)

    def step(sv, prec_tol):
        sv.build(H)
        return sv.solve(H, b, tol=prec_tol, out=x)

    res = None
    for _ in range(args.warmup):
        _, res = step(solver, args.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, step_ms = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, res = step(solver, args.tol)  # the solve returns once the device is done
        step_ms.append(1e3 * (time.perf_counter() - ts))
        iters.append(res["iterations"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    if res["status"] != 0:
        raise SystemExit(f"solve did not converge: {res}")
    log(f"FP64 solve: {ms_per_step:.3f} ms/step, {iters[-1]} iterations, true rel res {res['true_rel_residual']:.3e}")
    ph = solver.timings()

    out = {
        "metric": "MAS-PCG ms to 1e-4 rel. residual at 118k nodes; fwd+adjoint vs plain FP64",
        "value": round(ms_per_step, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"tet cube 48^3 (117,649 nodes, 352,947 DOF, 552,960 tets) + 20,000 contact couplings, "
            f"E={args.E:g} Pa, nu=0.49; full MAS hierarchy N={args.domain_size}; PCG to {args.tol:g}",
            "nodes": s.n,
            "dof": 3 * s.n,
            "nnzb": s.nnzb,
            "tol": args.tol,
            "domain_size": args.domain_size,
            "levels": info["levels"],
            "supernodes": info["units"][1:],
            "parallelism": "single GPU",
        },
        "median_ms_per_step": round(float(np.median(step_ms)), 4),
        "iterations": iters[-1],
        "true_rel_residual": res["true_rel_residual"],
        "phase_ms": {
            "coarse_sums": round(ph[0], 4),
            "inversion": round(ph[1], 4),
            "permute_H": round(ph[2], 4),
            "pcg": round(ph[3], 4),
        },
        "symbolic_ms": round(t_symbolic * 1e3, 1),
    }

    if not args.no_extras:
        # roofline: one instrumented solve, every launch bracketed by HIP events
        solver.set_kernel_timing(True)
        step(solver, args.tol)
        kt = solver.kernel_timing()
        solver.set_kernel_timing(False)
        nbytes = algorithmic_bytes(info, mixed=False)
        per = {}
        for k, nb in nbytes.items():
            tot, cnt = kt[k]
            if cnt:
                avg = tot / cnt
                per[k] = {
                    "avg_us": round(avg * 1e3, 3),
                    "launches": cnt,
                    "alg_bytes": nb,
                    "GBs": round(nb / (avg * 1e-3) / 1e9, 1),
                }
        dom = max(per, key=lambda k: per[k]["avg_us"] * per[k]["launches"])
        ach = per[dom]["GBs"]
        out["roofline"] = {
            "kernel": dom,
            "bound": "hbm",
            "achieved": ach,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom),
            "alg_bytes_per_launch": nbytes[dom],
            "avg_launch_us": per[dom]["avg_us"],
            "launches_averaged": per[dom]["launches"],
        }
        if dom == "spmv":
            # the same launches priced at the bytes of plain full 3x3-block CSR
            # (every block's values, column index, row pointers, x read, y written)
            full = s.nnzb * (72 + 4) + 4 * (s.n + 1) + 2 * 8 * 3 * s.n
            out["roofline"]["frac_on_full_bcsr_bytes"] = round(full / (per[dom]["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
            out["roofline"]["full_bcsr_bytes"] = full
        out["kernels"] = per
        log("kernels:", json.dumps(per))
        # the paper's breakdown of a solve (Table 1 columns): preconditioner
        # construction (coarse sums + inversion), preconditioner application
        # (MAS apply kernels) and the rest of the CG iteration (SpMV, x/r
        # update), from the instrumented solve's per-kernel totals
        tot = {k: kt[k][0] for k in kt}
        out["paper_breakdown_ms"] = {
            "PPC": round(ph[0] + ph[1], 4),
            "PPR": round(tot.get("apply_coarse", 0.0) + tot.get("apply_level0", 0.0) + tot.get("level0_update", 0.0), 4),
            "CGR": round(tot.get("spmv", 0.0) + tot.get("update", 0.0) + tot.get("residual", 0.0), 4),
            "note": "the level-0 apply fused with the x/r update counts as PPR",
        }

        # achievable HBM bandwidth for context: a triad a = b + s c over three
        # 1 GiB arrays (far beyond the 256 MB last-level cache), torch's own
        # elementwise kernel, timed with events on the current stream
        nt = (1 << 30) // 8
        ta, tb, tc = (torch.empty(nt, dtype=torch.float64, device=dev) for _ in range(3))
        tb.fill_(1.0)
        tc.fill_(2.0)
        torch.add(tb, tc, alpha=0.5, out=ta)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            torch.add(tb, tc, alpha=0.5, out=ta)
        e1.record()
        torch.cuda.synchronize()
        triad = 3 * nt * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del ta, tb, tc
        out["roofline"]["achievable_triad_GBs"] = round(triad, 1)
        out["roofline"]["frac_of_triad"] = round(ach / triad, 4)
        log(f"triad: {triad:.0f} GB/s")
        # the same triad on three 48 MiB arrays (144 MiB, within the 256 MB
        # last-level cache, about the size of the solver's working set),
        # repeated so that the arrays stay cache-resident
        nm = (48 << 20) // 8
        ta, tb, tc = (torch.empty(nm, dtype=torch.float64, device=dev) for _ in range(3))
        tb.fill_(1.0)
        tc.fill_(2.0)
        for _ in range(5):
            torch.add(tb, tc, alpha=0.5, out=ta)
        e0.record()
        for _ in range(100):
            torch.add(tb, tc, alpha=0.5, out=ta)
        e1.record()
        torch.cuda.synchronize()
        triad_c = 3 * nm * 8 * 100 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del ta, tb, tc
        out["roofline"]["triad_144MiB_GBs"] = round(triad_c, 1)
        log(f"triad on 144 MiB: {triad_c:.0f} GB/s")

        # batched domain inversion: about (3N)^3 flops per domain (FP64, MFMA)
        n3 = (3 * info["domain_size"]) ** 3
        inv_flop = sum(info["domains"][l] for l in range(info["levels"])) * n3
        out["inversion"] = {
            "ms": round(ph[1], 4),
            "gflop": round(inv_flop / 1e9, 3),
            "TFLOPs": round(inv_flop / (ph[1] * 1e-3) / 1e12, 2) if ph[1] > 0 else None,
            "frac_of_fp64_mfma_peak": round(inv_flop / (ph[1] * 1e-3) / 78.6e12, 4) if ph[1] > 0 else None,
        }

        # mixed precision on the same system
        msolver = mp.MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=args.domain_size, precision="mixed")
        for _ in range(max(args.warmup, 1)):
            step(msolver, args.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, mres = step(msolver, args.tol)
        torch.cuda.synchronize()
        ms_mixed = 1e3 * (time.perf_counter() - t0) / args.steps
        out["mixed"] = {
            "ms_per_solve": round(ms_mixed, 4),
            "iterations": mres["iterations"],
            "true_rel_residual": mres["true_rel_residual"],
            "speedup_vs_f64": round(ms_per_step / ms_mixed, 3),
        }
        x_mixed = x.cpu().numpy()
        log(f"mixed solve: {ms_mixed:.3f} ms, {mres['iterations']} its, true res {mres['true_rel_residual']:.3e}")
        # per-kernel times of the mixed solve against the FP64 ones
        msolver.set_kernel_timing(True)
        step(msolver, args.tol)
        mkt = msolver.kernel_timing()
        msolver.set_kernel_timing(False)
        mbytes = algorithmic_bytes(msolver.info(), mixed=True)
        mper = {}
        for k, nb in mbytes.items():
            tot, cnt = mkt[k]
            if cnt:
                avg = tot / cnt
                mper[k] = {"avg_us": round(avg * 1e3, 3), "launches": cnt, "alg_bytes": nb,
                           "GBs": round(nb / (avg * 1e-3) / 1e9, 1)}
        out["mixed"]["kernels"] = mper
        log("mixed kernels:", json.dumps(mper))
        msolver.close()

        # assembly of the system from its unassembled block list (element,
        # mass and contact blocks), the step before the solve (Sec. 6.2)
        rows_np, cols_np, blocks_np = s.meta["blocks"]
        arows = torch.as_tensor(rows_np, device=dev)
        acols = torch.as_tensor(cols_np, device=dev)
        ablocks = torch.as_tensor(blocks_np.reshape(-1, 3, 3), device=dev)
        Ha = mp.bcsr_assemble(s.n, arows, acols, ablocks)
        same = bool(torch.equal(Ha.col_idx.cpu(), torch.as_tensor(s.col_idx.astype(np.int32))))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Ha = mp.bcsr_assemble(s.n, arows, acols, ablocks, capacity=s.nnzb)
        torch.cuda.synchronize()
        ms_asm = 1e3 * (time.perf_counter() - t0) / args.steps
        m_in = int(rows_np.size)
        asm_bytes = m_in * (72 + 8) + s.nnzb * (72 + 4) + 4 * (s.n + 1)
        out["assembly"] = {
            "ms": round(ms_asm, 4),
            "blocks_in": m_in,
            "blocks_out": int(Ha.nnzb),
            "pattern_matches_generator": same,
            "alg_bytes": asm_bytes,
            "GBs": round(asm_bytes / (ms_asm * 1e-3) / 1e9, 1),
        }
        log(f"assembly: {m_in} blocks -> {Ha.nnzb} in {ms_asm:.3f} ms")
        del arows, acols, ablocks, Ha

        # ordering ablation (Sec. 4.1): level-0 domains of consecutive nodes in
        # Morton order of the positions instead of the connectivity-aware
        # partition; same hierarchy construction, same solver
        t0 = time.perf_counter()
        osolver = mp.MasPcg(s.row_ptr, s.col_idx, domain_size=args.domain_size,
                            partition=mp.morton_partition(s.meta["positions"], args.domain_size))
        t_sym_m = time.perf_counter() - t0
        step(osolver, args.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, ores = step(osolver, args.tol)
        torch.cuda.synchronize()
        ms_morton = 1e3 * (time.perf_counter() - t0) / args.steps
        oinf = osolver.info()
        out["ordering_ablation"] = {
            "connectivity": {"iterations": res["iterations"], "ms_per_solve": round(ms_per_step, 4),
                             "levels": info["levels"]},
            "morton": {"iterations": ores["iterations"], "ms_per_solve": round(ms_morton, 4),
                       "levels": oinf["levels"], "symbolic_ms": round(1e3 * t_sym_m, 1)},
        }
        log(f"Morton ordering: {ores['iterations']} its, {ms_morton:.3f} ms, {oinf['levels']} levels")
        osolver.close()

        # hierarchy depth ablation: the additive sum over levels (Supp. Eq. 6)
        # with the level cap at 1 (block Jacobi over the level-0 domains) and
        # 2, against the full hierarchy of the headline solve
        depth = {}
        for ml in (1, 2):
            dsolver = mp.MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=args.domain_size,
                                max_levels=ml)
            step(dsolver, args.tol)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, dres = step(dsolver, args.tol)
            torch.cuda.synchronize()
            depth[f"max_levels_{ml}"] = {"iterations": dres["iterations"],
                                         "ms_per_solve": round(1e3 * (time.perf_counter() - t0) / args.steps, 4)}
            dsolver.close()
        depth[f"full_{info['levels']}_levels"] = {"iterations": res["iterations"], "ms_per_solve": round(ms_per_step, 4)}
        out["depth_ablation"] = depth
        log("depth ablation:", json.dumps(depth))

        # supernode hierarchy rebuilt on the device from the device pattern
        # under the analysed partition (Sec. 4.1-4.2): the step repeated when
        # contacts change the pattern; no host round trip inside
        units_h, _ = solver.hierarchy_device(dev)
        units_d, _ = solver.hierarchy_rebuild(H.row_ptr, H.col_idx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            units_d, _ = solver.hierarchy_rebuild(H.row_ptr, H.col_idx)
        torch.cuda.synchronize()
        ms_hier = 1e3 * (time.perf_counter() - t0) / args.steps
        ud = units_d.cpu().numpy()
        got = [int(u) for u in ud[1:1 + ud[0]]]
        out["hierarchy_device"] = {
            "ms": round(ms_hier, 4),
            "levels": int(ud[0]),
            "matches_host_analysis": got == list(info["units"]) and [int(u) for u in units_h] == got,
            "host_symbolic_ms": round(t_symbolic * 1e3, 1),
        }
        log(f"device hierarchy: {ms_hier:.3f} ms, units {got}")

        # every solver plan re-derived on the device when contacts change the
        # pattern (mas_replan): a handle analysed on the contact-free mesh
        # pattern is re-planned for the pattern with the 20,000 contacts; the
        # partition comes from the same mesh graph as the headline solver's,
        # so the re-planned solve must repeat the headline solve bit for bit
        n = s.n
        deg = np.diff(s.gptr)
        key = np.unique(np.concatenate([np.arange(n) * (n + 1),
                                        np.repeat(np.arange(n), deg).astype(np.int64) * n + s.gadj]))
        rp_free = np.concatenate([[0], np.cumsum(np.bincount(key // n, minlength=n))]).astype(np.int32)
        ci_free = (key % n).astype(np.int32)
        rsolver = mp.MasPcg(rp_free, ci_free, graph=(s.gptr, s.gadj), domain_size=args.domain_size)
        rsolver.replan(H.row_ptr, H.col_idx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rsolver.replan(H.row_ptr, H.col_idx)
        torch.cuda.synchronize()
        ms_replan = 1e3 * (time.perf_counter() - t0) / args.steps
        mp_map, _, _ = rsolver.ordering()
        t0 = time.perf_counter()
        hsolver = mp.MasPcg(s.row_ptr, s.col_idx, domain_size=args.domain_size,
                            partition=mp_map // args.domain_size)
        ms_host_replan = 1e3 * (time.perf_counter() - t0)
        hsolver.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rsolver.build(H)  # places the plans, then the numeric build
        torch.cuda.synchronize()
        ms_place_build = 1e3 * (time.perf_counter() - t0)
        t0 = time.perf_counter()
        rsolver.build(H)
        torch.cuda.synchronize()
        ms_build = 1e3 * (time.perf_counter() - t0)
        xr, rres = rsolver.solve(H, b, tol=args.tol)
        x0, _ = step(solver, args.tol)
        torch.cuda.synchronize()
        out["replan_device"] = {
            "ms": round(ms_replan, 4),
            "host_analysis_same_partition_ms": round(ms_host_replan, 1),
            "first_build_ms": round(ms_place_build, 3),
            "build_ms": round(ms_build, 3),
            "iterations": rres["iterations"],
            "solve_equals_headline": bool(torch.equal(xr, x0)) and rres["iterations"] == res["iterations"],
        }
        log(f"device re-plan: {ms_replan:.3f} ms (host analysis {ms_host_replan:.1f} ms), "
            f"{rres['iterations']} its, equal: {out['replan_device']['solve_equals_headline']}")
        rsolver.close()

        # forward + adjoint (loss 0.5 ||x - x*||^2, FP32 dL/dH) vs forward
        xt = torch.as_tensor(np.random.default_rng(4).standard_normal(3 * s.n), device=dev)
        for _ in range(max(args.warmup, 1)):
            step(solver, args.tol)
            solver.adjoint(H, x, x - xt, dLdH_dtype=torch.float32, tol=args.tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(solver, args.tol)
            _, _, ares = solver.adjoint(H, x, x - xt, dLdH_dtype=torch.float32, tol=args.tol)
        torch.cuda.synchronize()
        ms_fb = 1e3 * (time.perf_counter() - t0) / args.steps
        out["fwd_adjoint"] = {
            "ms_fwd_plus_adjoint": round(ms_fb, 4),
            "ratio_vs_fwd": round(ms_fb / ms_per_step, 3),
            "adjoint_iterations": ares["iterations"],
        }
        log(f"fwd+adjoint: {ms_fb:.3f} ms ({ms_fb / ms_per_step:.2f}x)")

    if not args.no_cpu_baseline:
        ncores = len(os.sched_getaffinity(0))
        t_build, t_pcg, it, xo, core = oracle_solve(s, args.domain_size, args.tol)
        out["cpu_baseline"] = {
            "value": round(1e3 * (t_build + t_pcg), 1),
            "unit": "ms",
            "cores": 1,
            "kind": "oracle",
            "sample": f"the whole workload once: oracle partition+hierarchy+inversion ({t_build:.2f} s) and PCG "
            f"to {args.tol:g} ({it} iterations, {t_pcg:.2f} s), single-threaded C pinned to core {core}, "
            f"1 of {ncores} host cores ({cpu_model()})",
            "iterations": it,
            "cpu_model": cpu_model(),
        }
        log(f"cpu oracle: build {t_build:.2f}s pcg {t_pcg:.2f}s ({it} its)")
        solver.build(H)
        xg = solver.solve(H, b, tol=args.tol)[0].cpu().numpy()
        out["gpu_vs_oracle_rel_err"] = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
        if "mixed" in out:
            out["mixed"]["rel_err_vs_f64_oracle"] = float(np.linalg.norm(x_mixed - xo) / np.linalg.norm(xo))

    if not args.no_configs:
        out["configs"] = run_configs(args, s, H, b, dev, x_oracle=None if args.no_cpu_baseline else xo)

    print(json.dumps(out), flush=True)
    solver.close()


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_solve(s, N, tol, max_levels=0):
    """The CPU oracle on system s (single-threaded C), pinned to the first
    host core this process may use: (build s, pcg s, iterations, x, core)."""
    import oracle

    prev = os.sched_getaffinity(0)
    core = min(prev)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        P = oracle.MAS(s.row_ptr, s.col_idx, s.val, N=N, max_levels=max_levels, gptr=s.gptr, gadj=s.gadj)
        t_build = time.perf_counter() - t0
        t0 = time.perf_counter()
        xo, st, it, rr, tr = P.pcg(s.b, tol=tol)
        t_pcg = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, prev)
    return t_build, t_pcg, it, xo, core


def gpu_solves(mp, s, H, b, tol, steps, precision="f64", max_levels=0, N=16):
    """Build + solve steps times after two warm-ups: mean and median ms, the
    last result and x."""
    import numpy as np
    import torch

    sv = mp.MasPcg(s.row_ptr, s.col_idx, graph=(s.gptr, s.gadj), domain_size=N, precision=precision,
                   max_levels=max_levels)
    x = torch.empty_like(b)
    for _ in range(2):
        sv.build(H)
        sv.solve(H, b, tol=tol, out=x)
    ms = []
    for _ in range(steps):
        t0 = time.perf_counter()
        sv.build(H)
        _, res = sv.solve(H, b, tol=tol, out=x)
        ms.append(1e3 * (time.perf_counter() - t0))
    sv.close()
    if res["status"] != 0:
        raise SystemExit(f"solve did not converge: {res}")
    return float(np.mean(ms)), float(np.median(ms)), res, x


def run_configs(args, s1, H1, b1, dev, x_oracle):
    """The other workloads of the benchmark set, each timed on the GPU
    (build + solve, mean and median of the steps) with its iteration count
    and FP64 true residual, and the CPU oracle on the same system once
    (pinned to one core)."""
    import numpy as np
    import torch

    import synth
    import paper_2411_06224_amd as mp

    steps = max(3, min(args.steps, 10))
    cfg = {}

    def gpu_entry(mean, med, res):
        return {"ms": round(mean, 4), "median_ms": round(med, 4), "iterations": res["iterations"],
                "true_rel_residual": res["true_rel_residual"]}

    def with_oracle(entry, s, tol, max_levels=0):
        tb, tp, it, xo, _ = oracle_solve(s, 16, tol, max_levels)
        entry["oracle"] = {"ms": round(1e3 * (tb + tp), 1), "iterations": it, "cores": 1}
        return xo

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    # 8^3 cube, two-level MAS, FP64 to 1e-8: latency-bound, so us per iteration
    s0 = synth.config_small()
    H0 = mp.BlockMatrix.from_numpy(s0.row_ptr, s0.col_idx, s0.val, device=dev)
    b0 = torch.as_tensor(s0.b, device=dev)
    mean, med, res, _ = gpu_solves(mp, s0, H0, b0, 1e-8, 20, max_levels=2)
    e = gpu_entry(mean, med, res)
    e["us_per_iteration"] = round(1e3 * med / max(res["iterations"], 1), 2)
    with_oracle(e, s0, 1e-8, max_levels=2)
    cfg["cube8_f64_tol1e-8"] = e
    log("cube8:", json.dumps(e))

    # 48^3 at E = 1e6: FP64 to 1e-8, mixed to 1e-4 and 1e-6 (error against the
    # FP64 oracle's solution at the same tolerance)
    mean, med, res, _ = gpu_solves(mp, s1, H1, b1, 1e-8, steps)
    e = gpu_entry(mean, med, res)
    with_oracle(e, s1, 1e-8)
    cfg["cube48_E1e6_f64_tol1e-8"] = e
    log("cube48 E=1e6 1e-8:", json.dumps(e))
    for tol in (1e-4, 1e-6):
        mean, med, res, xm = gpu_solves(mp, s1, H1, b1, tol, steps, precision="mixed")
        e = gpu_entry(mean, med, res)
        xo = x_oracle if (tol == 1e-4 and x_oracle is not None) else with_oracle(e, s1, tol)
        e["rel_err_vs_f64_oracle"] = rel(xm.cpu().numpy(), xo)
        cfg[f"cube48_E1e6_mixed_tol{tol:g}"] = e
        log(f"cube48 E=1e6 mixed {tol:g}:", json.dumps(e))

    # 48^3 at E = 1e4 and 1e8 (FP64 to 1e-4; mixed at E = 1e8 to 1e-4, 1e-6)
    for E in (1e4, 1e8):
        sE = synth.config_large(E=E)
        HE = mp.BlockMatrix.from_numpy(sE.row_ptr, sE.col_idx, sE.val, device=dev)
        bE = torch.as_tensor(sE.b, device=dev)
        mean, med, res, _ = gpu_solves(mp, sE, HE, bE, 1e-4, steps)
        e = gpu_entry(mean, med, res)
        xo4 = with_oracle(e, sE, 1e-4)
        cfg[f"cube48_E{E:g}_f64_tol1e-4"] = e
        log(f"cube48 E={E:g}:", json.dumps(e))
        # FP64 to 1e-8 as well
        mean, med, res, _ = gpu_solves(mp, sE, HE, bE, 1e-8, steps)
        e8 = gpu_entry(mean, med, res)
        with_oracle(e8, sE, 1e-8)
        cfg[f"cube48_E{E:g}_f64_tol1e-8"] = e8
        log(f"cube48 E={E:g} 1e-8:", json.dumps(e8))
        if E == 1e8:
            f64_ms = mean
            # hierarchy depth at this stiffness: block Jacobi over the level-0
            # domains (1 level), two levels, all levels
            depth = {}
            for ml in (1, 2):
                dm, dmed, dres, _ = gpu_solves(mp, sE, HE, bE, 1e-4, steps, max_levels=ml)
                depth[f"max_levels_{ml}"] = {"ms": round(dm, 4), "iterations": dres["iterations"]}
            depth["all_levels"] = {"ms": round(f64_ms, 4), "iterations": cfg[f"cube48_E{E:g}_f64_tol1e-4"]["iterations"]}
            cfg["cube48_E1e8_depth_ablation"] = depth
            log("cube48 E=1e8 depth:", json.dumps(depth))
            for tol in (1e-4, 1e-6):
                mean, med, res, xm = gpu_solves(mp, sE, HE, bE, tol, steps, precision="mixed")
                e = gpu_entry(mean, med, res)
                xo = xo4 if tol == 1e-4 else with_oracle(e, sE, tol)
                e["rel_err_vs_f64_oracle"] = rel(xm.cpu().numpy(), xo)
                if tol == 1e-4:
                    e["speedup_vs_f64"] = round(f64_ms / mean, 3)
                cfg[f"cube48_E{E:g}_mixed_tol{tol:g}"] = e
                log(f"cube48 E={E:g} mixed {tol:g}:", json.dumps(e))
        del HE, bE, sE

    # 48^3 at E = 1e7: mixed forward to 1e-6, then the adjoint solve with
    # dL/dH in FP32 for L = 1/2 ||x - x*||^2
    s7 = synth.config_large(E=1e7)
    H7 = mp.BlockMatrix.from_numpy(s7.row_ptr, s7.col_idx, s7.val, device=dev)
    b7 = torch.as_tensor(s7.b, device=dev)
    sv = mp.MasPcg(s7.row_ptr, s7.col_idx, graph=(s7.gptr, s7.gadj), domain_size=16, precision="mixed")
    xt = torch.as_tensor(np.random.default_rng(4).standard_normal(3 * s7.n), device=dev)
    x7 = torch.empty_like(b7)
    fwd, both = [], []
    for i in range(steps + 2):
        t0 = time.perf_counter()
        sv.build(H7)
        _, fres = sv.solve(H7, b7, tol=1e-6, out=x7)
        t1 = time.perf_counter()
        _, _, ares = sv.adjoint(H7, x7, x7 - xt, dLdH_dtype=torch.float32, tol=1e-6)
        t2 = time.perf_counter()
        if i >= 2:
            fwd.append(1e3 * (t1 - t0))
            both.append(1e3 * (t2 - t0))
    sv.close()
    cfg["cube48_E1e7_mixed_fwd_adjoint_tol1e-6"] = {
        "ms_forward": round(float(np.mean(fwd)), 4),
        "ms_forward_plus_adjoint": round(float(np.mean(both)), 4),
        "ratio": round(float(np.mean(both) / np.mean(fwd)), 3),
        "forward_iterations": fres["iterations"],
        "adjoint_iterations": ares["iterations"],
        "forward_true_rel_residual": fres["true_rel_residual"],
    }
    log("cube48 E=1e7 fwd+adjoint:", json.dumps(cfg["cube48_E1e7_mixed_fwd_adjoint_tol1e-6"]))
    del H7, b7, s7

    # stiff membrane (512^2 cells) + 2,000 affine bodies: FP64 and mixed to 1e-4
    sm = synth.config_membrane()
    Hm = mp.BlockMatrix.from_numpy(sm.row_ptr, sm.col_idx, sm.val, device=dev)
    bm = torch.as_tensor(sm.b, device=dev)
    mean, med, res, _ = gpu_solves(mp, sm, Hm, bm, 1e-4, steps)
    e = gpu_entry(mean, med, res)
    e["levels"] = mp.MasPcg(sm.row_ptr, sm.col_idx, graph=(sm.gptr, sm.gadj), domain_size=16).info()["levels"]
    xo = with_oracle(e, sm, 1e-4)
    cfg["membrane512_bodies2000_f64_tol1e-4"] = e
    f64_ms = mean
    log("membrane f64:", json.dumps(e))
    # ordering ablation on this system (Sec. 4.1): level-0 domains of 16
    # consecutive nodes in Morton order against the connectivity-aware
    # partition; the bodies' couplings reach sheet nodes anywhere on the sheet
    t0 = time.perf_counter()
    part = mp.morton_partition(sm.meta["positions"], 16, device=dev)
    t_part = time.perf_counter() - t0
    sv = mp.MasPcg(sm.row_ptr, sm.col_idx, domain_size=16, partition=part)
    xm_ = torch.empty_like(bm)
    for _ in range(2):
        sv.build(Hm)
        sv.solve(Hm, bm, tol=1e-4, out=xm_)
    ms_m = []
    for _ in range(steps):
        t0 = time.perf_counter()
        sv.build(Hm)
        _, mres = sv.solve(Hm, bm, tol=1e-4, out=xm_)
        ms_m.append(1e3 * (time.perf_counter() - t0))
    cfg["membrane512_bodies2000_ordering_ablation"] = {
        "connectivity": {"iterations": e["iterations"], "ms": e["ms"], "levels": e["levels"]},
        "morton": {"iterations": mres["iterations"], "ms": round(float(np.mean(ms_m)), 4),
                   "true_rel_residual": mres["true_rel_residual"], "levels": sv.info()["levels"],
                   "partition_ms": round(1e3 * t_part, 2)},
    }
    sv.close()
    log("membrane ordering ablation:", json.dumps(cfg["membrane512_bodies2000_ordering_ablation"]))
    mean, med, res, xm = gpu_solves(mp, sm, Hm, bm, 1e-4, steps, precision="mixed")
    e = gpu_entry(mean, med, res)
    e["rel_err_vs_f64_oracle"] = rel(xm.cpu().numpy(), xo)
    e["speedup_vs_f64"] = round(f64_ms / mean, 3)
    cfg["membrane512_bodies2000_mixed_tol1e-4"] = e
    log("membrane mixed:", json.dumps(e))
    del Hm, xm_, xm
    from synth.abd import body_contacts

    d = body_contacts()
    cfg["membrane512_bodies2000_contact_assembly"] = abd_assembly_ablation(mp, dev, steps, d)
    cfg["membrane512_bodies2000_newton_step_device"] = newton_step_device(mp, dev, steps, sm, bm, d)
    return cfg


def newton_step_device(mp, dev, steps, sm, bm, d):
    """One Newton step's linear algebra with no host analysis: the contact
    Hessians of the 240,000 contacts reduced in two levels (Sec. 6.1) and
    assembled with the system's own blocks (Sec. 6.2), every solver plan of
    the new pattern derived on the device (Sec. 4.2), the MAS build and PCG
    to 1e-4.  The solver was analysed once on the contact-free system; the
    step's result is checked against a handle analysed on the host for the
    assembled pattern with the same partition (identical solution)."""
    import numpy as np
    import torch

    t = {k: torch.as_tensor(np.ascontiguousarray(d[k]), device=dev)
         for k in ("node_row", "node_is_body", "node_xbar", "rows", "cols", "blocks")}
    n = sm.n
    own_r = torch.as_tensor(np.repeat(np.arange(n, dtype=np.int32), np.diff(sm.row_ptr)), device=dev)
    own_c = torch.as_tensor(sm.col_idx, device=dev)
    own_v = torch.as_tensor(sm.val.reshape(-1, 3, 3), device=dev)
    S = mp.MasPcg(sm.row_ptr, sm.col_idx, graph=(sm.gptr, sm.gadj), domain_size=16)
    x = torch.empty_like(bm)
    marks = ("assemble", "replan", "build", "solve")

    def newton_step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        r2, c2, b2 = mp.abd_contact_blocks(d["n_nodes"], t["node_row"], t["node_is_body"], t["node_xbar"],
                                           t["rows"], t["cols"], t["blocks"], levels=2)
        Hg = mp.bcsr_assemble(n, torch.cat([own_r, r2]), torch.cat([own_c, c2]), torch.cat([own_v, b2]))
        ev[1].record()
        S.replan(Hg.row_ptr, Hg.col_idx)
        ev[2].record()
        S.build(Hg)
        ev[3].record()
        _, res = S.solve(Hg, bm, tol=1e-4, out=x)
        ev[4].record()
        torch.cuda.synchronize()
        return Hg, res, [ev[k].elapsed_time(ev[k + 1]) for k in range(4)]

    newton_step()
    rows = []
    for _ in range(steps):
        t0 = time.perf_counter()
        Hg, res, ph = newton_step()
        rows.append([1e3 * (time.perf_counter() - t0)] + ph)
    m = np.mean(np.array(rows), axis=0)
    rp, ci = Hg.row_ptr.cpu().numpy(), Hg.col_idx.cpu().numpy()
    part = S.ordering()[0] // 16
    B = mp.MasPcg(rp, ci, domain_size=16, partition=part)
    B.build(Hg)
    xb, bres = B.solve(Hg, bm, tol=1e-4)
    torch.cuda.synchronize()
    out = {
        "ms": round(float(m[0]), 4),
        "phase_ms": {k: round(float(v), 4) for k, v in zip(marks, m[1:])},
        "nnzb": int(Hg.nnzb),
        "levels": S.info()["levels"],
        "iterations": res["iterations"],
        "true_rel_residual": res["true_rel_residual"],
        "equals_host_planned_solve": bool(torch.equal(x, xb)) and bres["iterations"] == res["iterations"],
    }
    S.close()
    B.close()
    log("device Newton step:", json.dumps(out))
    return out


def abd_assembly_ablation(mp, dev, steps, d):
    """Contact Hessians of the 2,000 bodies on the 512^2 sheet (200,000
    vertex-face and 40,000 edge-edge contacts, 16 node-pair blocks each)
    assembled into the system's DOF blocks: the two-level reduction of
    Sec. 6.1 (equal node pairs summed, each pair mapped once, then the DOF
    blocks summed) against the single-level one (every block mapped, then
    summed), both ending in bcsr_assemble."""
    import numpy as np
    import torch

    t = {k: torch.as_tensor(np.ascontiguousarray(d[k]), device=dev)
         for k in ("node_row", "node_is_body", "node_xbar", "rows", "cols", "blocks")}
    nd = d["n_dof_rows"]
    out = {"contacts": d["contacts"], "blocks_in": int(d["rows"].size), "dof_rows": nd}

    def run(levels):
        r, c, b = mp.abd_contact_blocks(d["n_nodes"], t["node_row"], t["node_is_body"], t["node_xbar"],
                                        t["rows"], t["cols"], t["blocks"], levels=levels)
        A = mp.bcsr_assemble(nd, r, c, b)
        return A, int(r.numel())

    for levels in (2, 1):
        A, mid = run(levels)
        torch.cuda.synchronize()
        ts = []
        for _ in range(steps):
            t0 = time.perf_counter()
            A, mid = run(levels)
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
        out[f"levels{levels}"] = {"ms": round(float(np.mean(ts)), 4), "dof_blocks_listed": mid,
                                  "dof_blocks_out": int(A.nnzb)}
        if levels == 2:
            A2 = A
        else:
            # the two orders of summation agree to rounding
            num = (A.val - A2.val).abs().max().item()
            out["max_abs_diff_levels"] = num
            out["max_abs_value"] = A.val.abs().max().item()
        del A
    out["speedup_two_level"] = round(out["levels1"]["ms"] / out["levels2"]["ms"], 3)
    log("contact assembly:", json.dumps(out))
    return out


if __name__ == "__main__":
    main()
