#!/usr/bin/env python
"""Benchmark of the Krylov interior point method on one MI355X.

One step = one complete interior point solve (Algorithm 1: every Newton
system solved by Jacobi PCG on the doubly augmented KKT matrix, ratio test,
barrier update) of the radiation-therapy-shaped QP:
  200,000 voxels x 20,000 beamlets, P sparse with 0.5% density (log-normal
  values), objective 1/2 sum_v w_v (P_v x - d_v)^2 with w_v in {1, 10},
  x >= 0, and 10,000 max-dose rows P_k x <= 1.1.
Synthetic, seeded data (the paper's clinical problems are not available).

Prints one JSON line.  `value` is PCG iterations per second over the timed
solves (inputs resident in HBM); `roofline` describes the dominant PCG
kernel, timed with HIP events on the library's stream; `cpu_baseline` times
the CPU oracle's matrix-free PCG on the same Newton system for a bounded
number of iterations.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "IPM solve time & PCG iters/sec to 1e-6 KKT residual; achieved HBM GB/s vs peak"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rt_full",
                    choices=["rt_full", "rt_small", "svm_full", "tiny_dense"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16", "fp32x64", "bf16x64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="oracle PCG iterations for the CPU baseline (0: pick ~15 s)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--profile-cap", type=int, default=20000)
    return ap.parse_args()


def workload(name):
    from paper_2308_00637_amd import workloads as W
    return {"rt_full": W.rt_full, "rt_small": W.rt_small, "svm_full": W.svm_full,
            "tiny_dense": W.tiny_dense}[name]()


def kernel_bytes(spec, ob, cat, prec_bytes):
    """Algorithmic HBM bytes of one launch of a PCG matvec kernel: every stored
    operator entry once (value + int32 column), index arrays once, each vector
    the kernel reads or writes once."""
    n, m, me = spec.n, spec.m, spec.me
    p_rows = spec.P.shape[0] if spec.h_kind == "ptwp" else 0
    k = spec.U.shape[1] if spec.h_kind == "lowrank" else 0
    if cat == "rowpass":
        return (ob["row_bytes"] + 8 * n                      # operator, gathered p_x
                + 16 * p_rows                                # w read, u write
                + m * (16 + 16 + 16 + 16 + 8))               # lA,uA | p_lam | D | q_lam | wA
    if cat == "colpass":
        return (ob["col_bytes"] + n * k * prec_bytes         # operator, dense U rows
                + 8 * p_rows + 8 * m                         # gathered u, wA
                + 8 * n * 3 + 8 * n * me)                    # p_x, qdiag, q_x write, C
    if cat == "tsreduce":
        return n * k * prec_bytes + 8 * n * (1 + me)
    return 0


def cpu_baseline(spec, iters):
    """The oracle's textbook PCG with its matrix-free K v, at the first Newton
    system (default starting point, mu = 1)."""
    import numpy as np
    import oracle as O
    from oracle.pcg import pcg
    prob = O.from_spec(spec)
    st = O.initial_point(prob)
    rhs, _ = O.newton_rhs_doubly(prob, st, 1.0)
    dg = O.jacobi_diagonal(prob, st, 1.0)
    mv = lambda v: O.kkt_matvec(prob, st, 1.0, v)
    if iters <= 0:
        t0 = time.perf_counter()
        mv(rhs)
        one = time.perf_counter() - t0
        iters = int(max(3, min(200, 15.0 / max(one, 1e-6))))
    t0 = time.perf_counter()
    pcg(mv, rhs, dg, tol=1e-300, maxit=iters)
    dt = time.perf_counter() - t0
    return {"value": iters / dt, "unit": "PCG iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} iterations of the oracle's Jacobi PCG (matrix-free K v in "
                      f"NumPy/SciPy, float64, single-threaded) on the first Newton system "
                      f"of the same workload; {dt:.1f} s"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this method's solve runs on a single "
              "MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2308_00637_amd.qpk import QP, default_ipm_options

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    spec = workload(args.workload)
    t_gen = time.perf_counter() - t0
    print(f"[bench] workload {spec.name} generated in {t_gen:.1f}s", file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        qp = QP(spec, precision=args.precision)
        torch.cuda.synchronize()
        t_create = time.perf_counter() - t0
        print(f"[bench] qp_create {t_create:.2f}s", file=sys.stderr, flush=True)
        opts = default_ipm_options()
        for w in range(args.warmup):
            out = qp.solve(opts, want_state=False)
            inf = out["info"]
            print(f"[bench] warmup {w}: ipm={inf.iterations} cg={inf.total_cg_iters} "
                  f"{inf.time_ms / 1e3:.2f}s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        qp.profile_begin(args.profile_cap)
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            out = qp.solve(opts, want_state=False)
            infos.append(out["info"])
            print(f"[bench] step {s}: ipm={out['info'].iterations} cg={out['info'].total_cg_iters} "
                  f"{out['info'].time_ms / 1e3:.2f}s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = qp.profile_end()
        ob = qp.operator_bytes()
        if args.copy_calib_mb > 0:
            nb = args.copy_calib_mb * (1 << 20) // 8
            a = torch.empty(nb, dtype=torch.float64, device="cuda").fill_(1.0)
            b = torch.empty_like(a)
            b.copy_(a)
            torch.cuda.synchronize()
            del a, b
    total_cg = sum(i.total_cg_iters for i in infos)
    solve_s = sum(i.time_ms for i in infos) / 1e3
    info = infos[-1]

    prec_bytes = {"fp64": 8, "fp32": 4, "bf16": 2, "fp32x64": 4, "bf16x64": 2}[args.precision]
    kern = {}
    for cat in ("rowpass", "colpass", "tsreduce"):
        cnt, ms = prof[cat]
        if cnt:
            avg_s = ms / cnt / 1e3
            by = kernel_bytes(spec, ob, cat, prec_bytes)
            kern[cat] = {"launches_timed": cnt, "avg_us": avg_s * 1e6, "bytes": by,
                         "GBs": by / avg_s / 1e9}
    dom = max(kern, key=lambda c: kern[c]["avg_us"] * kern[c]["launches_timed"])
    d = kern[dom]
    cgv = prof["cgvec"]
    per_iter_us = sum(kern[c]["avg_us"] for c in kern) + (cgv[1] / cgv[0] * 1e3 if cgv[0] else 0.0)
    result = {
        "metric": METRIC,
        "value": total_cg / solve_s,
        "unit": "PCG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"{args.precision} matvec / f64",
        "data": "synthetic",
        "config": {"workload": spec.name, "n": spec.n, "m": spec.m, "me": spec.me,
                   "N_kkt": spec.n + spec.me + spec.m, "precision": args.precision,
                   "pcg_tol": 1e-7, "pcg_maxit": 5000},
        "ipm_solve_time_s": solve_s / args.steps,
        "ipm_iterations": info.iterations,
        "pcg_iterations_per_solve": total_cg / args.steps,
        "cg_maxiter_hits": info.cg_maxiter_hits,
        "cg_escalations_to_fp64": info.cg_escalations,
        "kkt_residual": info.rnorm,
        "objective": info.objective,
        "mu_final": info.mu_final,
        "qp_create_s": t_create,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": d["GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": d["GBs"] / HBM_PEAK_GBS, "traffic": None,
                     "avg_us": d["avg_us"], "algorithmic_bytes_per_launch": d["bytes"],
                     "launches_timed": d["launches_timed"]},
        "kernels": kern,
        "pcg_iteration_us": per_iter_us,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(spec, args.cpu_iters)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
