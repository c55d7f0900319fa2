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
solves (inputs resident in HBM).  `roofline` takes one PCG iteration as its
unit: the algorithmic bytes of an iteration (`iteration_bytes`: the operator
once per use the PCG data dependencies require, plus the vectors) over the
kernel time per iteration, which comes from dispatches sampled (one in
--profile-every) with HIP event pairs bound to the dispatch on the library's
stream; the dominant kernel's own figures sit beside it.  `traffic` (HBM
bytes per iteration) is read from the committed counter summary under
profiles/ when it was taken on the same kernel sources.  `cpu_baseline` times
the CPU oracle's matrix-free PCG on the same Newton system for a bounded
number of iterations, next to the oracle's exact (dense Cholesky) solve time
stored with the golden solution.

  python bench.py --summarize-stats rt_kernel_stats.csv --command "..."
  python bench.py --summarize-counters fetch.csv write.csv --bench-json b.json
turn rocprofv3 output into the summaries kept under profiles/.
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
                    choices=["rt_full", "rt_small", "svm_full", "svm_rbf", "qn_rt", "tiny_dense",
                             "batch3"])
    ap.add_argument("--batch-take", type=int, default=256,
                    help="batch3: instances of the 256-instance uneven batch, spread over its sizes "
                         "(all 256 by default; generating them takes about two minutes)")
    ap.add_argument("--batch-cg", type=int, default=40,
                    help="batch3: PCG iterations of the first Newton system timed per instance")
    ap.add_argument("--tune-table", default="",
                    help="batch3: team-size table of the autotuner (default: a file in the temp dir)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16", "fp32x64", "bf16x64"])
    ap.add_argument("--mu-rule", default="paper", choices=["paper", "mehrotra"],
                    help="the barrier parameter's rule: Algorithm 1's (default) or Mehrotra's "
                         "predictor-corrector (two PCG solves per IPM iteration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="oracle PCG iterations for the CPU baseline (0: pick ~15 s)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--profile-cap", type=int, default=20000)
    ap.add_argument("--profile-every", type=int, default=13,
                    help="time one dispatch in this many of each PCG kernel with HIP events")
    ap.add_argument("--summarize-stats", metavar="CSV",
                    help="print a markdown summary of a rocprofv3 --stats kernel_stats.csv and exit")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the per-kernel HBM traffic summary of two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) and exit; needs --bench-json")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="CSV",
                    help="print per-kernel means of every counter in rocprofv3 --pmc "
                         "counter_collection.csv files and exit; needs --bench-json")
    ap.add_argument("--bench-json", help="the JSON line printed by the profiled bench run")
    ap.add_argument("--command", default="", help="the profiled command, quoted in the summary")
    return ap.parse_args()


def workload(name):
    from paper_2308_00637_amd import workloads as W
    return {"rt_full": W.rt_full, "rt_small": W.rt_small, "svm_full": W.svm_full,
            "svm_rbf": W.svm_rbf, "qn_rt": W.qn_rt, "tiny_dense": W.tiny_dense}[name]()


def fused_bytes(spec, fz, prec_bytes):
    """Bytes of one dispatch of the fused single-read pass: each stored entry
    once (value + uint16 column offset), both halves' row pointers, w and the
    twin map per row of P, the gathered vector, each row's half dots written
    once and read once by the partner, the per-range x-parts written, and the
    lam-part data of the rows of A (six values in, two out)."""
    p_rows = spec.P.shape[0]
    return (fz["stored"] * (prec_bytes + 2) + 8 * (p_rows + 1) + 12 * p_rows + 8 * spec.n
            + 16 * p_rows + 8 * fz["ranges"] * spec.n + 64 * spec.m)


def kernel_bytes(spec, ob, lay, cat, prec_bytes, fz=None):
    """Algorithmic HBM bytes of one dispatch of a PCG kernel: every stored
    operator entry once (value + uint16 column offset, one row-pointer array
    per LDS chunk), and each vector the kernel must read or write once.  The
    per-chunk partial sums of a multi-chunk pass are an artefact of the LDS
    blocking and are not counted (the epilogue is charged the pass's outputs)."""
    n, m, me = spec.n, spec.m, spec.me
    N = n + me + m
    p_rows = spec.P.shape[0] if spec.h_kind == "ptwp" else 0
    k = spec.U.shape[1] if spec.h_kind == "lowrank" else 0
    row_out = 16 * p_rows + m * (16 + 16 + 16 + 16 + 8)   # w in, u out | lA,uA, p_lam, D, q_lam, wA
    col_out = 8 * n * 3 + 8 * n * me                       # p_x, qdiag, q_x out, C
    row_multi = lay["row"]["chunks"] > 1
    col_multi = lay["col"]["chunks"] > 1
    # PCG products on a multi-chunk column side leave its epilogue to the CG
    # update; the column pass then also reads p_x and diag(H) for p.q
    col_fused = col_multi and lay["col"]["work_items"] <= 2048
    if cat == "rowpass":
        return ob["row_bytes"] + 8 * n + (0 if row_multi else row_out)
    if cat == "colpass":
        return (ob["col_bytes"] + n * k * prec_bytes + 8 * p_rows + 8 * m
                + (16 * n if col_fused else 0 if col_multi else col_out))
    if cat == "epilogue":
        sides = [b for b, on in ((row_out, row_multi), (col_out, col_multi)) if on]
        return sum(sides) / max(1, len(sides))
    if cat == "tsreduce":
        return n * k * prec_bytes + 8 * n * (1 + me)
    if cat == "fused":
        return fused_bytes(spec, fz, prec_bytes)
    if cat == "cg_update":     # x, p, r, q, diag in; x, r, z out (fused: q_x from partials, diag(H) in)
        return 8 * 8 * N + (8 * n * me + 8 * n if col_fused else 0)
    if cat == "cg_pupdate":
        return 3 * 8 * N          # z, p in; p out
    return 0


def iteration_bytes(spec, precision):
    """Algorithmic HBM bytes of one PCG iteration: the operator data once per
    use that the PCG data dependencies require, plus fourteen touches of a
    float64 N-vector (a well-fused iteration reads p, x, r, z, diag and the
    lam-part data and writes q, x, r, z, p).

    * H = P^T W P (radiation therapy): P once.  The product is row-local,
      P^T (W (P v)) = sum_v P_v^T w_v (P_v . v), so one pass over the rows of P
      (and of A, whose row epilogue is local too) is enough; a second read of
      P, as in a two-pass design, is counted as overhead, not as algorithmic.
    * H = H0 + U W U^T (SVM Gram matrix, quasi-Newton): U twice, since
      U (W (U^T v)) needs all of U^T v before its second pass can start.
    * dense H: H once.
    Values take the stored precision's bytes, sparse column indices 4 bytes
    (2 bytes with bfloat16 values, which pair with 16-bit column offsets),
    row pointers 4 bytes."""
    import scipy.sparse as sp
    vb = {"fp64": 8, "fp32": 4, "bf16": 2, "fp32x64": 4, "bf16x64": 2}[precision]
    ib = 2 if vb == 2 else 4
    n, m, me = spec.n, spec.m, spec.me
    N = n + me + m
    total = 14 * 8 * N
    if spec.h_kind == "ptwp":
        total += spec.P.nnz * (vb + ib) + 4 * (spec.P.shape[0] + 1) + 8 * spec.P.shape[0]
    elif spec.h_kind == "lowrank":
        total += 2 * n * spec.U.shape[1] * vb
    else:
        total += n * n * vb
    if spec.A is not None:
        if sp.issparse(spec.A):
            total += spec.A.nnz * (vb + ib) + 4 * (m + 1)
        else:
            total += m * n * vb
    if spec.C is not None:
        total += me * n * 8
    return int(total)


# The sources of the single-instance path's kernels and their launches (the
# batched solver's kernel is a translation unit of its own).
PATH_SOURCES = ("qpk_api.hip", "qpk_internal.h", "qpk_kernels.hip")


def source_digest():
    """SHA-256 over the HIP sources of the single-instance path: counter
    figures taken on other sources do not describe the kernels that run now."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2308_00637_amd", "csrc")
    for f in PATH_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def stored_traffic(workload, precision, kernel):
    """HBM bytes per dispatch of `kernel` from the committed counter summary of
    this workload (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a plain device copy), or None when no summary exists or it was
    taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_json: "):
                rec = json.loads(line[len("traffic_json: "):])
    if not rec or rec.get("source_sha256") != source_digest():
        return None
    kk = rec["kernels"].get(kernel)
    if not kk:
        return None
    return 1024.0 * (kk["fetch_kib"] * rec["fetch_factor"] + kk["write_kib"] * rec["write_factor"])


def _short(name):
    return name.replace("void ", "").replace("qpk::", "").split("(")[0]


def summarize_stats(path, command):
    import csv
    rows = list(csv.DictReader(open(path)))
    out = ["# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
           "| kernel | calls | average us | total ms | % of kernel time |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    print("\n".join(out))


def kernel_category(lay):
    """Maps a rocprofv3 record to the bench's kernel category (None for the
    kernels outside the PCG iteration)."""
    grid = {"row": lay["row"]["work_items"], "col": lay["col"]["work_items"]}

    def category(r):
        name, g = _short(r["Kernel_Name"]), int(r["Grid_Size"])
        if name.startswith("k_chunked<"):
            epi = name[len("k_chunked<"):].split(",")[0].strip()
            if epi == "1":
                return "rowpass"
            if epi == "2":
                return "colpass"
            return "rowpass" if g == grid["row"] * 1024 and g != grid["col"] * 1024 else "colpass"
        if name.startswith("k_rowpass<0,"):
            return "rowpass"
        if name.startswith("k_colpass<0,"):
            return "colpass"
        if name.startswith("k_chunk_epilogue"):
            return "epilogue"
        if name.startswith("k_ts_reduce"):
            return "tsreduce"
        if name in ("k_cg_update", "k_cg_update_split", "k_cg_pupdate"):
            return "cg_update" if name.startswith("k_cg_update") else "cg_pupdate"
        if name.startswith("k_fused<"):
            return "fused"
        return None

    return category


def summarize_pmc(paths, bench_json, command):
    import csv
    rec = json.loads([ln for ln in open(bench_json) if ln.startswith("{")][-1])
    category = kernel_category(rec["layout"])
    agg = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            c = category(r)
            if c:
                agg.setdefault(c, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({n for v in agg.values() for n in v})
    out = ["# rocprofv3 counters per PCG kernel (mean per dispatch)", "",
           f"Command (one run per counter set): `{command}`", "",
           "| counter | " + " | ".join(agg) + " |", "|---|" + "---|" * len(agg)]
    for n in names:
        out.append(f"| {n} | " + " | ".join(
            f"{sum(agg[c][n]) / len(agg[c][n]):.4g}" if n in agg[c] else "" for c in agg) + " |")
    print("\n".join(out))


def summarize_counters(fetch_csv, write_csv, bench_json, command):
    """Per-category FETCH_SIZE / WRITE_SIZE (KiB per dispatch), the factors that
    map each counter onto the bytes of the bench's plain device copy, and the
    machine-readable line the bench reads back (keyed to the kernel sources)."""
    import csv
    rec = json.loads([ln for ln in open(bench_json) if ln.startswith("{")][-1])
    calib = rec["copy_calibration_bytes"]
    category = kernel_category(rec["layout"])

    def load(path, counter):
        per, copy = {}, 0.0
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if "copyBuffer" in r["Kernel_Name"]:
                copy = max(copy, v)
            c = category(r)
            if c:
                per.setdefault(c, []).append(v)
        return per, copy

    fetch, fcopy = load(fetch_csv, "FETCH_SIZE")
    write, wcopy = load(write_csv, "WRITE_SIZE")
    ff, wf = calib / (1024.0 * fcopy), calib / (1024.0 * wcopy)
    kern = {}
    for c in sorted(set(fetch) & set(write)):
        kern[c] = {"fetch_kib": sum(fetch[c]) / len(fetch[c]), "write_kib": sum(write[c]) / len(write[c]),
                   "dispatches": len(fetch[c])}
    out = ["# rocprofv3 HBM traffic counters", "",
           f"Command (twice, COUNTER = FETCH_SIZE then WRITE_SIZE): `{command}`", "",
           f"Calibration: a plain device copy of {calib / 2**20:.0f} MiB reads FETCH_SIZE "
           f"{fcopy:.0f} KiB and WRITE_SIZE {wcopy:.0f} KiB, so FETCH_SIZE is scaled by {ff:.3f} "
           f"and WRITE_SIZE by {wf:.3f}.", "",
           "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled HBM MB | algorithmic MB | ratio |",
           "|---|---|---|---|---|---|---|"]
    for c, v in kern.items():
        hbm = 1024.0 * (v["fetch_kib"] * ff + v["write_kib"] * wf)
        alg = rec["kernels"].get(c, {}).get("bytes")
        out.append(f"| {c} | {v['dispatches']} | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | "
                   f"{hbm / 1e6:.2f} | {alg / 1e6 if alg else float('nan'):.2f} | "
                   f"{hbm / alg if alg else float('nan'):.3f} |")
    out += ["", "traffic_json: " + json.dumps({"source_sha256": source_digest(), "fetch_factor": ff,
                                                "write_factor": wf, "kernels": kern})]
    print("\n".join(out))


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
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):   # one core: BLAS and OpenMP pools held to one thread
        if iters <= 0:
            t0 = time.perf_counter()
            mv(rhs)
            one = time.perf_counter() - t0
            iters = int(max(3, min(200, 15.0 / max(one, 1e-6))))
        t0 = time.perf_counter()
        pcg(mv, rhs, dg, tol=1e-300, maxit=iters)
        dt = time.perf_counter() - t0
    out = {"value": iters / dt, "unit": "PCG iters/s", "cores": 1, "kind": "oracle",
           "sample": f"{iters} iterations of the oracle's Jacobi PCG (matrix-free K v in "
                     f"NumPy/SciPy, float64, single-threaded) on the first Newton system "
                     f"of the same workload; {dt:.1f} s"}
    exact = stored_exact_solve(spec)
    if exact:
        out["exact_oracle_solve"] = exact
    return out


def stored_exact_solve(spec):
    """Wall time of the oracle's exact IPM solve (a dense Cholesky factor of
    the Schur complement Q + B^T D^-1 B at every Newton step) of this
    workload, as measured when tests/golden/make_golden.py stored its
    solution: a full solve of that size does not fit the bench's time budget,
    so it is read back with the host it ran on, not re-measured here."""
    names = {"rt_200000x20000_nnz0.5pct_maxdose10000": "rt_full.json"}
    path = os.path.join(ROOT, "tests", "golden", names.get(spec.name, ""))
    if spec.name not in names or not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    return {"ipm_iterations": rec["iterations"], "objective": rec["objective"],
            "timings": [{k: t[k] for k in ("threads", "ipm_seconds", "form_H_seconds", "nproc", "cpu")
                         if k in t} for t in rec.get("timings", [])],
            "how": "measured on the host that wrote tests/golden/rt_full.json (not this run)"}


def stream_rates(nbytes, reps=20):
    """Plain device copy and read (torch's copy and sum) of the dominant
    kernel's working-set size, timed with events on the current stream: the
    measured bandwidth beside the nominal peak."""
    import torch
    n = max(1, int(nbytes) // 8)
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
        a.sum()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(reps):
        b.copy_(a)
    ev[1].record()
    ev[2].record()
    for _ in range(reps):
        a.sum()
    ev[3].record()
    torch.cuda.synchronize()
    copy_s = ev[0].elapsed_time(ev[1]) / 1e3 / reps
    read_s = ev[2].elapsed_time(ev[3]) / 1e3 / reps
    del a, b
    return {"bytes": 8 * n, "copy_GBs": 2 * 8 * n / copy_s / 1e9, "read_GBs": 8 * n / read_s / 1e9,
            "how": "torch copy_ (read + write counted) and sum (read) of a float64 tensor "
                   "of this many bytes, mean of 20 after 3 warm-up"}


def main():
    args = parse()
    if args.summarize_stats:
        summarize_stats(args.summarize_stats, args.command)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.bench_json, args.command)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.bench_json, args.command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this method's solve runs on a single "
              "MI355X; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch3":
        bench_batch(args)
        return
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
        opts = default_ipm_options(mu_rule=1 if args.mu_rule == "mehrotra" else 0)
        for w in range(args.warmup):
            out = qp.solve(opts, want_state=False)
            inf = out["info"]
            print(f"[bench] warmup {w}: ipm={inf.iterations} cg={inf.total_cg_iters} "
                  f"{inf.time_ms / 1e3:.2f}s", file=sys.stderr, flush=True)
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
        graph = qp.graph_stats()
        # one more solve with a sample of dispatches timed by events, for the
        # per-kernel figures (the timed steps above replay their PCG chunks
        # from a graph, which event-timed launches cannot join)
        qp.profile_begin(args.profile_cap, args.profile_every)
        pout = qp.solve(opts, want_state=False)
        torch.cuda.synchronize()
        prof = qp.profile_end()
        prof_cg = pout["info"].total_cg_iters
        print(f"[bench] profiled solve: ipm={pout['info'].iterations} cg={prof_cg} "
              f"{pout['info'].time_ms / 1e3:.2f}s", file=sys.stderr, flush=True)
        ob = qp.operator_bytes()
        lay = qp.operator_layout()
        fz = qp.fused_layout()
        calib = 0
        if args.copy_calib_mb > 0:
            calib = args.copy_calib_mb * (1 << 20)
            nb = calib // 8
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
    for cat, (cnt, ms, seen) in prof.items():
        if cnt:
            # mean over the sampled dispatches (what a profiler's statistics
            # show), and the kernel time per CG iteration: the dispatches queued
            # past a converged PCG solve exit at once, so the whole category's
            # time (mean x dispatches) is spread over the real iterations
            avg_s = ms / cnt / 1e3
            per_it = avg_s * seen / prof_cg
            by = kernel_bytes(spec, ob, lay, cat, prec_bytes, fz)
            kern[cat] = {"launches_timed": cnt, "dispatches": seen, "dispatch_avg_us": avg_s * 1e6,
                         "avg_us": per_it * 1e6, "bytes": by, "GBs": by / per_it / 1e9}
    dom = max(kern, key=lambda c: kern[c]["avg_us"])
    d = kern[dom]
    with torch.cuda.stream(stream):
        rates = stream_rates(d["bytes"])
    per_iter_us = sum(v["avg_us"] for v in kern.values())
    wall_us = solve_s / max(1, total_cg) * 1e6
    # The roofline unit is one PCG iteration (every PCG kernel above, in
    # order): its algorithmic bytes over the kernel time per iteration.
    it_bytes = iteration_bytes(spec, args.precision)
    achieved = it_bytes / (per_iter_us * 1e-6) / 1e9
    measured = [stored_traffic(args.workload, args.precision, c) for c in kern]
    traffic = sum(measured) if measured and all(t is not None for t in measured) else None
    dom_traffic = stored_traffic(args.workload, args.precision, dom)
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
        "config": {"workload": spec.name, "mu_rule": args.mu_rule, "n": spec.n, "m": spec.m, "me": spec.me,
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
        "roofline": {"bound": "hbm", "kernel": "pcg_iteration (" + " + ".join(kern) + ")",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_over_algorithmic": traffic / it_bytes if traffic else None,
                     "algorithmic_bytes_per_iteration": it_bytes,
                     "kernel_us_per_iteration": per_iter_us, "wall_us_per_iteration": wall_us,
                     "frac_wall": it_bytes / (wall_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "measured_stream": rates,
                     "frac_of_copy": achieved / rates["copy_GBs"],
                     "dominant_kernel": {"name": dom, "dispatch_avg_us": d["dispatch_avg_us"],
                                         "avg_us": d["avg_us"], "bytes_per_launch": d["bytes"],
                                         "GBs": d["GBs"], "frac_of_peak": d["GBs"] / HBM_PEAK_GBS,
                                         "frac_of_copy": d["GBs"] / rates["copy_GBs"],
                                         "traffic": dom_traffic,
                                         "launches_timed": d["launches_timed"]}},
        "kernels": kern,
        "layout": lay,
        "fused": fz,
        "copy_calibration_bytes": calib,
        "pcg_graph": {"captures": graph[0], "replays": graph[1]},
        "profiled_solve_s": pout["info"].time_ms / 1e3,
        "pcg_kernel_us_per_iteration": per_iter_us,
        "pcg_wall_us_per_iteration": wall_us,
        # the same count over the time inside the PCG solves only (the IPM's
        # own kernels and host steps excluded); `value` keeps the whole solve
        "pcg_iters_per_s_inside_pcg": total_cg / max(1e-9, sum(i.pcg_time_ms for i in infos) / 1e3),
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(spec, args.cpu_iters)
    print(json.dumps(result), flush=True)


def bench_batch(args):
    """Batched PCG throughput at the uneven batch's shapes (256 dense QPs,
    n ~ U{500..8000}, m ~ U{n..2n}, G of n/2 x n, float32 storage): a stratified
    subset of them, each running one IPM iteration whose PCG is held to
    --batch-cg iterations (a whole solve of this batch takes hundreds of
    thousands of PCG iterations per instance), once with one workgroup per
    instance and once with the autotuner's teams.  `value` is PCG iterations
    per second over the batch with the teams; the bytes are each instance's
    operator per PCG iteration (A twice, U twice, float32)."""
    import tempfile
    import torch
    from paper_2308_00637_amd import workloads as W
    from paper_2308_00637_amd.qpk import QPBatch, default_ipm_options, default_pcg_options

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    specs = []
    for k in range(args.batch_take):   # one stratum at a time, keeping host memory to the data
        sp = W.batch_stratified(3, 256, args.batch_take, strata=[k])[0]
        sp.extra.clear()
        specs.append(sp)
        if (k + 1) % 16 == 0:
            print(f"[bench] {k + 1} instances generated ({time.perf_counter() - t0:.0f}s)",
                  file=sys.stderr, flush=True)
    print(f"[bench] {len(specs)} instances generated in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    per_it = [4 * (2 * sp.m * sp.n + 2 * sp.n * sp.U.shape[1]) for sp in specs]
    ns, ms = [sp.n for sp in specs], [sp.m for sp in specs]
    qb = QPBatch(specs, precision="fp32")
    for sp in specs:   # the device holds the operators now
        sp.A = sp.U = None
    opts = default_ipm_options(max_iter=1, pcg=default_pcg_options(tol=1e-300, maxit=args.batch_cg))

    def run(label):
        infos, st = qb.solve(opts)
        if st != 0:
            raise RuntimeError(f"batched solve returned {st}")
        ms = infos[0].time_ms
        cg = sum(f.total_cg_iters for f in infos)
        byts = sum(b * f.total_cg_iters for b, f in zip(per_it, infos))
        wg, teams = qb.launch_shape()
        # the launch's timeline from the device clock: how much of the
        # workgroups' time went to solving and when the last instance began
        t0, t1, g = qb.instance_times()
        span = max(t1)
        busy = sum(gi * (b - a) for a, b, gi in zip(t0, t1, g))
        longest = max(range(len(t0)), key=lambda i: t1[i] - t0[i])
        timeline = {"span_ms": span, "last_start_ms": max(t0),
                    "busy_fraction": busy / (wg * span) if span > 0 else None,
                    "longest_ms": t1[longest] - t0[longest], "longest_n": ns[longest],
                    "longest_team": g[longest]}
        print(f"[bench] {label}: {wg} workgroups, {teams} teams, {ms:.1f} ms, {cg} PCG iterations; "
              f"busy {timeline['busy_fraction']:.2f}, last start {timeline['last_start_ms']:.0f} ms, "
              f"longest {timeline['longest_ms']:.0f} ms (n {ns[longest]}, team {g[longest]})",
              file=sys.stderr, flush=True)
        return {"ms": ms, "pcg_iterations": cg, "pcg_iters_per_s": cg / (ms / 1e3),
                "GBs": byts / (ms / 1e3) / 1e9, "workgroups": wg, "teams": teams,
                "timeline": timeline}

    run("warm-up, one workgroup per instance")
    solo = run("one workgroup per instance")
    table = args.tune_table or os.path.join(tempfile.gettempdir(), "qpk_team_table.txt")
    t0 = time.perf_counter()
    sizes, probes = qb.autotune(table)
    tune_s = time.perf_counter() - t0
    print(f"[bench] autotune: {probes} measurements in {tune_s:.1f}s, team sizes {sizes}",
          file=sys.stderr, flush=True)
    run("warm-up, teams")
    team = run("teams")
    achieved = team["GBs"]
    result = {
        "metric": "batched PCG iterations/s at the uneven batch's shapes; achieved HBM GB/s vs peak",
        "value": team["pcg_iters_per_s"],
        "unit": "PCG iters/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": team["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 operator / f64",
        "data": "synthetic",
        "config": {"workload": f"batch_stratified_{len(specs)}_of_256", "n": ns,
                   "m": ms, "pcg_iterations_per_instance": args.batch_cg},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_sweep": sum(per_it)},
        "teams": {"sizes": sizes, "measurements": probes, "autotune_s": tune_s, **team},
        "one_workgroup_per_instance": solo,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
