"""Writes the stored expected values under tests/golden/ by running the CPU
oracle (and the seeded generators) only.  Run from the repository root:
    python tests/golden/make_golden.py [name ...]
Each fixture records the generator call it was made from."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2308_00637_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def svm_full():
    spec = W.svm_full()
    prob = O.from_spec(spec)
    d = lambda pr, st, mu, res: O.woodbury_direction(pr, st, mu, res, h0=spec.h0, U=spec.U, wd=spec.wd)
    t = time.perf_counter()
    r = O.solve(prob, direction=d)
    return dict(generator="workloads.svm_full()", oracle="oracle.solve with woodbury_direction",
                status=r.status, iterations=r.iterations, mu_final=r.mu, objective=r.objective,
                w_svm=(spec.U.T @ r.state.x).tolist(), sum_alpha=float(r.state.x.sum()),
                rnorm=r.log[-1]["rnorm"], seconds=time.perf_counter() - t)


def tiny_dense():
    spec = W.tiny_dense(0)
    r = O.solve(O.from_spec(spec))
    return dict(generator="workloads.tiny_dense(0)", oracle="oracle.solve (dense Cholesky)",
                status=r.status, iterations=r.iterations, mu_final=r.mu, objective=r.objective,
                x=r.state.x.tolist(), rnorm=r.log[-1]["rnorm"])


def rt_small():
    spec = W.rt_small(4)
    r = O.solve(O.from_spec(spec))
    return dict(generator="workloads.rt_small(4)", oracle="oracle.solve (dense Cholesky)",
                status=r.status, iterations=r.iterations, mu_final=r.mu, objective=r.objective,
                x=r.state.x.tolist(), rnorm=r.log[-1]["rnorm"])


def _host():
    import platform
    import subprocess
    lscpu = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
    model = next((ln.split(":", 1)[1].strip() for ln in lscpu.splitlines()
                  if ln.startswith("Model name")), platform.processor())
    return dict(nproc=os.cpu_count(), cpu=model, numpy=np.__version__)


def rt_full():
    """The 200,000 x 20,000 radiation-therapy QP solved by the oracle's IPM with
    exact Newton directions: the Schur complement Q + B^T D^-1 B (n = 20,000)
    factored densely by Cholesky at every step.  QPK_ORACLE_THREADS limits
    the BLAS threads (the survey asks for one thread and for all cores); with
    QPK_GOLDEN_TIME_ONLY=1 an existing rt_full.json only gains the time of
    this run (the solve must reproduce its objective)."""
    from threadpoolctl import threadpool_limits
    threads = int(os.environ.get("QPK_ORACLE_THREADS", "0")) or os.cpu_count()
    spec = W.rt_full()
    prob = O.from_spec(spec)
    steps = []

    def direction(pr, st, mu, res):
        t0 = time.perf_counter()
        d = O.schur_direction(pr, st, mu, res)
        steps.append(time.perf_counter() - t0)
        print(f"  newton step {len(steps)}: mu={mu:.1e} {steps[-1]:.1f}s", flush=True)
        return d

    with threadpool_limits(limits=threads):
        t = time.perf_counter()
        prob.Hdense()   # P^T W P, formed once (outside the IPM loop)
        t_h = time.perf_counter() - t
        t = time.perf_counter()
        r = O.solve(prob, direction=direction)
        secs = time.perf_counter() - t
    timing = dict(threads=threads, ipm_seconds=secs, form_H_seconds=t_h,
                  newton_step_seconds=steps, **_host())
    path = os.path.join(HERE, "rt_full.json")
    if os.environ.get("QPK_GOLDEN_TIME_ONLY") == "1":
        with open(path) as f:
            out = json.load(f)
        assert abs(r.objective - out["objective"]) <= 1e-12 * abs(out["objective"])
        out.setdefault("timings", []).append(timing)
        return out
    res = O.residuals(prob, r.state, r.mu)
    pr, du, co = O.infeasibilities(res)
    return dict(generator="workloads.rt_full()",
                oracle="oracle.solve with schur_direction (dense Cholesky of Q + B^T D^-1 B)",
                status=r.status, iterations=r.iterations, mu_final=r.mu, objective=r.objective,
                rnorm=O.stacked_norm(res), primal=pr, dual=du, compl=co,
                mus=[e["mu"] for e in r.log], x=r.state.x.tolist(),
                lam_uA=r.state.lam_uA.tolist(), timings=[timing])


MAKERS = {"svm_full": svm_full, "tiny_dense": tiny_dense, "rt_small": rt_small,
          "rt_full": rt_full}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(MAKERS)):
        out = MAKERS[name]()
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(out, f)
        print(name, out["status"], out["iterations"], out["objective"], flush=True)
