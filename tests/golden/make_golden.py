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


MAKERS = {"svm_full": svm_full, "tiny_dense": tiny_dense, "rt_small": rt_small}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(MAKERS)):
        out = MAKERS[name]()
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(out, f)
        print(name, out["status"], out["iterations"], out["objective"], flush=True)
