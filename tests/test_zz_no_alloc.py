"""ipm_solve_dense_noalloc, the entry point that allocates nothing (its
workspace is a fixed device array of the library), against the batched solve
it shares its kernel with (ipm_solve_batch on a batch of that one instance):
the same steps on the same data, so the results agree bitwise.  Two calls in a
row, the second smaller, then the first again (the array keeps the previous
call's contents); also against the oracle's solve.  The errors: a problem too
large for the array, and invalid bounds checked on the device."""
import numpy as np
import pytest

import oracle as O
from paper_2308_00637_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def noalloc(spec):
    from paper_2308_00637_amd.qpk import ipm_solve_dense_noalloc
    return ipm_solve_dense_noalloc(dev(spec.H), dev(spec.c), dev(spec.A), dev(spec.lA), dev(spec.uA),
                                   dev(spec.lx), dev(spec.ux))


def batched(spec):
    from paper_2308_00637_amd.qpk import QPBatch
    b = QPBatch([spec])
    infos, st = b.solve()
    x, lam, s = b.solution(0)
    return dict(x=x, lam=lam, s=s, info=infos[0], status=st)


CASES = [(51, 120, 200), (52, 40, 60), (51, 120, 200)]   # the second smaller, then the first again


@pytest.mark.parametrize("seed,n,m", CASES)
def test_noalloc_matches_batched_solve_bitwise(seed, n, m):
    spec = W.random_bounded_qp(seed, n, m, 0, max(2, n // 3))
    a = noalloc(spec)
    b = batched(spec)
    ia, ib = a["info"], b["info"]
    print(f"n={n} m={m}: ipm {ia.iterations}/{ib.iterations} cg {ia.total_cg_iters}/{ib.total_cg_iters} "
          f"obj {ia.objective:.12g}/{ib.objective:.12g}", flush=True)
    assert a["status"] == b["status"] == 0
    assert ia.result == ib.result == 0
    assert (ia.iterations, ia.total_cg_iters, ia.cg_maxiter_hits) == \
        (ib.iterations, ib.total_cg_iters, ib.cg_maxiter_hits)
    assert (ia.objective, ia.mu_final, ia.rnorm) == (ib.objective, ib.mu_final, ib.rnorm)
    for k in ("x", "lam", "s"):
        assert torch.equal(a[k], b[k]), k
    ref = O.solve(O.from_spec(spec))
    assert abs(ia.objective - ref.objective) <= 1e-6 * max(1.0, abs(ref.objective))


def workspace_values(n, m):
    """float64 values of the solver's per-instance block (29 n + 31 m)."""
    return 29 * n + 31 * m


def test_noalloc_rejects_a_problem_larger_than_its_array():
    """The size check runs on the host before any launch, so H is not read;
    the sizes are chosen (and checked here first) to need well over the 16 MiB
    array, as H here is far smaller than n x n."""
    from paper_2308_00637_amd.qpk import QPError, QP_ERR_ARG, ipm_solve_dense_noalloc
    n, m = 60_000, 60_000
    assert 8 * workspace_values(n, m) > 1.5 * (16 << 20)
    c = torch.zeros(n, dtype=torch.float64, device="cuda")
    H = torch.zeros(1, dtype=torch.float64, device="cuda")
    A = torch.zeros(m, dtype=torch.float64, device="cuda").reshape(m, 1)
    lA = torch.zeros(m, dtype=torch.float64, device="cuda")
    with pytest.raises(QPError) as e:
        ipm_solve_dense_noalloc(H, c, A, lA, lA)
    assert e.value.status == QP_ERR_ARG and "bytes of workspace" in str(e.value)


def test_noalloc_rejects_invalid_bounds_on_the_device():
    from paper_2308_00637_amd.qpk import QPError, QP_ERR_ARG
    spec = W.random_bounded_qp(53, 30, 20, 0, 10)
    spec.lA = spec.lA.copy()
    spec.uA = spec.uA.copy()
    spec.lA[3], spec.uA[3] = 1.0, 0.5     # lower side above the upper side
    with pytest.raises(QPError) as e:
        noalloc(spec)
    assert e.value.status == QP_ERR_ARG
    # the array is usable again afterwards
    ok = W.random_bounded_qp(52, 40, 60, 0, 13)
    assert noalloc(ok)["info"].result == 0
