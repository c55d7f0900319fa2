"""The seeded generators build the shapes and structure the workloads are
described with (CPU only): the radiation-therapy recipe's max-dose rows are
rows of P (the structure the blocked passes fold), its weights, targets and
row lengths follow the recipe, and the generators are reproducible."""
import numpy as np
import pytest

from paper_2308_00637_amd import workloads as W


@pytest.fixture(scope="module")
def rt():
    return W.rt_small(4)


def test_rt_max_dose_rows_are_rows_of_p(rt):
    K = rt.extra["maxdose_rows"]
    assert np.all(np.diff(K) > 0)                       # sorted, without repeats
    assert len(K) == rt.m == 1_000
    A, P = rt.A.tocsr(), rt.P.tocsr()
    assert (A != P[K]).nnz == 0
    assert np.array_equal(A.indptr, P[K].indptr) and np.array_equal(A.data, P[K].data)


def test_rt_recipe(rt):
    P = rt.P.tocsr()
    n_vox, n = P.shape
    assert (n_vox, n) == (20_000, 2_000)
    lengths = np.diff(P.indptr)
    # Binomial(2000, 0.005) before merging duplicate columns: mean 10
    assert 9.0 < lengths.mean() < 10.5
    for r in range(0, n_vox, 997):                      # columns sorted, in range
        c = P.indices[P.indptr[r]:P.indptr[r + 1]]
        assert np.all(np.diff(c) > 0) and (len(c) == 0 or (c[0] >= 0 and c[-1] < n))
    assert np.all(P.data > 0)
    assert set(np.unique(rt.w)) <= {1.0, 10.0} and 0.08 < np.mean(rt.w == 10.0) < 0.12
    assert np.all((rt.d >= 0.0) & (rt.d < 1.0))
    assert np.all(rt.uA == 1.1) and np.all(np.isneginf(rt.lA))
    assert np.all(rt.lx == 0.0) and np.all(np.isposinf(rt.ux))


def test_generators_are_reproducible():
    a, b = W.rt_qp(3, 500, 60, 0.05, 10), W.rt_qp(3, 500, 60, 0.05, 10)
    assert (a.P != b.P).nnz == 0 and np.array_equal(a.w, b.w) and np.array_equal(a.d, b.d)
    c = W.rt_qp(4, 500, 60, 0.05, 10)
    assert (a.P != c.P).nnz > 0
