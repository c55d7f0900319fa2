"""Seeded synthetic QP workloads.

This module only draws random problem data; it holds none of the solver's
arithmetic.  Both the HIP path (through the binding) and the CPU oracle read
the same `QPSpec`, each converting it with code of its own.

The QP form is the one of the paper's eq. (1) (Section 2.1), with variable
bounds kept apart from the general rows as in Section 3.1:

    min 1/2 x^T H x + c^T x   s.t.  lA <= A x <= uA,  C x = b,  lx <= x <= ux

Infinite entries of lA/uA/lx/ux mean "no bound on that side".

Hessian forms (`h_kind`):
  * "dense"   : H given as an n x n symmetric matrix.
  * "lowrank" : H = diag(h0) + U diag(wd) U^T with U dense n x k (the
                quasi-Newton form H0 + U W U^T of Section 2.2).
  * "ptwp"    : H = P^T diag(w) P with P sparse (rows = voxels); the
                objective is 1/2 sum_v w_v (P_v x - d_v)^2 + c^T x, so the
                linear term seen by the method is c - P^T W d.

The radiation-therapy-shaped and SVM-shaped instances are synthetic stand-ins
for the paper's RayStation and LIBSVM a1a problems (Section 4, Table 1), which
are not available; they reproduce shapes and value distributions only.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class QPSpec:
    n: int
    c: np.ndarray
    h_kind: str
    H: Optional[np.ndarray] = None            # dense
    h0: Optional[np.ndarray] = None           # lowrank
    U: Optional[np.ndarray] = None
    wd: Optional[np.ndarray] = None
    P: Optional[sp.csr_matrix] = None         # ptwp
    w: Optional[np.ndarray] = None
    d: Optional[np.ndarray] = None
    A: object = None                          # None, dense ndarray or csr_matrix
    lA: Optional[np.ndarray] = None
    uA: Optional[np.ndarray] = None
    C: Optional[np.ndarray] = None            # dense (me x n)
    b: Optional[np.ndarray] = None
    lx: Optional[np.ndarray] = None
    ux: Optional[np.ndarray] = None
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return 0 if self.A is None else int(self.A.shape[0])

    @property
    def me(self) -> int:
        return 0 if self.C is None else int(self.C.shape[0])

    def __post_init__(self):
        n = self.n
        if self.lx is None:
            self.lx = np.full(n, -np.inf)
        if self.ux is None:
            self.ux = np.full(n, np.inf)
        if self.A is not None:
            m = self.A.shape[0]
            if self.lA is None:
                self.lA = np.full(m, -np.inf)
            if self.uA is None:
                self.uA = np.full(m, np.inf)
        if self.C is not None and self.b is None:
            self.b = np.zeros(self.C.shape[0])


def _to_f32(a: np.ndarray) -> np.ndarray:
    """Round to the nearest float32 value, kept in float64 storage."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def dense_qp(rng: np.random.Generator, n: int, m: int, mg: int,
             round_f32: bool = False, name: str = "") -> QPSpec:
    """Dense QP with H = G^T G + 1e-3 I, Ax >= b strictly feasible at x0.

    Draw order: G (mg x n), c (n), A (m x n), x0 (n), slack u (m) ~ U(0.1, 1);
    b = A x0 - u so x0 satisfies every row with margin >= 0.1.
    """
    G = rng.standard_normal((mg, n))
    c = rng.standard_normal(n)
    A = rng.standard_normal((m, n))
    x0 = rng.standard_normal(n)
    u = rng.uniform(0.1, 1.0, m)
    if round_f32:
        G, c, A, x0, u = (_to_f32(v) for v in (G, c, A, x0, u))
    b = A @ x0 - u
    if round_f32:
        b = _to_f32(b)
    return QPSpec(n=n, c=c, h_kind="lowrank", h0=np.full(n, 1e-3),
                  U=np.ascontiguousarray(G.T), wd=np.ones(mg),
                  A=A, lA=b, uA=np.full(m, np.inf), name=name,
                  extra={"x0": x0, "G": G})


def tiny_dense(seed: int = 0) -> QPSpec:
    """Tiny dense QP: n=200, H=G^T G+1e-3 I with G 100x200, A 400x200, Ax>=b."""
    return dense_qp(np.random.default_rng(seed), 200, 400, 100, name="tiny_dense_n200_m400")


def sparse_rows(rng: np.random.Generator, nrows: int, ncols: int,
                density: float) -> sp.csr_matrix:
    """Random CSR with Binomial(ncols, density) entries per row.

    Column positions are uniform draws; duplicates within a row are merged
    away (so a row keeps slightly fewer entries), columns are sorted, and the
    values are log-normal exp(N(-3, 1)).
    """
    k = rng.binomial(ncols, density, size=nrows)
    rows = np.repeat(np.arange(nrows, dtype=np.int64), k)
    cols = rng.integers(0, ncols, size=rows.size, dtype=np.int64)
    key = rows * ncols + cols
    key = np.unique(key)                       # sorts and removes duplicates
    rows = key // ncols
    cols = (key - rows * ncols).astype(np.int32)
    vals = np.exp(rng.normal(-3.0, 1.0, size=key.size))
    indptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nrows), out=indptr[1:])
    return sp.csr_matrix((vals, cols, indptr.astype(np.int32)), shape=(nrows, ncols))


def rt_qp(seed: int, n_vox: int, n_beam: int, density: float, n_maxdose: int,
          maxdose: float = 1.1, name: str = "") -> QPSpec:
    """Radiation-therapy-shaped QP.

    objective 1/2 sum_v w_v (P_v x - d_v)^2 with P sparse (voxels x beamlets),
    w_v = 10 with probability 0.1 else 1, d ~ U(0, 1); constraints x >= 0 and
    max-dose rows P_k x <= maxdose on a sorted uniform sample of voxels.
    Draw order: P (row lengths, columns, values), w, d, max-dose voxel set.
    """
    rng = np.random.default_rng(seed)
    P = sparse_rows(rng, n_vox, n_beam, density)
    w = np.where(rng.random(n_vox) < 0.1, 10.0, 1.0)
    d = rng.uniform(0.0, 1.0, n_vox)
    K = np.sort(rng.choice(n_vox, size=n_maxdose, replace=False))
    A = P[K].tocsr()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    m = A.shape[0]
    return QPSpec(n=n_beam, c=np.zeros(n_beam), h_kind="ptwp", P=P, w=w, d=d,
                  A=A, lA=np.full(m, -np.inf), uA=np.full(m, maxdose),
                  lx=np.zeros(n_beam), ux=np.full(n_beam, np.inf), name=name,
                  extra={"maxdose_rows": K})


def rt_full(seed: int = 1) -> QPSpec:
    """200,000 voxels x 20,000 beamlets, 0.5% density, 10,000 max-dose rows."""
    return rt_qp(seed, 200_000, 20_000, 0.005, 10_000,
                 name="rt_200000x20000_nnz0.5pct_maxdose10000")


def rt_small(seed: int = 4) -> QPSpec:
    """20,000 voxels x 2,000 beamlets (~10 entries per row), 1,000 max-dose rows."""
    return rt_qp(seed, 20_000, 2_000, 0.005, 1_000,
                 name="rt_20000x2000_maxdose1000")


def svm_qp(seed: int, n_samples: int, n_feat: int, box: float = 1.0,
           name: str = "") -> QPSpec:
    """SVM-dual-shaped QP with a linear kernel.

    Labels y = +-1 with probability 1/2; features X_i ~ N(0.5 y_i 1, I) rounded
    to float32.  H = Z Z^T with Z = diag(y) X, c = -1, y^T alpha = 0,
    0 <= alpha <= box.  Draw order: y, X.
    """
    rng = np.random.default_rng(seed)
    y = np.where(rng.random(n_samples) < 0.5, 1.0, -1.0)
    X = _to_f32(rng.standard_normal((n_samples, n_feat)) + 0.5 * y[:, None])
    Z = y[:, None] * X
    return QPSpec(n=n_samples, c=-np.ones(n_samples), h_kind="lowrank",
                  h0=np.zeros(n_samples), U=Z, wd=np.ones(n_feat),
                  C=y[None, :].copy(), b=np.zeros(1),
                  lx=np.zeros(n_samples), ux=np.full(n_samples, box), name=name,
                  extra={"y": y})


def svm_rbf(seed: int = 7, n_samples: int = 1605, n_feat: int = 123, box: float = 1.0,
            name: str = "") -> QPSpec:
    """SVM dual with a precomputed dense RBF-kernel Hessian at the a1a shape of
    Table 1 (1,605 samples, one equality row, 3,210 bounds).  Synthetic
    two-Gaussian data stand in for a1a: y = +-1 with probability 1/2, features
    X_i ~ N(0.3 y_i 1, I); H_ij = y_i y_j exp(-g |X_i - X_j|^2) with
    g = 1 / n_feat.  Draw order: y, X.
    """
    rng = np.random.default_rng(seed)
    y = np.where(rng.random(n_samples) < 0.5, 1.0, -1.0)
    X = rng.standard_normal((n_samples, n_feat)) + 0.3 * y[:, None]
    sq = (X * X).sum(1)
    d2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * (X @ X.T), 0.0)
    H = np.exp(-d2 / n_feat) * np.outer(y, y)
    H = 0.5 * (H + H.T)
    return QPSpec(n=n_samples, c=-np.ones(n_samples), h_kind="dense", H=H,
                  C=y[None, :].copy(), b=np.zeros(1),
                  lx=np.zeros(n_samples), ux=np.full(n_samples, box),
                  name=name or f"svm_rbf_{n_samples}x{n_feat}", extra={"y": y, "X": X})


def svm_full(seed: int = 2) -> QPSpec:
    return svm_qp(seed, 500_000, 128, name="svm_500000x128")


def batch_sizes(seed: int = 3, count: int = 256, nmin: int = 500, nmax: int = 8000):
    """Per-instance (n, m, child seed) of the uneven batch: n ~ U{nmin..nmax},
    m ~ U{n..2n}, one spawned SeedSequence per instance."""
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for ch in children:
        r = np.random.default_rng(ch)
        n = int(r.integers(nmin, nmax + 1))
        m = int(r.integers(n, 2 * n + 1))
        out.append((n, m, r))
    return out


def batch_qps(seed: int = 3, count: int = 256, nmin: int = 500, nmax: int = 8000):
    """Uneven batch of dense QPs, each built like the tiny dense case with G
    of floor(n/2) x n, data rounded to float32."""
    return [dense_qp(r, n, m, n // 2, round_f32=True, name=f"batch{i}_n{n}_m{m}")
            for i, (n, m, r) in enumerate(batch_sizes(seed, count, nmin, nmax))]


def batch_stratified(seed: int = 3, count: int = 256, take: int = 32, nmin: int = 500,
                     nmax: int = 8000, strata=None):
    """`take` instances of the uneven batch above, spread evenly over its
    sizes: the batch's instances ranked by n, every (count / take)-th rank
    from the middle of each stratum; each is generated exactly as in the
    whole batch (same child seed).  `strata`: only these strata (0 = the
    smallest n)."""
    sizes = batch_sizes(seed, count, nmin, nmax)
    ranked = sorted(range(count), key=lambda i: (sizes[i][0], i))
    step = count / take
    ks = range(take) if strata is None else strata
    picks = sorted(ranked[int((k + 0.5) * step)] for k in ks)
    return [dense_qp(sizes[i][2], sizes[i][0], sizes[i][1], sizes[i][0] // 2, round_f32=True,
                     name=f"batch{i}_n{sizes[i][0]}_m{sizes[i][1]}") for i in picks]


def _csr_from_lengths(rng: np.random.Generator, lengths, ncols: int, col_hi: int) -> sp.csr_matrix:
    """CSR whose row i has lengths[i] distinct uniform columns in [0, col_hi),
    values exp(N(-3, 1))."""
    indptr = np.zeros(len(lengths) + 1, dtype=np.int64)
    cols = []
    for i, k in enumerate(lengths):
        c = np.sort(rng.choice(col_hi, size=int(k), replace=False)) if k else np.zeros(0, np.int64)
        cols.append(c)
        indptr[i + 1] = indptr[i] + len(c)
    cols = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    vals = np.exp(rng.normal(-3.0, 1.0, size=cols.size))
    return sp.csr_matrix((vals, cols, indptr.astype(np.int32)), shape=(len(lengths), ncols))


def ragged_qp(seed: int, n: int = 901, p_rows: int = 1503, m: int = 407) -> QPSpec:
    """Radiation-therapy-shaped QP with ragged structure: rows of P and A from
    empty to several hundred entries (longer than one batch of the blocked
    passes), the last tenth of the variables in no row of A, variables free,
    lower-, upper- and two-side bounded, rows two-sided, one-sided and free.
    Feasible around x0 ~ U(0.2, 0.8).

    Draw order: P lengths, P, A lengths, A, w, d, x0, variable bound kinds,
    row bound kinds, row margins, variable margins.
    """
    rng = np.random.default_rng(seed)
    pl = np.where(rng.random(p_rows) < 0.03, rng.integers(300, 600, p_rows), rng.poisson(25, p_rows))
    pl[rng.random(p_rows) < 0.05] = 0
    P = _csr_from_lengths(rng, np.minimum(pl, n), n, n)
    al = np.where(rng.random(m) < 0.1, rng.integers(150, 400, m), rng.poisson(6, m))
    al[rng.random(m) < 0.1] = 0
    col_hi = int(0.9 * n)
    A = _csr_from_lengths(rng, np.minimum(al, col_hi), n, col_hi)
    w = np.where(rng.random(p_rows) < 0.1, 10.0, 1.0)
    d = rng.uniform(0.0, 1.0, p_rows)
    x0 = rng.uniform(0.2, 0.8, n)
    vk = rng.integers(0, 4, n)                  # 0 free, 1 lower, 2 upper, 3 both
    rk = rng.integers(0, 4, m)                  # 0 both, 1 lower, 2 upper, 3 free row
    ax = A @ x0
    mlo, mhi = rng.uniform(0.05, 0.5, m), rng.uniform(0.05, 0.5, m)
    lA = np.where((rk == 0) | (rk == 1), ax - mlo, -np.inf)
    uA = np.where((rk == 0) | (rk == 2), ax + mhi, np.inf)
    vlo, vhi = rng.uniform(0.1, 0.2, n), rng.uniform(0.1, 0.2, n)
    lx = np.where((vk == 1) | (vk == 3), x0 - vlo, -np.inf)
    ux = np.where((vk == 2) | (vk == 3), x0 + vhi, np.inf)
    return QPSpec(n=n, c=np.zeros(n), h_kind="ptwp", P=P, w=w, d=d, A=A, lA=lA, uA=uA,
                  lx=lx, ux=ux, name=f"ragged_{n}x{p_rows}x{m}")


def qn_rt(seed: int = 6, n: int = 90_657, k: int = 20, m: int = 15) -> QPSpec:
    """Quasi-Newton radiation-therapy subproblem shape (the proton liver case
    of Table 1: 90,657 variables, 15 general rows, a bound on every variable):
    H = diag(h0) + U diag(w) U^T with mixed-sign w, as a limited-memory BFGS
    Hessian has, kept positive definite: h0 >= 0.5, the columns of U have norm
    about 1, and the negative weights sum to at most 0.4 in magnitude.
    Rows lA <= Ax <= uA two-sided around A x0, x >= 0.

    Draw order: h0, U, positive weights, negative weights, c, A, x0, row margins.
    """
    rng = np.random.default_rng(seed)
    h0 = rng.uniform(0.5, 1.5, n)
    U = rng.standard_normal((n, k)) / np.sqrt(n)
    kp = k - k // 2
    wpos = rng.uniform(0.5, 2.0, kp)
    wneg = -rng.uniform(0.2, 0.4, k - kp) / max(1, k - kp)
    c = rng.standard_normal(n)
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    x0 = rng.uniform(0.0, 1.0, n)
    ax = A @ x0
    mlo, mhi = rng.uniform(0.05, 0.5, m), rng.uniform(0.05, 0.5, m)
    return QPSpec(n=n, c=c, h_kind="lowrank", h0=h0, U=np.ascontiguousarray(U),
                  wd=np.concatenate([wpos, wneg]), A=A, lA=ax - mlo, uA=ax + mhi,
                  lx=np.zeros(n), ux=np.full(n, np.inf), name=f"qn_rt_{n}x{k}_m{m}")


def random_bounded_qp(seed: int, n: int, m: int, me: int, mg: int,
                      a_sparse: bool = False, two_sided: bool = True,
                      h_kind: str = "dense") -> QPSpec:
    """A general small QP exercising every block of the method: two-sided rows
    with some infinite sides, equality rows, and mixed variable bounds.
    Feasible by construction around a point x0."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((mg, n))
    c = rng.standard_normal(n)
    A = rng.standard_normal((m, n))
    if a_sparse:
        A = A * (rng.random((m, n)) < 0.3)
    x0 = rng.uniform(-0.5, 0.5, n)
    Ax0 = A @ x0
    lo = Ax0 - rng.uniform(0.1, 1.0, m)
    hi = Ax0 + rng.uniform(0.1, 1.0, m)
    side = rng.integers(0, 3, m) if two_sided else np.zeros(m, dtype=int)
    lA = np.where(side == 2, -np.inf, lo)     # side 0: both, 1: lower only, 2: upper only
    uA = np.where(side == 1, np.inf, hi)
    C = rng.standard_normal((me, n)) if me > 0 else None
    b = C @ x0 if me > 0 else None
    bside = rng.integers(0, 4, n)
    lx = np.where((bside == 0) | (bside == 1), x0 - rng.uniform(0.5, 2.0, n), -np.inf)
    ux = np.where((bside == 0) | (bside == 2), x0 + rng.uniform(0.5, 2.0, n), np.inf)
    kw = dict(n=n, c=c, A=(sp.csr_matrix(A) if a_sparse else A), lA=lA, uA=uA,
              C=C, b=b, lx=lx, ux=ux, name=f"general_n{n}_m{m}_me{me}",
              extra={"x0": x0, "G": G})
    if h_kind == "dense":
        return QPSpec(h_kind="dense", H=G.T @ G + 1e-2 * np.eye(n), **kw)
    return QPSpec(h_kind="lowrank", h0=np.full(n, 1e-2), U=np.ascontiguousarray(G.T),
                  wd=np.ones(mg), **kw)
