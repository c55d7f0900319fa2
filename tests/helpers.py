"""Shared test helpers: random interior states and conversions between the
oracle's compact block layout and the library's full-length masked layout.
No solver arithmetic lives here."""
import numpy as np

import oracle as O


def random_state(prob, rng, spread=1.0):
    """An arbitrary strictly interior iterate (positive slacks/multipliers)."""
    S = O.index_sets(prob)
    pos = lambda k: np.exp(spread * rng.standard_normal(k))
    return O.State(
        x=rng.standard_normal(prob.n), lam_e=rng.standard_normal(prob.me),
        lam_lA=pos(S.L.size), lam_uA=pos(S.U.size),
        lam_lx=pos(S.Lx.size), lam_ux=pos(S.Ux.size),
        s_lA=pos(S.L.size), s_uA=pos(S.U.size),
        s_lx=pos(S.Lx.size), s_ux=pos(S.Ux.size))


def to_masked(prob, st):
    """Compact oracle state -> library layout:
    x (n); lam = [lam_e (me) | lam_lA (m) | lam_uA (m) | lam_lx (n) | lam_ux (n)];
    s = [s_lA (m) | s_uA (m) | s_lx (n) | s_ux (n)]; absent sides hold 0."""
    S = O.index_sets(prob)
    n, m, me = prob.n, prob.m, prob.me
    lam = np.zeros(me + 2 * m + 2 * n)
    s = np.zeros(2 * m + 2 * n)
    lam[:me] = st.lam_e
    lam[me + S.L] = st.lam_lA
    lam[me + m + S.U] = st.lam_uA
    lam[me + 2 * m + S.Lx] = st.lam_lx
    lam[me + 2 * m + n + S.Ux] = st.lam_ux
    s[S.L] = st.s_lA
    s[m + S.U] = st.s_uA
    s[2 * m + S.Lx] = st.s_lx
    s[2 * m + n + S.Ux] = st.s_ux
    return np.array(st.x), lam, s


def from_masked(prob, x, lam, s):
    S = O.index_sets(prob)
    n, m, me = prob.n, prob.m, prob.me
    return O.State(
        x=np.array(x), lam_e=np.array(lam[:me]),
        lam_lA=lam[me + S.L], lam_uA=lam[me + m + S.U],
        lam_lx=lam[me + 2 * m + S.Lx], lam_ux=lam[me + 2 * m + n + S.Ux],
        s_lA=s[S.L], s_uA=s[m + S.U], s_lx=s[2 * m + S.Lx], s_ux=s[2 * m + n + S.Ux])


def kkt_to_masked(prob, v):
    """Compact doubly augmented vector (x | lam_e | lam_lA | lam_uA) -> the
    library's (x | lam_e | lam_l over all m rows | lam_u over all m rows)."""
    S = O.index_sets(prob)
    n, m, me = prob.n, prob.m, prob.me
    out = np.zeros(n + me + 2 * m)
    out[:n + me] = v[:n + me]
    out[n + me + S.L] = v[n + me:n + me + S.L.size]
    out[n + me + m + S.U] = v[n + me + S.L.size:]
    return out


def kkt_from_masked(prob, v):
    S = O.index_sets(prob)
    n, m, me = prob.n, prob.m, prob.me
    return np.concatenate([v[:n + me], v[n + me + S.L], v[n + me + m + S.U]])


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def res_to_masked(prob, res):
    """Oracle residual blocks -> the library's residual stack
    [rH n | re me | rlA m | ruA m | rlx n | rux n | rc1 m | rc2 m | rc3 n | rc4 n]."""
    S = O.index_sets(prob)
    n, m, me = prob.n, prob.m, prob.me
    out = []
    out.append(res.rH)
    out.append(res.re)
    for idx, blk, size in ((S.L, res.rlA, m), (S.U, res.ruA, m), (S.Lx, res.rlx, n),
                           (S.Ux, res.rux, n), (S.L, res.rc1, m), (S.U, res.rc2, m),
                           (S.Lx, res.rc3, n), (S.Ux, res.rc4, n)):
        v = np.zeros(size)
        v[idx] = blk
        out.append(v)
    return np.concatenate(out)


def dir_to_masked(prob, d):
    """Oracle Direction -> (dx, dlam, ds) in the library's iterate layouts."""
    st = O.State(d.dx, d.dlam_e, d.dlam_lA, d.dlam_uA, d.dlam_lx, d.dlam_ux,
                 d.ds_lA, d.ds_uA, d.ds_lx, d.ds_ux)
    return to_masked(prob, st)


def block_rel(a, b, sizes):
    """Largest relative error over consecutive blocks of the given sizes, each
    measured against its own norm (floored at 1e-14 of the whole vector's,
    so blocks that are rounding noise compare absolutely): an error confined
    to a block of small magnitude is not hidden by a large one elsewhere."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape and sum(sizes) == b.size, (a.shape, b.shape, sizes)
    floor = max(1e-14 * np.linalg.norm(b), 1e-300)
    worst, o = 0.0, 0
    for k in sizes:
        if k:
            worst = max(worst, float(np.linalg.norm(a[o:o + k] - b[o:o + k])
                                     / max(np.linalg.norm(b[o:o + k]), floor)))
        o += k
    return worst


def kkt_blocks(prob):
    """Block sizes of a compact doubly augmented vector: x, lam_e, lam_lA, lam_uA."""
    S = O.index_sets(prob)
    return [prob.n, prob.me, S.L.size, S.U.size]


def res_blocks(prob):
    """Block sizes of the library's residual stack (masked layout)."""
    n, m, me = prob.n, prob.m, prob.me
    return [n, me, m, m, n, n, m, m, n, n]


def lam_blocks(prob):
    n, m, me = prob.n, prob.m, prob.me
    return [me, m, m, n, n]


def s_blocks(prob):
    n, m = prob.n, prob.m
    return [m, m, n, n]
