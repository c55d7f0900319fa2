"""Python binding of libqpk (include/qpk.h): argument marshalling only.

Every call goes straight to the C ABI; device arrays are torch CUDA (HIP)
tensors, passed by data pointer on torch's current stream.  There is no
fallback: if libqpk.so is missing or cannot be loaded, importing this module
raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpk.so")

QP_OK = 0
QP_ERR_ARG = -1
QP_ERR_ALLOC = -2
QP_ERR_HIP = -3
QP_ERR_NOT_SPD = -4
QP_ERR_NUMERIC = -5
QP_ERR_STATE = -6
QP_ERR_UNSUPPORTED = -7
QP_MU_PAPER = 0
QP_MU_MEHROTRA = 1

H_DENSE, H_LOWRANK, H_PTWP = 0, 1, 2
A_NONE, A_DENSE, A_CSR = 0, 1, 2
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "fp32x64": 3, "bf16x64": 4}

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


class QpDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("m", C.c_int64), ("me", C.c_int64), ("h_kind", C.c_int32),
        ("H", _dp), ("k", C.c_int64), ("h0", _dp), ("U", _dp), ("wd", _dp),
        ("p_rows", C.c_int64), ("p_rowptr", _i64p), ("p_col", _i32p), ("p_val", _dp),
        ("p_w", _dp), ("p_d", _dp), ("c", _dp), ("a_kind", C.c_int32), ("A", _dp),
        ("a_rowptr", _i64p), ("a_col", _i32p), ("a_val", _dp), ("lA", _dp), ("uA", _dp),
        ("C", _dp), ("b", _dp), ("lx", _dp), ("ux", _dp), ("precision", C.c_int32),
    ]


class PcgOptions(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("check_every", C.c_int32),
                ("rr_period", C.c_int32), ("spectrum", C.c_int32), ("no_precond", C.c_int32)]


class PcgInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("status", C.c_int32),
                ("rel_residual", C.c_double), ("rhs_norm", C.c_double), ("escalated", C.c_int32),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double)]


class IpmOptions(C.Structure):
    _fields_ = [
        ("gamma", C.c_double), ("mu0", C.c_double), ("mu_tol", C.c_double),
        ("mu_div", C.c_double), ("max_iter", C.c_int32), ("warm_start", C.c_int32),
        ("pcg", PcgOptions), ("log_capacity", C.c_int32),
        ("log_mu", _dp), ("log_rnorm", _dp), ("log_primal", _dp), ("log_dual", _dp),
        ("log_compl", _dp), ("log_alpha_x", _dp), ("log_alpha_lam", _dp),
        ("log_cg_iters", _i32p), ("log_cg_relres", _dp), ("log_kappa", _dp),
        ("log_kappa_plain", _dp), ("mu_rule", C.c_int32), ("log_sigma", _dp),
    ]


class IpmInfo(C.Structure):
    _fields_ = [
        ("result", C.c_int32), ("iterations", C.c_int32), ("total_cg_iters", C.c_int64),
        ("cg_maxiter_hits", C.c_int32), ("cg_escalations", C.c_int32), ("mu_final", C.c_double), ("rnorm", C.c_double),
        ("primal", C.c_double), ("dual", C.c_double), ("compl_", C.c_double),
        ("objective", C.c_double), ("time_ms", C.c_double), ("pcg_time_ms", C.c_double),
    ]


EXPORTS = [
    "qp_default_pcg_options", "qp_default_ipm_options", "qp_status_string", "qp_last_error",
    "qp_create", "qp_destroy", "qp_set_stream", "qp_sizes", "qp_set_state", "qp_get_state",
    "qp_init_state", "qp_residuals", "qp_newton_rhs", "qp_kkt_matvec", "kkt_pcg_solve",
    "qp_newton_direction", "qp_step_lengths", "qp_take_step", "ipm_solve", "qp_backward",
    "qp_profile_begin", "qp_profile_end", "qp_operator_bytes", "qp_operator_layout",
    "qp_update_data", "qp_fused_layout",
    "qp_batch_create", "qp_batch_destroy", "ipm_solve_batch", "qp_batch_get_solution",
    "qp_batch_last_error", "ipm_solve_dense_noalloc", "qp_batch_set_teams", "qp_batch_launch_shape",
    "qp_batch_autotune", "qp_graph_stats", "qp_batch_instance_times",
]
PROF_CATEGORIES = ("rowpass", "colpass", "tsreduce", "epilogue", "cg_update", "cg_pupdate", "fused")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python -m paper_2308_00637_amd.build")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "qp_default_pcg_options": (None, [C.POINTER(PcgOptions)]),
        "qp_default_ipm_options": (None, [C.POINTER(IpmOptions)]),
        "qp_status_string": (C.c_char_p, [C.c_int32]),
        "qp_last_error": (C.c_char_p, [vp]),
        "qp_create": (C.c_int, [C.POINTER(QpDesc), vp, C.POINTER(vp)]),
        "qp_destroy": (None, [vp]),
        "qp_set_stream": (C.c_int, [vp, vp]),
        "qp_sizes": (C.c_int, [vp, _i64p, _i64p, _i64p, _i64p, _i64p]),
        "qp_set_state": (C.c_int, [vp, vp, vp, vp, C.c_double]),
        "qp_get_state": (C.c_int, [vp, vp, vp, vp, _dp]),
        "qp_init_state": (C.c_int, [vp, C.c_double]),
        "qp_residuals": (C.c_int, [vp, vp, _dp]),
        "qp_newton_rhs": (C.c_int, [vp, vp, vp]),
        "qp_kkt_matvec": (C.c_int, [vp, vp, vp]),
        "kkt_pcg_solve": (C.c_int, [vp, vp, vp, C.POINTER(PcgOptions), C.POINTER(PcgInfo)]),
        "qp_newton_direction": (C.c_int, [vp, C.POINTER(PcgOptions), vp, vp, vp, C.POINTER(PcgInfo)]),
        "qp_step_lengths": (C.c_int, [vp, vp, vp, C.c_double, _dp, _dp]),
        "qp_take_step": (C.c_int, [vp, vp, vp, vp, C.c_double, C.c_double]),
        "ipm_solve": (C.c_int, [vp, C.POINTER(IpmOptions), vp, vp, vp, C.POINTER(IpmInfo)]),
        "qp_backward": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, C.POINTER(PcgOptions), C.POINTER(PcgInfo)]),
        "qp_profile_begin": (C.c_int, [vp, C.c_int32, C.c_int32]),
        "qp_profile_end": (C.c_int, [vp, _i64p, _dp, _i64p]),
        "qp_operator_bytes": (C.c_int, [vp, _i64p, _i64p, _i64p, _i64p, _i64p]),
        "qp_operator_layout": (C.c_int, [vp, _i32p, _i32p, _i32p]),
        "qp_update_data": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "qp_fused_layout": (C.c_int, [vp, _i32p, _i32p, _i32p, _i64p, _i32p]),
        "qp_batch_create": (C.c_int, [C.POINTER(QpDesc), C.c_int32, vp, C.POINTER(vp)]),
        "qp_batch_destroy": (None, [vp]),
        "ipm_solve_batch": (C.c_int, [vp, C.POINTER(IpmOptions), C.c_int32, C.POINTER(IpmInfo)]),
        "qp_batch_get_solution": (C.c_int, [vp, C.c_int32, vp, vp, vp]),
        "qp_batch_last_error": (C.c_char_p, [vp]),
        "qp_batch_set_teams": (C.c_int, [vp, _i32p]),
        "qp_batch_launch_shape": (C.c_int, [vp, _i32p, _i32p]),
        "qp_batch_instance_times": (C.c_int, [vp, _dp, _dp, _i32p]),
        "qp_batch_autotune": (C.c_int, [vp, C.c_char_p, C.c_int32, _i32p, _i32p]),
        "qp_graph_stats": (C.c_int, [vp, _i64p, _i64p]),
        "ipm_solve_dense_noalloc": (C.c_int, [C.c_int64, C.c_int64, vp, vp, vp, vp, vp, vp, vp,
                                              C.POINTER(IpmOptions), vp, vp, vp, C.POINTER(IpmInfo), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


class QPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{LIB.qp_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _ptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return C.cast(None, C.POINTER(ctype))
    return a.ctypes.data_as(C.POINTER(ctype))


def _dev(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    assert t.is_cuda and t.dtype.itemsize == 8 and t.is_contiguous(), "need a contiguous float64 device tensor"
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_pcg_options(**kw) -> PcgOptions:
    o = PcgOptions()
    LIB.qp_default_pcg_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_ipm_options(**kw) -> IpmOptions:
    o = IpmOptions()
    LIB.qp_default_ipm_options(C.byref(o))
    for k, v in kw.items():
        if k == "pcg":
            o.pcg = v
        else:
            setattr(o, k, v)
    return o


@dataclass
class Sizes:
    n: int
    lam: int
    s: int
    kkt: int
    res: int


def make_desc(spec, precision: str = "fp64"):
    """QpDesc for a workload description; returns (desc, arrays it points into)."""
    f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    keep = []

    def hold(a):
        keep.append(a)
        return a

    d = QpDesc()
    n = int(spec.n)
    d.n, d.m, d.me = n, int(spec.m), int(spec.me)
    d.precision = PREC[precision]
    d.c = _ptr(hold(f64(spec.c)), C.c_double)
    if spec.h_kind == "dense":
        d.h_kind = H_DENSE
        d.H = _ptr(hold(f64(spec.H)), C.c_double)
    elif spec.h_kind == "lowrank":
        d.h_kind = H_LOWRANK
        d.k = int(spec.U.shape[1])
        d.h0 = _ptr(hold(f64(spec.h0)), C.c_double)
        d.U = _ptr(hold(f64(spec.U)), C.c_double)
        d.wd = _ptr(hold(f64(spec.wd)), C.c_double)
    elif spec.h_kind == "ptwp":
        d.h_kind = H_PTWP
        P = spec.P
        d.p_rows = int(P.shape[0])
        d.p_rowptr = _ptr(hold(np.ascontiguousarray(P.indptr, dtype=np.int64)), C.c_int64)
        d.p_col = _ptr(hold(np.ascontiguousarray(P.indices, dtype=np.int32)), C.c_int32)
        d.p_val = _ptr(hold(f64(P.data)), C.c_double)
        d.p_w = _ptr(hold(f64(spec.w)), C.c_double)
        d.p_d = _ptr(hold(f64(spec.d)), C.c_double)
    else:
        raise ValueError(spec.h_kind)
    if spec.A is None:
        d.a_kind = A_NONE
    elif hasattr(spec.A, "indptr"):
        d.a_kind = A_CSR
        d.a_rowptr = _ptr(hold(np.ascontiguousarray(spec.A.indptr, dtype=np.int64)), C.c_int64)
        d.a_col = _ptr(hold(np.ascontiguousarray(spec.A.indices, dtype=np.int32)), C.c_int32)
        d.a_val = _ptr(hold(f64(spec.A.data)), C.c_double)
    else:
        d.a_kind = A_DENSE
        d.A = _ptr(hold(f64(spec.A)), C.c_double)
    if spec.A is not None:
        d.lA = _ptr(hold(f64(spec.lA)), C.c_double)
        d.uA = _ptr(hold(f64(spec.uA)), C.c_double)
    if spec.C is not None:
        d.C = _ptr(hold(f64(spec.C)), C.c_double)
        d.b = _ptr(hold(f64(spec.b)), C.c_double)
    d.lx = _ptr(hold(f64(spec.lx)), C.c_double)
    d.ux = _ptr(hold(f64(spec.ux)), C.c_double)
    return d, keep


class QP:
    """Owns one qp_handle built from a workload description (`QPSpec`)."""

    def __init__(self, spec, precision: str = "fp64"):
        d, keep = make_desc(spec, precision)
        h = C.c_void_p()
        st = LIB.qp_create(C.byref(d), _stream(), C.byref(h))
        if st != QP_OK:
            raise QPError(st, LIB.qp_last_error(None).decode())
        self.h = h
        self.precision = precision
        # bumped by every call that changes the handle's data or iterate, so
        # a saved solve can tell whether the handle still holds it
        self.generation = 0
        self.p_rows = int(spec.P.shape[0]) if spec.h_kind == "ptwp" else 0
        sz = [C.c_int64() for _ in range(5)]
        LIB.qp_sizes(h, *[C.byref(v) for v in sz])
        self.sizes = Sizes(*[int(v.value) for v in sz])

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            LIB.qp_destroy(h)
            self.h = None

    def close(self):
        self.__del__()

    def _check(self, st):
        if st != QP_OK:
            raise QPError(st, LIB.qp_last_error(self.h).decode())

    def _empty(self, n):
        import torch
        return torch.empty(n, dtype=torch.float64, device="cuda")

    def set_stream(self):
        self._check(LIB.qp_set_stream(self.h, _stream()))

    # iterate I/O
    def set_state(self, x, lam, s, mu):
        self.generation += 1
        self._check(LIB.qp_set_state(self.h, _dev(x), _dev(lam), _dev(s), float(mu)))

    def get_state(self):
        x, lam, s = self._empty(self.sizes.n), self._empty(self.sizes.lam), self._empty(self.sizes.s)
        mu = C.c_double()
        self._check(LIB.qp_get_state(self.h, _dev(x), _dev(lam), _dev(s), C.byref(mu)))
        return x, lam, s, mu.value

    def init_state(self, mu=1.0):
        self.generation += 1
        self._check(LIB.qp_init_state(self.h, float(mu)))

    # steps a1..a8
    def residuals(self):
        r = self._empty(self.sizes.res)
        nrm = (C.c_double * 4)()
        self._check(LIB.qp_residuals(self.h, _dev(r), nrm))
        return r, list(nrm)

    def newton_rhs(self):
        rhs, dg = self._empty(self.sizes.kkt), self._empty(self.sizes.kkt)
        self._check(LIB.qp_newton_rhs(self.h, _dev(rhs), _dev(dg)))
        return rhs, dg

    def kkt_matvec(self, v):
        y = self._empty(self.sizes.kkt)
        self._check(LIB.qp_kkt_matvec(self.h, _dev(v), _dev(y)))
        return y

    def kkt_pcg_solve(self, rhs, opts: Optional[PcgOptions] = None):
        sol = self._empty(self.sizes.kkt)
        info = PcgInfo()
        self._check(LIB.kkt_pcg_solve(self.h, _dev(rhs), _dev(sol),
                                      C.byref(opts) if opts is not None else None, C.byref(info)))
        return sol, info

    def newton_direction(self, opts: Optional[PcgOptions] = None):
        dx, dl, ds = self._empty(self.sizes.n), self._empty(self.sizes.lam), self._empty(self.sizes.s)
        info = PcgInfo()
        self._check(LIB.qp_newton_direction(self.h, C.byref(opts) if opts is not None else None,
                                            _dev(dx), _dev(dl), _dev(ds), C.byref(info)))
        return dx, dl, ds, info

    def step_lengths(self, dlam, ds, gamma=0.99):
        ax, al = C.c_double(), C.c_double()
        self._check(LIB.qp_step_lengths(self.h, _dev(dlam), _dev(ds), float(gamma),
                                        C.byref(ax), C.byref(al)))
        return ax.value, al.value

    def take_step(self, dx, dlam, ds, ax, al):
        self.generation += 1
        self._check(LIB.qp_take_step(self.h, _dev(dx), _dev(dlam), _dev(ds), float(ax), float(al)))

    # Algorithm 1
    def solve(self, opts: Optional[IpmOptions] = None, log: bool = False, want_state: bool = True,
              log_kappa_plain: bool = False):
        """ipm_solve.  log: per-iteration arrays in out["log"]; log_kappa_plain
        (with log) also solves each Newton system by plain CG to log the
        condition number of K itself (out["log"]["kappa_plain"])."""
        if opts is None:
            opts = default_ipm_options()
        logs = None
        if log:
            cap = max(int(opts.max_iter), 1)
            keys = ["mu", "rnorm", "primal", "dual", "compl", "alpha_x", "alpha_lam", "cg_relres",
                    "kappa", "sigma"] + (["kappa_plain"] if log_kappa_plain else [])
            logs = {k: np.zeros(cap) for k in keys}
            logs["cg_iters"] = np.zeros(cap, dtype=np.int32)
            opts.log_capacity = cap
            for k, a in logs.items():
                setattr(opts, "log_" + k, _ptr(a, C.c_int32 if k == "cg_iters" else C.c_double))
        info = IpmInfo()
        if want_state:
            x, lam, s = self._empty(self.sizes.n), self._empty(self.sizes.lam), self._empty(self.sizes.s)
        else:
            x = lam = s = None
        self.generation += 1
        self._check(LIB.ipm_solve(self.h, C.byref(opts), _dev(x), _dev(lam), _dev(s), C.byref(info)))
        if logs is not None:
            k = info.iterations
            logs = {key: v[:k].copy() for key, v in logs.items()}
        return dict(x=x, lam=lam, s=s, info=info, log=logs)

    def update_data(self, c=None, lA=None, uA=None, b=None, w=None):
        self.generation += 1
        self._check(LIB.qp_update_data(self.h, _dev(c), _dev(lA), _dev(uA), _dev(b), _dev(w)))

    def profile_begin(self, max_launches: int, every: int = 1):
        """Time up to max_launches dispatches per PCG kernel, one in `every`."""
        self._check(LIB.qp_profile_begin(self.h, int(max_launches), int(every)))

    def profile_end(self):
        """Per category: (timed dispatches, their summed ms, all dispatches)."""
        cnt = (C.c_int64 * len(PROF_CATEGORIES))()
        ms = (C.c_double * len(PROF_CATEGORIES))()
        seen = (C.c_int64 * len(PROF_CATEGORIES))()
        self._check(LIB.qp_profile_end(self.h, cnt, ms, seen))
        return {k: (int(cnt[i]), float(ms[i]), int(seen[i])) for i, k in enumerate(PROF_CATEGORIES)}

    def operator_bytes(self):
        v = [C.c_int64() for _ in range(5)]
        self._check(LIB.qp_operator_bytes(self.h, *[C.byref(x) for x in v]))
        return dict(zip(("row_bytes", "col_bytes", "dense_bytes", "row_nnz", "col_nnz"),
                        [int(x.value) for x in v]))

    def operator_layout(self):
        """Blocked layout per side (row, column): LDS column chunks, work items
        per pass, columns per chunk."""
        arr = [(C.c_int32 * 2)() for _ in range(3)]
        self._check(LIB.qp_operator_layout(self.h, *arr))
        return {side: {"chunks": int(arr[0][i]), "work_items": int(arr[1][i]),
                       "chunk_cols": int(arr[2][i])} for i, side in enumerate(("row", "col"))}

    def graph_stats(self):
        """(captures, replays) of the PCG chunk graph (see qp_graph_stats)."""
        c, r = C.c_int64(), C.c_int64()
        self._check(LIB.qp_graph_stats(self.h, C.byref(c), C.byref(r)))
        return int(c.value), int(r.value)

    def fused_layout(self):
        """The fused single-read product: active, row ranges, columns of the
        first half, stored entries, failed (see qp_fused_layout)."""
        a, rg, hc, fl = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        st = C.c_int64()
        self._check(LIB.qp_fused_layout(self.h, C.byref(a), C.byref(rg), C.byref(hc), C.byref(st),
                                        C.byref(fl)))
        return {"active": bool(a.value), "ranges": int(rg.value), "half_cols": int(hc.value),
                "stored": int(st.value), "failed": bool(fl.value)}

    def backward(self, grad_x, want=("c", "lA", "uA", "b", "w"), opts: Optional[PcgOptions] = None):
        n, sz = self.sizes.n, self.sizes
        m = (sz.s - 2 * n) // 2
        me = sz.lam - 2 * m - 2 * n
        out = {}
        out["c"] = self._empty(n) if "c" in want else None
        out["lA"] = self._empty(m) if "lA" in want and m else None
        out["uA"] = self._empty(m) if "uA" in want and m else None
        out["b"] = self._empty(me) if "b" in want and me else None
        out["w"] = self._empty(self.p_rows) if "w" in want and getattr(self, "p_rows", 0) else None
        info = PcgInfo()
        self._check(LIB.qp_backward(self.h, _dev(grad_x), _dev(out["c"]), _dev(out["lA"]),
                                    _dev(out["uA"]), _dev(out["b"]), _dev(out["w"]),
                                    C.byref(opts) if opts is not None else None, C.byref(info)))
        return out, info


class QPBatch:
    """Owns one qp_batch: many independent dense QPs solved in one launch."""

    def __init__(self, specs, precision: str = "fp64"):
        descs = (QpDesc * len(specs))()
        self._keep = []
        for i, sp in enumerate(specs):
            d, keep = make_desc(sp, precision)
            descs[i] = d
            self._keep.append(keep)
        h = C.c_void_p()
        st = LIB.qp_batch_create(descs, len(specs), _stream(), C.byref(h))
        if st != QP_OK:
            raise QPError(st, LIB.qp_batch_last_error(None).decode())
        self.h = h
        self.specs = list(specs)
        self._keep = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            LIB.qp_batch_destroy(h)
            self.h = None

    def set_teams(self, sizes=None):
        """Workgroups per instance (powers of two, 1..64; None: all 1)."""
        arr = None
        if sizes is not None:
            arr = (C.c_int32 * len(self.specs))(*[int(g) for g in sizes])
        st = LIB.qp_batch_set_teams(self.h, arr)
        if st != QP_OK:
            raise QPError(st, LIB.qp_batch_last_error(self.h).decode())

    def autotune(self, table_path=None, max_team: int = 0):
        """Team sizes from measured times (see qp_batch_autotune); returns
        (team sizes, measurements taken)."""
        out = (C.c_int32 * len(self.specs))()
        probes = C.c_int32()
        path = None if table_path is None else str(table_path).encode()
        self._check_status(LIB.qp_batch_autotune(self.h, path, int(max_team), out, C.byref(probes)))
        return [int(v) for v in out], int(probes.value)

    def launch_shape(self):
        """(workgroups, teams) of the last solve's launch."""
        w, t = C.c_int32(), C.c_int32()
        self._check_status(LIB.qp_batch_launch_shape(self.h, C.byref(w), C.byref(t)))
        return int(w.value), int(t.value)

    def instance_times(self):
        """(start_ms, end_ms, team) per instance of the last completed solve:
        device wall-clock times from the earliest start, and the workgroups
        of the team that solved it."""
        k = len(self.specs)
        t0, t1, g = (C.c_double * k)(), (C.c_double * k)(), (C.c_int32 * k)()
        self._check_status(LIB.qp_batch_instance_times(self.h, t0, t1, g))
        return list(t0), list(t1), [int(v) for v in g]

    def _check_status(self, st):
        if st != QP_OK:
            raise QPError(st, LIB.qp_batch_last_error(self.h).decode())

    def solve(self, opts: Optional[IpmOptions] = None, workgroups: int = 0):
        if opts is None:
            opts = default_ipm_options()
        infos = (IpmInfo * len(self.specs))()
        st = LIB.ipm_solve_batch(self.h, C.byref(opts), int(workgroups), infos)
        if st not in (QP_OK, QP_ERR_NOT_SPD, QP_ERR_NUMERIC):
            raise QPError(st, LIB.qp_batch_last_error(self.h).decode())
        return list(infos), st

    def solution(self, i):
        import torch
        sp = self.specs[i]
        n, m = int(sp.n), int(sp.m)
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        lam = torch.empty(2 * m + 2 * n, dtype=torch.float64, device="cuda")
        s = torch.empty(2 * m + 2 * n, dtype=torch.float64, device="cuda")
        st = LIB.qp_batch_get_solution(self.h, int(i), _dev(x), _dev(lam), _dev(s))
        if st != QP_OK:
            raise QPError(st, LIB.qp_batch_last_error(self.h).decode())
        return x, lam, s


def ipm_solve_dense_noalloc(H, c, A=None, lA=None, uA=None, lx=None, ux=None,
                            opts: Optional[IpmOptions] = None, want_state: bool = True):
    """The allocation-free dense solve (see include/qpk.h): every argument a
    float64 device tensor (or None), the outputs allocated here by torch, the
    library allocates nothing.  Returns dict(x, lam, s, info)."""
    import torch
    n = int(c.shape[0])
    m = 0 if A is None else int(A.shape[0])
    info = IpmInfo()
    if want_state:
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        lam = torch.empty(2 * m + 2 * n, dtype=torch.float64, device="cuda")
        s = torch.empty(2 * m + 2 * n, dtype=torch.float64, device="cuda")
    else:
        x = lam = s = None
    st = LIB.ipm_solve_dense_noalloc(n, m, _dev(H), _dev(c), _dev(A), _dev(lA), _dev(uA), _dev(lx),
                                     _dev(ux), C.byref(opts) if opts is not None else None,
                                     _dev(x), _dev(lam), _dev(s), C.byref(info), _stream())
    if st not in (QP_OK, QP_ERR_NOT_SPD, QP_ERR_NUMERIC):
        raise QPError(st, LIB.qp_batch_last_error(None).decode())
    return dict(x=x, lam=lam, s=s, info=info, status=st)
