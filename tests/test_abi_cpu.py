"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every function include/qpk.h declares, and rejects bad problem data before
touching the device."""
import ctypes as C
import re
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpk.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:qp_status|void|const char\*)\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def qpk():
    from paper_2308_00637_amd import qpk as mod
    return mod


def test_library_loads_and_exports_every_declared_function(qpk):
    names = header_functions()
    assert len(names) >= 20
    lib = C.CDLL(qpk.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(qpk.EXPORTS) == names


@pytest.mark.parametrize("name", ["PcgOptions", "IpmOptions"])
def test_option_structs_match_the_library_layout(qpk, name):
    """The library fills a struct of its own size: a binding struct of
    another size would be overrun (the bytes after it must stay untouched)
    or left partly unset."""
    cls = getattr(qpk, name)
    size = C.sizeof(cls)
    buf = (C.c_ubyte * (size + 64))(*([0xAB] * (size + 64)))
    fill = qpk.LIB.qp_default_pcg_options if name == "PcgOptions" else qpk.LIB.qp_default_ipm_options
    fill(C.cast(buf, C.POINTER(cls)))
    assert bytes(buf[size:]) == b"\xab" * 64
    o = cls.from_buffer(buf)
    pcg = o if name == "PcgOptions" else o.pcg
    assert (pcg.tol, pcg.maxit, pcg.check_every, pcg.rr_period, pcg.spectrum, pcg.no_precond) == \
        (1e-7, 5000, 8, 0, 0, 0)
    if name == "IpmOptions":
        assert o.max_iter == 200 and not o.log_kappa and not o.log_kappa_plain


def test_default_options_match_the_paper(qpk):
    o = qpk.default_ipm_options()
    assert o.gamma == 0.99 and o.mu0 == 1.0 and o.mu_tol == 1e-6 and o.mu_div == 10.0
    assert o.pcg.tol == 1e-7 and o.pcg.maxit == 5000


def _desc(qpk, n=3, m=2):
    keep = []

    def arr(v, dt=np.float64):
        a = np.ascontiguousarray(v, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double if dt == np.float64 else C.c_int64))

    d = qpk.QpDesc()
    d.n, d.m, d.me = n, m, 0
    d.h_kind = qpk.H_DENSE
    d.H = arr(np.eye(n))
    d.c = arr(np.ones(n))
    d.a_kind = qpk.A_DENSE
    d.A = arr(np.ones((m, n)))
    d.lA = arr(np.zeros(m))
    d.uA = arr(np.ones(m))
    return d, keep, arr


@pytest.mark.parametrize("case", ["l_gt_u", "nan_c", "bad_n", "lx_eq_ux", "bad_prec", "bad_csr"])
def test_create_rejects_bad_data_on_the_host(qpk, case):
    d, keep, arr = _desc(qpk)
    if case == "l_gt_u":
        d.lA = arr([2.0, 0.0])
    elif case == "nan_c":
        d.c = arr([1.0, np.nan, 0.0])
    elif case == "bad_n":
        d.n = 0
    elif case == "lx_eq_ux":
        d.lx = arr([0.0, 1.0, 2.0])
        d.ux = arr([1.0, 1.0, 3.0])
    elif case == "bad_prec":
        d.precision = 7
    elif case == "bad_csr":
        d.a_kind = qpk.A_CSR
        d.a_rowptr = arr([0, 1, 5], np.int64)
        cols = np.array([0, 1, 2, 9, 1], dtype=np.int32)
        keep.append(cols)
        d.a_col = cols.ctypes.data_as(C.POINTER(C.c_int32))
        d.a_val = arr(np.ones(5))
    h = C.c_void_p()
    st = qpk.LIB.qp_create(C.byref(d), None, C.byref(h))
    assert st == qpk.QP_ERR_ARG
    assert not h.value
    assert len(qpk.LIB.qp_last_error(None)) > 0


def test_status_strings(qpk):
    for s in (0, -1, -2, -3, -4, -5, -6, -7):
        assert qpk.LIB.qp_status_string(s)
