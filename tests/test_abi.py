"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/rcb.h declares, and rejects invalid arguments on the
host before any launch."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rcb.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rcb_[a-z_]+)\s*\(", src)))


def _lib():
    from paper_1108_0028_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return L.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for req in ("rcb_build", "rcb_check_cells", "rcb_refresh", "rcb_walk", "rcb_neighbours_count", "rcb_neighbours_fill", "rcb_gravity",
                "rcb_gravity_vjp", "rcb_destroy", "rcb_last_error"):
        assert req in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_params_default_is_the_paper_default():
    from paper_1108_0028_amd._lib import RcbParams
    L = _lib()
    p = RcbParams()
    L.rcb_params_default(C.byref(p))
    assert p.n_ll == 12 and p.theta == 0.7 and p.precision == 0 and p.validate == 0
    assert p.pure_mac == 0 and p.split == 0 and p.taylor_reading == 0 and p.deterministic == 0


@pytest.mark.parametrize("case", ["null_out", "null_x", "n_zero", "n_neg", "n_huge", "nll_zero",
                                  "theta_neg", "theta_nan", "precision", "pure_mac", "split", "reading",
                                  "deterministic"])
def test_build_rejects_bad_arguments_on_host(case):
    from paper_1108_0028_amd._lib import RcbParams
    L = _lib()
    p = RcbParams()
    L.rcb_params_default(C.byref(p))
    fake = C.c_void_p(0x1000)   # never dereferenced: argument checks come first
    ptrs = [fake] * 5
    n = 100
    out = C.c_void_p()
    outp = C.byref(out)
    if case == "null_out":
        outp = None
    elif case == "null_x":
        ptrs[0] = None
    elif case == "n_zero":
        n = 0
    elif case == "n_neg":
        n = -5
    elif case == "n_huge":
        n = 1 << 31
    elif case == "nll_zero":
        p.n_ll = 0
    elif case == "theta_neg":
        p.theta = -0.1
    elif case == "theta_nan":
        p.theta = float("nan")
    elif case == "precision":
        p.precision = 7
    elif case == "pure_mac":
        p.pure_mac = 2
    elif case == "split":
        p.split = 3
    elif case == "reading":
        p.taylor_reading = 2
    elif case == "deterministic":
        p.deterministic = 2
    st = L.rcb_build(*ptrs, n, C.byref(p), None, outp)
    assert st == 1   # RCB_EINVAL
    assert L.rcb_last_error().decode().startswith("rcb_build")
    assert not out.value


def test_null_tree_arguments():
    L = _lib()
    tot = C.c_int64()
    assert L.rcb_walk(None, None) == 1
    assert L.rcb_refresh(None, *([C.c_void_p(8)] * 5), 1, 0, None) == 1
    assert L.rcb_refresh_noalloc(None, *([C.c_void_p(8)] * 5), 1, None) == 1
    assert L.rcb_check_cells(None, *([C.c_void_p(8)] * 3), 1, C.byref(tot), None) == 1
    assert L.rcb_neighbours_count(None, C.c_void_p(8), C.byref(tot), None) == 1
    assert L.rcb_neighbours_fill(None, C.c_void_p(8), C.c_void_p(8), 1, None) == 1
    assert L.rcb_gravity(None, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None) == 1
    assert L.rcb_gravity_vjp(None, *([C.c_void_p(8)] * 7), None) == 1
    assert L.rcb_tree_export(None, 0, C.c_void_p(8), 8, None) == 1
    L.rcb_destroy(None, None)


def test_noalloc_refresh_capacity_is_stated():
    L = _lib()
    assert L.rcb_refresh_noalloc_scratch(None) == 64 << 20
