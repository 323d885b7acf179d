"""ctypes wrapper of the plain FP64 C oracle (rcb_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use it; the product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rcb_oracle.c")
LIB = os.path.join(HERE, "_build", "librcb_oracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: FP64, no fused multiply-add, OpenMP."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        L.orc_build.restype = P
        L.orc_build.argtypes = [C.c_int64, dp, dp, dp, dp, dp, C.c_int, C.c_int]
        L.orc_free.argtypes = [P]
        L.orc_refresh.argtypes = [P, dp, dp, dp, dp, dp]
        L.orc_k.argtypes = [P]
        L.orc_k.restype = C.c_int
        L.orc_depth_for.argtypes = [C.c_int64, C.c_int]
        L.orc_depth_for.restype = C.c_int
        L.orc_topology.argtypes = [P, i64p, i64p, i64p, i32p]
        L.orc_nodes.argtypes = [P, dp, dp, dp, dp, dp, dp, dp]
        L.orc_walk.argtypes = [P, C.c_double, i64p, C.c_int64, C.c_int]
        L.orc_set_reading.argtypes = [P, C.c_int]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_threads.restype = C.c_int
        L.orc_list_sizes.argtypes = [P, i64p, i64p, i64p]
        L.orc_leaf_lists.argtypes = [P, C.c_int64, i32p, i32p]
        L.orc_neighbours_count.argtypes = [P, i64p]
        L.orc_neighbours_fill.argtypes = [P, i64p, i32p]
        L.orc_kernel_F.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc_deriv_tensor.argtypes = [C.c_int, dp, dp]
        L.orc_far_coeffs.argtypes = [C.c_double, dp, dp, dp, dp, dp, dp]
        L.orc_gravity.argtypes = [P, dp, dp, dp]
        L.orc_gravity_parts.argtypes = [P, dp, dp, dp, C.c_int]
        L.orc_vjp.argtypes = [P, dp, dp, dp, dp, dp, dp, dp]
        L.orc_psum.argtypes = [dp, C.c_int64]
        L.orc_psum.restype = C.c_double
        L.orc_init.argtypes = []
        L.orc_init()
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _i32(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def set_threads(n: int):
    """Threads of the oracle's OpenMP loops."""
    lib().orc_set_threads(int(n))


def threads() -> int:
    return int(lib().orc_threads())


def depth_for(n: int, n_ll: int) -> int:
    """Depth rule of Sec. 2.1: smallest k with N <= N_ll 2^k."""
    return int(lib().orc_depth_for(n, n_ll))


def psum(v) -> float:
    v, p = _d(v)
    return float(lib().orc_psum(p, v.shape[0]))


def kernel_F(r: float, h: float):
    F = C.c_double()
    dF = C.c_double()
    lib().orc_kernel_F(r, h, C.byref(F), C.byref(dF))
    return F.value, dF.value


def deriv_tensor(order: int, R) -> np.ndarray:
    R, p = _d(R)
    out = np.zeros(3 ** order)
    lib().orc_deriv_tensor(order, p, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out.reshape((3,) * order) if order else out


def far_coeffs(M: float, q6, R, with_t4: bool = False):
    q6, pq = _d(q6)
    R, pr = _d(R)
    f = np.zeros(3)
    J = np.zeros(9)
    H = np.zeros(27)
    T4 = np.zeros(81) if with_t4 else None
    dp = C.POINTER(C.c_double)
    lib().orc_far_coeffs(M, pq, pr, f.ctypes.data_as(dp), J.ctypes.data_as(dp), H.ctypes.data_as(dp),
                         T4.ctypes.data_as(dp) if with_t4 else None)
    out = (f, J.reshape(3, 3), H.reshape(3, 3, 3))
    if with_t4:
        out = out + (T4.reshape(3, 3, 3, 3),)
    return out


class OracleTree:
    """The oracle's RCB tree for one particle set (FP64, CPU)."""

    def __init__(self, x, y, z, m, h, n_ll: int, split: str = "mass"):
        """split: "mass" (centre of mass, the paper's choice), "number"
        (centre of number) or "median" (median position split, equal halves;
        Sec. 2.1 "Load balancing")."""
        L = lib()
        self._keep = [_d(a) for a in (x, y, z, m, h)]
        ps = [k[1] for k in self._keep]
        self.n = int(self._keep[0][0].shape[0])
        self.n_ll = n_ll
        self.ptr = L.orc_build(self.n, *ps, n_ll, {"mass": 0, "number": 1, "median": 2}[split])
        if not self.ptr:
            raise ValueError("oracle build rejected its arguments")
        self.k = int(L.orc_k(self.ptr))
        self.n_leaves = 1 << self.k
        self.nlab = 2 << self.k
        self.walked = None

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_free(self.ptr)
            self.ptr = None

    def refresh(self, x, y, z, m, h):
        arrs = [_d(a) for a in (x, y, z, m, h)]
        lib().orc_refresh(self.ptr, *[a[1] for a in arrs])
        self._keep = arrs

    def topology(self):
        perm = np.zeros(self.n, np.int64)
        first = np.zeros(self.nlab, np.int64)
        count = np.zeros(self.nlab, np.int64)
        axis = np.zeros(self.nlab, np.int32)
        lib().orc_topology(self.ptr, _i64(perm), _i64(first), _i64(count), _i32(axis))
        return dict(perm=perm, first=first, count=count, axis=axis)

    def nodes(self):
        L = self.nlab
        lo = np.zeros((L, 3)); hi = np.zeros((L, 3)); com = np.zeros((L, 3))
        M = np.zeros(L); Q = np.zeros((L, 6)); hint = np.zeros(L); hnode = np.zeros(L)
        dp = C.POINTER(C.c_double)
        lib().orc_nodes(self.ptr, *[a.ctypes.data_as(dp) for a in (lo, hi, com, M, Q, hint, hnode)])
        return dict(lo=lo, hi=hi, com=com, M=M, Q=Q, hint=hint, hnode=hnode)

    def walk(self, theta: float, leaves=None, pure_mac: bool = False):
        """Walk all leaves, or only the given leaf labels. pure_mac: gravity by
        the geometric MAC alone (Sec. 2.5 variant), neighbours by reachability."""
        pm = 1 if pure_mac else 0
        if leaves is None:
            lib().orc_walk(self.ptr, theta, None, 0, pm)
        else:
            lv = np.ascontiguousarray(leaves, dtype=np.int64)
            lib().orc_walk(self.ptr, theta, _i64(lv), lv.shape[0], pm)
        self.theta = theta
        self.walked = leaves

    def list_sizes(self):
        nn = np.zeros(self.n_leaves, np.int64)
        nf = np.zeros(self.n_leaves, np.int64)
        st = np.zeros((self.n_leaves, 5), np.int64)
        lib().orc_list_sizes(self.ptr, _i64(nn), _i64(nf), _i64(st))
        return nn, nf, st

    def leaf_lists(self, label: int):
        nn, nf, _ = self.list_sizes() if not hasattr(self, "_sizes") else self._sizes
        i = label - self.n_leaves
        near = np.zeros(max(1, nn[i]), np.int32)
        far = np.zeros(max(1, nf[i]), np.int32)
        lib().orc_leaf_lists(self.ptr, label, _i32(near), _i32(far))
        return near[: nn[i]].view(np.uint32), far[: nf[i]]

    def cache_sizes(self):
        self._sizes = self.list_sizes()
        return self._sizes

    def neighbours(self):
        """CSR (offsets, ids) in original particle order; -1 counts for unwalked leaves."""
        cnt = np.zeros(self.n, np.int64)
        lib().orc_neighbours_count(self.ptr, _i64(cnt))
        valid = cnt >= 0
        off = np.zeros(self.n + 1, np.int64)
        off[1:] = np.cumsum(np.where(valid, cnt, 0))
        ids = np.zeros(max(1, int(off[-1])), np.int32)
        lib().orc_neighbours_fill(self.ptr, _i64(off), _i32(ids))
        return off, ids[: int(off[-1])], valid

    def set_reading(self, reading: str):
        """Taylor coefficients of Eq. 6: "A" (J, H of the full field, default)
        or "B" (J, H of the monopole field only)."""
        self.reading = reading
        lib().orc_set_reading(self.ptr, {"A": 0, "B": 1}[reading])

    def gravity(self, parts: int = 3):
        """Accelerations of the walked leaves' particles (NaN elsewhere). parts:
        1 = near field only, 2 = far field only, 3 = both (for timing the two
        separately, as Table 1 does)."""
        ax = np.zeros(self.n); ay = np.zeros(self.n); az = np.zeros(self.n)
        dp = C.POINTER(C.c_double)
        if parts == 3:
            lib().orc_gravity(self.ptr, ax.ctypes.data_as(dp), ay.ctypes.data_as(dp), az.ctypes.data_as(dp))
        else:
            lib().orc_gravity_parts(self.ptr, ax.ctypes.data_as(dp), ay.ctypes.data_as(dp),
                                    az.ctypes.data_as(dp), parts)
        return ax, ay, az

    def vjp(self, gx, gy, gz):
        if getattr(self, "reading", "A") != "A":
            raise ValueError("the vector-Jacobian product is defined for reading A")
        g = [_d(a) for a in (gx, gy, gz)]
        out = [np.zeros(self.n) for _ in range(4)]
        dp = C.POINTER(C.c_double)
        lib().orc_vjp(self.ptr, *[a[1] for a in g], *[o.ctypes.data_as(dp) for o in out])
        return tuple(out)
