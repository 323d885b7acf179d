"""ctypes binding of librcb.so (the C ABI of include/rcb.h).

Argument marshalling only: torch tensors on the GPU are passed as device
pointers together with torch's current HIP stream; every step of the path
runs in the library's kernels. There is no CPU fallback: if librcb.so is
missing or a call fails, a RuntimeError is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librcb.so")

RCB_FP64, RCB_MIXED = 0, 1
FIELDS = dict(perm=0, first=1, count=2, lo=3, hi=4, com=5, mass=6, quad=7, hint=8, hnode=9,
              near_off=10, far_off=11, near=12, far=13)
STATUS = {0: "RCB_OK", 1: "RCB_EINVAL", 2: "RCB_ENOMEM", 3: "RCB_EHIP", 4: "RCB_ECAPACITY",
          5: "RCB_ESTATE", 6: "RCB_EINPUT"}


# workspace allocator callbacks (rcb_params.alloc / free)
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def _torch_alloc(nbytes, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream or 0)
    except Exception:       # out of memory: the library reports RCB_ENOMEM
        return None


def _torch_free(ptr, stream, ctx):
    torch.cuda.caching_allocator_delete(ptr)


_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_FREE = _FREE_FN(_torch_free)


class RcbParams(C.Structure):
    _fields_ = [("n_ll", C.c_int32), ("precision", C.c_int32), ("theta", C.c_double),
                ("validate", C.c_int32), ("pure_mac", C.c_int32),
                ("split", C.c_int32), ("taylor_reading", C.c_int32), ("deterministic", C.c_int32),
                ("alloc", _ALLOC_FN), ("free", _FREE_FN), ("alloc_ctx", C.c_void_p)]


class RcbTreeInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("k", C.c_int32), ("precision", C.c_int32),
                ("n_labels", C.c_int64), ("near_total", C.c_int64), ("far_total", C.c_int64),
                ("theta", C.c_double), ("walk_requeued", C.c_int64), ("walk_nodes", C.c_int64),
                ("walk_tests", C.c_int64)]


EXPORTED = ["rcb_params_default", "rcb_build", "rcb_check_cells", "rcb_refresh", "rcb_walk", "rcb_neighbours_count", "rcb_neighbours_fill",
            "rcb_gravity", "rcb_gravity_vjp", "rcb_get_info", "rcb_tree_export", "rcb_destroy",
            "rcb_release_cache", "rcb_refresh_noalloc", "rcb_refresh_noalloc_scratch", "rcb_last_error"]

_lib = None


class RcbError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


def lib():
    """Load librcb.so (built in-tree by build_lib.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.rcb_params_default.argtypes = [C.POINTER(RcbParams)]
        L.rcb_params_default.restype = None
        L.rcb_build.argtypes = [P, P, P, P, P, C.c_int64, C.POINTER(RcbParams), P, C.POINTER(P)]
        L.rcb_build.restype = C.c_int
        L.rcb_check_cells.argtypes = [P, P, P, P, C.c_int64, C.POINTER(C.c_int64), P]
        L.rcb_check_cells.restype = C.c_int
        L.rcb_refresh.argtypes = [P, P, P, P, P, P, C.c_int64, C.c_int32, P]
        L.rcb_refresh.restype = C.c_int
        L.rcb_refresh_noalloc.argtypes = [P, P, P, P, P, P, C.c_int64, P]
        L.rcb_refresh_noalloc.restype = C.c_int
        L.rcb_refresh_noalloc_scratch.argtypes = [P]
        L.rcb_refresh_noalloc_scratch.restype = C.c_size_t
        L.rcb_walk.argtypes = [P, P]
        L.rcb_walk.restype = C.c_int
        L.rcb_neighbours_count.argtypes = [P, P, C.POINTER(C.c_int64), P]
        L.rcb_neighbours_count.restype = C.c_int
        L.rcb_neighbours_fill.argtypes = [P, P, P, C.c_int64, P]
        L.rcb_neighbours_fill.restype = C.c_int
        L.rcb_gravity.argtypes = [P, P, P, P, P]
        L.rcb_gravity.restype = C.c_int
        L.rcb_gravity_vjp.argtypes = [P, P, P, P, P, P, P, P, P]
        L.rcb_gravity_vjp.restype = C.c_int
        L.rcb_get_info.argtypes = [P, C.POINTER(RcbTreeInfo)]
        L.rcb_get_info.restype = C.c_int
        L.rcb_tree_export.argtypes = [P, C.c_int32, P, C.c_size_t, P]
        L.rcb_tree_export.restype = C.c_int
        L.rcb_destroy.argtypes = [P, P]
        L.rcb_destroy.restype = None
        L.rcb_release_cache.argtypes = []
        L.rcb_release_cache.restype = None
        L.rcb_last_error.argtypes = []
        L.rcb_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != 0:
        raise RcbError(st, where, lib().rcb_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


class Tree:
    """An RCB tree built on the GPU (rcb_build) and its evaluations."""

    def __init__(self, x, y, z, m, h, n_ll: int = 12, theta: float = 0.7, precision: str = "fp64",
                 validate: bool = False, pure_mac: bool = False, split: str = "mass",
                 taylor_reading: str = "A", allocator: str = "library",
                 deterministic: bool = False):
        """split: "mass" (planes through the centre of mass, the paper's),
        "number" (through the centre of number) or "median" (median position
        split: equal halves). taylor_reading: "A" (J, H of the full field) or
        "B" (J, H of the monopole field; no VJP). allocator: "library" (the
        library's stream-ordered pool) or "torch" (workspace from PyTorch's
        caching allocator through rcb_params.alloc / free). deterministic:
        the VJP adds nothing atomically and repeats bit for bit."""
        L = lib()
        arrs = [_dev(a, torch.float64, nm) for a, nm in zip((x, y, z, m, h), "xyzmh")]
        n = arrs[0].numel()
        for a, nm in zip(arrs, "xyzmh"):
            if a.numel() != n or a.dim() != 1:
                raise ValueError(f"{nm} must be 1-D with {n} elements")
        p = RcbParams()
        L.rcb_params_default(C.byref(p))
        p.n_ll = int(n_ll)
        p.theta = float(theta)
        p.precision = RCB_MIXED if precision == "mixed" else RCB_FP64
        p.validate = 1 if validate else 0
        p.pure_mac = 1 if pure_mac else 0
        p.split = {"mass": 0, "number": 1, "median": 2}[split]
        p.taylor_reading = {"A": 0, "B": 1}[taylor_reading]
        p.deterministic = 1 if deterministic else 0
        if allocator == "torch":
            p.alloc = _TORCH_ALLOC
            p.free = _TORCH_FREE
        elif allocator != "library":
            raise ValueError(f"unknown allocator {allocator!r}")
        self.precision = precision
        self.device = arrs[0].device
        self.n = n
        h_ = C.c_void_p()
        st = L.rcb_build(*[_ptr(a) for a in arrs], n, C.byref(p), _stream(), C.byref(h_))
        _check(st, "rcb_build")
        self._h = h_
        self._total = None

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("tree was destroyed")
        return self._h

    def info(self) -> dict:
        i = RcbTreeInfo()
        _check(lib().rcb_get_info(self.handle, C.byref(i)), "rcb_get_info")
        return dict(n=i.n, k=i.k, precision=i.precision, n_labels=i.n_labels,
                    near_total=i.near_total, far_total=i.far_total, theta=i.theta,
                    walk_requeued=i.walk_requeued, walk_nodes=i.walk_nodes, walk_tests=i.walk_tests)

    def out_dtype(self):
        return torch.float32 if self.precision == "mixed" else torch.float64

    def cells_left(self, x, y, z) -> int:
        """Particles whose new position is outside their lowest-level cell."""
        xs = [_dev(a, torch.float64, nm) for a, nm in zip((x, y, z), "xyz")]
        out = C.c_int64()
        _check(lib().rcb_check_cells(self.handle, *[_ptr(a) for a in xs], self.n, C.byref(out),
                                     _stream()), "rcb_check_cells")
        return out.value

    def refresh(self, x, y, z, m, h, keep_lists: bool = False):
        """New inputs on the same tree: moments recomputed, topology kept.
        keep_lists=False walks again on demand (the paper's tree update);
        True keeps the interaction lists (the tree held fixed, as the VJP
        assumes; neighbours then need walk() first)."""
        xs = [_dev(a, torch.float64, nm) for a, nm in zip((x, y, z, m, h), "xyzmh")]
        _check(lib().rcb_refresh(self.handle, *[_ptr(a) for a in xs], self.n,
                                 1 if keep_lists else 0, _stream()), "rcb_refresh")
        self._keep = xs   # inputs stay alive until the stream has used them

    def walk(self):
        """Make the interaction lists now (the other calls make them on demand)."""
        _check(lib().rcb_walk(self.handle, _stream()), "rcb_walk")

    def neighbours(self):
        """(offsets int64[n+1], ids int32[total]) -- caller particle order."""
        off = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
        tot = C.c_int64()
        _check(lib().rcb_neighbours_count(self.handle, _ptr(off), C.byref(tot), _stream()),
               "rcb_neighbours_count")
        ids = torch.empty(max(1, tot.value), dtype=torch.int32, device=self.device)
        _check(lib().rcb_neighbours_fill(self.handle, _ptr(off), _ptr(ids), ids.numel(), _stream()),
               "rcb_neighbours_fill")
        return off, ids[: tot.value]

    def neighbours_count(self, off: torch.Tensor) -> int:
        tot = C.c_int64()
        _check(lib().rcb_neighbours_count(self.handle, _ptr(off), C.byref(tot), _stream()),
               "rcb_neighbours_count")
        return tot.value

    def neighbours_fill(self, off: torch.Tensor, ids: torch.Tensor):
        _check(lib().rcb_neighbours_fill(self.handle, _ptr(off), _ptr(ids), ids.numel(), _stream()),
               "rcb_neighbours_fill")

    def gravity(self, out=None):
        dt = self.out_dtype()
        if out is None:
            out = [torch.empty(self.n, dtype=dt, device=self.device) for _ in range(3)]
        _check(lib().rcb_gravity(self.handle, *[_ptr(o) for o in out], _stream()), "rcb_gravity")
        return tuple(out)

    def vjp(self, gx, gy, gz):
        dt = self.out_dtype()
        g = [_dev(a, dt, nm) for a, nm in zip((gx, gy, gz), ("gx", "gy", "gz"))]
        out = [torch.empty(self.n, dtype=dt, device=self.device) for _ in range(4)]
        _check(lib().rcb_gravity_vjp(self.handle, *[_ptr(a) for a in g], *[_ptr(o) for o in out],
                                     _stream()), "rcb_gravity_vjp")
        return tuple(out)

    def export(self, field: str) -> torch.Tensor:
        """Copy one of the tree's arrays (see rcb_field) into a new tensor."""
        inf = self.info()
        L, n, nleaf = inf["n_labels"], inf["n"], 1 << inf["k"]
        fid = FIELDS[field]
        if field in ("near", "far", "near_off", "far_off") and inf["near_total"] < 0:
            # the list fields run the walk first; sizes are known afterwards
            tmp = torch.empty(nleaf + 1, dtype=torch.int64, device=self.device)
            _check(lib().rcb_tree_export(self.handle, FIELDS["near_off"], _ptr(tmp), tmp.numel() * 8,
                                         _stream()), "rcb_tree_export")
            inf = self.info()
        spec = {"perm": (torch.int32, n), "first": (torch.int32, L), "count": (torch.int32, L),
                "lo": (torch.float64, 3 * L), "hi": (torch.float64, 3 * L),
                "com": (torch.float64, 3 * L), "mass": (torch.float64, L),
                "quad": (torch.float64, 6 * L), "hint": (torch.float64, L),
                "hnode": (torch.float64, L), "near_off": (torch.int64, nleaf + 1),
                "far_off": (torch.int64, nleaf + 1), "near": (torch.int32, inf["near_total"]),
                "far": (torch.int32, inf["far_total"])}[field]
        out = torch.empty(max(1, spec[1]), dtype=spec[0], device=self.device)
        _check(lib().rcb_tree_export(self.handle, fid, _ptr(out), out.numel() * out.element_size(),
                                     _stream()), "rcb_tree_export")
        return out[: spec[1]]

    def destroy(self):
        if self._h is not None:
            try:
                s = _stream()
            except Exception:   # interpreter shutdown: the tree's own stream
                s = None
            lib().rcb_destroy(self._h, s)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class RCBGravity(torch.autograd.Function):
    """Accelerations a(x, y, z, m; h) of the RCB tree with a hand-written
    backward: rcb_gravity_vjp on the tree of the forward pass (topology and
    lists held fixed). h receives no gradient."""

    @staticmethod
    def forward(ctx, x, y, z, m, h, n_ll=12, theta=0.7, precision="fp64", pure_mac=False,
                deterministic=False):
        tree = Tree(x.detach(), y.detach(), z.detach(), m.detach(), h.detach(), n_ll=n_ll,
                    theta=theta, precision=precision, pure_mac=pure_mac, deterministic=deterministic)
        ax, ay, az = tree.gravity()
        ctx.tree = tree
        return ax, ay, az

    @staticmethod
    def backward(ctx, gx, gy, gz):
        tree = ctx.tree
        dt = tree.out_dtype()
        g = [(torch.zeros(tree.n, dtype=dt, device=tree.device) if v is None else v.to(dt).contiguous())
             for v in (gx, gy, gz)]
        dx, dy, dz, dm = tree.vjp(*g)
        tree.destroy()
        ctx.tree = None
        return dx, dy, dz, dm, None, None, None, None, None, None


def release_cache():
    """Give back the device memory the library keeps for reuse (rcb_release_cache)."""
    lib().rcb_release_cache()


def gravity(x, y, z, m, h, n_ll: int = 12, theta: float = 0.7, precision: str = "fp64",
            pure_mac: bool = False, deterministic: bool = False):
    """Differentiable accelerations (see RCBGravity); deterministic: a
    backward that repeats bit for bit (no atomics)."""
    return RCBGravity.apply(x, y, z, m, h, n_ll, theta, precision, pure_mac, deterministic)
