"""rcb_refresh_noalloc (the refresh for callers that cannot allocate) against
rcb_refresh(keep_lists = 1) through the C ABI: two calls in a row on trees of
decreasing size share the static scratch array and must each reproduce the
allocating entry point bit for bit (moments, radii, then accelerations and
the VJP on the kept lists); the workspace allocator sees no call during the
no-alloc refresh; a tree larger than the array is refused."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("com", "mass", "quad", "hint", "hnode")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


class _Counting:
    """A workspace allocator (rcb_params.alloc / free) on PyTorch's caching
    allocator that counts its calls."""

    def __init__(self):
        import torch
        from paper_1108_0028_amd import _lib
        self.allocs = 0
        self.frees = 0

        def alloc(nbytes, stream, ctx):
            self.allocs += 1
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream or 0)

        def free(ptr, stream, ctx):
            self.frees += 1
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = _lib._ALLOC_FN(alloc)
        self.free_fn = _lib._FREE_FN(free)


def _build(arrs, n_ll, theta, prec, counting):
    from paper_1108_0028_amd._lib import RcbParams, _check, _ptr, _stream, lib
    L = lib()
    p = RcbParams()
    L.rcb_params_default(C.byref(p))
    p.n_ll, p.theta, p.precision = n_ll, theta, (1 if prec == "mixed" else 0)
    p.alloc, p.free = counting.alloc_fn, counting.free_fn
    h = C.c_void_p()
    _check(L.rcb_build(*[_ptr(a) for a in arrs], arrs[0].numel(), C.byref(p), _stream(), C.byref(h)),
           "rcb_build")
    return h


def _export(h, field, like):
    import torch
    from paper_1108_0028_amd._lib import FIELDS as F, _check, _ptr, _stream, lib
    out = torch.empty_like(like)
    _check(lib().rcb_tree_export(h, F[field], _ptr(out), out.numel() * out.element_size(), _stream()),
           "rcb_tree_export")
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_refresh_equals_refresh(prec):
    import torch
    from paper_1108_0028_amd import Tree
    from paper_1108_0028_amd._lib import _check, _ptr, _stream, lib
    L = lib()
    dev = torch.device("cuda:0")
    dt = torch.float32 if prec == "mixed" else torch.float64
    for n, seed in ((60000, 91), (9000, 92)):           # the second call is smaller
        _say("noalloc refresh", prec, n)
        c = W.small_random(n, seed, "clustered")
        arrs = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in c.arrays()]
        rng = np.random.default_rng(seed)
        moved = [torch.from_numpy(a).to(dev) for a in
                 (c.x + 1e-3 * rng.normal(size=n), c.y + 1e-3 * rng.normal(size=n),
                  c.z + 1e-3 * rng.normal(size=n), c.m * rng.uniform(0.9, 1.1, n),
                  c.h * rng.uniform(0.9, 1.2, n))]
        ref = Tree(*arrs, n_ll=8, theta=0.6, precision=prec)
        ref.walk()
        ref.refresh(*moved, keep_lists=True)
        counting = _Counting()
        h = _build(arrs, 8, 0.6, prec, counting)
        _check(L.rcb_walk(h, _stream()), "rcb_walk")
        need = L.rcb_refresh_noalloc_scratch(h)
        assert 0 < need <= L.rcb_refresh_noalloc_scratch(None)
        before = (counting.allocs, counting.frees)
        _check(L.rcb_refresh_noalloc(h, *[_ptr(a) for a in moved], n, _stream()), "rcb_refresh_noalloc")
        torch.cuda.synchronize()
        assert (counting.allocs, counting.frees) == before     # no workspace traffic
        nlab = ref.info()["n_labels"]
        for f in FIELDS:
            want = ref.export(f)
            got = _export(h, f, want).reshape(nlab, -1)[1:]      # label 0 is unused
            want = want.cpu().numpy().reshape(nlab, -1)[1:]
            np.testing.assert_array_equal(got.view(np.int64), want.view(np.int64), err_msg=f)
        acc = [torch.empty(n, dtype=dt, device=dev) for _ in range(3)]
        _check(L.rcb_gravity(h, *[_ptr(a) for a in acc], _stream()), "rcb_gravity")
        for a, b in zip(acc, ref.gravity()):
            np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
        g = [torch.from_numpy(v).to(dev, dt) for v in W.cotangents(n, seed=seed)]
        d = [torch.empty(n, dtype=dt, device=dev) for _ in range(4)]
        _check(L.rcb_gravity_vjp(h, *[_ptr(a) for a in g], *[_ptr(a) for a in d], _stream()), "vjp")
        tol = 1e-9 if prec == "fp64" else 1e-4      # atomics order differs between runs
        for a, b in zip(d, ref.vjp(*g)):
            a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
            assert np.abs(a - b).max() <= tol * np.abs(b).max()
        # the neighbour search needs a new walk after a refresh that kept the lists
        off = torch.empty(n + 1, dtype=torch.int64, device=dev)
        tot = C.c_int64()
        assert L.rcb_neighbours_count(h, _ptr(off), C.byref(tot), _stream()) == 5
        L.rcb_destroy(h, None)
        ref.destroy()


def test_noalloc_refresh_refuses_a_tree_beyond_the_array():
    import torch
    from paper_1108_0028_amd import Tree
    from paper_1108_0028_amd._lib import _ptr, _stream, lib
    L = lib()
    cap = L.rcb_refresh_noalloc_scratch(None)
    n = cap // 30                                         # ~33 bytes per particle are needed
    _say("noalloc refresh beyond capacity", n)
    rng = np.random.default_rng(93)
    arrs = [torch.from_numpy(v).to("cuda:0") for v in
            (rng.uniform(0, 1, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n), np.full(n, 1.0 / n),
             np.full(n, 0.01))]
    t = Tree(*arrs, n_ll=12, theta=0.7)
    assert L.rcb_refresh_noalloc_scratch(t.handle) > cap
    st = L.rcb_refresh_noalloc(t.handle, *[_ptr(a) for a in arrs], n, _stream())
    assert st == 4                                         # RCB_ECAPACITY
    assert b"rcb_refresh_noalloc" in L.rcb_last_error()
    t.destroy()
