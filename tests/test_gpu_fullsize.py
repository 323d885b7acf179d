"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times: the whole tree is compared bit for bit, and the
lists, neighbour lists and accelerations of a seeded sample of lowest-level
cells against the oracle walking only those cells (Sec. 2.2-2.4). The VJP at
full size is compared element by element with the oracle's for cotangents
that are non-zero on the sampled cells only (every particle still receives
source-side terms through the node adjoints, including those of nodes below
level 16), checked by central differences, and checked through properties
that hold at any size (translation invariance with the lists fixed;
accelerations are homogeneous of degree 1 in the masses, so
sum_b m_b dL/dm_b = L)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

from test_gpu_parity import TOL, _gpu_tree, _np, _say, compare_lists, compare_trees, gate
from test_gpu_vjp import TOL as VTOL

pytestmark = pytest.mark.gpu

SAMPLE = 192   # lowest-level cells compared per case


def _sample_leaves(ot, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(ot.n_leaves, SAMPLE, replace=False)) + ot.n_leaves


def _sampled_parity(c, n_ll, theta, precisions, seed):
    ot = O.OracleTree(*c.arrays(), n_ll=n_ll)
    leaves = _sample_leaves(ot, seed)
    ot.walk(theta, leaves)
    topo = ot.topology()
    first, count = topo["first"], topo["count"]
    pos = np.concatenate([np.arange(first[l], first[l] + count[l]) for l in leaves])
    sel = topo["perm"][pos]                          # caller indices of the sampled sinks
    ooff, oids, valid = ot.neighbours()
    assert valid[sel].all()
    ref = np.stack(ot.gravity(), 1)[sel]
    for prec in precisions:
        _say("full size", c.n, n_ll, theta, prec)
        gt = _gpu_tree(c, n_ll, theta, prec)
        if prec == precisions[0]:
            compare_trees(gt, ot)
            compare_lists(gt, ot, leaves)
        off, ids = gt.neighbours()
        off, ids = _np(off), _np(ids)
        for a in sel[:4096]:
            np.testing.assert_array_equal(ids[off[a]:off[a + 1]], oids[ooff[a]:ooff[a + 1]],
                                          err_msg=f"neighbours of particle {a}")
        np.testing.assert_array_equal(off[sel + 1] - off[sel], ooff[sel + 1] - ooff[sel])
        acc = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)[sel]
        g = gate(acc, ref)
        assert g <= TOL[prec], (prec, theta, g)
        if prec == "fp64":
            assert g <= 1e-11, (theta, g)
        gt.destroy()


def test_plummer_1m_theta_05_and_07():
    c = W.plummer()
    for k, theta in enumerate((0.5, 0.7)):
        _sampled_parity(c, 12, theta, ("fp64", "mixed"), seed=20 + k)


def test_plummer_background_4m_bench_configuration():
    c = W.plummer_background()
    _sampled_parity(c, 12, 0.7, ("mixed", "fp64"), seed=30)


def _cells_and_cotangents(ot, nleaves, seed):
    """Sampled lowest-level cells, their particles (caller indices) and N(0,1)
    cotangents on those particles only."""
    rng = np.random.default_rng(seed)
    leaves = np.sort(rng.choice(ot.n_leaves, nleaves, replace=False)) + ot.n_leaves
    topo = ot.topology()
    pos = np.concatenate([np.arange(topo["first"][l], topo["first"][l] + topo["count"][l]) for l in leaves])
    sel = topo["perm"][pos]
    g = [np.zeros(ot.n) for _ in range(3)]
    for a in g:
        a[sel] = rng.normal(size=sel.size)
    return leaves, sel, g


def _vjp(gt, g, prec):
    import torch
    dt = torch.float32 if prec == "mixed" else torch.float64
    return [_np(o).astype(np.float64) for o in gt.vjp(*[torch.from_numpy(a).to("cuda:0", dt) for a in g])]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("workload,nleaves", [("plummer", 128), ("plummer_background", 64)])
def test_vjp_elementwise_sampled_cells(workload, nleaves):
    c = getattr(W, workload)()
    ot = O.OracleTree(*c.arrays(), n_ll=12)
    leaves, sel, g = _cells_and_cotangents(ot, nleaves, 40 + nleaves)
    ot.walk(0.7, leaves)
    ot.cache_sizes()
    far_labels = np.concatenate([ot.leaf_lists(int(l))[1] for l in leaves])
    assert far_labels.max() >= 1 << 16     # node adjoints of the deep levels are exercised
    _say("vjp sampled cells: oracle", workload, len(leaves), "cells")
    ref = ot.vjp(*g)
    for prec in ("fp64", "mixed"):
        _say("vjp sampled cells", workload, prec)
        gt = _gpu_tree(c, 12, 0.7, prec)
        gt.gravity()
        got = _vjp(gt, g, prec)
        for name, a, b in zip(("dx", "dy", "dz", "dm"), got, ref):
            err = float(np.abs(a - b).max() / np.abs(b).max())
            print(f"   {name} rel err {err:.2e}", flush=True)
            assert err <= VTOL[prec], (prec, name, err)
        gt.destroy()


def test_vjp_mixed_against_fp64_1m():
    """Full N(0,1) cotangents at 1M particles: the mixed form's VJP (FP32
    pairs and FP32 atomic sums of node adjoints and source terms) against the
    FP64 form's on the same tree and lists, element by element. The FP64 VJP
    itself equals the oracle's (tests above and test_gpu_vjp.py)."""
    c = W.plummer()
    g = W.cotangents(c.n)
    out = {}
    for prec in ("fp64", "mixed"):
        _say("vjp full cotangents 1M", prec)
        gt = _gpu_tree(c, 12, 0.7, prec)
        gt.gravity()
        out[prec] = _vjp(gt, g, prec)
        gt.destroy()
    for name, a, b in zip(("dx", "dy", "dz", "dm"), out["mixed"], out["fp64"]):
        err = float(np.abs(a - b).max() / np.abs(b).max())
        print(f"   mixed vs fp64 {name} rel err {err:.2e}", flush=True)
        assert err <= VTOL["mixed"], (name, err)


def test_vjp_central_differences_1m():
    """Central differences (eps = 1e-6, relative for masses) of
    L = sum g . a on the fixed tree at 1M particles, FP64, for particles inside
    and outside the cells that carry the cotangents."""
    import torch
    from paper_1108_0028_amd import Tree
    c = W.plummer()
    ot = O.OracleTree(*c.arrays(), n_ll=12)
    _, sel, g = _cells_and_cotangents(ot, 128, 50)
    del ot
    dev = torch.device("cuda:0")
    base = [np.array(a, dtype=np.float64) for a in c.arrays()]
    tree = Tree(*[torch.from_numpy(a).to(dev) for a in base], n_ll=12, theta=0.7)
    tree.walk()
    grads = _vjp(tree, g, "fp64")
    gd = [torch.from_numpy(a).to(dev) for a in g]

    def L(comp, b, delta):
        vals = [torch.from_numpy(a).to(dev) for a in base]
        vals[comp][b] += delta
        tree.refresh(*vals, keep_lists=True)
        acc = tree.gravity()
        return float(sum((gi * ai).sum() for gi, ai in zip(gd, acc)))

    rng = np.random.default_rng(51)
    picks = list(rng.choice(sel, 3, replace=False)) + list(rng.choice(c.n, 3, replace=False))
    for b in picks:
        for comp in range(4):
            eps = 1e-6 if comp < 3 else 1e-6 * base[3][b]
            fd = (L(comp, b, eps) - L(comp, b, -eps)) / (2 * eps)
            grad = grads[comp]
            scale = np.max(np.abs(grad)) if comp < 3 else np.max(np.abs(grad * base[3]))
            err = abs(fd - grad[b]) * (1.0 if comp < 3 else base[3][b])
            _say("fd 1M", int(b), comp, fd, grad[b])
            assert err <= 1e-6 * scale, (int(b), comp, fd, grad[b])
    tree.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_vjp_properties_1m(precision):
    import torch
    c = W.plummer()
    _say("vjp properties", c.n, precision)
    gt = _gpu_tree(c, 12, 0.7, precision)
    dt = torch.float32 if precision == "mixed" else torch.float64
    g = [torch.from_numpy(v).to("cuda:0", dt) for v in W.cotangents(c.n)]
    acc = gt.gravity()
    dx, dy, dz, dm = gt.vjp(*g)
    dr = torch.stack([dx, dy, dz], 1).double()
    # translation invariance: the lists are fixed, so a common shift changes nothing
    scale = float(dr.abs().sum(0).max())
    drift = float(dr.sum(0).abs().max())
    tol = VTOL[precision]
    assert drift <= tol * scale, (drift, scale)
    # homogeneity of degree 1 in the masses
    L = float(sum((gi.double() * ai.double()).sum() for gi, ai in zip(g, acc)))
    m = torch.from_numpy(c.m).to("cuda:0", torch.float64)
    euler = float((m * dm.double()).sum())
    assert abs(euler - L) <= tol * float((m * dm.double()).abs().sum()), (euler, L)
    gt.destroy()


@pytest.mark.timeout(900)
def test_clumpy_cube_2p26_against_oracle():
    """The scaling workload at 2^26 particles (k = 23, the depth of the 10^8
    run): the oracle builds the same tree on the host, and the whole tree, the
    lists of 128 sampled lowest-level cells, their particles' neighbour lists
    and accelerations (both forms) are compared with it."""
    import torch
    n = 1 << 26
    c = W.clumpy_cube(n)
    _say("clumpy cube 2^26: oracle build")
    ot = O.OracleTree(*c.arrays(), n_ll=12)
    assert ot.k == 23
    leaves = _sample_leaves(ot, 60)
    ot.walk(0.7, leaves)
    topo = ot.topology()
    pos = np.concatenate([np.arange(topo["first"][l], topo["first"][l] + topo["count"][l]) for l in leaves])
    sel = topo["perm"][pos]
    del topo
    ooff, oids, valid = ot.neighbours()
    assert valid[sel].all()
    ref = np.stack(ot.gravity(), 1)[sel]
    for prec in ("mixed", "fp64"):
        _say("clumpy cube 2^26", prec)
        gt = _gpu_tree(c, 12, 0.7, prec)
        if prec == "mixed":
            compare_trees(gt, ot)
            compare_lists(gt, ot, leaves)
        off, ids = gt.neighbours()
        off = _np(off)
        np.testing.assert_array_equal(off[sel + 1] - off[sel], ooff[sel + 1] - ooff[sel])
        for a in sel[:2048]:
            np.testing.assert_array_equal(_np(ids[off[a]:off[a + 1]]), oids[ooff[a]:ooff[a + 1]],
                                          err_msg=f"neighbours of particle {a}")
        del off, ids
        acc = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)[sel]
        err = gate(acc, ref)
        assert err <= (1e-11 if prec == "fp64" else TOL[prec]), (prec, err)
        gt.destroy()
        torch.cuda.empty_cache()
    from paper_1108_0028_amd import release_cache
    release_cache()


def test_clumpy_cube_1e8_properties():
    """10^8 particles (the scaling workload's largest size), mixed and FP64:
    the neighbour lists of sampled particles equal an all-pairs search over
    all particles, and the two forms agree within the mixed form's bar on
    sampled particles (each form is checked against the oracle at the sizes
    above)."""
    import torch
    from paper_1108_0028_amd import Tree
    n = 100_000_000
    c = W.clumpy_cube(n)
    _say("clumpy cube", n)
    dev = torch.device("cuda:0")
    arrs = [torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in c.arrays()]
    del c
    rng = np.random.default_rng(8)
    sel = torch.from_numpy(np.sort(rng.choice(n, 4096, replace=False))).to(dev)
    acc = {}
    for prec in ("mixed", "fp64"):
        t = Tree(*arrs, n_ll=12, theta=0.7, precision=prec)
        assert t.info()["k"] == 23
        off, ids = t.neighbours()
        if prec == "mixed":
            x, y, z, h = arrs[0], arrs[1], arrs[2], arrs[4]
            for i in sel[:24].tolist():
                dx, dy, dz = x - x[i], y - y[i], z - z[i]
                d2 = (dx * dx + dy * dy) + dz * dz
                exact = torch.nonzero((d2 < (2.0 * h[i]) ** 2) & (torch.arange(n, device=dev) != i)).flatten()
                got = ids[int(off[i]):int(off[i + 1])].long()
                assert torch.equal(got, exact), i   # ascending by index
        del off, ids
        acc[prec] = torch.stack([v.double() for v in t.gravity()], 1)[sel].cpu().numpy()
        t.destroy()
        torch.cuda.empty_cache()
    from paper_1108_0028_amd import release_cache
    release_cache()
    g = gate(acc["mixed"], acc["fp64"])
    assert g <= TOL["mixed"], g
