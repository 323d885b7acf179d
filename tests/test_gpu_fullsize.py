"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times: the whole tree is compared bit for bit, and the
lists, neighbour lists and accelerations of a seeded sample of lowest-level
cells against the oracle walking only those cells (Sec. 2.2-2.4). The VJP at
full size is checked through properties that hold at any size (translation
invariance with the lists fixed; accelerations are homogeneous of degree 1 in
the masses, so sum_b m_b dL/dm_b = L)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

from test_gpu_parity import TOL, _gpu_tree, _np, _say, compare_lists, compare_trees, gate

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
    tol = 1e-9 if precision == "fp64" else 2e-3
    assert drift <= tol * scale, (drift, scale)
    # homogeneity of degree 1 in the masses
    L = float(sum((gi.double() * ai.double()).sum() for gi, ai in zip(g, acc)))
    m = torch.from_numpy(c.m).to("cuda:0", torch.float64)
    euler = float((m * dm.double()).sum())
    assert abs(euler - L) <= tol * float((m * dm.double()).abs().sum()), (euler, L)
    gt.destroy()


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
                assert torch.equal(torch.sort(got).values, exact), i
        del off, ids
        acc[prec] = torch.stack([v.double() for v in t.gravity()], 1)[sel].cpu().numpy()
        t.destroy()
        torch.cuda.empty_cache()
    g = gate(acc["mixed"], acc["fp64"])
    assert g <= TOL["mixed"], g
