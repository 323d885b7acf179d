"""GPU parity of the split variants of Sec. 2.1 "Load balancing" -- the
centre-of-number split (the centre of mass with unit weights) and the median
position split (equal halves, ties by caller index) -- against the oracle
built with the same split: tree bit-identical, lists and neighbour CSR
identical, accelerations within the bars."""
import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

from test_gpu_parity import SMALL, TOL, _np, _say, compare_lists, compare_trees, gate

pytestmark = pytest.mark.gpu


def _tree(c, n_ll, theta, precision="fp64", split="number"):
    import torch
    from paper_1108_0028_amd import Tree
    cv = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")
    return Tree(*[cv(a) for a in c.arrays()], n_ll=n_ll, theta=theta, precision=precision, split=split)


def _cloud(n, kind, seed):
    if kind == "ties":      # coordinates on a coarse grid, some -0: the median's tie rule
        c = W.small_random(n, seed, "uniform", h_scale=1.3)
        c.x[:] = np.round(c.x * 4) / 4
        c.y[:] = np.round(c.y * 3) / 3
        c.z[::3] = -0.0
        return c
    return W.small_random(n, seed, kind, h_scale=1.3)


@pytest.mark.parametrize("split", ["number", "median"])
@pytest.mark.parametrize("n,nll,kind", SMALL + [(5000, 4, "ties")])
def test_split_tree_lists_neighbours(n, nll, kind, split):
    c = _cloud(n, kind, 6000 + n)
    _say(split, "split", n, nll, kind)
    gt = _tree(c, nll, 0.7, split=split)
    ot = O.OracleTree(*c.arrays(), n_ll=nll, split=split)
    compare_trees(gt, ot)
    ot.walk(0.7)
    compare_lists(gt, ot)
    off, ids = gt.neighbours()
    ooff, oids, _ = ot.neighbours()
    np.testing.assert_array_equal(_np(off), ooff)
    np.testing.assert_array_equal(_np(ids), oids)
    ref = np.stack(ot.gravity(), 1)
    for prec in ("fp64", "mixed"):
        g = _tree(c, nll, 0.7, prec, split=split) if prec == "mixed" else gt
        a = np.stack([_np(v).astype(np.float64) for v in g.gravity()], 1)
        assert gate(a, ref) <= TOL[prec], (prec, gate(a, ref))
        g.destroy()


def test_number_split_equals_mass_split_for_power_of_two_masses():
    c = W.small_random(20000, 99, "plummer")
    c.m[:] = 2.0 ** -14
    _say("number vs mass split, equal masses 2^-14")
    a = _tree(c, 8, 0.7, split="mass")
    b = _tree(c, 8, 0.7, split="number")
    np.testing.assert_array_equal(_np(a.export("perm")), _np(b.export("perm")))
    nlab = a.info()["n_labels"]
    for f in ("lo", "hi", "com", "mass", "quad", "hint", "hnode"):   # label 0 is unused
        x, y = _np(a.export(f)).reshape(nlab, -1)[1:], _np(b.export(f)).reshape(nlab, -1)[1:]
        np.testing.assert_array_equal(x, y, err_msg=f)
    a.destroy()
    b.destroy()


@pytest.mark.parametrize("split", ["number", "median"])
def test_split_plummer_background_full_tree(split):
    c = W.plummer_background()
    _say(split, "split, plummer_background 4M: whole tree")
    gt = _tree(c, 12, 0.7, "mixed", split=split)
    ot = O.OracleTree(*c.arrays(), n_ll=12, split=split)
    compare_trees(gt, ot)
    gt.destroy()


def test_median_split_halves_and_renegades():
    # exact halves at every node, and on an unequal binary the median tree's
    # errors against the direct sum exceed the centre-of-mass tree's (Sec. 2.1)
    from oracle import brute
    c = W.binary_clumps()
    ref = brute.direct_accel(c.x, c.y, c.z, c.m, c.h)
    err = {}
    for split in ("mass", "median"):
        gt = _tree(c, 8, 0.7, split=split)
        cnt = _np(gt.export("count"))
        k = gt.info()["k"]
        if split == "median":
            for lab in range(1, 1 << k):
                assert cnt[2 * lab] == cnt[lab] // 2 and cnt[2 * lab + 1] == cnt[lab] - cnt[lab] // 2
        a = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)
        err[split] = np.mean(np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1))
        gt.destroy()
    assert err["median"] > 1.5 * err["mass"], err
