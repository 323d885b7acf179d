"""GPU parity of the centre-of-number split (Sec. 2.1 "Load balancing": the
split plane is the centre of mass with unit weights) against the oracle built
with the same split: tree bit-identical, lists and neighbour CSR identical,
accelerations within the bars."""
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


@pytest.mark.parametrize("n,nll,kind", SMALL)
def test_number_split_tree_lists_neighbours(n, nll, kind):
    c = W.small_random(n, 6000 + n, kind, h_scale=1.3)
    _say("number split", n, nll, kind)
    gt = _tree(c, nll, 0.7)
    ot = O.OracleTree(*c.arrays(), n_ll=nll, split="number")
    compare_trees(gt, ot)
    ot.walk(0.7)
    compare_lists(gt, ot)
    off, ids = gt.neighbours()
    ooff, oids, _ = ot.neighbours()
    np.testing.assert_array_equal(_np(off), ooff)
    np.testing.assert_array_equal(_np(ids), oids)
    ref = np.stack(ot.gravity(), 1)
    for prec in ("fp64", "mixed"):
        g = _tree(c, nll, 0.7, prec) if prec == "mixed" else gt
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


def test_number_split_plummer_background_full_tree():
    c = W.plummer_background()
    _say("number split, plummer_background 4M: whole tree")
    gt = _tree(c, 12, 0.7, "mixed")
    ot = O.OracleTree(*c.arrays(), n_ll=12, split="number")
    compare_trees(gt, ot)
    gt.destroy()
