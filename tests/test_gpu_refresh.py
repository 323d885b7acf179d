"""Tree update (Sec. 2.1 "Updating the tree") followed by the per-step walk:
after rcb_refresh with moved positions and larger smoothing lengths the tree
is kept, but the interaction lists are made again from the new moments and
radii, so the neighbour lists still equal an all-pairs search and the
accelerations still match the oracle walked on the refreshed tree. With the
lists kept (the fixed tree of the VJP) the neighbour calls refuse until the
tree has been walked again."""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
import workloads as W

from test_gpu_parity import TOL, compare_lists, compare_trees, gate
from test_gpu_vjp import _np, _say, _t

pytestmark = pytest.mark.gpu


def _moved(c, seed, grow):
    rng = np.random.default_rng(seed)
    return [c.x + 3e-3 * rng.normal(size=c.n), c.y + 3e-3 * rng.normal(size=c.n),
            c.z + 3e-3 * rng.normal(size=c.n), c.m * rng.uniform(0.9, 1.1, c.n),
            c.h * grow * rng.uniform(1.0, 1.1, c.n)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("kind,grow", [("clustered", 1.3), ("uniform", 1.5)])
def test_refresh_walks_again(kind, grow, prec):
    from paper_1108_0028_amd import Tree
    c = W.small_random(3000, 61, kind)
    _say("refresh + walk", kind, grow, prec)
    tree = Tree(*[_t(a) for a in c.arrays()], n_ll=8, theta=0.6, precision=prec)
    tree.neighbours()
    tree.gravity()
    moved = _moved(c, 62, grow)
    tree.refresh(*[_t(a) for a in moved])
    ot = O.OracleTree(*c.arrays(), n_ll=8)
    ot.refresh(*moved)
    ot.walk(0.6)
    compare_trees(tree, ot)
    compare_lists(tree, ot)
    off, ids = tree.neighbours()
    off, ids = _np(off).astype(np.int64), _np(ids).astype(np.int64)
    ooff, oids, _ = ot.neighbours()
    np.testing.assert_array_equal(off, ooff)
    np.testing.assert_array_equal(ids, oids)
    aoff, aids = brute.neighbours(*moved[:3], moved[4])   # ascending ids per list
    np.testing.assert_array_equal(off, aoff)
    np.testing.assert_array_equal(ids, aids)
    acc = np.stack([_np(v) for v in tree.gravity()], 1)
    ref = np.stack(ot.gravity(), 1)
    assert gate(acc, ref) <= TOL[prec]


def test_kept_lists_refuse_neighbours_until_walked():
    from paper_1108_0028_amd import RcbError, Tree
    c = W.small_random(2000, 63, "clustered")
    _say("refresh keep_lists")
    tree = Tree(*[_t(a) for a in c.arrays()], n_ll=8, theta=0.6)
    tree.walk()
    moved = _moved(c, 64, 1.3)
    tree.refresh(*[_t(a) for a in moved], keep_lists=True)
    with pytest.raises(RcbError) as e:
        tree.neighbours()
    assert e.value.status == 5   # RCB_ESTATE
    # gravity keeps the old lists: the oracle refreshed without a new walk
    ot = O.OracleTree(*c.arrays(), n_ll=8)
    ot.walk(0.6)
    ot.refresh(*moved)
    acc = np.stack([_np(v) for v in tree.gravity()], 1)
    assert gate(acc, np.stack(ot.gravity(), 1)) <= 1e-11
    tree.walk()
    ot.walk(0.6)
    compare_lists(tree, ot)
    off, ids = tree.neighbours()
    ooff, oids, _ = ot.neighbours()
    np.testing.assert_array_equal(_np(off).astype(np.int64), ooff)
    np.testing.assert_array_equal(_np(ids).astype(np.int64), oids)
