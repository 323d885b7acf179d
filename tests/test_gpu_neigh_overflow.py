"""Neighbour lists longer than the per-particle slab of the count call
(Sec. 2.3 "Neighbour list"): the ranks past it go through an overflow pool
that the fill call places, and when the pool itself runs out the groups
holding such particles are searched again. Both routes must give the
oracle's CSR exactly (lists in tree order), and the all-pairs sets.

  uniform, h x 2:    mean ~190, max ~680 neighbours; ~3.5e5 entries past the
                     slab, which the pool (>= 2^20 entries) holds
  uniform, h x 40:   every pair; ~8.4e6 entries past the slab, more than the
                     pool: the re-search route
"""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
import workloads as W

from test_gpu_parity import _gpu_tree, _np, _say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,kind,hs,nll", [(6000, "uniform", 2.0, 8), (3000, "uniform", 40.0, 6)])
def test_long_neighbour_lists(n, kind, hs, nll):
    c = W.small_random(n, 11 + n, kind, h_scale=hs)
    _say("long neighbour lists", n, kind, hs)
    ot = O.OracleTree(*c.arrays(), n_ll=nll)
    ot.walk(0.7)
    ooff, oids, valid = ot.neighbours()
    assert valid.all()
    assert np.diff(ooff).max() > 192
    gt = _gpu_tree(c, nll, 0.7)
    for _ in range(2):   # a second count/fill on the same tree reuses the slab and pool
        off, ids = gt.neighbours()
        np.testing.assert_array_equal(_np(off), ooff)
        np.testing.assert_array_equal(_np(ids), oids)
    boff, bids = brute.neighbours(c.x, c.y, c.z, c.h)
    np.testing.assert_array_equal(ooff, boff)
    g = _np(ids)
    for i in range(0, n, 97):
        assert sorted(g[ooff[i]:ooff[i + 1]].tolist()) == bids[boff[i]:boff[i + 1]].tolist()
    gt.destroy()
