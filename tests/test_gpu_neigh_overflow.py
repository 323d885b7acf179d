"""Neighbour lists longer than the per-particle slab of the count call
(Sec. 2.3 "Neighbour list"): the count call keeps the first 192 ids of each
particle and queues the lowest-level cells holding a longer list; the fill
call searches those cells again, one wave each, writing whole lists. The CSR
must be the oracle's exactly (lists in tree order), and the all-pairs sets.

  uniform, h x 2:    mean ~190, max ~680 neighbours (~40% of the particles
                     past the slab)
  uniform, h x 40:   every pair (all cells queued)
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
