"""Neighbour lists longer than the per-particle row of the count call
(Sec. 2.3.2 "Neighbour list"): the count call keeps the first 64 ids of each
particle in its row and the next ones in up to three 64-slot chunks from a
shared pool, and queues the lowest-level cells holding a list that fit
neither (longer than 256, or the pool ran out); the fill call sorts the kept
lists, searches the queued cells again, one wave each, writing only those
lists, and sorts each of them in one workgroup (in LDS up to 4096 ids, in
place in the CSR beyond). The CSR must be the oracle's exactly (every list
ascending by caller index) and equal the all-pairs search.

  plummer, h x 1:    ~50 neighbours, a few percent of the lists past the row
  clumpy cube 40000: mean ~77, 21% of the lists past the row, 7% past 256: the
                     row and 1-3 chunks, and the pool runs out (both paths)
  uniform, h x 2:    mean ~190, max ~680 neighbours (most lists past the row)
  uniform, h x 40:   every pair: lists of n - 1 (3000: sorted in LDS; 5000:
                     sorted in place, 4999 > 4096)
"""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
import workloads as W

from test_gpu_parity import _gpu_tree, _np, _say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,kind,hs,nll", [(20000, "plummer", 1.0, 12), (40000, "clumpy", 1.0, 12),
                                           (6000, "uniform", 2.0, 8), (3000, "uniform", 40.0, 6),
                                           (5000, "uniform", 40.0, 6)])
def test_long_neighbour_lists(n, kind, hs, nll):
    c = W.clumpy_cube(n) if kind == "clumpy" else W.small_random(n, 11 + n, kind, h_scale=hs)
    _say("long neighbour lists", n, kind, hs)
    ot = O.OracleTree(*c.arrays(), n_ll=nll)
    ot.walk(0.7)
    ooff, oids, valid = ot.neighbours()
    assert valid.all()
    cnt = np.diff(ooff)
    assert (cnt > 64).any() and cnt.max() > 64
    boff, bids = brute.neighbours(c.x, c.y, c.z, c.h)
    np.testing.assert_array_equal(ooff, boff)
    np.testing.assert_array_equal(oids, bids)
    gt = _gpu_tree(c, nll, 0.7)
    for _ in range(2):   # a second count/fill on the same tree reuses the slab
        off, ids = gt.neighbours()
        np.testing.assert_array_equal(_np(off), ooff)
        np.testing.assert_array_equal(_np(ids), oids)
    gt.destroy()
