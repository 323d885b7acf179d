"""The wide group walk (a FIFO of 1024 nodes, then 8192 for the groups that
outgrow it) and the 8-wide walk that takes the groups outgrowing both make
the same per-leaf decisions (Sec. 2.2-2.4.1). With the FIFOs capped through
RCB_WALK_WIDE_STACK, so that all, many or a few groups are walked again over
what the first walk wrote, and at the default sizes (where the clustered
cases send groups to the 8192-node FIFO), the lists, neighbours and
accelerations still match the oracle, in both walk modes and through the
exact second pass that long lists take."""
import os

import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

from test_gpu_parity import TOL, _gpu_tree, _np, _say, compare_lists, gate

pytestmark = pytest.mark.gpu

CASES = [(777, 3, "uniform", 1.5), (12305, 6, "clustered", 1.5), (40000, 12, "plummer", 1.5),
         (9000, 6, "clustered", 40.0)]   # the last: near lists past the slab (exact pass)


@pytest.fixture
def wide_cap():
    old = os.environ.get("RCB_WALK_WIDE_STACK")

    def set_cap(v):
        if v is None:
            os.environ.pop("RCB_WALK_WIDE_STACK", None)
        else:
            os.environ["RCB_WALK_WIDE_STACK"] = str(v)

    yield set_cap
    set_cap(old)


@pytest.mark.parametrize("pure", [False, True])
@pytest.mark.parametrize("n,nll,kind,hs", CASES)
def test_capped_wide_stack_gives_the_same_lists(n, nll, kind, hs, pure, wide_cap):
    c = W.small_random(n, 7000 + n, kind, h_scale=hs)
    ot = O.OracleTree(*c.arrays(), n_ll=nll)
    ot.walk(0.6, pure_mac=pure)
    ref = np.stack(ot.gravity(), 1)
    if hs < 10:
        ooff, oids, _ = ot.neighbours()
    requeued = {}
    for cap in (None, 2, 24, 96):
        _say("walk fallback", n, nll, kind, hs, "pure" if pure else "paper", "cap", cap)
        wide_cap(cap)
        gt = _gpu_tree(c, nll, 0.6, pure_mac=pure)
        compare_lists(gt, ot)
        requeued[cap] = gt.info()["walk_requeued"]
        if hs < 10:
            off, ids = gt.neighbours()
            np.testing.assert_array_equal(_np(off), ooff)
            np.testing.assert_array_equal(_np(ids), oids)
        ax, ay, az = gt.gravity()
        assert gate(np.stack([_np(ax), _np(ay), _np(az)], 1), ref) < TOL["fp64"]
        gt.destroy()
    wide_cap(None)
    assert requeued[2] > 0 and requeued[2] >= requeued[24] >= requeued[96] >= requeued[None]
    if (n, kind, pure) == (12305, "clustered", False):
        assert requeued[None] > 0   # wide frontiers: the 8192-node FIFO took these groups
