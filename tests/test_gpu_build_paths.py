"""The two ways the device build reaches the lowest level (Sec. 2.1
"Strategy"): by default, nodes of at most 512 particles and 6 levels are
finished by one wave each in LDS (subtrees) and only the bigger ones go
through the device-wide level passes; with RCB_BUILD_LEVELS set in the
environment every level is one device-wide pass (the path the median split
and the moments-only refresh always take). Both must give the oracle's tree
bit for bit, and so the same lists, neighbours and accelerations."""
import os

import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

from test_gpu_parity import _gpu_tree, _np, _say, compare_lists, compare_trees

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,nll,kind", [(3000, 8, "clustered"), (40000, 12, "plummer"), (9000, 1, "uniform")])
def test_level_passes_and_subtrees_build_the_same_tree(n, nll, kind):
    c = W.small_random(n, 500 + n, kind)
    ot = O.OracleTree(*c.arrays(), n_ll=nll)
    ot.walk(0.7)
    out = {}
    for path in ("subtrees", "levels"):
        _say("build path", path, n, nll, kind)
        if path == "levels":
            os.environ["RCB_BUILD_LEVELS"] = "1"
        try:
            gt = _gpu_tree(c, nll, 0.7)
            compare_trees(gt, ot)
            compare_lists(gt, ot)
            off, ids = gt.neighbours()
            acc = np.stack([_np(v) for v in gt.gravity()], 1)
            out[path] = (_np(off), _np(ids), acc)
            gt.destroy()
        finally:
            os.environ.pop("RCB_BUILD_LEVELS", None)
    for a, b in zip(out["subtrees"], out["levels"]):
        np.testing.assert_array_equal(a, b)
