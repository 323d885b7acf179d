"""Workspace from the caller's allocator (rcb_params.alloc / free, here
PyTorch's caching allocator): the same results as with the library's own
pool, and every block returned when the tree is destroyed."""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import _np, _say

pytestmark = pytest.mark.gpu


def test_torch_allocator_gives_the_same_results_and_returns_every_block():
    import torch
    from paper_1108_0028_amd import Tree
    c = W.small_random(60000, 91, "plummer")
    arrs = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in c.arrays()]
    g = [torch.from_numpy(v).to("cuda:0") for v in W.cotangents(c.n, seed=3)]
    out = {}
    for alloc in ("library", "torch"):
        _say("allocator", alloc)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        t = Tree(*arrs, n_ll=8, theta=0.7, precision="fp64", allocator=alloc)
        off, ids = t.neighbours()
        acc = t.gravity()
        vjp = t.vjp(*g)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - before
        out[alloc] = ([_np(off), _np(ids)], [_np(v) for v in acc], [_np(v) for v in vjp], held)
        t.destroy()
        del off, ids, acc, vjp
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before, alloc
    lib, tor = out["library"], out["torch"]
    for a, b in zip(lib[0], tor[0]):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(lib[1], tor[1]):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(lib[2], tor[2]):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    # the tree's workspace came from torch: it held more than the outputs alone
    assert tor[3] > lib[3] + 8 * c.n
