"""Trees on two streams at once, destroyed without waiting: the library keeps
freed blocks per stream and reads small values back through pinned host
memory, so steps on different streams, of different sizes, back to back,
must give exactly the results of one tree on the default stream."""
import numpy as np
import pytest

import workloads as W

from test_gpu_parity import _np, _say

pytestmark = pytest.mark.gpu


def _step(arrs, prec):
    from paper_1108_0028_amd import Tree
    t = Tree(*arrs, n_ll=8, theta=0.7, precision=prec)
    off, ids = t.neighbours()
    acc = t.gravity()
    t.destroy()   # returns at once: the frees are ordered on the stream
    return off, ids, acc


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_two_streams_back_to_back_match_the_default_stream(prec):
    import torch
    from paper_1108_0028_amd import release_cache
    clouds = [W.small_random(30000, 7, "clustered"), W.small_random(21000, 8, "plummer")]
    arrs = [[torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in c.arrays()] for c in clouds]
    ref = []
    for a in arrs:
        off, ids, acc = _step(a, prec)
        torch.cuda.synchronize()
        ref.append((_np(off), _np(ids), [_np(v) for v in acc]))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for a in arrs:
        for v in a:   # inputs were made on the default stream
            for st in streams:
                v.record_stream(st)
    torch.cuda.synchronize()
    outs = []
    for rep in range(3):
        for si, st in enumerate(streams):
            with torch.cuda.stream(st):
                ci = (rep + si) % 2   # each stream alternates between the two sizes
                _say("stream", si, "repeat", rep, "cloud", ci, prec)
                outs.append((ci, st, _step(arrs[ci], prec)))
    torch.cuda.synchronize()
    for ci, st, (off, ids, acc) in outs:
        r_off, r_ids, r_acc = ref[ci]
        np.testing.assert_array_equal(_np(off), r_off)
        np.testing.assert_array_equal(_np(ids), r_ids)
        for a, b in zip(acc, r_acc):
            np.testing.assert_array_equal(_np(a), b)
    release_cache()
    off, ids, acc = _step(arrs[0], prec)   # after the kept blocks went back to the pool
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(ids), ref[0][1])
