"""The VJP takes the far-field coefficients that rcb_gravity kept for the
current moments, and computes them itself when none are kept: after a
gravity call, after rcb_refresh (which discards them) and after gravity on
the refreshed moments, rcb_gravity_vjp must equal the oracle's fixed-tree
VJP (the FP64 bar of 1e-9 exposes coefficients of the wrong moments), and a
VJP that takes kept coefficients must equal one that computed them."""
import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

from test_gpu_vjp import TOL, _np, _say, _t

pytestmark = pytest.mark.gpu


def _rel(got, ref):
    return max(np.abs(a - b).max() / np.abs(b).max() for a, b in zip(got, ref))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_vjp_with_kept_and_computed_coefficients(prec):
    import torch
    from paper_1108_0028_amd import Tree
    c = W.small_random(3000, 41, "clustered")
    g = W.cotangents(c.n, seed=9)
    dt = torch.float32 if prec == "mixed" else torch.float64
    gt = [_t(a, dt) for a in g]
    ot = O.OracleTree(*c.arrays(), n_ll=8)
    ot.walk(0.6)
    ref = ot.vjp(*g)

    _say("vjp without a gravity call", prec)
    fresh = Tree(*[_t(a) for a in c.arrays()], n_ll=8, theta=0.6, precision=prec)
    computed = [_np(o) for o in fresh.vjp(*gt)]
    fresh.destroy()
    assert _rel(computed, ref) <= TOL[prec]

    _say("vjp after gravity", prec)
    tree = Tree(*[_t(a) for a in c.arrays()], n_ll=8, theta=0.6, precision=prec)
    tree.gravity()
    kept = [_np(o) for o in tree.vjp(*gt)]
    assert _rel(kept, ref) <= TOL[prec]
    assert _rel(kept, computed) <= (1e-12 if prec == "fp64" else 1e-5)

    rng = np.random.default_rng(5)
    moved = [c.x + 2e-3 * rng.normal(size=c.n), c.y + 2e-3 * rng.normal(size=c.n),
             c.z + 2e-3 * rng.normal(size=c.n), c.m * rng.uniform(0.9, 1.1, c.n), c.h]
    tree.refresh(*[_t(a) for a in moved], keep_lists=True)   # the VJP's fixed tree
    ot.refresh(*moved)
    ref2 = ot.vjp(*g)
    stale = _rel(ref2, ref)
    _say("vjp after refresh", prec, "moved-input VJP change", stale)
    got2 = [_np(o) for o in tree.vjp(*gt)]
    assert _rel(got2, ref2) <= TOL[prec]
    _say("vjp after gravity on the refreshed moments", prec)
    tree.gravity()
    got3 = [_np(o) for o in tree.vjp(*gt)]
    assert _rel(got3, ref2) <= TOL[prec]
    if prec == "fp64":
        assert stale > 1e3 * TOL[prec]   # old coefficients would fail the bar
    tree.destroy()
