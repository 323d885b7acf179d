"""GPU parity of the pure-MAC walk (the variant of Sec. 2.5 in which
reachability does not override the MAC) against the oracle's pure-MAC walk:
lists bit-identical (candidate-only entries included), neighbour CSR
identical, accelerations and VJP within the same bars as the paper's walk,
and at 1M Plummer particles on sampled cells."""
import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

from test_gpu_parity import SMALL, TOL, _gpu_tree, _np, _say, compare_lists, gate
from test_gpu_vjp import TOL as VJP_TOL
from test_gpu_vjp import _t

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,nll,kind", SMALL)
def test_pure_mac_lists_and_neighbours_identical(n, nll, kind):
    c = W.small_random(n, 4000 + n, kind, h_scale=1.5)
    ot = O.OracleTree(*c.arrays(), n_ll=nll)
    for theta in (0.5, 0.9):
        _say("pure-MAC lists", n, nll, kind, theta)
        gt = _gpu_tree(c, nll, theta, pure_mac=True)
        ot.walk(theta, pure_mac=True)
        compare_lists(gt, ot)
        off, ids = gt.neighbours()
        ooff, oids, _ = ot.neighbours()
        np.testing.assert_array_equal(_np(off), ooff)
        np.testing.assert_array_equal(_np(ids), oids)
        gt.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n,nll,kind", SMALL)
def test_pure_mac_gravity_matches_oracle(n, nll, kind, precision):
    c = W.small_random(n, 5000 + n, kind)
    ot = O.OracleTree(*c.arrays(), n_ll=nll)
    for theta in (0.0, 0.5, 0.8):
        _say("pure-MAC gravity", precision, n, nll, kind, theta)
        gt = _gpu_tree(c, nll, theta, precision, pure_mac=True)
        a = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)
        ot.walk(theta, pure_mac=True)
        g = gate(a, np.stack(ot.gravity(), 1))
        assert g <= TOL[precision], (precision, theta, g)
        if precision == "fp64":
            assert g <= 1e-11, (theta, g)
        gt.destroy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pure_mac_vjp_matches_oracle(prec):
    import torch
    from paper_1108_0028_amd import Tree
    c = W.small_random(3000, 77, "clustered")
    g = W.cotangents(c.n, seed=78)
    ot = O.OracleTree(*c.arrays(), n_ll=6)
    dt = torch.float32 if prec == "mixed" else torch.float64
    for theta in (0.5, 0.8):
        _say("pure-MAC vjp", prec, theta)
        ot.walk(theta, pure_mac=True)
        ref = ot.vjp(*g)
        tree = Tree(*[_t(a) for a in c.arrays()], n_ll=6, theta=theta, precision=prec, pure_mac=True)
        got = [_np(o).astype(np.float64) for o in tree.vjp(*[_t(a, dt) for a in g])]
        for name, a, b in zip(("dx", "dy", "dz", "dm"), got, ref):
            err = np.abs(a - b).max() / np.abs(b).max()
            assert err <= VJP_TOL[prec], (name, theta, err)
        tree.destroy()


def test_pure_mac_plummer_1m_sampled():
    c = W.plummer()
    ot = O.OracleTree(*c.arrays(), n_ll=12)
    rng = np.random.default_rng(41)
    leaves = np.sort(rng.choice(ot.n_leaves, 128, replace=False)) + ot.n_leaves
    ot.walk(0.7, leaves, pure_mac=True)
    topo = ot.topology()
    first, count = topo["first"], topo["count"]
    pos = np.concatenate([np.arange(first[l], first[l] + count[l]) for l in leaves])
    sel = topo["perm"][pos]
    ooff, oids, valid = ot.neighbours()
    assert valid[sel].all()
    ref = np.stack(ot.gravity(), 1)[sel]
    for prec in ("mixed", "fp64"):
        _say("pure-MAC 1M sampled", prec)
        gt = _gpu_tree(c, 12, 0.7, prec, pure_mac=True)
        if prec == "mixed":
            compare_lists(gt, ot, leaves)
        off, ids = gt.neighbours()
        off, ids = _np(off), _np(ids)
        np.testing.assert_array_equal(off[sel + 1] - off[sel], ooff[sel + 1] - ooff[sel])
        for a in sel[:2048]:
            np.testing.assert_array_equal(ids[off[a]:off[a + 1]], oids[ooff[a]:ooff[a + 1]])
        acc = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)[sel]
        g = gate(acc, ref)
        assert g <= TOL[prec], (prec, g)
        gt.destroy()
