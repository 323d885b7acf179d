"""GPU parity of Taylor reading B (the quadrupole in f only, J and H of the
monopole field; the default is reading A) against the oracle with the same
reading, and the VJP's refusal of such trees."""
import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

from test_gpu_parity import SMALL, TOL, _np, _say, gate

pytestmark = pytest.mark.gpu


def _tree(c, n_ll, theta, precision):
    import torch
    from paper_1108_0028_amd import Tree
    cv = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")
    return Tree(*[cv(a) for a in c.arrays()], n_ll=n_ll, theta=theta, precision=precision,
                taylor_reading="B")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n,nll,kind", SMALL)
def test_reading_b_gravity_matches_oracle(n, nll, kind, precision):
    c = W.small_random(n, 7000 + n, kind)
    ot = O.OracleTree(*c.arrays(), n_ll=nll)
    ot.set_reading("B")
    for theta in (0.5, 0.8):
        _say("reading B", precision, n, nll, kind, theta)
        gt = _tree(c, nll, theta, precision)
        a = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)
        ot.walk(theta)
        g = gate(a, np.stack(ot.gravity(), 1))
        assert g <= TOL[precision], (precision, theta, g)
        if precision == "fp64":
            assert g <= 1e-11, (theta, g)
        gt.destroy()


def test_reading_b_plummer_1m_sampled_and_no_vjp():
    import torch
    c = W.plummer()
    ot = O.OracleTree(*c.arrays(), n_ll=12)
    ot.set_reading("B")
    rng = np.random.default_rng(51)
    leaves = np.sort(rng.choice(ot.n_leaves, 128, replace=False)) + ot.n_leaves
    ot.walk(0.7, leaves)
    topo = ot.topology()
    pos = np.concatenate([np.arange(topo["first"][l], topo["first"][l] + topo["count"][l]) for l in leaves])
    sel = topo["perm"][pos]
    ref = np.stack(ot.gravity(), 1)[sel]
    for prec in ("mixed", "fp64"):
        _say("reading B 1M sampled", prec)
        gt = _tree(c, 12, 0.7, prec)
        acc = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)[sel]
        assert gate(acc, ref) <= TOL[prec]
        if prec == "fp64":
            g = [torch.zeros(c.n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
            with pytest.raises(RuntimeError, match="reading A"):
                gt.vjp(*g)
        gt.destroy()
