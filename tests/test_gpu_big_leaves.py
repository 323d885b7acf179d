"""Lowest-level cells of more than 64 particles (Table 1's large N_ll rows,
Sec. 3.2.1): the interaction kernels then take a cell's sinks in several
passes of 64 lanes. Gravity and the VJP are compared element by element with
the oracle on the same tree, in both forms, on clouds whose cells hold up to
a few hundred particles; the neighbour CSR must be identical."""
import numpy as np
import pytest

from oracle import oracle as O
import workloads as W

from test_gpu_parity import TOL, _gpu_tree, _np, _say, compare_lists, compare_trees, gate
from test_gpu_vjp import TOL as VTOL, _t

pytestmark = pytest.mark.gpu


def _largest_cell(ot):
    cnt = ot.topology()["count"]
    return int(cnt[ot.n_leaves:].max())


def _vjp_gpu(gt, g, prec):
    import torch
    dt = torch.float32 if prec == "mixed" else torch.float64
    return [_np(o).astype(np.float64) for o in gt.vjp(*[_t(a, dt) for a in g])]


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


CASES = [(30000, 64, "plummer", 0.7), (30000, 128, "plummer", 0.5), (20000, 128, "clustered", 0.7)]


@pytest.mark.parametrize("n,nll,kind,theta", CASES)
def test_gravity_vjp_neighbours_with_large_cells(n, nll, kind, theta):
    c = W.small_random(n, 7000 + nll, kind, h_scale=0.5)
    ot = O.OracleTree(*c.arrays(), n_ll=nll)
    big = _largest_cell(ot)
    assert big > 128, big            # several 64-sink passes per cell
    ot.walk(theta)
    ref = np.stack(ot.gravity(), 1)
    ooff, oids, _ = ot.neighbours()
    g = W.cotangents(c.n, seed=nll)
    vref = ot.vjp(*g)
    for prec in ("fp64", "mixed"):
        _say("large cells", n, nll, kind, theta, prec, "largest cell", big)
        gt = _gpu_tree(c, nll, theta, prec)
        if prec == "fp64":
            compare_trees(gt, ot)
            compare_lists(gt, ot)
        off, ids = gt.neighbours()
        np.testing.assert_array_equal(_np(off), ooff)
        np.testing.assert_array_equal(_np(ids), oids)
        a = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)
        err = gate(a, ref)
        assert err <= TOL[prec], (prec, err)
        if prec == "fp64":
            assert err <= 1e-11, err
        got = _vjp_gpu(gt, g, prec)
        for name, x, r in zip(("dx", "dy", "dz", "dm"), got, vref):
            e = _rel(x, r)
            print(f"   vjp {name} rel err {e:.2e}", flush=True)
            assert e <= VTOL[prec], (prec, name, e)
        gt.destroy()


def test_coincident_particles_gravity_and_vjp():
    """700 particles at one point plus a ragged cloud around them: the point
    is one cell of hundreds of particles whose pair terms are all exactly 0
    (Sec. 2.4.3 with r = 0), next to ordinary cells."""
    c = W.small_random(1500, 71, "uniform")
    c.x[:700] = 0.25
    c.y[:700] = -0.5
    c.z[:700] = 0.125
    ot = O.OracleTree(*c.arrays(), n_ll=4)
    assert _largest_cell(ot) >= 700
    g = W.cotangents(c.n, seed=72)
    for theta in (0.0, 0.7):
        ot.walk(theta)
        ref = np.stack(ot.gravity(), 1)
        vref = ot.vjp(*g)
        for prec in ("fp64", "mixed"):
            _say("coincident gravity", theta, prec)
            gt = _gpu_tree(c, 4, theta, prec)
            a = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)
            assert gate(a, ref) <= (1e-11 if prec == "fp64" else TOL[prec])
            got = _vjp_gpu(gt, g, prec)
            for name, x, r in zip(("dx", "dy", "dz", "dm"), got, vref):
                assert _rel(x, r) <= VTOL[prec], (theta, prec, name, _rel(x, r))
            gt.destroy()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("nll", [1, 128])
def test_sobol_sphere_table1_extremes(nll):
    """The 500,000-particle Sobol sphere of Table 1 (about 105 neighbours) at
    its smallest and largest N_ll, theta = 0.7: the whole tree bit for bit,
    and lists, neighbours, accelerations and the VJP (cotangents on the
    sampled cells only) of 128 sampled lowest-level cells against the oracle
    walking only those cells."""
    import torch
    c = W.sobol_sphere()
    ot = O.OracleTree(*c.arrays(), n_ll=nll)
    assert ot.k == {1: 19, 128: 12}[nll]
    rng = np.random.default_rng(80 + nll)
    leaves = np.sort(rng.choice(ot.n_leaves, 128, replace=False)) + ot.n_leaves
    ot.walk(0.7, leaves)
    topo = ot.topology()
    pos = np.concatenate([np.arange(topo["first"][l], topo["first"][l] + topo["count"][l]) for l in leaves])
    sel = topo["perm"][pos]
    ooff, oids, valid = ot.neighbours()
    assert valid[sel].all()
    ref = np.stack(ot.gravity(), 1)[sel]
    g = [np.zeros(c.n) for _ in range(3)]
    for a in g:
        a[sel] = rng.normal(size=sel.size)
    vref = ot.vjp(*g)
    for prec in ("fp64", "mixed"):
        _say("sobol", nll, prec, "largest cell", _largest_cell(ot))
        gt = _gpu_tree(c, nll, 0.7, prec)
        if prec == "fp64":
            compare_trees(gt, ot)
            compare_lists(gt, ot, leaves)
        off, ids = gt.neighbours()
        off, ids = _np(off), _np(ids)
        np.testing.assert_array_equal(off[sel + 1] - off[sel], ooff[sel + 1] - ooff[sel])
        for a in sel:
            np.testing.assert_array_equal(ids[off[a]:off[a + 1]], oids[ooff[a]:ooff[a + 1]])
        acc = np.stack([_np(v).astype(np.float64) for v in gt.gravity()], 1)[sel]
        err = gate(acc, ref)
        assert err <= (1e-11 if prec == "fp64" else TOL[prec]), (prec, err)
        got = _vjp_gpu(gt, g, prec)
        for name, x, r in zip(("dx", "dy", "dz", "dm"), got, vref):
            e = _rel(x, r)
            print(f"   vjp {name} rel err {e:.2e}", flush=True)
            assert e <= VTOL[prec], (prec, name, e)
        gt.destroy()
        del off, ids
        torch.cuda.empty_cache()
