"""Pins of the oracle's two walk modes (Sec. 2.2-2.4.1 and the pure-MAC
variant of Sec. 2.5) that do not reuse the oracle's recursion.

The lists of a top-down walk have a closed description over ancestor chains:
a node is tested iff every strict ancestor below the root was tested, is
non-empty and was opened. Written vectorised over all labels from the
oracle's node data, that description must give exactly the oracle's lists.
The remaining pins are brute force (all-pairs neighbours, the direct sum at
theta = 0), set inclusions between the modes that follow from the
definitions, and the VJP against central differences.
"""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
import workloads as W

CAND, NBONLY, LABEL = np.uint32(1 << 31), np.uint32(1 << 30), np.uint32((1 << 30) - 1)
PAD = 1.0 + 2.0 ** -32


def _tests(t, A, theta):
    """Per-label predicates for sink leaf A: non-empty, reachable, MAC, B contains A."""
    nd, topo = t.nodes(), t.topology()
    g = 0.5 * (nd["lo"] + nd["hi"])
    d = g - g[A]
    dg2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    rs = (nd["hnode"][A] + nd["hint"]) * PAD
    reach = dg2 < rs * rs
    H = (nd["hi"] - nd["lo"]).max(1)
    dc = nd["com"] - nd["com"][A]
    R2 = (dc[:, 0] * dc[:, 0] + dc[:, 1] * dc[:, 1]) + dc[:, 2] * dc[:, 2]
    mac = H * H < (theta * theta) * R2
    lab = np.arange(t.nlab)
    lvl = np.zeros(t.nlab, np.int64)
    lvl[1:] = np.floor(np.log2(lab[1:])).astype(np.int64)
    contains = np.zeros(t.nlab, bool)
    contains[1:] = (A >> (t.k - lvl[1:])) == lab[1:]
    return topo["count"] > 0, reach, mac, contains, lvl


def _chain(t, lvl, passes):
    """tested[B]: every strict ancestor of B at level >= 1 passes (labels in
    increasing order visit parents first). The walk starts at level 1, or at
    the root when the root is the only leaf."""
    top = 0 if t.k == 0 else 1
    tested = np.zeros(t.nlab, bool)
    for B in range(1, t.nlab):
        tested[B] = lvl[B] == top or (lvl[B] > top and tested[B >> 1] and passes[B >> 1])
    return tested


def expected_lists(t, A, theta, pure):
    nonempty, reach, mac, contains, lvl = _tests(t, A, theta)
    leaf = np.arange(t.nlab) >= t.n_leaves
    if pure:
        acc = nonempty & mac & ~contains
        g_tested = _chain(t, lvl, nonempty & ~acc)
        n_tested = _chain(t, lvl, nonempty & reach)
        far = np.nonzero(g_tested & acc)[0]
        gnear = g_tested & nonempty & ~acc & leaf
        cand = n_tested & nonempty & reach & leaf
    else:
        acc = nonempty & ~reach & mac
        tested = _chain(t, lvl, nonempty & ~acc)
        far = np.nonzero(tested & acc)[0]
        gnear = tested & nonempty & ~acc & leaf
        cand = gnear & reach
    near = []
    for B in np.nonzero(gnear | cand)[0]:
        e = np.uint32(B)
        if cand[B]:
            e |= CAND
        if not gnear[B]:
            e |= NBONLY
        near.append(e)
    return np.array(near, np.uint32), far


CASES = [(700, 5, "plummer"), (500, 3, "clustered"), (300, 6, "uniform"), (9, 12, "uniform")]


@pytest.mark.parametrize("pure", [False, True])
@pytest.mark.parametrize("theta", [0.0, 0.5, 0.7, 1.2])
@pytest.mark.parametrize("n,nll,kind", CASES)
def test_lists_equal_the_ancestor_chain_description(n, nll, kind, theta, pure):
    c = W.small_random(n, 60 + n, kind)
    t = O.OracleTree(*c.arrays(), n_ll=nll)
    t.walk(theta, pure_mac=pure)
    t.cache_sizes()
    count = t.topology()["count"]
    for A in range(t.n_leaves, 2 * t.n_leaves):
        near, far = t.leaf_lists(A)
        if count[A] == 0:
            assert len(near) == 0 and len(far) == 0
            continue
        en, ef = expected_lists(t, A, theta, pure)
        np.testing.assert_array_equal(near, en, err_msg=f"near list of leaf {A}")
        np.testing.assert_array_equal(np.sort(far), ef, err_msg=f"far list of leaf {A}")


@pytest.mark.parametrize("theta", [0.0, 0.5, 0.7, 1.0])
def test_pure_mac_gravity_cover(theta):
    # the gravity near field and the far nodes hold every particle exactly
    # once; A is in its own near field; no far node contains A
    c = W.small_random(900, 7, "plummer")
    t = O.OracleTree(*c.arrays(), n_ll=5)
    t.walk(theta, pure_mac=True)
    t.cache_sizes()
    topo = t.topology()
    for A in range(t.n_leaves, 2 * t.n_leaves):
        if topo["count"][A] == 0:
            continue
        near, far = t.leaf_lists(A)
        grav = (near[(near & NBONLY) == 0] & LABEL).astype(np.int64)
        assert A in set(grav.tolist())
        if theta == 0.0:
            assert len(far) == 0 and not np.any(near & NBONLY)
        cover = np.zeros(t.n, np.int64)
        for lab in list(grav) + list(far):
            cover[topo["first"][lab]:topo["first"][lab] + topo["count"][lab]] += 1
            B = int(lab)
            a = A
            while a > B:
                a >>= 1
            assert a != B or B == A, (A, B)
        assert np.all(cover == 1)


def test_pure_mac_lists_are_subsets_of_the_paper_walk():
    # a cell the paper's walk accepts satisfies the MAC and is not reachable,
    # so it does not contain A: the pure walk accepts it or an ancestor, and
    # its near field can only shrink; a leaf reached through reachable cells
    # only is a candidate of both walks
    c = W.small_random(1500, 9, "clustered")
    t = O.OracleTree(*c.arrays(), n_ll=6)
    lists = {}
    for pure in (False, True):
        t.walk(0.7, pure_mac=pure)
        t.cache_sizes()
        lists[pure] = {A: t.leaf_lists(A)[0].copy() for A in range(t.n_leaves, 2 * t.n_leaves)}
        lists[pure, "sizes"] = t.list_sizes()[2]
    shorter = 0
    for A in range(t.n_leaves, 2 * t.n_leaves):
        d, p = lists[False][A], lists[True][A]
        dg = set((d & LABEL).tolist())
        pg = set((p[(p & NBONLY) == 0] & LABEL).tolist())
        assert pg <= dg
        assert set((p[(p & CAND) != 0] & LABEL).tolist()) <= set((d[(d & CAND) != 0] & LABEL).tolist())
        shorter += len(pg) < len(dg)
    assert shorter > 0
    st_d, st_p = lists[False, "sizes"], lists[True, "sizes"]
    assert np.all(st_p[:, 3] <= st_d[:, 3]) and st_p[:, 3].sum() < st_d[:, 3].sum()


@pytest.mark.parametrize("n,nll,kind,hs", [(1, 12, "uniform", 1.0), (333, 5, "clustered", 1.0),
                                           (1000, 12, "plummer", 1.0), (500, 3, "uniform", 3.0)])
def test_pure_mac_neighbours_equal_all_pairs(n, nll, kind, hs):
    c = W.small_random(n, 100 + n, kind, h_scale=hs)
    t = O.OracleTree(*c.arrays(), n_ll=nll)
    t.walk(0.7, pure_mac=True)
    off, ids, valid = t.neighbours()
    assert valid.all()
    boff, bids = brute.neighbours(c.x, c.y, c.z, c.h)
    np.testing.assert_array_equal(off, boff)
    np.testing.assert_array_equal(ids, bids)   # each list ascending by index


@pytest.mark.parametrize("n,nll,kind", [(400, 4, "clustered"), (513, 8, "plummer")])
def test_pure_mac_theta_zero_equals_brute_force(n, nll, kind):
    c = W.small_random(n, 3 + n, kind)
    t = O.OracleTree(*c.arrays(), n_ll=nll)
    t.walk(0.0, pure_mac=True)
    a = np.stack(t.gravity(), 1)
    ref = brute.direct_accel(c.x, c.y, c.z, c.m, c.h)
    assert np.abs(a - ref).max() <= 1e-13 * np.abs(ref).max()


def test_pure_mac_accuracy_on_uniform_sphere():
    # shorter near lists cost accuracy (Sec. 2.5), but the error still falls
    # with theta and stays at the per-mille level at theta = 0.5
    c = W.uniform_sphere()
    t = O.OracleTree(*c.arrays(), n_ll=8)
    ref = brute.direct_accel(c.x, c.y, c.z, c.m, c.h)
    stats = {}
    for pure in (False, True):
        for th in (0.4, 0.5, 0.7):
            t.walk(th, pure_mac=pure)
            stats[pure, th] = brute.error_stats(np.stack(t.gravity(), 1), ref)
    assert stats[True, 0.4]["mean"] < stats[True, 0.5]["mean"] < stats[True, 0.7]["mean"]
    for th in (0.4, 0.5, 0.7):
        assert stats[True, th]["mean"] >= stats[False, th]["mean"]
    assert stats[True, 0.5]["mean"] < 3e-3


def _L(t, c, g, x, y, z, m):
    t.refresh(x, y, z, m, c.h)
    a = t.gravity()
    return float(sum((gi * ai).sum() for gi, ai in zip(g, a)))


def test_pure_mac_vjp_finite_differences_and_invariants():
    c = W.small_random(140, 33, "clustered")
    g = W.cotangents(c.n, seed=8)
    t = O.OracleTree(*c.arrays(), n_ll=4)
    t.walk(0.8, pure_mac=True)
    t.cache_sizes()
    assert any(np.any(t.leaf_lists(A)[0] & NBONLY) for A in range(t.n_leaves, 2 * t.n_leaves))
    dx, dy, dz, dm = t.vjp(*g)
    base = [c.x.copy(), c.y.copy(), c.z.copy(), c.m.copy()]
    L0 = _L(t, c, g, *base)
    scale = np.abs(np.concatenate([dx, dy, dz])).sum()
    for d in (dx, dy, dz):
        assert abs(d.sum()) < 1e-11 * scale
    assert (c.m * dm).sum() == pytest.approx(L0, rel=1e-10)
    rng = np.random.default_rng(1)
    for i in rng.choice(c.n, 10, replace=False):
        for comp, grad in zip(range(4), (dx, dy, dz, dm)):
            eps = 1e-6 if comp < 3 else 1e-6 * c.m[i]
            p = [b.copy() for b in base]; p[comp][i] += eps
            q = [b.copy() for b in base]; q[comp][i] -= eps
            num = (_L(t, c, g, *p) - _L(t, c, g, *q)) / (2 * eps)
            assert abs(num - grad[i]) < 2e-6 * np.abs(grad).max() + 1e-7 * abs(num), (i, comp)
    t.refresh(*base, c.h)
