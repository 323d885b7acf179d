"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each checks a printed value
(Table 1), a closed form, a library routine (scipy quad, sympy, torch
autograd), brute force on tiny inputs, or an invariant that a plausible
mistake (dropped term, wrong sign, transposed index) would break.
"""
import math
import os

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Sec. 2.1 depth rule, pinned by Table 1's L column
# --------------------------------------------------------------------------
def test_depth_rule_matches_table1():
    rows = [l.split() for l in open(os.path.join(GOLD, "table1_depth.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 8
    for n, nll, L in rows:
        assert O.depth_for(int(n), int(nll)) == int(L), (n, nll, L)


def test_depth_rule_edges():
    assert O.depth_for(1, 12) == 0
    assert O.depth_for(12, 12) == 0       # "dropped below": average <= N_ll
    assert O.depth_for(13, 12) == 1
    assert O.depth_for(4096, 8) == 9
    assert O.depth_for(1 << 20, 12) == 17
    assert O.depth_for(1 << 22, 12) == 19
    assert O.depth_for(100_000_000, 12) == 23


# --------------------------------------------------------------------------
# canonical pairwise sum
# --------------------------------------------------------------------------
def test_psum_adjacent_pairing_and_padding():
    big = 2.0 ** 53
    # adjacent pairs first: (2^53 + 1) + (1 - 2^53) = 2^53 + (1 - 2^53) = 1
    assert O.psum([big, 1.0, 1.0, -big]) == 1.0
    # left-to-right would give 0, (2^53 + (1 + 1)) - 2^53 would give 2
    # five values pad to eight: ((2^53+1)+(1+1)) + ((1+0)+0) = 2^53+2 + 1 -> 2^53+4
    assert O.psum([big, 1.0, 1.0, 1.0, 1.0]) == big + 4.0
    assert O.psum([]) == 0.0
    assert math.copysign(1.0, O.psum([-0.0])) == 1.0
    assert O.psum([3.0]) == 3.0


def test_psum_error_bound_vs_fsum():
    rng = np.random.default_rng(0)
    for n in (1, 7, 64, 1000, 4097):
        v = rng.normal(size=n) * 10.0 ** rng.uniform(-3, 3, n)
        ex = math.fsum(v)
        bound = math.ceil(math.log2(max(n, 2))) * 2.0 ** -53 * np.abs(v).sum() * 1.01
        assert abs(O.psum(v) - ex) <= bound
        iv = rng.integers(-1000, 1000, n).astype(float)
        assert O.psum(iv) == float(iv.sum())


# --------------------------------------------------------------------------
# kernel softening, Sec. 2.4.3
# --------------------------------------------------------------------------
def _enclosed_mass_fraction(r, h):
    from scipy.integrate import quad
    f = lambda s: 4.0 * math.pi * s * s * float(brute.cubic_spline_W(s, h))
    pts = [p for p in (h, 2 * h) if p < r]
    return quad(f, 0.0, r, points=pts or None, epsabs=1e-14, epsrel=1e-13, limit=200)[0]


@pytest.mark.parametrize("h", [0.3, 1.0, 2.5])
def test_kernel_F_is_enclosed_mass_over_r3(h):
    # eta = 4 pi int_0^r r'^2 W dr' (Sec. 2.4.3) and the pair acceleration is
    # m_b eta / r^2 along e_ab, i.e. F = eta / r^3 in the division-safe form.
    for q in (0.05, 0.4, 0.999, 1.0, 1.3, 1.9999, 2.0, 2.7, 6.0):
        r = q * h
        F, _ = O.kernel_F(r, h)
        eta = _enclosed_mass_fraction(r, h)
        assert F == pytest.approx(eta / r ** 3, rel=1e-10, abs=1e-12 / h ** 3), q


def test_kernel_S_continuity_and_newton_limit():
    h = 1.7
    for q, S_h2 in ((1.0, 19.0 / 30.0), (2.0, 0.25)):
        lo, _ = O.kernel_F(q * h * (1 - 1e-12), h)
        hi, _ = O.kernel_F(q * h * (1 + 1e-12), h)
        assert lo * q * h * h * h == pytest.approx(S_h2, rel=1e-9)
        assert hi * q * h * h * h == pytest.approx(S_h2, rel=1e-9)
    F, _ = O.kernel_F(5.0, h)
    assert F == 1.0 / 125.0
    F0, _ = O.kernel_F(0.0, h)
    assert F0 == pytest.approx(4.0 / 3.0 / h ** 3)
    # the oracle's F matches the brute-force S(q)/r form
    r = np.linspace(0.01, 4.0, 97) * h
    Fs = np.array([O.kernel_F(v, h)[0] for v in r])
    np.testing.assert_allclose(Fs * r, brute.S_of_q(r, h), rtol=1e-13)


def test_kernel_derivative_by_finite_differences():
    h = 0.8
    for q in (0.2, 0.7, 0.99, 1.01, 1.5, 1.98, 2.02, 3.0):
        r = q * h
        _, dFr = O.kernel_F(r, h)
        e = 1e-6 * h
        num = (O.kernel_F(r + e, h)[0] - O.kernel_F(r - e, h)[0]) / (2 * e)
        assert dFr * r == pytest.approx(num, rel=1e-6, abs=1e-9 / h ** 4), q


# --------------------------------------------------------------------------
# derivative tensors of 1/r and the far field, Sec. 2.4.2
# --------------------------------------------------------------------------
def test_derivative_tensors_match_sympy():
    import itertools
    import sympy as sp
    X = sp.symbols("x0 x1 x2")
    f = 1 / sp.sqrt(X[0] ** 2 + X[1] ** 2 + X[2] ** 2)
    R = np.array([0.7, -1.3, 0.45])
    sub = dict(zip(X, [sp.Rational(7, 10), sp.Rational(-13, 10), sp.Rational(45, 100)]))
    cache = {(): f}
    for order in range(1, 7):
        T = O.deriv_tensor(order, R)
        for idx in itertools.product(range(3), repeat=order):
            key = tuple(sorted(idx))
            if key not in cache:
                cache[key] = sp.diff(cache[key[:-1]], X[key[-1]])
            ref = float(cache[key].subs(sub))
            assert T[idx] == pytest.approx(ref, rel=1e-12, abs=1e-13), (order, idx)


def test_derivative_tensors_traceless_and_symmetric():
    R = np.array([-0.3, 0.9, 1.7])
    for order in range(2, 7):
        T = O.deriv_tensor(order, R)
        tr = np.trace(T, axis1=0, axis2=1)
        assert np.abs(tr).max() < 1e-11 * np.abs(T).max()          # Laplace
        assert np.allclose(T, np.swapaxes(T, 0, order - 1), rtol=0, atol=1e-13 * np.abs(T).max())


def test_far_field_point_mass_is_newton():
    R = np.array([2.0, -1.0, 0.5])
    f, J, H = O.far_coeffs(3.0, np.zeros(6), R)
    r = np.linalg.norm(R)
    np.testing.assert_allclose(f, -3.0 * R / r ** 3, rtol=1e-14)


def _cluster(seed, n=40, s=1.0):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(n, 3)) * s * np.array([1.0, 0.6, 0.3])
    m = rng.uniform(0.5, 1.5, n)
    return p, m


def test_far_field_jacobian_and_hessian_are_derivatives():
    p, m = _cluster(3)
    t = O.OracleTree(p[:, 0], p[:, 1], p[:, 2], m, np.full(len(m), 0.1), n_ll=len(m))
    nd = t.nodes()
    M, q6, com = nd["M"][1], nd["Q"][1], nd["com"][1]
    R = np.array([6.0, -3.0, 4.5])
    f, J, H, T4 = O.far_coeffs(M, q6, R, with_t4=True)
    e = 1e-5
    for l in range(3):
        dR = np.zeros(3); dR[l] = e
        fp, Jp, Hp = O.far_coeffs(M, q6, R + dR)
        fm, Jm, Hm = O.far_coeffs(M, q6, R - dR)
        np.testing.assert_allclose((fp - fm) / (2 * e), J[:, l], rtol=1e-7, atol=1e-12)
        np.testing.assert_allclose((Jp - Jm) / (2 * e), H[:, :, l], rtol=1e-7, atol=1e-12)
        np.testing.assert_allclose((Hp - Hm) / (2 * e), T4[:, :, :, l], rtol=1e-6, atol=1e-12)
    assert np.allclose(J, J.T, atol=1e-15)
    assert abs(np.trace(J)) < 1e-12 * np.abs(J).max()


def test_multipole_error_falls_as_third_power():
    p, m = _cluster(4)
    t = O.OracleTree(p[:, 0], p[:, 1], p[:, 2], m, np.full(len(m), 0.1), n_ll=len(m))
    nd = t.nodes()
    M, q6, com = nd["M"][1], nd["Q"][1], nd["com"][1]
    u = np.array([0.6, 0.64, 0.48])
    errs = []
    for dist in (20.0, 40.0, 80.0):
        x = com + dist * u
        v = x[None, :] - p
        exact = -(m[:, None] * v / np.linalg.norm(v, axis=1)[:, None] ** 3).sum(0)
        f, _, _ = O.far_coeffs(M, q6, x - com)
        errs.append(np.linalg.norm(f - exact) / np.linalg.norm(exact))
    # the truncation after the quadrupole leaves an O((s/R)^3) relative error
    assert errs[1] / errs[0] == pytest.approx(1 / 8, rel=0.15)
    assert errs[2] / errs[1] == pytest.approx(1 / 8, rel=0.08)


def test_taylor_error_falls_as_third_power():
    # Eq. 6: f(r_A + d) ~ f + J d + 1/2 H[d, d]; error O(|d|^3)
    M, q6 = 2.0, np.array([0.3, -0.1, 0.2, 0.5, 0.05, -0.8])
    RA = np.array([4.0, 1.0, -2.0])
    f, J, H = O.far_coeffs(M, q6, RA)
    u = np.array([0.48, -0.6, 0.64])
    errs = []
    for s in (0.4, 0.2, 0.1):
        d = s * u
        exact, _, _ = O.far_coeffs(M, q6, RA + d)
        approx = f + J @ d + 0.5 * np.einsum("ilm,l,m->i", H, d, d)
        errs.append(np.linalg.norm(approx - exact))
    assert errs[1] / errs[0] == pytest.approx(1 / 8, rel=0.1)
    assert errs[2] / errs[1] == pytest.approx(1 / 8, rel=0.05)


# --------------------------------------------------------------------------
# tree build, Sec. 2.1
# --------------------------------------------------------------------------
@pytest.mark.parametrize("split", ["mass", "number", "median"])
@pytest.mark.parametrize("n,nll,kind", [(1, 12, "uniform"), (5, 12, "uniform"), (300, 4, "clustered"),
                                        (1001, 8, "plummer"), (777, 3, "uniform"), (600, 5, "ties")])
def test_tree_rules(n, nll, kind, split):
    if kind == "ties":          # many equal coordinates: the median split's tie rule
        c = W.small_random(n, 10 + n, "uniform")
        c.x[:] = np.round(c.x * 4) / 4
        c.y[:] = np.round(c.y * 3) / 3
        c.z[::3] = -0.0
    else:
        c = W.small_random(n, 10 + n, kind)
    t = O.OracleTree(*c.arrays(), n_ll=nll, split=split)
    topo, nd = t.topology(), t.nodes()
    perm, first, count, axis = topo["perm"], topo["first"], topo["count"], topo["axis"]
    assert sorted(perm) == list(range(n))
    assert t.k == O.depth_for(n, nll)
    P = np.stack([c.x, c.y, c.z], 1)
    assert first[1] == 0 and count[1] == n
    np.testing.assert_array_equal(nd["lo"][1], P.min(0))
    np.testing.assert_array_equal(nd["hi"][1], P.max(0))
    for lab in range(1, 1 << t.k):
        L, R = 2 * lab, 2 * lab + 1
        assert first[L] == first[lab] and count[L] + count[R] == count[lab]
        assert first[R] == first[lab] + count[L]
        if count[lab] == 0:
            continue
        side = nd["hi"][lab] - nd["lo"][lab]
        ax = int(np.argmax(side))                       # first maximum
        assert axis[lab] == ax
        ids = np.sort(perm[first[lab]:first[lab] + count[lab]])
        plane = nd["hi"][L][ax]
        assert plane == nd["lo"][R][ax]
        left = perm[first[L]:first[L] + count[L]]
        right = perm[first[R]:first[R] + count[R]]
        if split == "median":
            # equal halves: the floor(c/2) first in (coordinate, index) order go left
            order = np.lexsort((ids, P[ids, ax]))
            assert count[L] == len(ids) // 2
            np.testing.assert_array_equal(np.sort(left), np.sort(ids[order[:len(ids) // 2]]))
            assert plane == P[ids[order[len(ids) // 2]], ax]
            assert plane != 0.0 or math.copysign(1.0, plane) == 1.0     # -0 is stored as +0
            assert np.all(P[left, ax] <= plane) and np.all(P[right, ax] >= plane)
            continue
        if split == "mass":
            com = np.array([math.fsum(c.m[ids] * P[ids, d]) / math.fsum(c.m[ids]) for d in range(3)])
        else:                                            # centre of number: weights 1
            com = np.array([math.fsum(P[ids, d]) / len(ids) for d in range(3)])
        assert abs(plane - com[ax]) <= 1e-14 * (1 + abs(com[ax]))
        assert np.all(P[left, ax] < plane) and np.all(P[right, ax] >= plane)
    for lab in range(1 << t.k, 2 << t.k):
        ids = perm[first[lab]:first[lab] + count[lab]]
        assert np.all(np.diff(ids) > 0)          # stable partitions starting from input order
        assert np.all(P[ids] >= nd["lo"][lab]) and np.all(P[ids] <= nd["hi"][lab])
        if count[lab]:
            g = 0.5 * (nd["lo"][lab] + nd["hi"][lab])
            d = np.linalg.norm(P[ids] - g, axis=1)
            assert nd["hint"][lab] == pytest.approx(d.max(), rel=1e-15)
            assert nd["hnode"][lab] == pytest.approx((d + 2 * c.h[ids]).max(), rel=1e-15)


def test_centre_of_number_split_equals_mass_split_for_equal_power_of_two_masses():
    # m = 2^-j scales every product m x exactly, so both planes are the same number
    c = W.small_random(1500, 12, "clustered")
    c.m[:] = 2.0 ** -11
    a = O.OracleTree(*c.arrays(), n_ll=5, split="mass")
    b = O.OracleTree(*c.arrays(), n_ll=5, split="number")
    np.testing.assert_array_equal(a.topology()["perm"], b.topology()["perm"])
    for key in ("lo", "hi", "com", "M", "Q", "hint", "hnode"):
        np.testing.assert_array_equal(a.nodes()[key], b.nodes()[key])
    # with unequal masses the planes differ and so do the trees
    c2 = W.small_random(1500, 12, "clustered")
    a2 = O.OracleTree(*c2.arrays(), n_ll=5, split="mass")
    b2 = O.OracleTree(*c2.arrays(), n_ll=5, split="number")
    assert not np.array_equal(a2.nodes()["hi"], b2.nodes()["hi"])


def test_median_split_renegades_cost_accuracy():
    # Sec. 2.1 "Load balancing": in a binary with more particles in one star the
    # median split cuts the heavier star and puts part of it into the lighter
    # star's cell; the centre-of-mass split keeps the stars apart. The
    # truncation errors of the median tree are larger.
    c = W.binary_clumps()
    ref = brute.direct_accel(c.x, c.y, c.z, c.m, c.h)
    err = {}
    for split in ("mass", "median"):
        t = O.OracleTree(*c.arrays(), n_ll=8, split=split)
        t.walk(0.7)
        err[split] = brute.error_stats(np.stack(t.gravity(), 1), ref)
    assert err["median"]["mean"] > 1.5 * err["mass"]["mean"]
    assert err["median"]["p99"] > 1.5 * err["mass"]["p99"]


def test_quadrupole_eq1_traceless_and_eq2_equals_direct():
    c = W.small_random(600, 21, "clustered")
    t = O.OracleTree(*c.arrays(), n_ll=6)
    topo, nd = t.topology(), t.nodes()
    P = np.stack([c.x, c.y, c.z], 1)
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for lab in [1, 2, 3, 5, 12, 40]:
        ids = topo["perm"][topo["first"][lab]:topo["first"][lab] + topo["count"][lab]]
        d = P[ids] - nd["com"][lab]
        mm = c.m[ids]
        direct = np.einsum("a,ai,aj->ij", 3 * mm, d, d) - np.eye(3) * (mm * (d * d).sum(1)).sum()
        q = nd["Q"][lab]
        full = np.array([[q[0], q[1], q[2]], [q[1], q[3], q[4]], [q[2], q[4], q[5]]])
        assert abs(np.trace(full)) < 1e-13 * np.abs(full).max()
        np.testing.assert_allclose(full, direct, rtol=1e-11, atol=1e-14 * np.abs(direct).max())


# --------------------------------------------------------------------------
# walk invariants, Sec. 2.2 - 2.4.1
# --------------------------------------------------------------------------
def _cover_check(t, theta):
    topo = t.topology()
    nn, nf, st = t.cache_sizes()
    for A in range(t.n_leaves, 2 * t.n_leaves):
        if topo["count"][A] == 0:
            assert nn[A - t.n_leaves] == 0 and nf[A - t.n_leaves] == 0
            continue
        near, far = t.leaf_lists(A)
        labs = near & 0x7FFFFFFF
        cand = near >> 31
        assert A in set(labs.tolist())
        assert cand[list(labs).index(A)] == 1
        assert np.all(np.diff(labs.astype(np.int64)) > 0)          # ascending leaf labels
        if theta == 0.0:
            assert len(far) == 0
        # every particle is represented exactly once: by a near leaf or a far node
        cover = np.zeros(t.n, np.int64)
        for lab in list(labs) + list(far):
            cover[topo["first"][lab]:topo["first"][lab] + topo["count"][lab]] += 1
        assert np.all(cover == 1)


@pytest.mark.parametrize("theta", [0.0, 0.5, 0.7, 1.0])
def test_walk_lists_cover_every_particle_once(theta):
    c = W.small_random(700, 5, "plummer")
    t = O.OracleTree(*c.arrays(), n_ll=6)
    t.walk(theta)
    _cover_check(t, theta)


def test_walk_single_leaf_tree():
    c = W.small_random(9, 2, "uniform")
    t = O.OracleTree(*c.arrays(), n_ll=12)
    assert t.k == 0
    t.walk(0.7)
    near, far = t.leaf_lists(1)
    assert list(near) == [1 | (1 << 31)] and len(far) == 0


# --------------------------------------------------------------------------
# neighbours, Sec. 2.3: equal to the all-pairs search
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,nll,kind,hs", [(1, 12, "uniform", 1.0), (2, 1, "uniform", 20.0),
                                           (333, 5, "clustered", 1.0), (1000, 12, "plummer", 1.0),
                                           (500, 3, "uniform", 3.0)])
def test_neighbours_equal_all_pairs(n, nll, kind, hs):
    c = W.small_random(n, 100 + n, kind, h_scale=hs)
    t = O.OracleTree(*c.arrays(), n_ll=nll)
    t.walk(0.6)
    off, ids, valid = t.neighbours()
    assert valid.all()
    boff, bids = brute.neighbours(c.x, c.y, c.z, c.h)
    np.testing.assert_array_equal(off, boff)
    np.testing.assert_array_equal(ids, bids)   # each list ascending by index


def test_neighbours_with_coincident_particles():
    c = W.small_random(200, 8, "uniform")
    c.x[50:60] = c.x[50]; c.y[50:60] = c.y[50]; c.z[50:60] = c.z[50]
    t = O.OracleTree(*c.arrays(), n_ll=4)
    t.walk(0.5)
    off, ids, _ = t.neighbours()
    boff, bids = brute.neighbours(c.x, c.y, c.z, c.h)
    np.testing.assert_array_equal(off, boff)
    assert 50 not in ids[off[50]:off[51]].tolist() and 51 in ids[off[50]:off[51]].tolist()


def test_uniform_sphere_has_exactly_50_neighbours():
    c = W.uniform_sphere()
    t = O.OracleTree(*c.arrays(), n_ll=8)
    assert t.k == 9
    t.walk(0.5)
    off, ids, _ = t.neighbours()
    assert np.all(np.diff(off) == 50)


# --------------------------------------------------------------------------
# gravity, Sec. 2.4: theta = 0 is the direct sum; conservation in direct sum
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,nll,kind", [(400, 4, "clustered"), (513, 8, "plummer"), (7, 12, "uniform")])
def test_theta_zero_equals_brute_force(n, nll, kind):
    c = W.small_random(n, 3 + n, kind)
    t = O.OracleTree(*c.arrays(), n_ll=nll)
    t.walk(0.0)
    a = np.stack(t.gravity(), 1)
    ref = brute.direct_accel(c.x, c.y, c.z, c.m, c.h)
    assert np.abs(a - ref).max() <= 1e-13 * np.abs(ref).max()
    # symmetric h_ab and central forces: zero net force and torque
    P = np.stack([c.x, c.y, c.z], 1)
    scale = (c.m[:, None] * np.abs(a)).sum()
    assert np.abs((c.m[:, None] * a).sum(0)).max() < 1e-14 * scale
    tq = np.cross(P, c.m[:, None] * a).sum(0)
    assert np.abs(tq).max() < 1e-13 * scale * np.abs(P).max()


def test_gravity_parts_add_up():
    """The near-only and far-only evaluations (used to time Table 1's NG and
    FG columns) are the two terms of the full sum: at theta = 0 the far part
    is zero and the near part is the whole; at theta = 0.7 they add up to the
    full acceleration to rounding."""
    c = W.small_random(2000, 77, "clustered")
    t = O.OracleTree(*c.arrays(), n_ll=6)
    t.walk(0.0)
    assert np.all(np.stack(t.gravity(parts=2), 1) == 0.0)
    np.testing.assert_array_equal(np.stack(t.gravity(parts=1), 1), np.stack(t.gravity(), 1))
    t.walk(0.7)
    full = np.stack(t.gravity(), 1)
    near, far = np.stack(t.gravity(parts=1), 1), np.stack(t.gravity(parts=2), 1)
    assert np.abs(far).max() > 1e-3 * np.abs(full).max()
    assert np.abs(near + far - full).max() <= 1e-14 * np.abs(full).max()


def test_reading_b_changes_only_the_sink_expansion():
    # Reading B keeps f and takes J, H from the monopole field: a particle alone
    # in its cell sits at the cell's centre of mass (d = 0 up to the rounding
    # of m x / m), where Eq. 6 is f alone, so both readings agree to rounding;
    # the others differ by the quadrupole parts of J d + H[d, d] / 2.
    c = W.small_random(3000, 77, "plummer")
    t = O.OracleTree(*c.arrays(), n_ll=1)
    t.walk(0.7)
    t.set_reading("A")
    aA = np.stack(t.gravity(), 1)
    t.set_reading("B")
    aB = np.stack(t.gravity(), 1)
    topo = t.topology()
    cnt = topo["count"][t.n_leaves:]
    first = topo["first"][t.n_leaves:]
    alone = topo["perm"][first[cnt == 1]]
    shared = np.setdiff1d(np.arange(c.n), alone)
    assert len(alone) > 100 and len(shared) > 100
    np.testing.assert_allclose(aA[alone], aB[alone], rtol=1e-13, atol=1e-15 * np.abs(aA).max())
    d = np.linalg.norm(aA[shared] - aB[shared], axis=1) / np.linalg.norm(aA[shared], axis=1)
    assert np.count_nonzero(d) > len(shared) // 2 and d.max() < 0.05
    with pytest.raises(ValueError):
        t.vjp(*W.cotangents(c.n, seed=1))


def test_reading_a_is_the_more_accurate_at_the_working_angles():
    c = W.uniform_sphere()
    t = O.OracleTree(*c.arrays(), n_ll=8)
    ref = brute.direct_accel(c.x, c.y, c.z, c.m, c.h)
    for th in (0.5, 0.7):
        t.walk(th)
        err = {}
        for r in "AB":
            t.set_reading(r)
            err[r] = brute.error_stats(np.stack(t.gravity(), 1), ref)
        assert err["A"]["mean"] < err["B"]["mean"] and err["A"]["p99"] < err["B"]["p99"], th


def _line16(y):
    """16 equal masses on the x axis at x = 0, 1, ..., 15 (y given per
    particle, z = 0), one particle per lowest-level cell (N_ll = 1, k = 4).
    Every split is along x through a half-integer centre of mass, so the
    cells are known by hand: particle i sits in leaf 16 + i; node 2 holds
    particles 0..7 (box x in [0, 7.5]), node 3 particles 8..15 (box x in
    [7.5, 15]), node 6 particles 8..11 (box x in [7.5, 11.5]), node 7
    particles 12..15 (box x in [11.5, 15]). h is tiny, so no cell that does
    not hold the sink's particle is reachable (Sec. 2.3.1)."""
    n = 16
    x = np.arange(n, dtype=np.float64)
    z = np.zeros(n)
    m = np.full(n, 1.0 / n)
    h = np.full(n, 1e-4)
    return O.OracleTree(x, np.asarray(y, np.float64), z, m, h, n_ll=1)


def _far(t, leaf):
    return set(int(v) for v in t.leaf_lists(leaf)[1])


def test_mac_decisions_on_hand_built_cells():
    """Eq. 4 (Sec. 2.4.1) decided by hand: cell B is accepted for sink cell A
    iff H_B < theta R_AB, with H_B the longest side of B's box and R_AB the
    distance of the two centres of mass.

    y alternates -0.25, +0.25, so every box is 0.5 high and its centre of
    mass has y = 0 (equal numbers of each sign) unless it holds one particle.
    Sink leaf 16 (particle 0 at (0, -0.25, 0)) against node 3: H_3 = 7.5
    (box 7.5 x 0.5 x 0), COM_3 = (11.5, 0, 0), R^2 = 11.5^2 + 0.25^2, so the
    critical angle is theta* = 7.5 / sqrt(132.3125) = 0.65202... Just above it
    node 3 is accepted; just below it node 3 is opened and its children 6
    (H = 4, R ~ 9.5) and 7 (H = 3.5, R ~ 13.5) are accepted instead. The
    readings that would move the decision: box centres instead of centres of
    mass (R = 11 -> theta* = 0.68), the sink's own side (H_16 = 0.5 -> always
    accepted), the box diagonal (sqrt(7.5^2 + 0.5^2) -> theta* = 0.6535) or
    theta instead of theta^2 (accepted at theta*)."""
    y = np.where(np.arange(16) % 2 == 0, -0.25, 0.25)
    t = _line16(y)
    assert t.k == 4
    crit = 7.5 / math.sqrt(11.5 ** 2 + 0.25 ** 2)
    t.walk(crit * (1 + 1e-9))
    assert 3 in _far(t, 16)
    t.walk(crit * (1 - 1e-9))
    far = _far(t, 16)
    assert 3 not in far and {6, 7} <= far
    # the other way round: sink leaf 31 (particle 15, x = 15, box 14.5..15)
    # against node 2: H_2 = 7.5, COM_2 = (3.5, 0, 0), same critical angle
    t.walk(crit * (1 + 1e-9))
    assert 2 in _far(t, 31)
    t.walk(crit * (1 - 1e-9))
    assert 2 not in _far(t, 31)
    # between the geometric-centre angle and the diagonal's: accepted only
    # by the centre-of-mass distance and the longest side
    t.walk(0.6530)
    assert 3 in _far(t, 16)


def test_mac_is_strict_at_equality():
    """All particles on the x axis: sink leaf 20 (particle 4 at x = 4)
    against node 3 has H_3 = 7.5 and R = 11.5 - 4 = 7.5 exactly, so at
    theta = 1 the ratio equals theta and Eq. 4's strict inequality rejects
    the cell; one ulp above 1 it is accepted."""
    t = _line16(np.zeros(16))
    t.walk(1.0)
    assert 3 not in _far(t, 20)
    t.walk(float(np.nextafter(1.0, 2.0)))
    assert 3 in _far(t, 20)


def test_accuracy_on_uniform_sphere():
    # Sec. 3.1: error falls with theta; at theta = 0.5 on the homogeneous
    # sphere the mean relative error is well below 0.1%.
    c = W.uniform_sphere()
    t = O.OracleTree(*c.arrays(), n_ll=8)
    ref = brute.direct_accel(c.x, c.y, c.z, c.m, c.h)
    stats = {}
    for th in (0.4, 0.5, 0.7, 1.0):
        t.walk(th)
        stats[th] = brute.error_stats(np.stack(t.gravity(), 1), ref)
    assert stats[0.4]["mean"] < stats[0.5]["mean"] < stats[0.7]["mean"] < stats[1.0]["mean"]
    assert stats[0.5]["mean"] < 1e-3 and stats[0.7]["frac_below_1pct"] > 0.99


# --------------------------------------------------------------------------
# vector-Jacobian product on the fixed tree
# --------------------------------------------------------------------------
def _L_fixed(t, c, gx, gy, gz, x, y, z, m):
    t.refresh(x, y, z, m, c.h)
    ax, ay, az = t.gravity()
    return float((gx * ax).sum() + (gy * ay).sum() + (gz * az).sum())


@pytest.mark.parametrize("theta", [0.5, 0.8])
def test_vjp_finite_differences(theta):
    c = W.small_random(120, 31, "clustered")
    gx, gy, gz = W.cotangents(c.n, seed=4)
    t = O.OracleTree(*c.arrays(), n_ll=4)
    t.walk(theta)
    nn, nf, _ = t.list_sizes()
    assert nf.sum() > 0
    dx, dy, dz, dm = t.vjp(gx, gy, gz)
    base = [c.x.copy(), c.y.copy(), c.z.copy(), c.m.copy()]
    rng = np.random.default_rng(0)
    for i in rng.choice(c.n, 12, replace=False):
        for comp, grad in zip(range(4), (dx, dy, dz, dm)):
            eps = 1e-6 if comp < 3 else 1e-6 * c.m[i]
            p = [b.copy() for b in base]; p[comp][i] += eps
            mm = [b.copy() for b in base]; mm[comp][i] -= eps
            num = (_L_fixed(t, c, gx, gy, gz, *p) - _L_fixed(t, c, gx, gy, gz, *mm)) / (2 * eps)
            scale = np.abs(grad).max() if comp < 3 else np.abs(grad).max()
            assert abs(num - grad[i]) < 2e-6 * scale + 1e-7 * abs(num), (i, comp, num, grad[i])
    t.refresh(*base, c.h)


def test_vjp_invariants():
    c = W.small_random(300, 41, "plummer")
    gx, gy, gz = W.cotangents(c.n, seed=5)
    t = O.OracleTree(*c.arrays(), n_ll=5)
    t.walk(0.7)
    dx, dy, dz, dm = t.vjp(gx, gy, gz)
    ax, ay, az = t.gravity()
    L = (gx * ax).sum() + (gy * ay).sum() + (gz * az).sum()
    scale = np.abs(np.concatenate([dx, dy, dz])).sum()
    # translation invariance with fixed lists
    for d in (dx, dy, dz):
        assert abs(d.sum()) < 1e-11 * scale
    # accelerations are homogeneous of degree one in the masses
    assert (c.m * dm).sum() == pytest.approx(L, rel=1e-10)


def test_vjp_theta_zero_equals_autograd_of_direct_sum():
    c = W.small_random(150, 51, "clustered")
    gx, gy, gz = W.cotangents(c.n, seed=6)
    t = O.OracleTree(*c.arrays(), n_ll=4)
    t.walk(0.0)
    dx, dy, dz, dm = t.vjp(gx, gy, gz)
    rx, ry, rz, rm, _ = brute.direct_accel_torch_grad(c.x, c.y, c.z, c.m, c.h, gx, gy, gz)
    for a, b in ((dx, rx), (dy, ry), (dz, rz), (dm, rm)):
        assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()
