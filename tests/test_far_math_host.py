"""Host build of the library's far-field algebra (csrc/far_math.h) against
the oracle's generic derivative-tensor code (pinned by sympy and finite
differences). Checks the forward f, J, H of one source and every output of
the backward pair adjoint: dPsi/dR, the sink-centre part, dPsi/dM, dPsi/dQ."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SHIM = os.path.join(HERE, "native", "far_math_shim.cpp")
OUT = os.path.join(HERE, "native", "_build", "libfar_math_shim.so")
HDR = os.path.join(ROOT, "paper_1108_0028_amd", "csrc", "far_math.h")


def _shim():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    if not os.path.exists(OUT) or os.path.getmtime(OUT) < max(os.path.getmtime(SHIM), os.path.getmtime(HDR)):
        subprocess.check_call(["g++", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-std=c++17",
                               "-I", os.path.dirname(HDR), "-o", OUT, SHIM])
    L = C.CDLL(OUT)
    dp = C.POINTER(C.c_double)
    L.shim_m2l.argtypes = [C.c_double] * 4 + [dp, dp]
    L.shim_m2l_b.argtypes = [C.c_double] * 4 + [dp, dp]
    L.shim_pair_adjoint.argtypes = [C.c_double] * 4 + [dp] * 8
    L.shim_pair_adjoint_sym.argtypes = [C.c_double] * 4 + [dp] * 8
    L.shim_jidx.argtypes = [C.c_int, C.c_int]
    L.shim_hidx.argtypes = [C.c_int] * 3
    return L


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


JI = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
HI = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2), (1, 2, 2),
      (2, 2, 2)]


def test_index_maps():
    L = _shim()
    for k, (i, l) in enumerate(JI):
        assert L.shim_jidx(i, l) == k and L.shim_jidx(l, i) == k
    import itertools
    for k, t in enumerate(HI):
        for perm in itertools.permutations(t):
            assert L.shim_hidx(*perm) == k


@pytest.mark.parametrize("seed", range(6))
def test_forward_m2l_matches_oracle(seed):
    L = _shim()
    rng = np.random.default_rng(seed)
    R = rng.normal(size=3) * 3
    M = rng.uniform(0.1, 2)
    q = rng.normal(size=6)
    q[5] = -(q[0] + q[3])                     # traceless
    c = np.zeros(19)
    L.shim_m2l(R[0], R[1], R[2], M, _p(q), _p(c))
    f, J, H = O.far_coeffs(M, q, R)
    np.testing.assert_allclose(c[:3], f, rtol=1e-12, atol=1e-14 * np.abs(f).max())
    for k, (i, l) in enumerate(JI):
        assert c[3 + k] == pytest.approx(J[i, l], rel=1e-11, abs=1e-13 * np.abs(J).max())
    for k, (i, l, m) in enumerate(HI):
        assert c[9 + k] == pytest.approx(H[i, l, m], rel=1e-11, abs=1e-13 * np.abs(H).max())


@pytest.mark.parametrize("seed", range(4))
def test_forward_m2l_reading_b_matches_oracle(seed):
    # reading B: f of the full field, J and H of the monopole field
    L = _shim()
    rng = np.random.default_rng(50 + seed)
    R = rng.normal(size=3) * 3
    M = rng.uniform(0.1, 2)
    q = rng.normal(size=6)
    q[5] = -(q[0] + q[3])
    c = np.zeros(19)
    L.shim_m2l_b(R[0], R[1], R[2], M, _p(q), _p(c))
    f, _, _ = O.far_coeffs(M, q, R)
    _, J, H = O.far_coeffs(M, np.zeros(6), R)
    np.testing.assert_allclose(c[:3], f, rtol=1e-12, atol=1e-14 * np.abs(f).max())
    for k, (i, l) in enumerate(JI):
        assert c[3 + k] == pytest.approx(J[i, l], rel=1e-11, abs=1e-13 * np.abs(J).max())
    for k, (i, l, m) in enumerate(HI):
        assert c[9 + k] == pytest.approx(H[i, l, m], rel=1e-11, abs=1e-13 * np.abs(H).max())


@pytest.mark.parametrize("form", ["shim_pair_adjoint", "shim_pair_adjoint_sym"])
@pytest.mark.parametrize("seed", range(6))
def test_pair_adjoint_matches_oracle_tensors(seed, form):
    L = _shim()
    rng = np.random.default_rng(100 + seed)
    R = rng.normal(size=3) * 2.5
    M = rng.uniform(0.1, 2)
    q = rng.normal(size=6)
    q[5] = -(q[0] + q[3])
    G0 = rng.normal(size=3)
    G1 = rng.normal(size=(3, 3))
    G2 = rng.normal(size=(3, 3, 3))
    G2 = 0.5 * (G2 + G2.transpose(0, 2, 1))   # symmetric in the last two indices
    G2u = np.array([[G2[i, l, m] for (l, m) in JI] for i in range(3)]).ravel()
    rho = np.zeros(3); cot = np.zeros(3); aM = np.zeros(1); aQ = np.zeros(6)
    getattr(L, form)(R[0], R[1], R[2], M, _p(q), _p(G0), _p(np.ascontiguousarray(G1.ravel())),
                     _p(G2u), _p(rho), _p(cot), _p(aM), _p(aQ))
    f, J, H, T4 = O.far_coeffs(M, q, R, with_t4=True)
    g = [None] + [O.deriv_tensor(n, R) for n in range(1, 6)]
    rho_ref = (np.einsum("i,il->l", G0, J) + np.einsum("im,iml->l", G1, H)
               + 0.5 * np.einsum("imn,imnl->l", G2, T4))
    cot_ref = 0.5 * np.einsum("imn,imnl->l", G2, T4)
    aM_ref = (np.einsum("i,i", g[1], G0) + np.einsum("il,il", g[2], G1)
              + 0.5 * np.einsum("ilm,ilm", g[3], G2))
    aQ_ref = (np.einsum("ijk,i->jk", g[3], G0) + np.einsum("ijkl,il->jk", g[4], G1)
              + 0.5 * np.einsum("ijklm,ilm->jk", g[5], G2)) / 6.0
    sc = np.abs(rho_ref).max()
    np.testing.assert_allclose(rho, rho_ref, rtol=1e-10, atol=1e-12 * sc)
    np.testing.assert_allclose(cot, cot_ref, rtol=1e-10, atol=1e-12 * np.abs(cot_ref).max())
    assert aM[0] == pytest.approx(aM_ref, rel=1e-10)
    # Q is traceless and so is every dQ/d(input): only the deviatoric part of
    # dPsi/dQ reaches the gradients, and the closed forms drop tr(Q) terms.
    full = np.zeros((3, 3))
    for k, (j, l) in enumerate(JI):
        full[j, l] = full[l, j] = aQ[k]
    dev = lambda a: a - np.trace(a) / 3.0 * np.eye(3)
    np.testing.assert_allclose(dev(full), dev(aQ_ref), rtol=1e-9, atol=1e-12 * np.abs(aQ_ref).max())
