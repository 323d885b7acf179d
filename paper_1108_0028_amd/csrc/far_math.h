// far_math.h -- far-field algebra of one source node B seen from a sink leaf
// A (Sec. 2.4.2), written once for the device kernels and for host tests.
//
// Source B: mass M, traceless quadrupole Q (Eq. 1 / Eq. 2) about its centre
// of mass; x = R = com_A - com_B, r = |x|. With the potential of Eq. 5,
// Phi = -M/r - (1/6) Q_jk d_jk(1/r), the sink coefficients of Eq. 6 are
// f = -grad Phi, J = grad f, H = grad J. Writing q = Q x, s = x.q and
// D_n = (-1)^n (2n-1)!! / r^(2n+1):
//   f_i   = a1 x_i + c0 q_i
//   J_il  = b2 x_i x_l + a1 d_il + c1 (q_i x_l + q_l x_i) + c0 Q_il
//   H_ilm = e3 x_i x_l x_m + b2 (d_il x_m + d_im x_l + d_lm x_i)
//           + c2 (q_i x_l x_m + q_l x_i x_m + q_m x_i x_l)
//           + c1 (Q_lm x_i + Q_im x_l + Q_il x_m + q_i d_lm + q_l d_im + q_m d_il)
//   a1 = M D1 + s D3 / 6, b2 = M D2 + s D4 / 6, e3 = M D3 + s D5 / 6,
//   c0 = D2 / 3, c1 = D3 / 3, c2 = D4 / 3.
//
// Backward: with the sink leaf's cotangent moments
//   G0_i = sum_a g_ai, G1_il = sum_a g_ai d_al, G2_ilm = sum_a g_ai d_al d_am
// (d_a = r_a - com_A), leaf A's far-field share of L = sum g . a is, per B,
//   Psi = G0.f + G1:J + G2:H / 2,
// and the backward pass needs dPsi/dM, dPsi/dQ, dPsi/dR and d(G2:H/2)/dR,
// the part that moves with the sink's centre of mass. far_pair_adjoint
// carries dPsi/dR by forward-mode dual numbers through the forward closed
// forms (a cross-check for the tests); far_pair_adjoint_sym, used by the
// kernels, has every output in closed form over symmetrised moments.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define RCB_HD __host__ __device__ __forceinline__
#else
#define RCB_HD inline
#endif

namespace rcbfar {

// 1/sqrt(x) and 1/x in FP64: the hardware estimates refined by two Newton
// steps on the device (the estimate's error squares each step); the plain
// expressions on the host.
RCB_HD double rsqrt64(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * (1.5 - h * y * y);
    y = y * (1.5 - h * y * y);
    return y;
#else
    return 1.0 / sqrt(x);
#endif
}
RCB_HD double rcp64(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rcp(x);
    y = y * (2.0 - x * y);
    y = y * (2.0 - x * y);
    return y;
#else
    return 1.0 / x;
#endif
}

RCB_HD constexpr int jidx(int i, int l) {
    // (00)(01)(02)(11)(12)(22)
    return (i < l ? i : l) == 0 ? (i < l ? l : i) : ((i < l ? i : l) == 1 ? 2 + (i < l ? l : i) : 5);
}
RCB_HD constexpr int hidx(int i, int l, int m) {
    // (000)(001)(002)(011)(012)(022)(111)(112)(122)(222)
    int a = i, b = l, c = m, t = 0;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    return a == 0 ? (b == 0 ? c : (b == 1 ? 2 + c : 5)) : (a == 1 ? (b == 1 ? 5 + c : 8) : 9);
}

// One source's f, J, H added into a reduced accumulator of kAcc doubles.
// With ri = 1/r the coefficients are powers of ri:
//   c0 = ri^5, c1 = -5 ri^7, c2 = 35 ri^9,
//   a1 = -M ri^3 + c1 s / 2, b2 = 3 M ri^5 + c2 s / 2,
//   e3 / 3 = M c1 - 105 ri^11 s / 2,
// and with g = b2 x + c1 q, u = e3 x / 3 + c2 q and cx = c1 x the closed
// forms above regroup as
//   f_i = a1 x_i + c0 q_i
//   J_il = g_i x_l + q_l cx_i + c0 Q_il + a1 d_il
//   H_ilm = sum over the three choices of the single index j (the other
//           two, k and n): u_j x_k x_n + Q_kn cx_j + d_kn g_j
// The field of Eq. 5 is harmonic, so J and H are traceless in every index
// pair; only 5 components of J and 7 of H are accumulated, and the
// Kronecker-delta terms are summed once (sum of a1, sum of g) instead of
// into every diagonal component. Within one H component the three choices
// of j coincide in pairs or all three when indices repeat; such terms are
// accumulated once and weighted by their multiplicity in m2l_finish:
//   H_000 = 3 [u0 x0x0 + Q00 cx0]            (h0)
//   H_001 = 2 [u0 x0x1 + Q01 cx0] + [u1 x0x0 + Q00 cx1]   (h1, h2)
//   H_002 = 2 [u0 x0x2 + Q02 cx0] + [u2 x0x0 + Q00 cx2]   (h3, h4)
//   H_011 = [u0 x1x1 + Q11 cx0] + 2 [u1 x0x1 + Q01 cx1]   (h5, h6)
//   H_012 = u0 x1x2 + u1 x0x2 + u2 x0x1 + Q12 cx0 + Q02 cx1 + Q01 cx2 (h7)
//   H_111 = 3 [u1 x1x1 + Q11 cx1]            (h8)
//   H_112 = 2 [u1 x1x2 + Q12 cx1] + [u2 x1x1 + Q11 cx2]   (h9, h10)
// (each plus its delta terms). Layout: f (0..2); J xx xy xz yy yz without
// a1 (3..7); h0..h10 (8..18); sum g (19..21); sum a1 (22).
//
// RB (Taylor reading B): f as above, but J and H of the monopole field
// alone, J_il = M g_il and H_ilm = M g_ilm, i.e. the same expressions with
// Q = 0 in them (g = M D2 x, u = M D3 x / 3, a1 = M D1).
constexpr int kAcc = 23;

template <bool RB = false>
RCB_HD void m2l_accumulate(double x, double y, double z, double M, const double qq[6], double (&c)[kAcc]) {
    const double X[3] = {x, y, z};
    const double r2 = (x * x + y * y) + z * z;
    const double ri = rsqrt64(r2);
    const double w = ri * ri;
    const double p3 = ri * w;
    const double c0 = p3 * w;
    const double p7 = c0 * w;
    const double p9 = p7 * w;
    const double c1 = -5.0 * p7;
    const double c2 = 35.0 * p9;
    double q[3];
    for (int i = 0; i < 3; ++i) q[i] = qq[jidx(i, 0)] * x + qq[jidx(i, 1)] * y + qq[jidx(i, 2)] * z;
    const double hs = 0.5 * ((q[0] * x + q[1] * y) + q[2] * z);
    const double a1 = hs * c1 - M * p3;
    // f (both readings)
    for (int i = 0; i < 3; ++i) {
        c[i] += a1 * X[i];
        c[i] += c0 * q[i];
    }
    const double xx[5] = {x * x, x * y, x * z, y * y, y * z};   // 00 01 02 11 12
    double g[3], u[3];
    if constexpr (RB) {
        const double gm = 3.0 * (M * c0), um = M * c1, am = -(M * p3);
        for (int i = 0; i < 3; ++i) {
            g[i] = gm * X[i];
            u[i] = um * X[i];
        }
        c[3] += g[0] * x;
        c[4] += g[0] * y;
        c[5] += g[0] * z;
        c[6] += g[1] * y;
        c[7] += g[1] * z;
        c[8] += u[0] * xx[0];
        c[9] += u[0] * xx[1];
        c[10] += u[1] * xx[0];
        c[11] += u[0] * xx[2];
        c[12] += u[2] * xx[0];
        c[13] += u[0] * xx[3];
        c[14] += u[1] * xx[1];
        c[15] += u[0] * xx[4];
        c[15] += u[1] * xx[2];
        c[15] += u[2] * xx[1];
        c[16] += u[1] * xx[3];
        c[17] += u[1] * xx[4];
        c[18] += u[2] * xx[3];
        for (int i = 0; i < 3; ++i) c[19 + i] += g[i];
        c[22] += am;
        return;
    }
    const double b2 = hs * c2 + 3.0 * (M * c0);
    const double e3t = (hs * (p9 * w)) * -105.0 + M * c1;
    double cx[3];
    for (int i = 0; i < 3; ++i) {
        const double cq = c1 * q[i];
        g[i] = b2 * X[i] + cq;
        u[i] = e3t * X[i] + c2 * q[i];
        cx[i] = c1 * X[i];
    }
    // J: xx xy xz yy yz
    for (int i = 0; i < 2; ++i)
        for (int l = i; l < 3; ++l) {
            double &v = c[3 + jidx(i, l)];
            v += g[i] * X[l];
            v += q[l] * cx[i];
            v += c0 * qq[jidx(i, l)];
        }
    const double Q00 = qq[0], Q01 = qq[1], Q02 = qq[2], Q11 = qq[3], Q12 = qq[4];
    c[8] += u[0] * xx[0];
    c[8] += Q00 * cx[0];
    c[9] += u[0] * xx[1];
    c[9] += Q01 * cx[0];
    c[10] += u[1] * xx[0];
    c[10] += Q00 * cx[1];
    c[11] += u[0] * xx[2];
    c[11] += Q02 * cx[0];
    c[12] += u[2] * xx[0];
    c[12] += Q00 * cx[2];
    c[13] += u[0] * xx[3];
    c[13] += Q11 * cx[0];
    c[14] += u[1] * xx[1];
    c[14] += Q01 * cx[1];
    c[15] += u[0] * xx[4];
    c[15] += u[1] * xx[2];
    c[15] += u[2] * xx[1];
    c[15] += Q12 * cx[0];
    c[15] += Q02 * cx[1];
    c[15] += Q01 * cx[2];
    c[16] += u[1] * xx[3];
    c[16] += Q11 * cx[1];
    c[17] += u[1] * xx[4];
    c[17] += Q12 * cx[1];
    c[18] += u[2] * xx[3];
    c[18] += Q11 * cx[2];
    for (int i = 0; i < 3; ++i) c[19 + i] += g[i];
    c[22] += a1;
}

// the reduced accumulator of m2l_accumulate -> f (0..2), J (3..8, jidx),
// H (9..18, hidx)
RCB_HD void m2l_finish(const double (&a)[kAcc], double (&c)[19]) {
    for (int i = 0; i < 3; ++i) c[i] = a[i];
    const double *G = a + 19;
    c[3 + jidx(0, 0)] = a[3] + a[22];
    c[3 + jidx(0, 1)] = a[4];
    c[3 + jidx(0, 2)] = a[5];
    c[3 + jidx(1, 1)] = a[6] + a[22];
    c[3 + jidx(1, 2)] = a[7];
    c[3 + jidx(2, 2)] = -(c[3 + jidx(0, 0)] + c[3 + jidx(1, 1)]);
    c[9 + hidx(0, 0, 0)] = 3.0 * (a[8] + G[0]);
    c[9 + hidx(0, 0, 1)] = (2.0 * a[9] + a[10]) + G[1];
    c[9 + hidx(0, 0, 2)] = (2.0 * a[11] + a[12]) + G[2];
    c[9 + hidx(0, 1, 1)] = (a[13] + 2.0 * a[14]) + G[0];
    c[9 + hidx(0, 1, 2)] = a[15];
    c[9 + hidx(1, 1, 1)] = 3.0 * (a[16] + G[1]);
    c[9 + hidx(1, 1, 2)] = (2.0 * a[17] + a[18]) + G[2];
    c[9 + hidx(0, 2, 2)] = -(c[9 + hidx(0, 0, 0)] + c[9 + hidx(0, 1, 1)]);
    c[9 + hidx(1, 2, 2)] = -(c[9 + hidx(0, 0, 1)] + c[9 + hidx(1, 1, 1)]);
    c[9 + hidx(2, 2, 2)] = -(c[9 + hidx(0, 0, 2)] + c[9 + hidx(1, 1, 2)]);
}

// a + J d + H[d, d] / 2 for the 19 stored coefficients
template <typename T>
RCB_HD void l2p(const double (&c)[19], const T d[3], T out[3]) {
    for (int i = 0; i < 3; ++i) {
        T t1 = (T)c[i];
        T t2 = (T)0;
        for (int l = 0; l < 3; ++l) {
            t1 += (T)c[3 + jidx(i, l)] * d[l];
            for (int m = 0; m < 3; ++m) t2 += (T)c[9 + hidx(i, l, m)] * d[l] * d[m];
        }
        out[i] = t1 + (T)0.5 * t2;
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
struct Dual {   // value and gradient with respect to x = R
    double v, d0, d1, d2;
};
RCB_HD Dual dconst(double c) { return Dual{c, 0.0, 0.0, 0.0}; }
RCB_HD Dual operator+(const Dual &a, const Dual &b) { return Dual{a.v + b.v, a.d0 + b.d0, a.d1 + b.d1, a.d2 + b.d2}; }
RCB_HD Dual operator-(const Dual &a, const Dual &b) { return Dual{a.v - b.v, a.d0 - b.d0, a.d1 - b.d1, a.d2 - b.d2}; }
RCB_HD Dual operator*(const Dual &a, const Dual &b) {
    return Dual{a.v * b.v, a.v * b.d0 + a.d0 * b.v, a.v * b.d1 + a.d1 * b.v, a.v * b.d2 + a.d2 * b.v};
}
RCB_HD Dual operator*(double c, const Dual &a) { return Dual{c * a.v, c * a.d0, c * a.d1, c * a.d2}; }
RCB_HD Dual operator+(const Dual &a, double c) { return Dual{a.v + c, a.d0, a.d1, a.d2}; }

// Sink-leaf cotangent moments and their x-independent traces.
struct SinkMoments {
    double G0[3];
    double G1[9];    // G1[3 i + l]
    double G2[18];   // G2[6 i + jidx(l, m)], symmetric in (l, m)
    double t1;       // tr G1
    double sig[3];   // sig_m = sum_i G2_iim
    double tau[3];   // tau_i = sum_l G2_ill
};

RCB_HD void sink_traces(SinkMoments &G) {
    G.t1 = G.G1[0] + G.G1[4] + G.G1[8];
    for (int m = 0; m < 3; ++m) {
        G.sig[m] = G.G2[6 * 0 + jidx(0, m)] + G.G2[6 * 1 + jidx(1, m)] + G.G2[6 * 2 + jidx(2, m)];
        G.tau[m] = G.G2[6 * m + jidx(0, 0)] + G.G2[6 * m + jidx(1, 1)] + G.G2[6 * m + jidx(2, 2)];
    }
}

// One (A, B) pair of the backward pass.
//   rho   = dPsi/dR                 (B's centre of mass receives -rho)
//   cot   = d(G2:H/2)/dR            (A's centre of mass receives +cot)
//   adjM  = dPsi/dM_B
//   adjQ  = dPsi/dQ_B, symmetrised, unique order xx xy xz yy yz zz
//           (an off-diagonal entry is the derivative w.r.t. Q_jk = Q_kj
//            taken once; the push counts it for both (j,k) and (k,j)).
RCB_HD void far_pair_adjoint(double x, double y, double z, double M, const double qq[6],
                             const SinkMoments &G, double rho[3], double cot[3], double &adjM,
                             double adjQ[6]) {
    const Dual X[3] = {Dual{x, 1.0, 0.0, 0.0}, Dual{y, 0.0, 1.0, 0.0}, Dual{z, 0.0, 0.0, 1.0}};
    const double r2v = (x * x + y * y) + z * z;
    const double ri = 1.0 / sqrt(r2v);
    const double ri3 = ri * ri * ri;
    const Dual rinv = Dual{ri, -ri3 * x, -ri3 * y, -ri3 * z};
    const Dual rinv2 = rinv * rinv;
    const Dual D1 = -1.0 * (rinv * rinv2);
    const Dual D2 = -3.0 * (D1 * rinv2);
    const Dual D3 = -5.0 * (D2 * rinv2);
    const Dual D4 = -7.0 * (D3 * rinv2);
    const Dual D5 = -9.0 * (D4 * rinv2);
    const double Qm[3][3] = {{qq[0], qq[1], qq[2]}, {qq[1], qq[3], qq[4]}, {qq[2], qq[4], qq[5]}};
    Dual q[3];
    for (int i = 0; i < 3; ++i) q[i] = Qm[i][0] * X[0] + Qm[i][1] * X[1] + Qm[i][2] * X[2];
    const Dual s = q[0] * X[0] + q[1] * X[1] + q[2] * X[2];
    // sink contractions with x
    const Dual u0 = G.G0[0] * X[0] + G.G0[1] * X[1] + G.G0[2] * X[2];
    Dual v1[3], v1t[3];
    for (int i = 0; i < 3; ++i) {
        v1[i] = G.G1[3 * i] * X[0] + G.G1[3 * i + 1] * X[1] + G.G1[3 * i + 2] * X[2];
        v1t[i] = G.G1[i] * X[0] + G.G1[3 + i] * X[1] + G.G1[6 + i] * X[2];
    }
    const Dual w11 = X[0] * v1[0] + X[1] * v1[1] + X[2] * v1[2];
    Dual P[6];    // P_lm = sum_i G2_ilm x_i
    for (int k = 0; k < 6; ++k) P[k] = G.G2[k] * X[0] + G.G2[6 + k] * X[1] + G.G2[12 + k] * X[2];
    Dual Rm[9];   // Rm_il = sum_m G2_ilm x_m
    for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l)
            Rm[3 * i + l] = G.G2[6 * i + jidx(l, 0)] * X[0] + G.G2[6 * i + jidx(l, 1)] * X[1] +
                            G.G2[6 * i + jidx(l, 2)] * X[2];
    Dual p[3], pt[3];   // p_i = sum_lm G2_ilm x_l x_m ; pt_l = sum_im G2_ilm x_i x_m
    for (int i = 0; i < 3; ++i) {
        p[i] = Rm[3 * i] * X[0] + Rm[3 * i + 1] * X[1] + Rm[3 * i + 2] * X[2];
        pt[i] = P[jidx(i, 0)] * X[0] + P[jidx(i, 1)] * X[1] + P[jidx(i, 2)] * X[2];
    }
    const Dual w2 = p[0] * X[0] + p[1] * X[1] + p[2] * X[2];
    const Dual sx = G.sig[0] * X[0] + G.sig[1] * X[1] + G.sig[2] * X[2];
    const Dual tx = G.tau[0] * X[0] + G.tau[1] * X[1] + G.tau[2] * X[2];
    const double sixth = 1.0 / 6.0, third = 1.0 / 3.0;
    const Dual a1 = M * D1 + sixth * (D3 * s);
    const Dual b2 = M * D2 + sixth * (D4 * s);
    const Dual e3 = M * D3 + sixth * (D5 * s);
    const Dual c0 = third * D2, c1 = third * D3, c2 = third * D4;
    double G1Q = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l) G1Q += G.G1[3 * i + l] * Qm[i][l];
    const Dual G0q = G.G0[0] * q[0] + G.G0[1] * q[1] + G.G0[2] * q[2];
    const Dual qv1 = q[0] * v1[0] + q[1] * v1[1] + q[2] * v1[2];
    const Dual qv1t = q[0] * v1t[0] + q[1] * v1t[1] + q[2] * v1t[2];
    Dual QP = dconst(0.0), QRm = dconst(0.0);
    for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) {
            QP = QP + Qm[l][m] * P[jidx(l, m)];
            QRm = QRm + Qm[l][m] * Rm[3 * l + m];
        }
    const Dual tq = G.tau[0] * q[0] + G.tau[1] * q[1] + G.tau[2] * q[2];
    const Dual sq = G.sig[0] * q[0] + G.sig[1] * q[1] + G.sig[2] * q[2];
    const Dual qp = q[0] * p[0] + q[1] * p[1] + q[2] * p[2];
    const Dual qpt = q[0] * pt[0] + q[1] * pt[1] + q[2] * pt[2];
    const Dual psi01 = a1 * (u0 + G.t1) + c0 * (G0q + G1Q) + b2 * w11 + c1 * (qv1 + qv1t);
    const Dual psi2 = b2 * (sx + 0.5 * tx) + c1 * (0.5 * QP + QRm + 0.5 * tq + sq) + 0.5 * (e3 * w2) +
                      0.5 * (c2 * (qp + 2.0 * qpt));
    rho[0] = psi01.d0 + psi2.d0;
    rho[1] = psi01.d1 + psi2.d1;
    rho[2] = psi01.d2 + psi2.d2;
    cot[0] = psi2.d0;
    cot[1] = psi2.d1;
    cot[2] = psi2.d2;
    const double kA = u0.v + G.t1;
    const double kB = w11.v + sx.v + 0.5 * tx.v;
    const double kE = 0.5 * w2.v;
    adjM = D1.v * kA + D2.v * kB + D3.v * kE;
    const double sig_s = sixth * (D3.v * kA + D4.v * kB + D5.v * kE);
    double psq[3];
    for (int j = 0; j < 3; ++j)
        psq[j] = c0.v * G.G0[j] + c1.v * (v1[j].v + v1t[j].v + 0.5 * G.tau[j] + G.sig[j]) +
                 0.5 * c2.v * (p[j].v + 2.0 * pt[j].v);
    const double xs[3] = {x, y, z};
    double A[3][3];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
            A[j][k] = sig_s * xs[j] * xs[k] + psq[j] * xs[k] + c0.v * G.G1[3 * j + k] +
                      c1.v * (0.5 * P[jidx(j, k)].v + Rm[3 * j + k].v);
    adjQ[0] = A[0][0];
    adjQ[1] = 0.5 * (A[0][1] + A[1][0]);
    adjQ[2] = 0.5 * (A[0][2] + A[2][0]);
    adjQ[3] = A[1][1];
    adjQ[4] = 0.5 * (A[1][2] + A[2][1]);
    adjQ[5] = A[2][2];
}


// Symmetrised sink moments. Psi contracts G1 with the symmetric J and G2
// with the fully symmetric H, so only sym(G1) and the full symmetrisation of
// G2 enter Psi and all its derivatives:
//   S1 = G0, S2_il = (G1_il + G1_li)/2, S3_ilm = (G2_ilm + G2_lim + G2_mil)/3,
//   t1 = tr S2, sg_m = sum_i S3_iim.
struct SymMoments {
    double S1[3];
    double S2[6];    // jidx order
    double S3[10];   // hidx order
    double t1;
    double sg[3];
};

RCB_HD void sym_moments(const double G0[3], const double G1[9], const double G2[18], SymMoments &S) {
    for (int i = 0; i < 3; ++i) S.S1[i] = G0[i];
    for (int i = 0; i < 3; ++i)
        for (int l = i; l < 3; ++l) S.S2[jidx(i, l)] = 0.5 * (G1[3 * i + l] + G1[3 * l + i]);
    for (int i = 0; i < 3; ++i)
        for (int l = i; l < 3; ++l)
            for (int m = l; m < 3; ++m)
                S.S3[hidx(i, l, m)] =
                    (G2[6 * i + jidx(l, m)] + G2[6 * l + jidx(i, m)] + G2[6 * m + jidx(i, l)]) / 3.0;
    S.t1 = S.S2[0] + S.S2[3] + S.S2[5];
    for (int m = 0; m < 3; ++m) S.sg[m] = S.S3[hidx(0, 0, m)] + S.S3[hidx(1, 1, m)] + S.S3[hidx(2, 2, m)];
}

// Closed form of the pair adjoint with symmetrised moments (no dual numbers).
// With u0 = S1.x, v = S2 x, w11 = x.v, sx = sg.x, P_lm = S3_ilm x_i, p = P x,
// w2 = x.p, q = Q x, s = x.q and the scalars of the forward pass, the pair's
// share of L is
//   Psi = a1 K1 + b2 K2 + e3 w2/2 + c0 K3 + 2 c1 q.v + 3/2 c1 K4 + 3/2 c2 q.p,
//   K1 = u0 + t1, K2 = w11 + 3/2 sx, K3 = S1.q + S2:Q, K4 = Q:P + sg.q.
// Using dD_k/dx = D_(k+1) x, ds/dx = 2 q, dq_i/dx_n = Q_in and
//   da1 = b2 x + c1 q, db2 = e3 x + c2 q, de3 = e4 x + c3 q, dc_k = c_(k+1) x
// (e4 = M D4 + s D6/6, c3 = D5/3):
//   dPsi/dM = D1 K1 + D2 K2 + D3 w2/2
//   dPsi/dQ = sym[ ss x x^T + psq x^T ] + c0 S2 + 3/2 c1 P,
//             ss = (D3 K1 + D4 K2 + D5 w2/2)/6,
//             psq = c0 S1 + 2 c1 v + 3/2 c1 sg + 3/2 c2 p
//   rho = dPsi/dR = ax x + aq q + a1 S1 + b2 (2 v + 3/2 sg) + 3/2 e3 p + Q psq
//                   + 2 c1 S2 q + 3/2 c1 (S3:Q) + 3 c2 P q,
//         ax = b2 K1 + e3 K2 + e4 w2/2 + c1 K3 + 2 c2 q.v + 3/2 c2 K4 + 3/2 c3 q.p,
//         aq = c1 K1 + c2 K2 + c3 w2/2
//   cot = d(S3:H/2)/dR = bx x + bq q + 3/2 b2 sg + 3/2 e3 p + 3/2 c1 (S3:Q)
//                        + Q (3/2 c1 sg + 3/2 c2 p) + 3 c2 P q,
//         bx = 3/2 e3 sx + 3/2 c2 K4 + e4 w2/2 + 3/2 c3 q.p, bq = 3/2 c2 sx + c3 w2/2
// where (S3:Q)_n = S3_nlm Q_lm.
RCB_HD void far_pair_adjoint_sym(double x, double y, double z, double M, const double qq[6],
                                 const SymMoments &S, double rho[3], double cot[3], double &adjM,
                                 double adjQ[6]) {
    const double X[3] = {x, y, z};
    const double r2 = (x * x + y * y) + z * z;
    const double ri = rsqrt64(r2);
    const double ri2 = ri * ri;
    const double D1 = -ri * ri2;
    const double D2 = -3.0 * D1 * ri2;
    const double D3 = -5.0 * D2 * ri2;
    const double D4 = -7.0 * D3 * ri2;
    const double D5 = -9.0 * D4 * ri2;
    const double D6 = -11.0 * D5 * ri2;
    double q[3];
    for (int i = 0; i < 3; ++i) q[i] = qq[jidx(i, 0)] * x + qq[jidx(i, 1)] * y + qq[jidx(i, 2)] * z;
    const double s = q[0] * x + q[1] * y + q[2] * z;
    const double sixth = 1.0 / 6.0, third = 1.0 / 3.0;
    const double a1 = M * D1 + sixth * D3 * s;
    const double b2 = M * D2 + sixth * D4 * s;
    const double e3 = M * D3 + sixth * D5 * s;
    const double e4 = M * D4 + sixth * D6 * s;
    const double c0 = third * D2, c1 = third * D3, c2 = third * D4, c3 = third * D5;
    // sink contractions with x
    const double u0 = S.S1[0] * x + S.S1[1] * y + S.S1[2] * z;
    double v[3];
    for (int i = 0; i < 3; ++i) v[i] = S.S2[jidx(i, 0)] * x + S.S2[jidx(i, 1)] * y + S.S2[jidx(i, 2)] * z;
    const double w11 = v[0] * x + v[1] * y + v[2] * z;
    const double sx = S.sg[0] * x + S.sg[1] * y + S.sg[2] * z;
    double P[6];
    for (int l = 0; l < 3; ++l)
        for (int m = l; m < 3; ++m)
            P[jidx(l, m)] = S.S3[hidx(0, l, m)] * x + S.S3[hidx(1, l, m)] * y + S.S3[hidx(2, l, m)] * z;
    double p[3];
    for (int l = 0; l < 3; ++l) p[l] = P[jidx(l, 0)] * x + P[jidx(l, 1)] * y + P[jidx(l, 2)] * z;
    const double w2 = p[0] * x + p[1] * y + p[2] * z;
    // contractions with Q (symmetric: off-diagonal pairs counted twice)
    const double S2Q = (S.S2[0] * qq[0] + S.S2[3] * qq[3] + S.S2[5] * qq[5]) +
                       2.0 * (S.S2[1] * qq[1] + S.S2[2] * qq[2] + S.S2[4] * qq[4]);
    const double QP = (P[0] * qq[0] + P[3] * qq[3] + P[5] * qq[5]) +
                      2.0 * (P[1] * qq[1] + P[2] * qq[2] + P[4] * qq[4]);
    const double K1 = u0 + S.t1;
    const double K2 = w11 + 1.5 * sx;
    const double K3 = (S.S1[0] * q[0] + S.S1[1] * q[1] + S.S1[2] * q[2]) + S2Q;
    const double K4 = QP + (S.sg[0] * q[0] + S.sg[1] * q[1] + S.sg[2] * q[2]);
    const double qv = q[0] * v[0] + q[1] * v[1] + q[2] * v[2];
    const double qp = q[0] * p[0] + q[1] * p[1] + q[2] * p[2];
    adjM = D1 * K1 + D2 * K2 + 0.5 * D3 * w2;
    const double ss = sixth * (D3 * K1 + D4 * K2 + 0.5 * D5 * w2);
    double psq[3], psc[3];
    for (int j = 0; j < 3; ++j) {
        psc[j] = 1.5 * (c1 * S.sg[j] + c2 * p[j]);
        psq[j] = c0 * S.S1[j] + 2.0 * c1 * v[j] + psc[j];
    }
    for (int j = 0; j < 3; ++j)
        for (int k = j; k < 3; ++k)
            adjQ[jidx(j, k)] = ss * X[j] * X[k] + 0.5 * (psq[j] * X[k] + psq[k] * X[j]) +
                               c0 * S.S2[jidx(j, k)] + 1.5 * c1 * P[jidx(j, k)];
    const double ax = b2 * K1 + e3 * K2 + 0.5 * e4 * w2 + c1 * K3 + 2.0 * c2 * qv + 1.5 * c2 * K4 +
                      1.5 * c3 * qp;
    const double aq = c1 * K1 + c2 * K2 + 0.5 * c3 * w2;
    const double bx = 1.5 * e3 * sx + 1.5 * c2 * K4 + 0.5 * e4 * w2 + 1.5 * c3 * qp;
    const double bq = 1.5 * c2 * sx + 0.5 * c3 * w2;
    for (int n = 0; n < 3; ++n) {
        double S3Q = 0.0, Pq = 0.0, S2q = 0.0, Qpsq = 0.0, Qpsc = 0.0;
        for (int m = 0; m < 3; ++m) {
            for (int l = 0; l < 3; ++l) S3Q += S.S3[hidx(n, l, m)] * qq[jidx(l, m)];
            Pq += P[jidx(n, m)] * q[m];
            S2q += S.S2[jidx(n, m)] * q[m];
            Qpsq += qq[jidx(n, m)] * psq[m];
            Qpsc += qq[jidx(n, m)] * psc[m];
        }
        const double common = 1.5 * e3 * p[n] + 1.5 * c1 * S3Q + 3.0 * c2 * Pq;
        cot[n] = bx * X[n] + bq * q[n] + 1.5 * b2 * S.sg[n] + Qpsc + common;
        rho[n] = ax * X[n] + aq * q[n] + a1 * S.S1[n] + b2 * (2.0 * v[n] + 1.5 * S.sg[n]) + Qpsq +
                 2.0 * c1 * S2q + common;
    }
}

}  // namespace rcbfar
