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
// and the backward pass needs dPsi/dM, dPsi/dQ (closed forms below),
// dPsi/dR (forward-mode dual numbers through the same closed forms, which
// carries the fourth derivative of the field without forming it), and
// d(G2:H/2)/dR, the part that moves with the sink's centre of mass.
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

// f (0..2), J (3..8, jidx), H (9..18, hidx) of one source, accumulated.
RCB_HD void m2l_accumulate(double x, double y, double z, double M, const double qq[6], double (&c)[19]) {
    const double r2 = (x * x + y * y) + z * z;
    const double rinv = rsqrt64(r2);
    const double rinv2 = rinv * rinv;
    const double D1 = -rinv * rinv2;
    const double D2 = -3.0 * D1 * rinv2;
    const double D3 = -5.0 * D2 * rinv2;
    const double D4 = -7.0 * D3 * rinv2;
    const double D5 = -9.0 * D4 * rinv2;
    const double X[3] = {x, y, z};
    const double Qm[3][3] = {{qq[0], qq[1], qq[2]}, {qq[1], qq[3], qq[4]}, {qq[2], qq[4], qq[5]}};
    double qv[3];
    for (int i = 0; i < 3; ++i) qv[i] = Qm[i][0] * x + Qm[i][1] * y + Qm[i][2] * z;
    const double s = qv[0] * x + qv[1] * y + qv[2] * z;
    const double sixth = 1.0 / 6.0, third = 1.0 / 3.0;
    const double a1 = M * D1 + sixth * D3 * s;
    const double b2 = M * D2 + sixth * D4 * s;
    const double e3 = M * D3 + sixth * D5 * s;
    const double c0 = third * D2, c1 = third * D3, c2 = third * D4;
    for (int i = 0; i < 3; ++i) c[i] += a1 * X[i] + c0 * qv[i];
    for (int i = 0; i < 3; ++i)
        for (int l = i; l < 3; ++l) {
            double v = b2 * X[i] * X[l] + c1 * (qv[i] * X[l] + qv[l] * X[i]) + c0 * Qm[i][l];
            if (i == l) v += a1;
            c[3 + jidx(i, l)] += v;
        }
    for (int i = 0; i < 3; ++i)
        for (int l = i; l < 3; ++l)
            for (int m = l; m < 3; ++m) {
                double v = e3 * X[i] * X[l] * X[m];
                double dd = 0.0;
                if (i == l) dd += X[m];
                if (i == m) dd += X[l];
                if (l == m) dd += X[i];
                v += b2 * dd;
                v += c2 * (qv[i] * X[l] * X[m] + qv[l] * X[i] * X[m] + qv[m] * X[i] * X[l]);
                double w = Qm[l][m] * X[i] + Qm[i][m] * X[l] + Qm[i][l] * X[m];
                if (l == m) w += qv[i];
                if (i == m) w += qv[l];
                if (i == l) w += qv[m];
                v += c1 * w;
                c[9 + hidx(i, l, m)] += v;
            }
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


// Closed-form version of far_pair_adjoint (no dual numbers). With ' = d/dR
// and the recursions dD_k/dx_n = D_(k+1) x_n, ds/dx_n = 2 q_n, dq_i/dx_n = Q_in,
//   e4 = M D4 + s D6/6, c3 = D5/3,
// the fourth derivative T4_ilmn = dH_ilm/dx_n contracted with G2/2 gives
//   2 cot_n = (e4 x_n + c3 q_n) w2 + e3 (p_n + 2 pt_n) + (e3 x_n + c2 q_n)(2 sig.x + tau.x)
//           + b2 (2 sig_n + tau_n) + c3 x_n (q.p + 2 q.pt)
//           + c2 [Q p + 2 Rm^T q + 2 Q pt + 2 Rm q + 2 P q]_n
//           + c2 x_n (Q:P + 2 Q:Rm + tau.q + 2 sig.q)
//           + c1 [G2_n..:Q + 2 sum_im G2_inm Q_im + Q tau + 2 Q sig]_n
// with w2 = G2_ilm x_i x_l x_m, p_i = G2_ilm x_l x_m, pt_l = G2_ilm x_i x_m,
// P_lm = G2_ilm x_i, Rm_il = G2_ilm x_m; and
//   (G0.J)_n  = b2 u0 x_n + a1 G0_n + c1 ((G0.q) x_n + q_n u0) + c0 (Q G0)_n
//   (G1:H)_n  = e3 w11 x_n + b2 (t1 x_n + v1_n + v1t_n) + c2 ((q.v1 + q.v1t) x_n + q_n w11)
//             + c1 ((Q v1t)_n + (Q v1)_n + (G1:Q) x_n + (G1^T q)_n + (G1 q)_n + t1 q_n)
//   rho = G0.J + G1:H + cot.
RCB_HD void far_pair_adjoint_cf(double x, double y, double z, double M, const double qq[6],
                                const SinkMoments &G, double rho[3], double cot[3], double &adjM,
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
    const double Qm[3][3] = {{qq[0], qq[1], qq[2]}, {qq[1], qq[3], qq[4]}, {qq[2], qq[4], qq[5]}};
    double q[3];
    for (int i = 0; i < 3; ++i) q[i] = Qm[i][0] * x + Qm[i][1] * y + Qm[i][2] * z;
    const double s = q[0] * x + q[1] * y + q[2] * z;
    const double sixth = 1.0 / 6.0, third = 1.0 / 3.0;
    const double a1 = M * D1 + sixth * D3 * s;
    const double b2 = M * D2 + sixth * D4 * s;
    const double e3 = M * D3 + sixth * D5 * s;
    const double e4 = M * D4 + sixth * D6 * s;
    const double c0 = third * D2, c1 = third * D3, c2 = third * D4, c3 = third * D5;
    // sink contractions
    const double u0 = G.G0[0] * x + G.G0[1] * y + G.G0[2] * z;
    double v1[3], v1t[3];
    for (int i = 0; i < 3; ++i) {
        v1[i] = G.G1[3 * i] * x + G.G1[3 * i + 1] * y + G.G1[3 * i + 2] * z;
        v1t[i] = G.G1[i] * x + G.G1[3 + i] * y + G.G1[6 + i] * z;
    }
    const double w11 = x * v1[0] + y * v1[1] + z * v1[2];
    double P[6];
    for (int k = 0; k < 6; ++k) P[k] = G.G2[k] * x + G.G2[6 + k] * y + G.G2[12 + k] * z;
    double Rm[9];
    for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l)
            Rm[3 * i + l] = G.G2[6 * i + jidx(l, 0)] * x + G.G2[6 * i + jidx(l, 1)] * y +
                            G.G2[6 * i + jidx(l, 2)] * z;
    double p[3], pt[3];
    for (int i = 0; i < 3; ++i) {
        p[i] = Rm[3 * i] * x + Rm[3 * i + 1] * y + Rm[3 * i + 2] * z;
        pt[i] = P[jidx(i, 0)] * x + P[jidx(i, 1)] * y + P[jidx(i, 2)] * z;
    }
    const double w2 = p[0] * x + p[1] * y + p[2] * z;
    const double sx = G.sig[0] * x + G.sig[1] * y + G.sig[2] * z;
    const double tx = G.tau[0] * x + G.tau[1] * y + G.tau[2] * z;
    double G1Q = 0.0, QP = 0.0, QRm = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l) {
            G1Q += G.G1[3 * i + l] * Qm[i][l];
            QP += Qm[i][l] * P[jidx(i, l)];
            QRm += Qm[i][l] * Rm[3 * i + l];
        }
    const double G0q = G.G0[0] * q[0] + G.G0[1] * q[1] + G.G0[2] * q[2];
    const double qv1 = q[0] * v1[0] + q[1] * v1[1] + q[2] * v1[2];
    const double qv1t = q[0] * v1t[0] + q[1] * v1t[1] + q[2] * v1t[2];
    const double tq = G.tau[0] * q[0] + G.tau[1] * q[1] + G.tau[2] * q[2];
    const double sq = G.sig[0] * q[0] + G.sig[1] * q[1] + G.sig[2] * q[2];
    const double qp = q[0] * p[0] + q[1] * p[1] + q[2] * p[2];
    const double qpt = q[0] * pt[0] + q[1] * pt[1] + q[2] * pt[2];
    const double k3 = 2.0 * sx + tx;
    const double k7 = QP + 2.0 * QRm + tq + 2.0 * sq;
    const double k5 = qp + 2.0 * qpt;
    for (int n = 0; n < 3; ++n) {
        double Qp = 0.0, RmTq = 0.0, Qpt = 0.0, Rmq = 0.0, Pq = 0.0, QG0 = 0.0, Qv1t = 0.0, Qv1 = 0.0;
        double G1Tq = 0.0, G1q = 0.0, Qtau = 0.0, Qsig = 0.0, G2nQ = 0.0, G2inmQ = 0.0;
        for (int i = 0; i < 3; ++i) {
            Qp += Qm[n][i] * p[i];
            RmTq += Rm[3 * i + n] * q[i];
            Qpt += Qm[n][i] * pt[i];
            Rmq += Rm[3 * n + i] * q[i];
            Pq += P[jidx(n, i)] * q[i];
            QG0 += Qm[n][i] * G.G0[i];
            Qv1t += Qm[n][i] * v1t[i];
            Qv1 += Qm[n][i] * v1[i];
            G1Tq += G.G1[3 * i + n] * q[i];
            G1q += G.G1[3 * n + i] * q[i];
            Qtau += Qm[n][i] * G.tau[i];
            Qsig += Qm[n][i] * G.sig[i];
            for (int m = 0; m < 3; ++m) {
                G2nQ += G.G2[6 * n + jidx(i, m)] * Qm[i][m];
                G2inmQ += G.G2[6 * i + jidx(n, m)] * Qm[i][m];
            }
        }
        const double two_cot = (e4 * X[n] + c3 * q[n]) * w2 + e3 * (p[n] + 2.0 * pt[n]) +
                               (e3 * X[n] + c2 * q[n]) * k3 + b2 * (2.0 * G.sig[n] + G.tau[n]) +
                               c3 * X[n] * k5 + c2 * (Qp + 2.0 * RmTq + 2.0 * Qpt + 2.0 * Rmq + 2.0 * Pq) +
                               c2 * X[n] * k7 + c1 * (G2nQ + 2.0 * G2inmQ + Qtau + 2.0 * Qsig);
        const double g0j = b2 * u0 * X[n] + a1 * G.G0[n] + c1 * (G0q * X[n] + q[n] * u0) + c0 * QG0;
        const double g1h = e3 * w11 * X[n] + b2 * (G.t1 * X[n] + v1[n] + v1t[n]) +
                           c2 * ((qv1 + qv1t) * X[n] + q[n] * w11) +
                           c1 * (Qv1t + Qv1 + G1Q * X[n] + G1Tq + G1q + G.t1 * q[n]);
        cot[n] = 0.5 * two_cot;
        rho[n] = g0j + g1h + cot[n];
    }
    const double kA = u0 + G.t1;
    const double kB = w11 + sx + 0.5 * tx;
    const double kE = 0.5 * w2;
    adjM = D1 * kA + D2 * kB + D3 * kE;
    const double sig_s = sixth * (D3 * kA + D4 * kB + D5 * kE);
    double psq[3];
    for (int j = 0; j < 3; ++j)
        psq[j] = c0 * G.G0[j] + c1 * (v1[j] + v1t[j] + 0.5 * G.tau[j] + G.sig[j]) + 0.5 * c2 * (p[j] + 2.0 * pt[j]);
    double A[3][3];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
            A[j][k] = sig_s * X[j] * X[k] + psq[j] * X[k] + c0 * G.G1[3 * j + k] +
                      c1 * (0.5 * P[jidx(j, k)] + Rm[3 * j + k]);
    adjQ[0] = A[0][0];
    adjQ[1] = 0.5 * (A[0][1] + A[1][0]);
    adjQ[2] = 0.5 * (A[0][2] + A[2][0]);
    adjQ[3] = A[1][1];
    adjQ[4] = 0.5 * (A[1][2] + A[2][1]);
    adjQ[5] = A[2][2];
}

}  // namespace rcbfar
