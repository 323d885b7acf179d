// Host build of the library's far-field algebra (csrc/far_math.h) for the
// CPU tests, which compare it with the oracle's generic tensor code.
#include "far_math.h"

extern "C" {

void shim_m2l(double x, double y, double z, double M, const double *q6, double *c19) {
    double a[rcbfar::kAcc], c[19];
    for (int i = 0; i < rcbfar::kAcc; ++i) a[i] = 0.0;
    rcbfar::m2l_accumulate(x, y, z, M, q6, a);
    rcbfar::m2l_finish(a, c);
    for (int i = 0; i < 19; ++i) c19[i] = c[i];
}

void shim_m2l_b(double x, double y, double z, double M, const double *q6, double *c19) {
    double a[rcbfar::kAcc], c[19];
    for (int i = 0; i < rcbfar::kAcc; ++i) a[i] = 0.0;
    rcbfar::m2l_accumulate<true>(x, y, z, M, q6, a);
    rcbfar::m2l_finish(a, c);
    for (int i = 0; i < 19; ++i) c19[i] = c[i];
}

void shim_pair_adjoint(double x, double y, double z, double M, const double *q6, const double *G0,
                       const double *G1, const double *G2, double *rho, double *cot, double *adjM,
                       double *adjQ) {
    rcbfar::SinkMoments G;
    for (int i = 0; i < 3; ++i) G.G0[i] = G0[i];
    for (int i = 0; i < 9; ++i) G.G1[i] = G1[i];
    for (int i = 0; i < 18; ++i) G.G2[i] = G2[i];
    rcbfar::sink_traces(G);
    rcbfar::far_pair_adjoint(x, y, z, M, q6, G, rho, cot, *adjM, adjQ);
}

void shim_pair_adjoint_sym(double x, double y, double z, double M, const double *q6, const double *G0,
                           const double *G1, const double *G2, double *rho, double *cot, double *adjM,
                           double *adjQ) {
    rcbfar::SymMoments S;
    rcbfar::sym_moments(G0, G1, G2, S);
    rcbfar::far_pair_adjoint_sym(x, y, z, M, q6, S, rho, cot, *adjM, adjQ);
}

int shim_jidx(int i, int l) { return rcbfar::jidx(i, l); }
int shim_hidx(int i, int l, int m) { return rcbfar::hidx(i, l, m); }
}
