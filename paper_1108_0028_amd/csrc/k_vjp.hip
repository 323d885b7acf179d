// k_vjp.hip -- vector-Jacobian product of the accelerations with the tree
// held fixed (topology, particle-to-leaf map and interaction lists frozen;
// M, COM and Q of every node are functions of the inputs). For
// L = sum_a g_a . a_a it returns dL/dx, dL/dy, dL/dz, dL/dm.
//
// Near field (Sec. 2.4.3), pair (a, b), v = r_a - r_b:
//   K = F I + (dF/dr / r) v v^T;  dr_a -= m_b K g_a;  dr_b += m_b K g_a;
//   dm_b -= F (v . g_a).
// Pairs are recomputed from the lists, not stored. The source-side terms
// are summed over the wave's sinks and added with FP64 atomics.
// Far field (Sec. 2.4.2, Eq. 6): per sink leaf the cotangent moments G0, G1,
// G2, stored symmetrised (far_math.h: only their symmetric parts reach Psi),
// then
//   dr_a += J g_a + H[g_a, d_a]                       (d_a = r_a - com_A)
//   com_A receives cot = sum_B d(G2:H/2)/dR  ->  dr_a += m_a/M_A cot,
//                                              dm_a += cot . d_a / M_A
//   node B receives dM, -dPsi/dR, dQ: summed over the group's leaves that
//   accepted B, then added with FP64 atomics.
// Push: every node's adjoint reaches its particles b through
//   M = sum m, COM = sum m r / M, Q = sum m (3 d d^T - |d|^2 I), d = r - COM:
//   dr_b += aR m_b / M + m_b (6 aQ d - 2 tr(aQ) d)
//   dm_b += aM + aR . d / M + 3 d.aQ.d - |d|^2 tr(aQ)
// (dQ/dCOM = 0 because sum m d = 0).
// Kernels: moments (per group) -> far (per group) -> near (per group, leaf by
// leaf) -> push.
#include <cstdlib>

#include "far_math.h"
#include "near_tile.h"
#include "rcb_internal.h"
#include "soft.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
// M, R(3) and the traceless part of the Q adjoint, (xx, xy, xz, yy, yz) with
// zz = -(xx + yy): Q is traceless, so the push (the only reader) sees the
// adjoint's traceless part alone (6 aQ d - 2 tr(aQ) d = 6 (aQ - tr/3 I) d, and
// likewise for dm), and one atomic per entry fewer goes out
constexpr int kAdj = 9;
constexpr int kAdjCopies = 8;   // node-adjoint copies filled by k_vjp_far
// Nodes of the levels above kMidLevel sit in the far lists of many groups at
// once, and the atomics on their adjoints contend: they get kAdjMidCopies
// copies (kAdjCopies / XCD), in their own array of kAdj * 2^kMidLevel per copy.
constexpr int kMidLevel = 16;
constexpr int kAdjMidCopies = 64;
constexpr int kAcc = 30;    // G0(3), G1(9), G2(18) while accumulating
constexpr int kMom = 23;    // S1(3), S2(6), S3(10), t1, sg(3): far_math.h SymMoments

using rcbfar::hidx;
using rcbfar::jidx;

struct VjpArgs {
    int64_t nleaf;
    int gk;
    int64_t ngroup;
    const int32_t *nfirst, *ncount;
    const double *ncom, *nM, *nQ;
    const int64_t *gnear_beg, *gnear_end, *gfar_beg, *gfar_end;
    const uint64_t *gnear, *gfar;
    const double *px, *py, *pz, *pm, *ph;
    const float *fdx, *fdy, *fdz, *fm, *fh;
    const int32_t *pid;
    const void *gx, *gy, *gz;
    double *mom;    // kMom per leaf: symmetrised cotangent moments
    double *leafc;  // kLeafC per leaf
    double *sink;   // 4 n, tree order: dx dy dz dm
    double *src;    // 4 n, tree order, atomics (FP64 form)
    float *srcf;    // the same in the mixed form (FP32 atomics, its contract's accumulation)
    double *adj;    // kAdj per label (summed copies); component q of label B at q * nlab + B
    double *adjm;   // unused
    int64_t nmid;   // labels below nmid have kAdjMidCopies adjoint copies, q * nmid + B
    int64_t n;
    int64_t nlab;
    // deterministic form: each far entry's node adjoint (kAdj FP64) at row
    // cbase[group] + (entry - the group's first entry)
    double *contrib;
    const int64_t *cbase;
    // deterministic form: the cotangents in tree order, 3 n values of the
    // output type (component c of tree position p at c * n + p)
    void *gtree;
};

template <bool MIXED>
__device__ __forceinline__ double load_g(const void *p, int32_t i) {
    if constexpr (MIXED) return (double)((const float *)p)[i];
    else return ((const double *)p)[i];
}

// leaf slot (within the group) of tree position pa
__device__ __forceinline__ int leaf_slot(const int32_t (&lf)[8], int32_t pa) {
    int la = 0;
#pragma unroll
    for (int i = 1; i < 8; ++i)
        if (lf[i] <= pa) la = i;
    return la;
}

// cotangent moments G0, G1, G2 of every leaf of the group, stored symmetrised
template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_vjp_moments(VjpArgs a) {
    __shared__ double acc_all[kWaves][8][kAcc];
    double(*acc)[kAcc] = acc_all[threadIdx.x / kWave];
    const int64_t gi = wave_index();
    if (gi >= a.ngroup) return;
    const int lane = lane_id();
    const int G = 1 << a.gk;
    const int64_t GL = (a.nleaf >> a.gk) + gi;
    const int32_t sG = a.nfirst[GL], nG = a.ncount[GL];
    for (int i = lane; i < 8 * kAcc; i += kWave) acc[i / kAcc][i % kAcc] = 0.0;
    __builtin_amdgcn_wave_barrier();
    int32_t lf[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) lf[i] = i < G ? a.nfirst[a.nleaf + gi * G + i] : 0x7fffffff;
    for (int s0 = 0; s0 < nG; s0 += kWave) {
        const int si = s0 + lane;
        if (si < nG) {
            const int32_t p = sG + si;
            const int la = leaf_slot(lf, p);
            const int64_t A = a.nleaf + gi * G + la;
            const int32_t o = a.pid[p];
            const double g[3] = {load_g<MIXED>(a.gx, o), load_g<MIXED>(a.gy, o), load_g<MIXED>(a.gz, o)};
            const double d[3] = {a.px[p] - a.ncom[3 * A], a.py[p] - a.ncom[3 * A + 1],
                                 a.pz[p] - a.ncom[3 * A + 2]};
            double *m = acc[la];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                atomicAdd(&m[u], g[u]);
#pragma unroll
                for (int l = 0; l < 3; ++l) atomicAdd(&m[3 + 3 * u + l], g[u] * d[l]);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const int l = k < 3 ? 0 : (k < 5 ? 1 : 2);
                    const int mm = k < 3 ? k : (k < 5 ? k - 2 : 2);
                    atomicAdd(&m[12 + 6 * u + k], g[u] * d[l] * d[mm]);
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (lane < G) {
        const double *m = acc[lane];
        rcbfar::SymMoments S;
        rcbfar::sym_moments(m, m + 3, m + 12, S);
        double *o = a.mom + (gi * G + lane) * kMom;
#pragma unroll
        for (int q = 0; q < 3; ++q) o[q] = S.S1[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) o[3 + q] = S.S2[q];
#pragma unroll
        for (int q = 0; q < 10; ++q) o[9 + q] = S.S3[q];
        o[19] = S.t1;
#pragma unroll
        for (int q = 0; q < 3; ++q) o[20 + q] = S.sg[q];
    }
}

// far field: per group, lanes = far entries; the group's leaves are taken in
// turn with their centre of mass and cotangent moments held uniform (scalar
// registers), so each lane sums its entry's node adjoint over the leaves that
// accepted it and issues one set of atomics. The sink-centre term is kept per
// lane and leaf in LDS and summed over the lanes once per group.
struct VjpFarShared {
    double cot[8][3][kWave / 2];   // per lane pair and leaf
    double mom[8][kMom];       // the group's leaves: symmetrised moments
    double com[8][3];          // and centres of mass
};

// AT: the type of the node-adjoint copies (FP64; FP32 in the mixed form, whose
// contract allows FP32 accumulation), summed in FP64 by k_adj_reduce
// MODE kFarAtomic: node adjoints added atomically to the copies. The
// deterministic form: kFarStore writes each entry's node adjoint (its sum over
// the group's leaves, in leaf order) to a.contrib, summed per node later;
// kFarCot computes the sink-centre sums only (k_vjp_far_node then computes
// the node adjoints itself).
constexpr int kFarAtomic = 0, kFarCot = 1, kFarStore = 2;
template <typename AT, int MODE>
__global__ __launch_bounds__(kBlock) void k_vjp_far(VjpArgs a, AT *__restrict__ adjc, AT *__restrict__ adjmc) {
    __shared__ VjpFarShared sh_all[kWaves];
    VjpFarShared &sh = sh_all[threadIdx.x / kWave];
    double(*cotp)[3][kWave / 2] = sh.cot;
    const int64_t gi = wave_index();
    if (gi >= a.ngroup) return;
    const int lane = lane_id();
    const int G = 1 << a.gk;
    for (int i = lane; i < 8 * 3 * (kWave / 2); i += kWave) (&cotp[0][0][0])[i] = 0.0;
    for (int i = lane; i < G * kMom; i += kWave) sh.mom[i / kMom][i % kMom] = a.mom[gi * G * kMom + i];
    if (lane < 3 * G) sh.com[lane / 3][lane % 3] = a.ncom[3 * (a.nleaf + gi * G) + lane];
    tile_sync();
    const int64_t f0 = a.gfar_beg[gi], f1 = a.gfar_end[gi];
    for (int64_t e0 = f0; e0 < f1; e0 += kWave) {
        const int64_t e = e0 + lane;
        const uint64_t ent = e < f1 ? a.gfar[e] : 0ull;
        const uint32_t emask = (uint32_t)(ent >> 32) & 0xffu;
        const int64_t B = (uint32_t)ent & 0x7fffffffu;
        double qq[6], cB[3], MB = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) qq[q] = 0.0;
        cB[0] = cB[1] = cB[2] = 0.0;
        if (emask) {
#pragma unroll
            for (int q = 0; q < 6; ++q) qq[q] = a.nQ[6 * B + q];
            cB[0] = a.ncom[3 * B];
            cB[1] = a.ncom[3 * B + 1];
            cB[2] = a.ncom[3 * B + 2];
            MB = a.nM[B];
        }
        double ad[kAdj];
#pragma unroll
        for (int q = 0; q < kAdj; ++q) ad[q] = 0.0;
        for (int i = 0; i < G; ++i) {
            const bool mine = (emask >> i) & 1u;
            if (ballot(mine) == 0) continue;
            const int64_t leaf = gi * G + i;
            const int64_t A = a.nleaf + leaf;
            // the leaf's moments and centre are the same on every lane
            const double *mo = sh.mom[i];
            rcbfar::SymMoments Sm;
#pragma unroll
            for (int q = 0; q < 3; ++q) Sm.S1[q] = uniform_f64(mo[q]);
#pragma unroll
            for (int q = 0; q < 6; ++q) Sm.S2[q] = uniform_f64(mo[3 + q]);
#pragma unroll
            for (int q = 0; q < 10; ++q) Sm.S3[q] = uniform_f64(mo[9 + q]);
            Sm.t1 = uniform_f64(mo[19]);
#pragma unroll
            for (int q = 0; q < 3; ++q) Sm.sg[q] = uniform_f64(mo[20 + q]);
            const double cA[3] = {uniform_f64(sh.com[i][0]), uniform_f64(sh.com[i][1]),
                                  uniform_f64(sh.com[i][2])};
            double ct[3] = {0.0, 0.0, 0.0};
            if (mine) {
                double rho[3], aM, aQ[6];
                rcbfar::far_pair_adjoint_sym(cA[0] - cB[0], cA[1] - cB[1], cA[2] - cB[2], MB, qq, Sm,
                                             rho, ct, aM, aQ);
                ad[0] += aM;
#pragma unroll
                for (int u = 0; u < 3; ++u) ad[1 + u] -= rho[u];
                const double tq = (aQ[0] + aQ[3] + aQ[5]) / 3.0;
                ad[4] += aQ[0] - tq;
                ad[5] += aQ[1];
                ad[6] += aQ[2];
                ad[7] += aQ[3] - tq;
                ad[8] += aQ[4];
            }
            // lanes 2j and 2j + 1 add their terms, the even lane keeps the sum
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const double t = ct[u] + swap_adjacent_lanes(ct[u]);
                if (!(lane & 1)) cotp[i][u][lane >> 1] += t;
            }
        }
        if (MODE == kFarStore && emask) {
            double *row = a.contrib + (a.cbase[gi] + (e - f0)) * kAdj;
#pragma unroll
            for (int q = 0; q < kAdj; ++q) row[q] = ad[q];
        }
        if (MODE == kFarAtomic && emask) {
            // each copy takes the blocks of one residue mod the number of
            // copies, i.e. of one XCD under round-robin dispatch (8 | copies)
            if (B < a.nmid) {
                AT *adj = adjmc + (int64_t)(blockIdx.x % kAdjMidCopies) * kAdj * a.nmid;
#pragma unroll
                for (int q = 0; q < kAdj; ++q)
                    __hip_atomic_fetch_add(adj + q * a.nmid + B, (AT)ad[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                AT *adj = adjc + (int64_t)(blockIdx.x % kAdjCopies) * kAdj * a.nlab;
#pragma unroll
                for (int q = 0; q < kAdj; ++q)
                    __hip_atomic_fetch_add(adj + q * a.nlab + B, (AT)ad[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    tile_sync();
    if (lane < 3 * G) {
        const int i = lane / 3, u = lane % 3;
        double v = 0.0;
        for (int l = 0; l < kWave / 2; ++l) v += cotp[i][u][l];
        a.leafc[(gi * G + i) * kLeafC + 19 + u] = v;
    }
}

// near field and the sink-side far terms: per group, the leaves in turn, lanes
// (sink slot, slice) over the leaf's particles as in the forward kernel
// (near_tile.h). Sources of the leaf's near cells are staged 64 at a time in
// LDS as T = ceil(nt / J) rows of J. Sink slot s visits the rows in the
// rotated order (s + t) mod T, so at each step the lanes of one slice touch
// different sources and the source-side terms are summed with LDS atomics
// without conflicts; each tile's sums then go out with one set of FP64
// atomics per source.
template <typename T>
struct VjpTile {
    T x[kWave], y[kWave], z[kWave], m[kWave], h[kWave];
    int32_t pb[kWave];
    double acc[4][kWave];
};
template <typename T>
struct VjpShared {
    EntryChunk ec;
    VjpTile<T> t;
};

// SRC = false (the deterministic form): sink-side terms only; the source-side
// terms are summed per source cell by k_vjp_near_src instead.
template <bool MIXED, bool SRC>
__global__ __launch_bounds__(kBlock) void k_vjp_near(VjpArgs a) {
    using T = typename std::conditional<MIXED, float, double>::type;
    __shared__ VjpShared<T> sh_all[kWaves];
    VjpShared<T> &sh = sh_all[threadIdx.x / kWave];
    const int64_t gi = wave_index();
    if (gi >= a.ngroup) return;
    const int lane = lane_id();
    const int G = 1 << a.gk;
    const int64_t GL = (a.nleaf >> a.gk) + gi;
    if (a.ncount[GL] == 0) return;
    const int64_t n0 = a.gnear_beg[gi], n1 = a.gnear_end[gi];
    for (int li = 0; li < G; ++li) {
        const int64_t A = a.nleaf + gi * G + li;
        const int32_t sA = a.nfirst[A], c = a.ncount[A];
        if (c == 0) continue;
        const LeafLanes L = leaf_lanes(c);
        const double cA[3] = {a.ncom[3 * A], a.ncom[3 * A + 1], a.ncom[3 * A + 2]};
        for (int g0 = 0; g0 < c; g0 += L.S) {
            const int si = g0 + L.sslot;
            const bool has_sink = L.sslot < L.S && si < c;
            const int32_t pa = sA + (has_sink ? si : 0);
            const int32_t oa = a.pid[pa];
            T ga[3] = {(T)0, (T)0, (T)0};
            double gd[3] = {0.0, 0.0, 0.0};
            if (has_sink) {
                gd[0] = load_g<MIXED>(a.gx, oa);
                gd[1] = load_g<MIXED>(a.gy, oa);
                gd[2] = load_g<MIXED>(a.gz, oa);
                ga[0] = (T)gd[0];
                ga[1] = (T)gd[1];
                ga[2] = (T)gd[2];
            }
            T sx, sy, sz, ha;
            if constexpr (MIXED) {   // leaf frame
                sx = a.fdx[pa];
                sy = a.fdy[pa];
                sz = a.fdz[pa];
                ha = a.fh[pa];
            } else {
                sx = a.px[pa];
                sy = a.py[pa];
                sz = a.pz[pa];
                ha = a.ph[pa];
            }
            double acc[3] = {0.0, 0.0, 0.0};
            for (int64_t e0 = n0; e0 < n1; e0 += kWave) {
                const int tot = load_entry_chunk(a.gnear, a.nfirst, a.ncount, e0, n1, 1u << li, sh.ec);
                for (int t = 0; t < tot; t += kWave) {
                    const int q = t + lane;
                    if (q < tot) {
                        const int k = entry_of(sh.ec, q);
                        const int32_t pb = sh.ec.fB[k] + (q - sh.ec.pos[k]);
                        if constexpr (MIXED) {
                            const int64_t B = sh.ec.label[k];
                            sh.t.x[lane] = (float)(a.ncom[3 * B] - cA[0]) + a.fdx[pb];
                            sh.t.y[lane] = (float)(a.ncom[3 * B + 1] - cA[1]) + a.fdy[pb];
                            sh.t.z[lane] = (float)(a.ncom[3 * B + 2] - cA[2]) + a.fdz[pb];
                            sh.t.m[lane] = a.fm[pb];
                            sh.t.h[lane] = a.fh[pb];
                        } else {
                            sh.t.x[lane] = a.px[pb];
                            sh.t.y[lane] = a.py[pb];
                            sh.t.z[lane] = a.pz[pb];
                            sh.t.m[lane] = a.pm[pb];
                            sh.t.h[lane] = a.ph[pb];
                        }
                        sh.t.pb[lane] = pb;
                    }
#pragma unroll
                    for (int cc = 0; cc < 4; ++cc) sh.t.acc[cc][lane] = 0.0;
                    tile_sync();
                    const int nt = tot - t < kWave ? tot - t : kWave;
                    const int rows = (nt + L.J - 1) / L.J;
                    // sink slot s starts at row s mod rows, so that the lanes of
                    // one step add into different sources
                    const int span = rows * L.J;
                    int j = (L.sslot % rows) * L.J + L.slice;
                    for (int st = 0; st < rows; ++st, j = j + L.J < span ? j + L.J : j + L.J - span) {
                        // the deterministic form leaves out the self pair, whose sink and
                        // source terms cancel exactly (v = 0) but would be computed in two
                        // kernels there
                        if (has_sink && j < nt && (SRC || sh.t.pb[j] != pa)) {
                            const T v[3] = {sx - sh.t.x[j], sy - sh.t.y[j], sz - sh.t.z[j]};
                            const T r2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
                            const T hsum = ha + sh.t.h[j];
                            const T ri = rsq_t(r2);
                            const T ri2 = ri * ri;
                            const T r3 = ri2 * ri;
                            const T r5 = r3 * ri2;
                            T F = r3, dFr = (T)-3 * r5;
                            if (!soft_outside<T>(r2, hsum)) soft_FdF<T>(r2, ri, r3, r5, hsum, F, dFr);
                            const T vg = v[0] * ga[0] + v[1] * ga[1] + v[2] * ga[2];
                            const T mb = sh.t.m[j];
#pragma unroll
                            for (int cc = 0; cc < 3; ++cc) {
                                const T Kg = mb * (F * ga[cc] + dFr * v[cc] * vg);
                                acc[cc] -= (double)Kg;
                                if (SRC) atomicAdd(&sh.t.acc[cc][j], (double)Kg);
                            }
                            if (SRC) atomicAdd(&sh.t.acc[3][j], (double)(-F * vg));
                        }
                    }
                    tile_sync();
                    if (SRC && lane < nt) {
                        const double s0 = sh.t.acc[0][lane], s1 = sh.t.acc[1][lane],
                                     s2 = sh.t.acc[2][lane], s3 = sh.t.acc[3][lane];
                        if (s0 != 0.0 || s1 != 0.0 || s2 != 0.0 || s3 != 0.0) {
                            const int32_t pb = sh.t.pb[lane];
                            if constexpr (MIXED) {
                                __hip_atomic_fetch_add(a.srcf + pb, (float)s0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                __hip_atomic_fetch_add(a.srcf + a.n + pb, (float)s1, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                                __hip_atomic_fetch_add(a.srcf + 2 * a.n + pb, (float)s2, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                                __hip_atomic_fetch_add(a.srcf + 3 * a.n + pb, (float)s3, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                            } else {
                                atomicAdd(a.src + pb, s0);
                                atomicAdd(a.src + a.n + pb, s1);
                                atomicAdd(a.src + 2 * a.n + pb, s2);
                                atomicAdd(a.src + 3 * a.n + pb, s3);
                            }
                        }
                    }
                    tile_sync();
                }
            }
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) acc[cc] = seg_sum(acc[cc], L.slice, L.J);
            if (has_sink && L.slice == 0) {
                const double *lc = a.leafc + (gi * G + li) * kLeafC;
                const double d[3] = {a.px[pa] - cA[0], a.py[pa] - cA[1], a.pz[pa] - cA[2]};
                const double ma = a.pm[pa];
                const double MA = a.nM[A];
                const double cot[3] = {lc[19], lc[20], lc[21]};
                double out[3];
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    double v = acc[l] + ma / MA * cot[l];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        v += gd[i] * lc[3 + jidx(i, l)];
#pragma unroll
                        for (int m = 0; m < 3; ++m) v += gd[i] * lc[9 + hidx(i, l, m)] * d[m];
                    }
                    out[l] = v;
                }
                a.sink[pa] = out[0];
                a.sink[a.n + pa] = out[1];
                a.sink[2 * a.n + pa] = out[2];
                a.sink[3 * a.n + pa] = (cot[0] * d[0] + cot[1] * d[1] + cot[2] * d[2]) / MA;
            }
        }
    }
}

// One node's adjoint (aM, aR, aQ) pushed to a particle at r of mass mb
// through M, COM and Q of the node.
__device__ __forceinline__ void push_node(const double (&ad)[kAdj], double MB, const double (&cB)[3],
                                          const double (&r)[3], double mb, double (&dr)[3],
                                          double &dmb) {
    const double Q[3][3] = {{ad[4], ad[5], ad[6]}, {ad[5], ad[7], ad[8]}, {ad[6], ad[8], -(ad[4] + ad[7])}};
    const double d[3] = {r[0] - cB[0], r[1] - cB[1], r[2] - cB[2]};
    double Qd[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) Qd[l] = Q[l][0] * d[0] + Q[l][1] * d[1] + Q[l][2] * d[2];
#pragma unroll
    for (int l = 0; l < 3; ++l) dr[l] += ad[1 + l] * mb / MB + mb * (6.0 * Qd[l]);
    dmb += ad[0] + (ad[1] * d[0] + ad[2] * d[1] + ad[3] * d[2]) / MB +
           3.0 * (d[0] * Qd[0] + d[1] * Qd[1] + d[2] * Qd[2]);
}

// node adjoints -> particles along each particle's ancestor chain; then the
// three parts are summed and written in caller order. One wave per group,
// lanes over the group's particles: the chain below the group node differs
// per lane, the chain from the group node up is the same for every lane.
template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_vjp_push(VjpArgs a, const double *__restrict__ adj,
                                                     const double *__restrict__ ncom,
                                                     const double *__restrict__ nM, void *dx, void *dy,
                                                     void *dz, void *dm) {
    const int64_t gi = wave_index();
    if (gi >= a.ngroup) return;
    const int G = 1 << a.gk;
    const int64_t GL = (a.nleaf >> a.gk) + gi;
    const int32_t sG = a.nfirst[GL], nG = a.ncount[GL];
    int32_t lf[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) lf[i] = i < G ? a.nfirst[a.nleaf + gi * G + i] : 0x7fffffff;
    for (int s0 = 0; s0 < nG; s0 += kWave) {
        const int si = s0 + lane_id();
        if (si >= nG) continue;
        const int64_t p = (int64_t)sG + si;
        const double r[3] = {a.px[p], a.py[p], a.pz[p]};
        const double mb = a.pm[p];
        double sr[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) sr[c] = MIXED ? (double)a.srcf[c * a.n + p] : a.src[c * a.n + p];
        double dr[3] = {a.sink[p] + sr[0], a.sink[a.n + p] + sr[1], a.sink[2 * a.n + p] + sr[2]};
        double dmb = a.sink[3 * a.n + p] + sr[3];
        const int64_t A = a.nleaf + gi * G + leaf_slot(lf, (int32_t)p);
        for (int64_t B = A; B > GL; B >>= 1) {
            double ad[kAdj];
#pragma unroll
            for (int q = 0; q < kAdj; ++q) ad[q] = adj[q * a.nlab + B];
            const double cB[3] = {ncom[3 * B], ncom[3 * B + 1], ncom[3 * B + 2]};
            push_node(ad, nM[B], cB, r, mb, dr, dmb);
        }
        for (int64_t B = GL; B >= 1; B >>= 1) {   // wave-uniform
            double ad[kAdj];
#pragma unroll
            for (int q = 0; q < kAdj; ++q) ad[q] = adj[q * a.nlab + B];
            const double cB[3] = {ncom[3 * B], ncom[3 * B + 1], ncom[3 * B + 2]};
            push_node(ad, nM[B], cB, r, mb, dr, dmb);
        }
        const int32_t o = a.pid[p];
        if constexpr (MIXED) {
            ((float *)dx)[o] = (float)dr[0];
            ((float *)dy)[o] = (float)dr[1];
            ((float *)dz)[o] = (float)dr[2];
            ((float *)dm)[o] = (float)dmb;
        } else {
            ((double *)dx)[o] = dr[0];
            ((double *)dy)[o] = dr[1];
            ((double *)dz)[o] = dr[2];
            ((double *)dm)[o] = dmb;
        }
    }
}

// node adjoints: the copies summed in FP64 in a fixed order into out (labels
// below nmid from the mid-level copies, the others from the kAdjCopies ones);
// out may be copy 0 of adjc (each thread reads its own element first)
template <typename A>
__global__ void k_adj_reduce(double *out, const A *adjc, const A *__restrict__ adjmc, int64_t nlab,
                             int64_t nmid) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= kAdj * nlab) return;
    const int64_t q = i / nlab, B = i % nlab;
    double v;
    if (B < nmid) {
        const int64_t len = kAdj * nmid, k = q * nmid + B;
        v = (double)adjmc[k];
        for (int c = 1; c < kAdjMidCopies; ++c) v += (double)adjmc[(int64_t)c * len + k];
    } else {
        const int64_t len = kAdj * nlab;
        v = (double)adjc[i];
        for (int c = 1; c < kAdjCopies; ++c) v += (double)adjc[(int64_t)c * len + i];
    }
    out[i] = v;
}

// ---------------------------------------------------------------------------
// Deterministic form: no atomics. The per-group lists are turned into lists
// of the groups that hold each node (far) or each lowest-level cell (near),
// ascending by group (k_sort.hip), and every sum runs in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kDetChunk = 512;   // far entries per wave of k_vjp_far_node

// cotangent moments without atomics: the group's leaves in turn, 64 particles
// at a time, each of the 30 sums a canonical wave sum (wave_sum)
template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_vjp_moments_det(VjpArgs a) {
    const int64_t gi = wave_index();
    if (gi >= a.ngroup) return;
    const int lane = lane_id();
    const int G = 1 << a.gk;
    for (int li = 0; li < G; ++li) {
        const int64_t A = a.nleaf + gi * G + li;
        const int32_t sA = a.nfirst[A], c = a.ncount[A];
        double m[kAcc];
#pragma unroll
        for (int q = 0; q < kAcc; ++q) m[q] = 0.0;
        for (int s0 = 0; s0 < c; s0 += kWave) {
            const int si = s0 + lane;
            double g[3] = {0.0, 0.0, 0.0}, d[3] = {0.0, 0.0, 0.0};
            if (si < c) {
                const int32_t p = sA + si;
                const int32_t o = a.pid[p];
                g[0] = load_g<MIXED>(a.gx, o);
                g[1] = load_g<MIXED>(a.gy, o);
                g[2] = load_g<MIXED>(a.gz, o);
                d[0] = a.px[p] - a.ncom[3 * A];
                d[1] = a.py[p] - a.ncom[3 * A + 1];
                d[2] = a.pz[p] - a.ncom[3 * A + 2];
            }
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                m[u] += wave_sum(g[u]);
#pragma unroll
                for (int l = 0; l < 3; ++l) m[3 + 3 * u + l] += wave_sum(g[u] * d[l]);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    const int l = k < 3 ? 0 : (k < 5 ? 1 : 2);
                    const int mm = k < 3 ? k : (k < 5 ? k - 2 : 2);
                    m[12 + 6 * u + k] += wave_sum(g[u] * d[l] * d[mm]);
                }
            }
        }
        if (lane == 0) {
            rcbfar::SymMoments S;
            rcbfar::sym_moments(m, m + 3, m + 12, S);
            double *o = a.mom + (gi * G + li) * kMom;
#pragma unroll
            for (int q = 0; q < 3; ++q) o[q] = S.S1[q];
#pragma unroll
            for (int q = 0; q < 6; ++q) o[3 + q] = S.S2[q];
#pragma unroll
            for (int q = 0; q < 10; ++q) o[9 + q] = S.S3[q];
            o[19] = S.t1;
#pragma unroll
            for (int q = 0; q < 3; ++q) o[20 + q] = S.sg[q];
        }
    }
}

// the cotangents in tree order (contiguous per cell for the source-side pass)
template <bool MIXED>
__global__ void k_det_gather_g(VjpArgs a) {
    using T = typename std::conditional<MIXED, float, double>::type;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int32_t o = a.pid[p];
    T *gt = (T *)a.gtree;
    gt[p] = (T)load_g<MIXED>(a.gx, o);
    gt[a.n + p] = (T)load_g<MIXED>(a.gy, o);
    gt[2 * a.n + p] = (T)load_g<MIXED>(a.gz, o);
}

// entries per group
__global__ void k_det_count(const int64_t *__restrict__ beg, const int64_t *__restrict__ end,
                            int64_t ngroup, int64_t *__restrict__ cnt) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g < ngroup) cnt[g] = end[g] - beg[g];
}

// item = label << 32 | group << 8 | mask (bits 32-39 of the list entry: the far
// mask, or the near mask), or with compact = true label << 32 | the item's own
// index; written in group order at the group's offset
__global__ __launch_bounds__(kBlock) void k_det_items(const int64_t *__restrict__ beg,
                                                      const int64_t *__restrict__ end,
                                                      const uint64_t *__restrict__ list, int64_t ngroup,
                                                      const int64_t *__restrict__ base, bool compact,
                                                      uint64_t *__restrict__ items) {
    const int64_t gi = wave_index();
    if (gi >= ngroup) return;
    const int64_t e0 = beg[gi], ne = end[gi] - e0, o = base[gi];
    for (int64_t j = lane_id(); j < ne; j += kWave) {
        const uint64_t ent = list[e0 + j];
        const uint64_t lab = (uint32_t)ent & 0x7fffffffu;
        const uint64_t mask = (ent >> 32) & 0xffu;
        items[o + j] = (lab << 32) | (compact ? (uint64_t)(o + j) : (((uint64_t)gi << 8) | mask));
    }
}

// each label's range [lb, le) in the sorted items (lb = le = 0 if absent)
__global__ void k_det_bounds(const uint64_t *__restrict__ it, int64_t n, int64_t *__restrict__ lb,
                             int64_t *__restrict__ le) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t B = (uint32_t)(it[i] >> 32);
    if (i == 0 || (uint32_t)(it[i - 1] >> 32) != B) lb[B] = i;
    if (i == n - 1 || (uint32_t)(it[i + 1] >> 32) != B) le[B] = i + 1;
}

// chunks of kDetChunk entries per label
__global__ void k_det_nchunk(const int64_t *__restrict__ lb, const int64_t *__restrict__ le,
                             int64_t nlab, int64_t *__restrict__ nc) {
    const int64_t B = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (B < nlab) nc[B] = (le[B] - lb[B] + kDetChunk - 1) / kDetChunk;
}

__global__ void k_det_owner(const int64_t *__restrict__ cb, int64_t nlab, int32_t *__restrict__ owner) {
    const int64_t B = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (B >= nlab) return;
    for (int64_t c = cb[B]; c < cb[B + 1]; ++c) owner[c] = (int32_t)B;
}

// node adjoints, one wave per chunk of one node's entries: lanes over the
// entries, each taking the entry's adjoint stored by k_vjp_far (STORED) or
// summing it over the leaves of the entry's far mask in order; the chunk's
// sum is a canonical wave sum
template <bool STORED>
__global__ __launch_bounds__(kBlock) void k_vjp_far_node(VjpArgs a, const uint64_t *__restrict__ items,
                                                         const int64_t *__restrict__ lb,
                                                         const int64_t *__restrict__ le,
                                                         const int64_t *__restrict__ cb,
                                                         const int32_t *__restrict__ owner, int64_t nchunk,
                                                         double *__restrict__ part) {
    const int64_t c = wave_index();
    if (c >= nchunk) return;
    const int lane = lane_id();
    const int G = 1 << a.gk;
    const int64_t B = __builtin_amdgcn_readfirstlane(owner[c]);
    const int64_t e_beg = lb[B] + (c - cb[B]) * kDetChunk;
    const int64_t e_end = e_beg + kDetChunk < le[B] ? e_beg + kDetChunk : le[B];
    double qq[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) qq[q] = a.nQ[6 * B + q];
    const double cB[3] = {a.ncom[3 * B], a.ncom[3 * B + 1], a.ncom[3 * B + 2]};
    const double MB = a.nM[B];
    double ad[kAdj];
#pragma unroll
    for (int q = 0; q < kAdj; ++q) ad[q] = 0.0;
    for (int64_t e0 = e_beg; e0 < e_end; e0 += kWave) {
        const int64_t e = e0 + lane;
        if (e >= e_end) continue;
        const uint64_t it = items[e];
        if constexpr (STORED) {
            const double *row = a.contrib + (int64_t)(uint32_t)it * kAdj;
#pragma unroll
            for (int q = 0; q < kAdj; ++q) ad[q] += row[q];
            continue;
        }
        const int64_t gi = (uint32_t)it >> 8;
        const uint32_t mask = (uint32_t)it & 0xffu;
        for (int i = 0; i < G; ++i) {
            if (!((mask >> i) & 1u)) continue;
            const int64_t leaf = gi * G + i;
            const int64_t A = a.nleaf + leaf;
            const double *mo = a.mom + leaf * kMom;
            rcbfar::SymMoments Sm;
#pragma unroll
            for (int q = 0; q < 3; ++q) Sm.S1[q] = mo[q];
#pragma unroll
            for (int q = 0; q < 6; ++q) Sm.S2[q] = mo[3 + q];
#pragma unroll
            for (int q = 0; q < 10; ++q) Sm.S3[q] = mo[9 + q];
            Sm.t1 = mo[19];
#pragma unroll
            for (int q = 0; q < 3; ++q) Sm.sg[q] = mo[20 + q];
            double rho[3], ct[3] = {0.0, 0.0, 0.0}, aM, aQ[6];
            rcbfar::far_pair_adjoint_sym(a.ncom[3 * A] - cB[0], a.ncom[3 * A + 1] - cB[1],
                                         a.ncom[3 * A + 2] - cB[2], MB, qq, Sm, rho, ct, aM, aQ);
            ad[0] += aM;
#pragma unroll
            for (int u = 0; u < 3; ++u) ad[1 + u] -= rho[u];
            const double tq = (aQ[0] + aQ[3] + aQ[5]) / 3.0;
            ad[4] += aQ[0] - tq;
            ad[5] += aQ[1];
            ad[6] += aQ[2];
            ad[7] += aQ[3] - tq;
            ad[8] += aQ[4];
        }
    }
#pragma unroll
    for (int q = 0; q < kAdj; ++q) {
        const double v = wave_sum(ad[q]);
        if (lane == 0) part[c * kAdj + q] = v;
    }
}

// adj[q * nlab + B] = sum of the node's chunk sums in chunk order (0 if none)
__global__ void k_det_adj_sum(const double *__restrict__ part, const int64_t *__restrict__ cb, int64_t nlab,
                              double *__restrict__ adj) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= kAdj * nlab) return;
    const int64_t q = i / nlab, B = i % nlab;
    double v = 0.0;
    for (int64_t c = cb[B]; c < cb[B + 1]; ++c) v += part[c * kAdj + q];
    adj[i] = v;
}

// source-side near terms, one wave per lowest-level cell B: lanes (source
// slot, slice) over B's particles as in leaf_lanes. The sink cells A whose
// near list holds B (the groups ascending, then the cells of each group's
// near mask) are taken 8 groups (64 cells) at a time; an exclusive scan of
// their sizes gives each cell's first sink, and the sinks are staged 64 at a
// time in LDS (near_tile.h's chunk layout), each slice taking every J-th.
// In the mixed form a staged sink carries the FP32 shift from its cell's
// centre of mass to B's, so the pair arithmetic is exactly that of
// k_vjp_near. The slices' sums are combined by seg_sum and written (no
// atomics: B owns its particles).
template <typename T>
struct SinkTile {
    T x[kWave], y[kWave], z[kWave], h[kWave], g[3][kWave];
    float sx[kWave], sy[kWave], sz[kWave];   // mixed form: (float)(com_B - com_A)
    int32_t pa[kWave];                       // tree position (the self pair is left out)
};
template <typename T>
struct SrcShared {
    EntryChunk ec;
    SinkTile<T> t;
};

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_vjp_near_src(VjpArgs a, const uint64_t *__restrict__ items,
                                                         const int64_t *__restrict__ lb,
                                                         const int64_t *__restrict__ le) {
    using T = typename std::conditional<MIXED, float, double>::type;
    __shared__ SrcShared<T> sh_all[kWaves];
    SrcShared<T> &sh = sh_all[threadIdx.x / kWave];
    const int64_t bl = wave_index();
    if (bl >= a.nleaf) return;
    const int lane = lane_id();
    const int G = 1 << a.gk;
    const int64_t B = a.nleaf + bl;
    const int32_t sB = a.nfirst[B], c = a.ncount[B];
    if (c == 0) return;
    const LeafLanes L = leaf_lanes(c);
    const int64_t e_beg = lb[B], e_end = le[B];
    const double cB[3] = {a.ncom[3 * B], a.ncom[3 * B + 1], a.ncom[3 * B + 2]};
    for (int g0 = 0; g0 < c; g0 += L.S) {
        const int si = g0 + L.sslot;
        const bool has_src = L.sslot < L.S && si < c;
        const int32_t pb = sB + (has_src ? si : 0);
        T mb, hb, bx, by, bz;   // bx..: FP64 position, or the FP32 offset from com_B
        if constexpr (MIXED) {
            mb = a.fm[pb];
            hb = a.fh[pb];
            bx = a.fdx[pb];
            by = a.fdy[pb];
            bz = a.fdz[pb];
        } else {
            mb = a.pm[pb];
            hb = a.ph[pb];
            bx = a.px[pb];
            by = a.py[pb];
            bz = a.pz[pb];
        }
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t e0 = e_beg; e0 < e_end; e0 += kWave / 8) {
            // lane = (group entry e0 + lane / 8, cell lane % 8 of its mask)
            const int64_t e = e0 + (lane >> 3);
            const int li = lane & 7;
            int32_t fA = 0, cA = 0, A = 0;
            if (e < e_end && li < G) {
                const uint64_t it = items[e];
                if (((uint32_t)it >> li) & 1u) {
                    A = (int32_t)(a.nleaf + (int64_t)((uint32_t)it >> 8) * G + li);
                    fA = a.nfirst[A];
                    cA = a.ncount[A];
                }
            }
            const int p = wave_excl_scan(cA);
            sh.ec.fB[lane] = fA;
            sh.ec.pos[lane] = p;
            sh.ec.label[lane] = A;
            if (lane == kWave - 1) sh.ec.pos[kWave] = p + cA;
            tile_sync();
            const int tot = __builtin_amdgcn_readfirstlane(sh.ec.pos[kWave]);
            for (int t = 0; t < tot; t += kWave) {
                const int q = t + lane;
                if (q < tot) {
                    const int k = entry_of(sh.ec, q);
                    const int32_t pa = sh.ec.fB[k] + (q - sh.ec.pos[k]);
                    sh.t.pa[lane] = pa;
                    if constexpr (MIXED) {
                        const int64_t Ak = sh.ec.label[k];
                        sh.t.x[lane] = a.fdx[pa];
                        sh.t.y[lane] = a.fdy[pa];
                        sh.t.z[lane] = a.fdz[pa];
                        sh.t.h[lane] = a.fh[pa];
                        sh.t.sx[lane] = (float)(cB[0] - a.ncom[3 * Ak]);
                        sh.t.sy[lane] = (float)(cB[1] - a.ncom[3 * Ak + 1]);
                        sh.t.sz[lane] = (float)(cB[2] - a.ncom[3 * Ak + 2]);
                    } else {
                        sh.t.x[lane] = a.px[pa];
                        sh.t.y[lane] = a.py[pa];
                        sh.t.z[lane] = a.pz[pa];
                        sh.t.h[lane] = a.ph[pa];
                    }
                    const T *gt = (const T *)a.gtree;
                    sh.t.g[0][lane] = gt[pa];
                    sh.t.g[1][lane] = gt[a.n + pa];
                    sh.t.g[2][lane] = gt[2 * a.n + pa];
                }
                tile_sync();
                const int nt = tot - t < kWave ? tot - t : kWave;
                if (has_src) {
                    for (int j = L.slice; j < nt; j += L.J) {
                        if (sh.t.pa[j] == pb) continue;   // the self pair: v = 0, no term
                        T v[3];
                        if constexpr (MIXED) {   // the source in the sink cell's frame, as in k_vjp_near
                            v[0] = sh.t.x[j] - (sh.t.sx[j] + bx);
                            v[1] = sh.t.y[j] - (sh.t.sy[j] + by);
                            v[2] = sh.t.z[j] - (sh.t.sz[j] + bz);
                        } else {
                            v[0] = sh.t.x[j] - bx;
                            v[1] = sh.t.y[j] - by;
                            v[2] = sh.t.z[j] - bz;
                        }
                        const T r2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
                        const T hsum = sh.t.h[j] + hb;
                        const T ri = rsq_t(r2);
                        const T ri2 = ri * ri;
                        const T r3 = ri2 * ri;
                        const T r5 = r3 * ri2;
                        T F = r3, dFr = (T)-3 * r5;
                        if (!soft_outside<T>(r2, hsum)) soft_FdF<T>(r2, ri, r3, r5, hsum, F, dFr);
                        const T ga[3] = {sh.t.g[0][j], sh.t.g[1][j], sh.t.g[2][j]};
                        const T vg = v[0] * ga[0] + v[1] * ga[1] + v[2] * ga[2];
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) acc[cc] += (double)(mb * (F * ga[cc] + dFr * v[cc] * vg));
                        acc[3] += (double)(-F * vg);
                    }
                }
                tile_sync();
            }
        }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) acc[cc] = seg_sum(acc[cc], L.slice, L.J);
        if (has_src && L.slice == 0) {
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                if constexpr (MIXED) a.srcf[cc * a.n + pb] = (float)acc[cc];
                else a.src[cc * a.n + pb] = acc[cc];
            }
        }
    }
}

// per-node lists of one list kind: the items sorted by label and each
// label's range in them
struct DetLists {
    int64_t *base = nullptr;   // each group's first item (exclusive scan of the list sizes)
    int64_t total = 0;
    uint64_t *items = nullptr;
    int64_t *lb = nullptr, *le = nullptr;
};

rcb_status det_count(rcb_tree *t, const int64_t *beg, const int64_t *end, Scratch &tmp, hipStream_t s,
                     DetLists &out) {
    const int64_t NG = t->ngroup;
    int64_t *cnt = (int64_t *)dalloc(t, sizeof(int64_t) * (NG + 1), s, tmp);
    if (!cnt) return RCB_ENOMEM;
    k_det_count<<<(unsigned)((NG + 255) / 256), 256, 0, s>>>(beg, end, NG, cnt);
    RCB_LAUNCH_CHECK("k_det_count");
    rcb_status st = scan_i64(t, cnt, cnt, NG, s);
    if (st != RCB_OK) return st;
    HostRead rd{cnt + NG, &out.total, (int)sizeof(int64_t)};
    st = read_small(s, &rd, 1, "deterministic VJP: list size");
    if (st != RCB_OK) return st;
    out.base = cnt;
    return RCB_OK;
}

rcb_status det_sort(rcb_tree *t, const int64_t *beg, const int64_t *end, const uint64_t *list, bool compact,
                    Scratch &tmp, hipStream_t s, DetLists &out) {
    const int64_t NG = t->ngroup, total = out.total;
    const int64_t cap = total > 0 ? total : 1;
    uint64_t *ia = (uint64_t *)dalloc(t, sizeof(uint64_t) * cap, s, tmp);
    uint64_t *ib = (uint64_t *)dalloc(t, sizeof(uint64_t) * cap, s, tmp);
    int64_t *lbe = (int64_t *)dalloc(t, sizeof(int64_t) * 2 * t->nlab, s, tmp);
    if (!ia || !ib || !lbe) return RCB_ENOMEM;
    k_det_items<<<(unsigned)((NG + kWaves - 1) / kWaves), kBlock, 0, s>>>(beg, end, list, NG, out.base, compact,
                                                                          ia);
    RCB_LAUNCH_CHECK("k_det_items");
    rcb_status st = sort_by_label(t, ia, ib, total, t->k + 1, s, &out.items);
    if (st != RCB_OK) return st;
    RCB_ZERO(lbe, sizeof(int64_t) * 2 * t->nlab, s);
    out.lb = lbe;
    out.le = lbe + t->nlab;
    if (total > 0) {
        k_det_bounds<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(out.items, total, out.lb, out.le);
        RCB_LAUNCH_CHECK("k_det_bounds");
    }
    return RCB_OK;
}

// The deterministic form after the cotangent moments and far coefficients:
// sink-centre sums and node adjoints (FP64, q * nlab + B) of the far field,
// and the source-side near terms. Each far entry's node adjoint is stored by
// k_vjp_far and summed per node (72 B per entry); if that array cannot be had
// (or RCB_VJP_DET_RECOMPUTE is set) k_vjp_far_node recomputes it per node.
rcb_status vjp_det(rcb_tree *t, VjpArgs a, double *adj, bool mixed, Scratch &tmp, hipStream_t s) {
    const int64_t nlab = t->nlab;
    const unsigned gridg = (unsigned)((t->ngroup + kWaves - 1) / kWaves);
    DetLists far, near;
    rcb_status st = det_count(t, t->gfar_beg, t->gfar_end, tmp, s, far);
    if (st != RCB_OK) return st;
    double *contrib = nullptr;
    if (far.total > 0 && far.total < (int64_t(1) << 32) && getenv("RCB_VJP_DET_RECOMPUTE") == nullptr)
        contrib = (double *)dalloc(t, sizeof(double) * kAdj * far.total, s, tmp);
    a.contrib = contrib;
    a.cbase = far.base;
    if (contrib) k_vjp_far<double, kFarStore><<<gridg, kBlock, 0, s>>>(a, nullptr, nullptr);
    else k_vjp_far<double, kFarCot><<<gridg, kBlock, 0, s>>>(a, nullptr, nullptr);
    RCB_LAUNCH_CHECK("k_vjp_far");
    st = det_sort(t, t->gfar_beg, t->gfar_end, t->gfar, contrib != nullptr, tmp, s, far);
    if (st != RCB_OK) return st;
    int64_t *cb = (int64_t *)dalloc(t, sizeof(int64_t) * (nlab + 1), s, tmp);
    if (!cb) return RCB_ENOMEM;
    const unsigned gl = (unsigned)((nlab + 255) / 256);
    k_det_nchunk<<<gl, 256, 0, s>>>(far.lb, far.le, nlab, cb);
    RCB_LAUNCH_CHECK("k_det_nchunk");
    st = scan_i64(t, cb, cb, nlab, s);
    if (st != RCB_OK) return st;
    int64_t nchunk = 0;
    HostRead rd{cb + nlab, &nchunk, (int)sizeof(int64_t)};
    st = read_small(s, &rd, 1, "deterministic VJP: chunk count");
    if (st != RCB_OK) return st;
    const int64_t ncap = nchunk > 0 ? nchunk : 1;
    int32_t *owner = (int32_t *)dalloc(t, sizeof(int32_t) * ncap, s, tmp);
    double *part = (double *)dalloc(t, sizeof(double) * kAdj * ncap, s, tmp);
    if (!owner || !part) return RCB_ENOMEM;
    if (nchunk > 0) {
        k_det_owner<<<gl, 256, 0, s>>>(cb, nlab, owner);
        RCB_LAUNCH_CHECK("k_det_owner");
        const unsigned gc = (unsigned)((nchunk + kWaves - 1) / kWaves);
        if (contrib) k_vjp_far_node<true><<<gc, kBlock, 0, s>>>(a, far.items, far.lb, far.le, cb, owner, nchunk, part);
        else k_vjp_far_node<false><<<gc, kBlock, 0, s>>>(a, far.items, far.lb, far.le, cb, owner, nchunk, part);
        RCB_LAUNCH_CHECK("k_vjp_far_node");
    }
    k_det_adj_sum<<<(unsigned)((kAdj * nlab + 255) / 256), 256, 0, s>>>(part, cb, nlab, adj);
    RCB_LAUNCH_CHECK("k_det_adj_sum");
    st = det_count(t, t->gnear_beg, t->gnear_end, tmp, s, near);
    if (st != RCB_OK) return st;
    st = det_sort(t, t->gnear_beg, t->gnear_end, t->gnear, false, tmp, s, near);
    if (st != RCB_OK) return st;
    a.gtree = dalloc(t, (mixed ? sizeof(float) : sizeof(double)) * 3 * t->n, s, tmp);
    if (!a.gtree) return RCB_ENOMEM;
    const unsigned gp = (unsigned)((t->n + 255) / 256);
    if (mixed) k_det_gather_g<true><<<gp, 256, 0, s>>>(a);
    else k_det_gather_g<false><<<gp, 256, 0, s>>>(a);
    RCB_LAUNCH_CHECK("k_det_gather_g");
    const unsigned gn = (unsigned)((t->nleaf + kWaves - 1) / kWaves);
    if (mixed) k_vjp_near_src<true><<<gn, kBlock, 0, s>>>(a, near.items, near.lb, near.le);
    else k_vjp_near_src<false><<<gn, kBlock, 0, s>>>(a, near.items, near.lb, near.le);
    RCB_LAUNCH_CHECK("k_vjp_near_src");
    return RCB_OK;
}

}  // namespace

rcb_status gravity_vjp(rcb_tree *t, const void *gx, const void *gy, const void *gz, void *dx,
                       void *dy, void *dz, void *dm, hipStream_t s) {
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    Scratch tmp(t, s);
    const int64_t n = t->n;
    double *sink = (double *)dalloc(t, sizeof(double) * 4 * n, s, tmp);
    const bool mixed = t->p.precision == RCB_MIXED;
    void *srcv = dalloc(t, (mixed ? sizeof(float) : sizeof(double)) * 4 * n, s, tmp);
    const bool det = t->p.deterministic != 0;
    if (det && t->ngroup > (int64_t(1) << 24)) {
        set_error("rcb_gravity_vjp: the deterministic form takes at most 2^24 groups of 8 cells (k <= 27)");
        return RCB_ECAPACITY;
    }
    const int64_t nmid = std::min<int64_t>(t->nlab, int64_t(1) << kMidLevel);
    // node-adjoint copies: FP64 (summed into copy 0 of adj) or, in the mixed
    // form, FP32 (summed into adj); the deterministic form writes adj alone
    const size_t adj_n = det ? 0 : (size_t)kAdjCopies * kAdj * t->nlab;
    const size_t adjm_n = det ? 0 : (size_t)kAdjMidCopies * kAdj * nmid;
    double *adj = (double *)dalloc(t, sizeof(double) * (mixed || det ? (size_t)kAdj * t->nlab : adj_n), s, tmp);
    void *adjc = det ? (void *)adj : mixed ? dalloc(t, sizeof(float) * adj_n, s, tmp) : (void *)adj;
    void *adjmc = det ? (void *)adj : dalloc(t, (mixed ? sizeof(float) : sizeof(double)) * adjm_n, s, tmp);
    double *mom = (double *)dalloc(t, sizeof(double) * kMom * t->nleaf, s, tmp);
    if (!t->farc) {
        t->farc = (double *)dalloc(t, sizeof(double) * kLeafC * t->nleaf, s, t->list_allocs);
        t->farc_valid = false;
    }
    double *leafc = t->farc;   // 19 far coefficients + the leaf's cotangent sum per leaf
    if (!sink || !srcv || !adj || !adjc || !adjmc || !mom || !leafc) return RCB_ENOMEM;
    RCB_ZERO(srcv, (mixed ? sizeof(float) : sizeof(double)) * 4 * n, s);
    if (!det) {
        RCB_ZERO(adjc, (mixed ? sizeof(float) : sizeof(double)) * adj_n, s);
        RCB_ZERO(adjmc, (mixed ? sizeof(float) : sizeof(double)) * adjm_n, s);
    }
    VjpArgs a{t->nleaf, t->gk, t->ngroup, t->nfirst, t->ncount, t->ncom, t->nM, t->nQ,
              t->gnear_beg, t->gnear_end, t->gfar_beg, t->gfar_end, t->gnear, t->gfar, t->px, t->py, t->pz, t->pm, t->ph,
              t->fdx, t->fdy, t->fdz, t->fm, t->fh, t->pid, gx, gy, gz, mom, leafc, sink, mixed ? nullptr : (double *)srcv,
              mixed ? (float *)srcv : nullptr, adj, nullptr, nmid, n, t->nlab};
    const unsigned gridg = (unsigned)((t->ngroup + kWaves - 1) / kWaves);
    if (det && mixed) k_vjp_moments_det<true><<<gridg, kBlock, 0, s>>>(a);
    else if (det) k_vjp_moments_det<false><<<gridg, kBlock, 0, s>>>(a);
    else if (mixed) k_vjp_moments<true><<<gridg, kBlock, 0, s>>>(a);
    else k_vjp_moments<false><<<gridg, kBlock, 0, s>>>(a);
    RCB_LAUNCH_CHECK("k_vjp_moments");
    if (!t->farc_valid) {   // else kept by the last rcb_gravity on these moments
        st = far_coefficients(t, leafc, kLeafC, s);
        if (st != RCB_OK) return st;
        t->farc_valid = true;
    }

    const int64_t alen = kAdj * t->nlab;
    const unsigned gridr = (unsigned)((alen + 255) / 256);
    if (det) {
        // far field, then node adjoints and source-side terms from the
        // per-node lists
        st = vjp_det(t, a, adj, mixed, tmp, s);
        if (st != RCB_OK) return st;
        if (mixed) k_vjp_near<true, false><<<gridg, kBlock, 0, s>>>(a);
        else k_vjp_near<false, false><<<gridg, kBlock, 0, s>>>(a);
        RCB_LAUNCH_CHECK("k_vjp_near");
    } else {
        if (mixed) {
            k_vjp_far<float, kFarAtomic><<<gridg, kBlock, 0, s>>>(a, (float *)adjc, (float *)adjmc);
            RCB_LAUNCH_CHECK("k_vjp_far");
            k_adj_reduce<float><<<gridr, 256, 0, s>>>(adj, (const float *)adjc, (const float *)adjmc, t->nlab,
                                                      nmid);
        } else {
            k_vjp_far<double, kFarAtomic><<<gridg, kBlock, 0, s>>>(a, (double *)adjc, (double *)adjmc);
            RCB_LAUNCH_CHECK("k_vjp_far");
            k_adj_reduce<double><<<gridr, 256, 0, s>>>(adj, (const double *)adjc, (const double *)adjmc, t->nlab,
                                                       nmid);
        }
        RCB_LAUNCH_CHECK("k_adj_reduce");
        if (mixed) k_vjp_near<true, true><<<gridg, kBlock, 0, s>>>(a);
        else k_vjp_near<false, true><<<gridg, kBlock, 0, s>>>(a);
        RCB_LAUNCH_CHECK("k_vjp_near");
    }
    if (mixed) k_vjp_push<true><<<gridg, kBlock, 0, s>>>(a, adj, t->ncom, t->nM, dx, dy, dz, dm);
    else k_vjp_push<false><<<gridg, kBlock, 0, s>>>(a, adj, t->ncom, t->nM, dx, dy, dz, dm);
    RCB_LAUNCH_CHECK("k_vjp_push");
    return RCB_OK;
}

}  // namespace rcb
