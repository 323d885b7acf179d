// k_grav.hip -- gravitational accelerations from the interaction lists
// (Sec. 2.4: near field by kernel-softened direct summation, far field by
// quadrupole cell-cell interaction, Taylor-expanded about the sink leaf's
// centre of mass).
//
// One wave per sink leaf A:
//  far:  lanes run over far(A); each evaluates the field of node B at
//        R = com_A - com_B in FP64 -- f_i, J_il, H_ilm of the potential
//        Phi = -M/r - Q_jk x_j x_k / (2 r^5) (Eq. 5) -- and the 19 unique
//        coefficients are summed over the wave.
//  near: lanes are (sink slot, slice) as in the neighbour search; slice j of
//        sink a runs over particles first_B + t J + j of every near cell B:
//        a_a -= m_b F(r, h_ab) (r_a - r_b), F = S(q)/r (Sec. 2.4.3).
//  L2P:  a_a += f + J d + H[d, d] / 2,  d = r_a - com_A  (Eq. 6).
// FP64 form: everything in FP64. Mixed form: particles as FP32 offsets from
// their leaf's centre of mass; per (A, B) the FP64 offset com_A - com_B is
// rounded to FP32 once; P2P, accumulation and L2P in FP32; M2L in FP64.
//
// The far-field closed forms are in far_math.h.
#include "far_math.h"
#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;

using rcbfar::hidx;
using rcbfar::jidx;
using rcbfar::m2l_accumulate;

// F = S(q)/r of the cubic-spline softening; FP64
__device__ __forceinline__ double soft_F(double r2, double hab) {
    const double rinv = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
    const double r = r2 * rinv;
    const double hinv = 1.0 / hab;
    const double q = r * hinv;
    const double h3 = hinv * hinv * hinv;
    const double r3 = rinv * rinv * rinv;
    const double in = h3 * (4.0 / 3.0 + q * q * (-6.0 / 5.0 + 0.5 * q));
    const double mid = h3 * (8.0 / 3.0 + q * (-3.0 + q * (6.0 / 5.0 - q * (1.0 / 6.0)))) -
                       r3 * (1.0 / 15.0);
    return q < 1.0 ? in : (q < 2.0 ? mid : r3);
}

__device__ __forceinline__ float soft_Ff(float r2, float hab) {
    const float rinv = r2 > 0.0f ? __frsqrt_rn(r2) : 0.0f;
    const float r = r2 * rinv;
    const float hinv = __frcp_rn(hab);
    const float q = r * hinv;
    const float h3 = hinv * hinv * hinv;
    const float r3 = rinv * rinv * rinv;
    const float in = h3 * (4.0f / 3.0f + q * q * (-1.2f + 0.5f * q));
    const float mid = h3 * (8.0f / 3.0f + q * (-3.0f + q * (1.2f - q * (1.0f / 6.0f)))) -
                      r3 * (1.0f / 15.0f);
    return q < 1.0f ? in : (q < 2.0f ? mid : r3);
}

struct GravArgs {
    int64_t nleaf;
    const int32_t *nfirst, *ncount;
    const double *ncom, *nM, *nQ;
    const int64_t *near_off, *far_off;
    const int32_t *near_list, *far_list;
    const double *px, *py, *pz, *pm, *ph;
    const float *fdx, *fdy, *fdz, *fm, *fh;
    const int32_t *pid;
    void *ax, *ay, *az;
};

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_gravity(GravArgs g) {
    const int64_t li = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kWave;
    if (li >= g.nleaf) return;
    const int lane = lane_id();
    const int64_t A = g.nleaf + li;
    const int32_t sA = g.nfirst[A], nA = g.ncount[A];
    if (nA == 0) return;
    const double cAx = g.ncom[3 * A], cAy = g.ncom[3 * A + 1], cAz = g.ncom[3 * A + 2];

    // far field: 19 FP64 coefficients at com_A
    double c[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) c[q] = 0.0;
    const int64_t f0 = g.far_off[li], f1 = g.far_off[li + 1];
    for (int64_t e = f0 + lane; e < f1; e += kWave) {
        const int64_t B = g.far_list[e];
        double qq[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) qq[q] = g.nQ[6 * B + q];
        m2l_accumulate(cAx - g.ncom[3 * B], cAy - g.ncom[3 * B + 1], cAz - g.ncom[3 * B + 2], g.nM[B],
                       qq, c);
    }
#pragma unroll
    for (int q = 0; q < 19; ++q) c[q] = wave_sum(c[q]);

    // near field
    int S = 1;
    while (S < nA && S < kWave) S <<= 1;
    const int J = kWave / S;
    const int sslot = lane / J;
    const int slice = lane % J;
    const int64_t l0 = g.near_off[li], l1 = g.near_off[li + 1];
    for (int g0 = 0; g0 < nA; g0 += kWave) {
        const int si = g0 + sslot;
        const bool has_sink = si < nA;
        const int64_t pa = (int64_t)sA + (has_sink ? si : 0);
        if constexpr (!MIXED) {
            const double xa = g.px[pa], ya = g.py[pa], za = g.pz[pa], ha = g.ph[pa];
            double ax = 0.0, ay = 0.0, az = 0.0;
            for (int64_t e = l0; e < l1; ++e) {
                const int64_t B = (uint32_t)g.near_list[e] & 0x7fffffffu;
                const int32_t fB = g.nfirst[B], cB = g.ncount[B];
                for (int32_t t0 = slice; t0 < cB; t0 += J) {
                    const int64_t pb = (int64_t)fB + t0;
                    const double vx = xa - g.px[pb], vy = ya - g.py[pb], vz = za - g.pz[pb];
                    const double r2 = (vx * vx + vy * vy) + vz * vz;
                    const double F = soft_F(r2, 0.5 * (ha + g.ph[pb])) * g.pm[pb];
                    ax -= F * vx;
                    ay -= F * vy;
                    az -= F * vz;
                }
            }
            for (int o = 1; o < J; o <<= 1) {
                ax += __shfl_xor(ax, o, kWave);
                ay += __shfl_xor(ay, o, kWave);
                az += __shfl_xor(az, o, kWave);
            }
            if (has_sink && slice == 0) {
                const double d[3] = {xa - cAx, ya - cAy, za - cAz};
                double out[3] = {ax, ay, az};
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    double t1 = c[i];
                    double t2 = 0.0;
#pragma unroll
                    for (int l = 0; l < 3; ++l) {
                        t1 += c[3 + jidx(i, l)] * d[l];
#pragma unroll
                        for (int m = 0; m < 3; ++m) t2 += c[9 + hidx(i, l, m)] * d[l] * d[m];
                    }
                    out[i] += t1 + 0.5 * t2;
                }
                const int32_t o = g.pid[pa];
                ((double *)g.ax)[o] = out[0];
                ((double *)g.ay)[o] = out[1];
                ((double *)g.az)[o] = out[2];
            }
        } else {
            const float xa = g.fdx[pa], ya = g.fdy[pa], za = g.fdz[pa], ha = g.fh[pa];
            float ax = 0.0f, ay = 0.0f, az = 0.0f;
            for (int64_t e = l0; e < l1; ++e) {
                const int64_t B = (uint32_t)g.near_list[e] & 0x7fffffffu;
                const int32_t fB = g.nfirst[B], cB = g.ncount[B];
                const float ox = (float)(cAx - g.ncom[3 * B]);
                const float oy = (float)(cAy - g.ncom[3 * B + 1]);
                const float oz = (float)(cAz - g.ncom[3 * B + 2]);
                const float bx = xa + ox, by = ya + oy, bz = za + oz;
                for (int32_t t0 = slice; t0 < cB; t0 += J) {
                    const int64_t pb = (int64_t)fB + t0;
                    const float vx = bx - g.fdx[pb], vy = by - g.fdy[pb], vz = bz - g.fdz[pb];
                    const float r2 = (vx * vx + vy * vy) + vz * vz;
                    const float F = soft_Ff(r2, 0.5f * (ha + g.fh[pb])) * g.fm[pb];
                    ax -= F * vx;
                    ay -= F * vy;
                    az -= F * vz;
                }
            }
            for (int o = 1; o < J; o <<= 1) {
                ax += __shfl_xor(ax, o, kWave);
                ay += __shfl_xor(ay, o, kWave);
                az += __shfl_xor(az, o, kWave);
            }
            if (has_sink && slice == 0) {
                const float d[3] = {xa, ya, za};
                float out[3] = {ax, ay, az};
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    float t1 = (float)c[i];
                    float t2 = 0.0f;
#pragma unroll
                    for (int l = 0; l < 3; ++l) {
                        t1 += (float)c[3 + jidx(i, l)] * d[l];
#pragma unroll
                        for (int m = 0; m < 3; ++m) t2 += (float)c[9 + hidx(i, l, m)] * d[l] * d[m];
                    }
                    out[i] += t1 + 0.5f * t2;
                }
                const int32_t o = g.pid[pa];
                ((float *)g.ax)[o] = out[0];
                ((float *)g.ay)[o] = out[1];
                ((float *)g.az)[o] = out[2];
            }
        }
    }
}

}  // namespace

rcb_status gravity(rcb_tree *t, void *ax, void *ay, void *az, hipStream_t s) {
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    GravArgs g{t->nleaf, t->nfirst, t->ncount, t->ncom, t->nM, t->nQ, t->near_off, t->far_off,
               t->near_list, t->far_list, t->px, t->py, t->pz, t->pm, t->ph, t->fdx, t->fdy,
               t->fdz, t->fm, t->fh, t->pid, ax, ay, az};
    const unsigned grid = (unsigned)((t->nleaf + kWaves - 1) / kWaves);
    if (t->p.precision == RCB_MIXED) {
        k_gravity<true><<<grid, kBlock, 0, s>>>(g);
    } else {
        k_gravity<false><<<grid, kBlock, 0, s>>>(g);
    }
    RCB_LAUNCH_CHECK("k_gravity");
    return RCB_OK;
}

}  // namespace rcb
