// k_grav.hip -- gravitational accelerations from the interaction lists
// (Sec. 2.4: near field by kernel-softened direct summation, far field by
// quadrupole cell-cell interaction, Taylor-expanded about the sink leaf's
// centre of mass).
//
// One wave per group of up to 8 sibling leaves (k_walk.hip):
//  far:  lanes are (far entry e = lane/8, leaf slot i = lane%8); the lane
//        evaluates node B of entry e at R = com_A(i) - com_B in FP64 if leaf i
//        accepted B (mask bit), accumulating f_i, J_il, H_ilm of Eq. 5's field
//        (far_math.h). B's record is loaded once for the 8 leaves. Lanes of
//        the same leaf are summed at the end; coefficients go to LDS.
//  near: lanes are (sink slot, slice) over the group's particles (contiguous
//        in tree order); slice j of sink a runs over particles
//        first_B + t J + j of every near entry B whose mask has a's leaf:
//        a_a -= m_b F(r, h_ab) (r_a - r_b), F = S(q)/r (Sec. 2.4.3).
//  L2P:  a_a += f + J d + H[d, d] / 2,  d = r_a - com_A  (Eq. 6).
// FP64 form: everything in FP64. Mixed form: particles as FP32 offsets from
// their leaf's centre of mass; per (A, B) the FP64 offset com_A - com_B is
// rounded to FP32 once; P2P, accumulation and L2P in FP32; M2L in FP64.
#include "far_math.h"
#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;

using rcbfar::hidx;
using rcbfar::jidx;
using rcbfar::m2l_accumulate;

// F = S(q)/r of the cubic-spline softening
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
    int gk;
    int64_t ngroup;
    const int32_t *nfirst, *ncount;
    const double *ncom, *nM, *nQ;
    const int64_t *gnear_off, *gfar_off;
    const uint64_t *gnear, *gfar;
    const double *px, *py, *pz, *pm, *ph;
    const float *fdx, *fdy, *fdz, *fm, *fh;
    const int32_t *pid;
    void *ax, *ay, *az;
};

// Far-field coefficients of the group's leaves into coef[8][19] (LDS).
__device__ __forceinline__ void group_far(const GravArgs &g, int64_t gi, double (*coef)[19]) {
    const int lane = lane_id();
    const int slot = lane >> 3, li = lane & 7;
    const int G = 1 << g.gk;
    const int64_t A = g.nleaf + gi * G + (li < G ? li : 0);
    const double cA[3] = {g.ncom[3 * A], g.ncom[3 * A + 1], g.ncom[3 * A + 2]};
    double c[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) c[q] = 0.0;
    const int64_t f0 = g.gfar_off[gi], f1 = g.gfar_off[gi + 1];
    for (int64_t e0 = f0; e0 < f1; e0 += 8) {
        const int64_t e = e0 + slot;
        if (e < f1) {
            const uint64_t ent = g.gfar[e];
            if ((ent >> (32 + li)) & 1ull) {
                const int64_t B = (uint32_t)ent & 0x7fffffffu;
                double qq[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) qq[q] = g.nQ[6 * B + q];
                m2l_accumulate(cA[0] - g.ncom[3 * B], cA[1] - g.ncom[3 * B + 1],
                               cA[2] - g.ncom[3 * B + 2], g.nM[B], qq, c);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        double v = c[q];
        v += __shfl_xor(v, 8, kWave);
        v += __shfl_xor(v, 16, kWave);
        v += __shfl_xor(v, 32, kWave);
        c[q] = v;
    }
    if (slot == 0) {
#pragma unroll
        for (int q = 0; q < 19; ++q) coef[li][q] = c[q];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_gravity(GravArgs g) {
    __shared__ double coef_all[kWaves][8][19];
    double(*coef)[19] = coef_all[threadIdx.x / kWave];
    const int64_t gi = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kWave;
    if (gi >= g.ngroup) return;
    const int lane = lane_id();
    const int G = 1 << g.gk;
    const int64_t GL = (g.nleaf >> g.gk) + gi;   // group node label
    const int32_t sG = g.nfirst[GL], nG = g.ncount[GL];
    if (nG == 0) return;
    group_far(g, gi, coef);

    // leaf boundaries of the group (leaf ranges are contiguous and ordered)
    int32_t lf[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) lf[i] = i < G ? g.nfirst[g.nleaf + gi * G + i] : 0x7fffffff;
    int S = 1;
    while (S < nG && S < kWave) S <<= 1;
    const int J = kWave / S;
    const int sslot = lane / J;
    const int slice = lane % J;
    const int64_t n0 = g.gnear_off[gi], n1 = g.gnear_off[gi + 1];
    for (int g0 = 0; g0 < nG; g0 += S) {
        const int si = g0 + sslot;
        const bool has_sink = si < nG;
        const int32_t pa = sG + (has_sink ? si : 0);
        int la = 0;
#pragma unroll
        for (int i = 1; i < 8; ++i)
            if (lf[i] <= pa) la = i;
        const uint32_t bit = has_sink ? (1u << la) : 0u;
        const int64_t A = g.nleaf + gi * G + la;
        const double cAx = g.ncom[3 * A], cAy = g.ncom[3 * A + 1], cAz = g.ncom[3 * A + 2];
        if constexpr (!MIXED) {
            const double xa = g.px[pa], ya = g.py[pa], za = g.pz[pa], ha = g.ph[pa];
            double ax = 0.0, ay = 0.0, az = 0.0;
            for (int64_t e = n0; e < n1; ++e) {
                const uint64_t ent = g.gnear[e];
                const int64_t B = (uint32_t)ent & 0x7fffffffu;
                const int32_t fB = g.nfirst[B], cB = g.ncount[B];
                if (!(((uint32_t)(ent >> 32)) & bit)) continue;
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
                double c[19];
#pragma unroll
                for (int q = 0; q < 19; ++q) c[q] = coef[la][q];
                double out[3];
                rcbfar::l2p<double>(c, d, out);
                const int32_t o = g.pid[pa];
                ((double *)g.ax)[o] = ax + out[0];
                ((double *)g.ay)[o] = ay + out[1];
                ((double *)g.az)[o] = az + out[2];
            }
        } else {
            const float xa = g.fdx[pa], ya = g.fdy[pa], za = g.fdz[pa], ha = g.fh[pa];
            float ax = 0.0f, ay = 0.0f, az = 0.0f;
            for (int64_t e = n0; e < n1; ++e) {
                const uint64_t ent = g.gnear[e];
                const int64_t B = (uint32_t)ent & 0x7fffffffu;
                const int32_t fB = g.nfirst[B], cB = g.ncount[B];
                if (!(((uint32_t)(ent >> 32)) & bit)) continue;
                const float bx = xa + (float)(cAx - g.ncom[3 * B]);
                const float by = ya + (float)(cAy - g.ncom[3 * B + 1]);
                const float bz = za + (float)(cAz - g.ncom[3 * B + 2]);
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
                double c[19];
#pragma unroll
                for (int q = 0; q < 19; ++q) c[q] = coef[la][q];
                float out[3];
                rcbfar::l2p<float>(c, d, out);
                const int32_t o = g.pid[pa];
                ((float *)g.ax)[o] = ax + out[0];
                ((float *)g.ay)[o] = ay + out[1];
                ((float *)g.az)[o] = az + out[2];
            }
        }
    }
}

}  // namespace

rcb_status gravity(rcb_tree *t, void *ax, void *ay, void *az, hipStream_t s) {
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    GravArgs g{t->nleaf, t->gk, t->ngroup, t->nfirst, t->ncount, t->ncom, t->nM, t->nQ,
               t->gnear_off, t->gfar_off, t->gnear, t->gfar, t->px, t->py, t->pz, t->pm, t->ph,
               t->fdx, t->fdy, t->fdz, t->fm, t->fh, t->pid, ax, ay, az};
    const unsigned grid = (unsigned)((t->ngroup + kWaves - 1) / kWaves);
    if (t->p.precision == RCB_MIXED) {
        k_gravity<true><<<grid, kBlock, 0, s>>>(g);
    } else {
        k_gravity<false><<<grid, kBlock, 0, s>>>(g);
    }
    RCB_LAUNCH_CHECK("k_gravity");
    return RCB_OK;
}

}  // namespace rcb
