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
//  near: the group's leaves in turn. Lanes are (sink slot, slice) over the
//        leaf's particles (near_tile.h: S = min(c, 64) sinks, J = 64 / S
//        slices). The cells of the group's near list whose mask has the leaf
//        are staged 64 sources at a time in LDS; slice j of a sink takes tile
//        entries j, j + J, ...: a_a -= m_b F(r, h_ab) (r_a - r_b),
//        F = S(q)/r (Sec. 2.4.3); the slices are summed at the end.
//  L2P:  a_a += f + J d + H[d, d] / 2,  d = r_a - com_A  (Eq. 6).
// FP64 form: everything in FP64. Mixed form: the sink leaf's frame. Sinks
// are their FP32 offsets from the leaf centre of mass; a source of cell B is
// its FP32 offset plus the FP64 difference com_B - com_A rounded to FP32;
// pairs, accumulation and L2P in FP32; M2L in FP64.
#include "far_math.h"
#include "near_tile.h"
#include "rcb_internal.h"
#include "soft.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;

using rcbfar::hidx;
using rcbfar::jidx;
using rcbfar::m2l_accumulate;

struct GravArgs {
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
    void *ax, *ay, *az;
    double *farc;   // if given: each leaf's far coefficients at farc[leaf * kLeafC]
};

// Far-field coefficients of the group's leaves into coef[8][19] (LDS).
// The union far list is taken in windows of kFarWin entries, whose node data
// (centre of mass, mass, quadrupole) are staged in LDS by one coalesced pass.
// For each window every leaf gets the list of the window positions whose mask
// has it (ballot ranks, in list order); then lane (s, i) evaluates entries
// s, s + 8, ... of leaf i's list, so a leaf's lanes only idle at the end of
// the window rather than on every entry the leaf did not accept.
constexpr int kFarWin = 64;
struct FarWindow {
    int32_t lab[kFarWin];
    uint8_t idx[8][kFarWin];
    double nd[kFarWin][10];
};

template <bool RB>
__device__ __forceinline__ void group_far(const GravArgs &g, int64_t gi, FarWindow &fw, double (*coef)[19]) {
    const int lane = lane_id();
    const int slot = lane >> 3, li = lane & 7;
    const int G = 1 << g.gk;
    const int64_t A = g.nleaf + gi * G + (li < G ? li : 0);
    const double cA[3] = {g.ncom[3 * A], g.ncom[3 * A + 1], g.ncom[3 * A + 2]};
    double c[rcbfar::kAcc];
#pragma unroll
    for (int q = 0; q < rcbfar::kAcc; ++q) c[q] = 0.0;
    const int64_t f0 = g.gfar_beg[gi], f1 = g.gfar_end[gi];
    for (int64_t w0 = f0; w0 < f1; w0 += kFarWin) {
        const int nw = (int)(f1 - w0 < kFarWin ? f1 - w0 : kFarWin);
        int base[8];
#pragma unroll
        for (int l = 0; l < 8; ++l) base[l] = 0;
        for (int p0 = 0; p0 < nw; p0 += kWave) {
            const int p = p0 + lane;
            uint32_t m = 0;
            if (p < nw) {
                const uint64_t ent = g.gfar[w0 + p];
                fw.lab[p] = (int32_t)((uint32_t)ent & 0x7fffffffu);
                m = (uint32_t)(ent >> 32) & 0xffu;
                const int64_t Bn = (uint32_t)ent & 0x7fffffffu;
                fw.nd[p][0] = g.ncom[3 * Bn];
                fw.nd[p][1] = g.ncom[3 * Bn + 1];
                fw.nd[p][2] = g.ncom[3 * Bn + 2];
                fw.nd[p][3] = g.nM[Bn];
#pragma unroll
                for (int q = 0; q < 6; ++q) fw.nd[p][4 + q] = g.nQ[6 * Bn + q];
            }
#pragma unroll
            for (int l = 0; l < 8; ++l) {
                const bool has = (m >> l) & 1u;
                const uint64_t bl = ballot(has);
                if (has) fw.idx[l][base[l] + rank_below(bl)] = (uint8_t)p;
                base[l] += __popcll(bl);
            }
        }
        int most = 0, mine = 0;
#pragma unroll
        for (int l = 0; l < 8; ++l) {
            most = base[l] > most ? base[l] : most;
            mine = li == l ? base[l] : mine;
        }
        tile_sync();
        const int rounds = (most + 7) >> 3;
        for (int r = 0; r < rounds; ++r) {
            const int k = 8 * r + slot;
            if (k < mine) {
                const double *nd = fw.nd[fw.idx[li][k]];
                double qq[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) qq[q] = nd[4 + q];
                m2l_accumulate<RB>(cA[0] - nd[0], cA[1] - nd[1], cA[2] - nd[2], nd[3], qq, c);
            }
        }
        tile_sync();
    }
#pragma unroll
    for (int q = 0; q < rcbfar::kAcc; ++q) {
        double v = c[q];
        v += __shfl_xor(v, 8, kWave);
        v += __shfl_xor(v, 16, kWave);
        v += __shfl_xor(v, 32, kWave);
        c[q] = v;
    }
    if (slot == 0) {
        double full[19];
        rcbfar::m2l_finish(c, full);
#pragma unroll
        for (int q = 0; q < 19; ++q) coef[li][q] = full[q];
    }
    tile_sync();
}

struct alignas(16) SrcF {
    float x, y, z, m, h;
};
struct alignas(16) SrcD {
    double x, y, z, m, h;
};

// tile: 64 staged sources, then 64 zero-mass sources that pad the last
// partial row of slices, so the pair loop needs no bounds test
template <bool MIXED>
struct NearStage {
    EntryChunk ec;
    typename std::conditional<MIXED, SrcF, SrcD>::type tile[2 * kWave];
};
// the far window and the near staging are used one after the other
template <bool MIXED>
struct GravShared {
    double coef[8][19];
    union {
        FarWindow fw;
        NearStage<MIXED> np;
    };
};

// RB: Taylor reading B for the sink coefficients (J, H of the monopole field)
template <bool MIXED, bool RB>
__global__ __launch_bounds__(kBlock) void k_gravity(GravArgs g) {
    using T = typename std::conditional<MIXED, float, double>::type;
    __shared__ GravShared<MIXED> sh_all[kWaves];
    GravShared<MIXED> &sh = sh_all[threadIdx.x / kWave];
    const int64_t gi = wave_index();
    if (gi >= g.ngroup) return;
    const int lane = lane_id();
    const int G = 1 << g.gk;
    const int64_t GL = (g.nleaf >> g.gk) + gi;   // group node label
    if (g.ncount[GL] == 0) return;
    group_far<RB>(g, gi, sh.fw, sh.coef);
    if (g.farc)
        for (int i = lane; i < G * 19; i += kWave) g.farc[(gi * G + i / 19) * kLeafC + i % 19] = sh.coef[i / 19][i % 19];
    using Src = typename std::conditional<MIXED, SrcF, SrcD>::type;
    Src dummy;
    dummy.x = dummy.y = dummy.z = dummy.m = 0;
    dummy.h = 1;
    sh.np.tile[kWave + lane] = dummy;
    const int64_t n0 = g.gnear_beg[gi], n1 = g.gnear_end[gi];
    for (int li = 0; li < G; ++li) {
        const int64_t A = g.nleaf + gi * G + li;
        const int32_t sA = g.nfirst[A], c = g.ncount[A];
        if (c == 0) continue;
        const LeafLanes L = leaf_lanes(c);
        const double cA[3] = {g.ncom[3 * A], g.ncom[3 * A + 1], g.ncom[3 * A + 2]};
        for (int g0 = 0; g0 < c; g0 += L.S) {
            const int si = g0 + L.sslot;
            const bool has_sink = L.sslot < L.S && si < c;
            const int32_t pa = sA + (has_sink ? si : 0);
            T xa, ya, za, ha;
            if constexpr (MIXED) {   // leaf frame
                xa = g.fdx[pa];
                ya = g.fdy[pa];
                za = g.fdz[pa];
                ha = g.fh[pa];
            } else {
                xa = g.px[pa];
                ya = g.py[pa];
                za = g.pz[pa];
                ha = g.ph[pa];
            }
            T ax = 0, ay = 0, az = 0;
            for (int64_t e0 = n0; e0 < n1; e0 += kWave) {
                const int tot = load_entry_chunk(g.gnear, g.nfirst, g.ncount, e0, n1, 1u << li, sh.np.ec);
                for (int t = 0; t < tot; t += kWave) {
                    const int q = t + lane;
                    if (q >= tot) sh.np.tile[lane] = dummy;
                    if (q < tot) {
                        const int k = entry_of(sh.np.ec, q);
                        const int64_t pb = (int64_t)sh.np.ec.fB[k] + (q - sh.np.ec.pos[k]);
                        if constexpr (MIXED) {
                            const int64_t B = sh.np.ec.label[k];
                            SrcF s;
                            s.x = (float)(g.ncom[3 * B] - cA[0]) + g.fdx[pb];
                            s.y = (float)(g.ncom[3 * B + 1] - cA[1]) + g.fdy[pb];
                            s.z = (float)(g.ncom[3 * B + 2] - cA[2]) + g.fdz[pb];
                            s.m = g.fm[pb];
                            s.h = g.fh[pb];
                            sh.np.tile[lane] = s;
                        } else {
                            SrcD s;
                            s.x = g.px[pb];
                            s.y = g.py[pb];
                            s.z = g.pz[pb];
                            s.m = g.pm[pb];
                            s.h = g.ph[pb];
                            sh.np.tile[lane] = s;
                        }
                    }
                    tile_sync();
                    const int nt = tot - t < kWave ? tot - t : kWave;
                    const int rows = (nt + L.J - 1) / L.J;
                    for (int r = 0; r < rows; ++r) {
                        const auto s = sh.np.tile[r * L.J + L.slice];
                        const T vx = xa - s.x, vy = ya - s.y, vz = za - s.z;
                        const T r2 = (vx * vx + vy * vy) + vz * vz;
                        const T hsum = ha + s.h;
                        const T ri = rsq_t(r2);
                        const T r3 = ri * ri * ri;
                        T F = r3;
                        if (!soft_outside<T>(r2, hsum)) F = soft_F<T>(r2, ri, r3, hsum);
                        F *= s.m;
                        ax -= F * vx;
                        ay -= F * vy;
                        az -= F * vz;
                    }
                    tile_sync();
                }
            }
            ax = seg_sum(ax, L.slice, L.J);
            ay = seg_sum(ay, L.slice, L.J);
            az = seg_sum(az, L.slice, L.J);
            if (has_sink && L.slice == 0) {
                double c19[19];
#pragma unroll
                for (int q = 0; q < 19; ++q) c19[q] = sh.coef[li][q];
                T d[3], out[3];
                if constexpr (MIXED) {
                    d[0] = xa;
                    d[1] = ya;
                    d[2] = za;
                } else {
                    d[0] = xa - cA[0];
                    d[1] = ya - cA[1];
                    d[2] = za - cA[2];
                }
                rcbfar::l2p<T>(c19, d, out);
                const int32_t o = g.pid[pa];
                ((T *)g.ax)[o] = ax + out[0];
                ((T *)g.ay)[o] = ay + out[1];
                ((T *)g.az)[o] = az + out[2];
            }
        }
    }
}

// far-field coefficients of every leaf, stride doubles per leaf (first 19 used)
struct FarShared {
    double coef[8][19];
    FarWindow fw;
};
__global__ __launch_bounds__(kBlock) void k_far_coeffs(GravArgs g, double *out, int stride) {
    __shared__ FarShared sh_all[kWaves];
    FarShared &sh = sh_all[threadIdx.x / kWave];
    double(*coef)[19] = sh.coef;
    const int64_t gi = wave_index();
    if (gi >= g.ngroup) return;
    const int G = 1 << g.gk;
    group_far<false>(g, gi, sh.fw, coef);
    for (int i = lane_id(); i < G * 19; i += kWave) out[(gi * G + i / 19) * stride + i % 19] = coef[i / 19][i % 19];
}

}  // namespace

rcb_status far_coefficients(rcb_tree *t, double *out, int stride, hipStream_t s) {
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    GravArgs g{t->nleaf, t->gk, t->ngroup, t->nfirst, t->ncount, t->ncom, t->nM, t->nQ,
               t->gnear_beg, t->gnear_end, t->gfar_beg, t->gfar_end, t->gnear, t->gfar, t->px, t->py, t->pz, t->pm, t->ph,
               t->fdx, t->fdy, t->fdz, t->fm, t->fh, t->pid, nullptr, nullptr, nullptr, nullptr};
    const unsigned grid = (unsigned)((t->ngroup + kWaves - 1) / kWaves);
    k_far_coeffs<<<grid, kBlock, 0, s>>>(g, out, stride);
    RCB_LAUNCH_CHECK("k_far_coeffs");
    return RCB_OK;
}

rcb_status gravity(rcb_tree *t, void *ax, void *ay, void *az, hipStream_t s) {
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    const bool rb = t->p.taylor_reading == RCB_READING_B;
    // the far coefficients are kept for a VJP on the same moments (if the
    // array cannot be had, gravity goes on without keeping them)
    if (!rb && !t->farc) t->farc = (double *)dalloc(t, sizeof(double) * kLeafC * t->nleaf, s, t->list_allocs);
    double *farc = rb ? nullptr : t->farc;
    GravArgs g{t->nleaf, t->gk, t->ngroup, t->nfirst, t->ncount, t->ncom, t->nM, t->nQ,
               t->gnear_beg, t->gnear_end, t->gfar_beg, t->gfar_end, t->gnear, t->gfar, t->px, t->py, t->pz, t->pm, t->ph,
               t->fdx, t->fdy, t->fdz, t->fm, t->fh, t->pid, ax, ay, az, farc};
    const unsigned grid = (unsigned)((t->ngroup + kWaves - 1) / kWaves);
    if (t->p.precision == RCB_MIXED) {
        if (rb) k_gravity<true, true><<<grid, kBlock, 0, s>>>(g);
        else k_gravity<true, false><<<grid, kBlock, 0, s>>>(g);
    } else {
        if (rb) k_gravity<false, true><<<grid, kBlock, 0, s>>>(g);
        else k_gravity<false, false><<<grid, kBlock, 0, s>>>(g);
    }
    RCB_LAUNCH_CHECK("k_gravity");
    if (farc) t->farc_valid = true;
    return RCB_OK;
}

}  // namespace rcb
