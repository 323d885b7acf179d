// k_build.hip -- top-down RCB build on the device, one pass per level
// (Sec. 2.1: "Strategy", "Load balancing", "Particle sorting", "Node
// labelling", "Multipole moments").
//
// Each level l = 0 .. k-1 splits every node through its centre of mass,
// perpendicular to the longest side of its box, with a stable partition
// (coordinate < plane -> child 2n). Node sums are canonical pairwise sums
// over the node's particles in their order at split time, which is ascending
// input index because every partition is stable and starts from input
// order. The pairwise tree is aligned at the node's first particle and padded
// with +0.0 to a power of two; a final "+ 0.0" maps -0.0 to +0.0, so any
// wider padding gives the same bits.
//
// Work split: a node of <= 512 particles is handled by one wave end to end
// (sums, split, partition) from registers. Larger nodes register in a list;
// their 512-particle chunks are reduced by one wave each, a wave per node
// combines the chunk sums, and the partition runs as count / scan / scatter
// over the same chunks. Kernels are HBM-bound: each level reads 32 B and
// writes 36 B per particle.
#include <chrono>
#include <mutex>
#include <string>
#include <type_traits>

#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------------------
// bounds, validation, initial copy
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bounds_partial(const double *__restrict__ x,
                                                           const double *__restrict__ y,
                                                           const double *__restrict__ z, int64_t n,
                                                           double *__restrict__ part,
                                                           int32_t *__restrict__ iota = nullptr) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        if (iota) iota[i] = (int32_t)i;   // the order of level 0
        double v[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], v[d]);
            hi[d] = fmax(hi[d], v[d]);
        }
    }
    __shared__ double red[6][kWavesPerBlock];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double a = lo[d], b = hi[d];
        for (int o = 1; o < kWave; o <<= 1) {
            a = fmin(a, __shfl_xor(a, o, kWave));
            b = fmax(b, __shfl_xor(b, o, kWave));
        }
        if (lane_id() == 0) {
            red[d][threadIdx.x / kWave] = a;
            red[3 + d][threadIdx.x / kWave] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double r = red[threadIdx.x][0];
        for (int w = 1; w < kWavesPerBlock; ++w)
            r = threadIdx.x < 3 ? fmin(r, red[threadIdx.x][w]) : fmax(r, red[threadIdx.x][w]);
        part[6 * blockIdx.x + threadIdx.x] = r;
    }
}

// one block of 256 threads: per-thread minima / maxima over the partials,
// then a tree over the block (min and max do not depend on the order)
// Also sets the root's range and clears the nclr control words of clr.
__global__ __launch_bounds__(256) void k_bounds_final(const double *__restrict__ part, int nb,
                                                      double *__restrict__ nlo, double *__restrict__ nhi,
                                                      int32_t *__restrict__ nfirst, int32_t *__restrict__ ncount,
                                                      int32_t n, int32_t *__restrict__ clr, int nclr) {
    __shared__ double red[6][256];
    const int t = threadIdx.x;
    if (t == 0) {
        nfirst[1] = 0;
        ncount[1] = n;
    }
    for (int i = t; i < nclr; i += 256) clr[i] = 0;
    double r[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) r[d] = part[d];
    for (int b = t; b < nb; b += 256) {
#pragma unroll
        for (int d = 0; d < 6; ++d) r[d] = d < 3 ? fmin(r[d], part[6 * b + d]) : fmax(r[d], part[6 * b + d]);
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) red[d][t] = r[d];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int d = 0; d < 6; ++d)
                red[d][t] = d < 3 ? fmin(red[d][t], red[d][t + w]) : fmax(red[d][t], red[d][t + w]);
        }
        __syncthreads();
    }
    if (t < 3) nlo[3 + t] = red[t][0];   // label 1
    else if (t < 6) nhi[3 + t - 3] = red[t][0];
}

__global__ void k_validate(const double *__restrict__ x, const double *__restrict__ y,
                           const double *__restrict__ z, const double *__restrict__ m,
                           const double *__restrict__ h, int64_t n, int32_t *__restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool bad = !isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i]) || !(m[i] > 0.0) ||
                   !(h[i] > 0.0) || !isfinite(m[i]) || !isfinite(h[i]);
        if (bad) atomicOr(flag, 1);
    }
}

__global__ void k_init(const double *__restrict__ x, const double *__restrict__ y,
                       const double *__restrict__ z, const double *__restrict__ m, int64_t n,
                       double *__restrict__ ox, double *__restrict__ oy, double *__restrict__ oz,
                       double *__restrict__ om, int32_t *__restrict__ oid) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        ox[i] = x[i];
        oy[i] = y[i];
        oz[i] = z[i];
        om[i] = m[i];
        oid[i] = (int32_t)i;
    }
}

__global__ void k_gather_h(const double *__restrict__ h, const int32_t *__restrict__ id, int64_t n,
                           double *__restrict__ oh) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        oh[i] = h[id[i]];
}

// refresh: new inputs into one level's particle order (h only if ph != null)
__global__ void k_refresh_gather(const double *__restrict__ x, const double *__restrict__ y,
                                 const double *__restrict__ z, const double *__restrict__ m,
                                 const double *__restrict__ h, const int32_t *__restrict__ id, int64_t n,
                                 double *__restrict__ px, double *__restrict__ py,
                                 double *__restrict__ pz, double *__restrict__ pm,
                                 double *__restrict__ ph) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = id[i];
        px[i] = x[j];
        py[i] = y[j];
        pz[i] = z[j];
        pm[i] = m[j];
        if (ph) ph[i] = h[j];
    }
}

// ---------------------------------------------------------------------------
// chunk sums. Payload A: m, m x, m y, m z and max |r - g|^2 (g = box centre).
// Payload B (leaves): the six Eq. 1 components about the leaf centre of mass
// and max(|r - g| + 2h). Lane l holds the 8 consecutive elements
// [base + 8l, base + 8l + 8); pairs, quads and octets are summed in the lane,
// the remaining 6 levels of the 512-wide tree across lanes.
// ---------------------------------------------------------------------------
template <int P>
struct Pay;
template <>
struct Pay<0> {
    static constexpr int NS = 4;
};
template <>
struct Pay<1> {
    static constexpr int NS = 6;
};

struct PartIn {
    const double *x, *y, *z, *m, *h;
};

// Sum and max over the LANES lanes of this lane's group (xor butterfly: the
// canonical pairwise tree across lanes, as for the whole wave).
template <int LANES>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
template <int LANES>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// LANES = 64: one node per wave (512 elements); LANES = 8: one node per 8-lane
// group (64 elements). Narrower trees padded with zeros give the same bits.
// Wave-private LDS staging of one 512-element chunk: elements are loaded
// coalesced (lane l takes base + 64 t + l) and read back as each lane's 8
// consecutive ones; one pad slot per 8 keeps the read-back off shared banks.
constexpr int kStage = kChunk + kChunk / 8;
__device__ __forceinline__ int stage_slot(int e) { return e + (e >> 3); }

// Staging of a wave's contiguous range [w0, wend) of at most kChunk elements
// in two halves, so that a caller can issue the global loads of all its
// fields before the first LDS round trip: load8c takes lane l's elements
// w0 + 64 t + l (coalesced, zero past wend); transpose8 passes them through
// LDS and returns this lane's [p0, p0 + 8), zero at and past `end`.
template <typename V>
__device__ __forceinline__ void load8c(const V *__restrict__ a, int64_t w0, int64_t wend, V (&r)[8]) {
    const int l = lane_id();
#pragma unroll
    for (int t = 0; t < 8; ++t) r[t] = w0 + 64 * t + l < wend ? a[w0 + 64 * t + l] : (V)0;
}
template <typename V>
__device__ __forceinline__ void transpose8(const V (&r)[8], int64_t w0, int64_t p0, int64_t end, V *buf,
                                           V (&out)[8]) {
    const int l = lane_id();
#pragma unroll
    for (int t = 0; t < 8; ++t) buf[stage_slot(64 * t + l)] = r[t];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int t = 0; t < 8; ++t) out[t] = p0 + t < end ? buf[stage_slot((int)(p0 + t - w0))] : (V)0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}
// The reverse: value t of this lane goes to position w0 + dl[t] (dl < 0: none),
// then the range [w0, wend) is stored coalesced.
template <typename V>
__device__ __forceinline__ void scatter8w(V *__restrict__ a, int64_t w0, int64_t wend, const int (&dl)[8],
                                          const V (&val)[8], V *buf) {
    const int l = lane_id();
#pragma unroll
    for (int t = 0; t < 8; ++t)
        if (dl[t] >= 0) buf[stage_slot(dl[t])] = val[t];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = 64 * t + l;
        if (w0 + e < wend) a[w0 + e] = buf[stage_slot(e)];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// `stage`: a wave-private buffer of kStage doubles (LANES == 64) or null
// (direct loads of each lane's 8 consecutive elements).
// The tree sums of one node from its elements [p0, p0 + 8) held by this lane
// (zero past `end`), as loaded by chunk_sums or by a caller that staged them.
template <int P, int LANES = kWave>
__device__ __forceinline__ void chunk_sums_regs(const double (&X)[8], const double (&Y)[8],
                                                const double (&Z)[8], const double (&Mm)[8],
                                                const double (&H)[8], int64_t p0, int64_t end,
                                                const double g[3], const double c[3],
                                                double (&sums)[Pay<P>::NS], double &mx) {
    constexpr int NS = Pay<P>::NS;
    double v[8][NS];
    double ml = -1.0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int64_t i = p0 + t;
        if (i < end) {
            const double xi = X[t], yi = Y[t], zi = Z[t], mi = Mm[t];
            if constexpr (P == 0) {
                v[t][0] = mi;
                v[t][1] = mi * xi;
                v[t][2] = mi * yi;
                v[t][3] = mi * zi;
                ml = fmax(ml, dist2(xi, yi, zi, g[0], g[1], g[2]));
            } else {
                const double d0 = xi - c[0], d1 = yi - c[1], d2 = zi - c[2];
                const double r2 = (d0 * d0 + d1 * d1) + d2 * d2;
                const double m3 = 3.0 * mi;
                const double mr2 = mi * r2;
                v[t][0] = (m3 * d0) * d0 - mr2;
                v[t][1] = (m3 * d0) * d1;
                v[t][2] = (m3 * d0) * d2;
                v[t][3] = (m3 * d1) * d1 - mr2;
                v[t][4] = (m3 * d1) * d2;
                v[t][5] = (m3 * d2) * d2 - mr2;
                const double rg = sqrt(dist2(xi, yi, zi, g[0], g[1], g[2]));
                ml = fmax(ml, rg + 2.0 * H[t]);
            }
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s) v[t][s] = 0.0;
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double a = (v[0][s] + v[1][s]) + (v[2][s] + v[3][s]);
        const double b = (v[4][s] + v[5][s]) + (v[6][s] + v[7][s]);
        sums[s] = group_sum<LANES>(a + b);
    }
    mx = group_max<LANES>(ml);
}

template <int P, int LANES = kWave>
__device__ __forceinline__ void chunk_sums(const PartIn &in, int64_t base, int64_t end,
                                           const double g[3], const double c[3],
                                           double (&sums)[Pay<P>::NS], double &mx,
                                           double *stage = nullptr) {
    const int64_t p0 = base + 8 * (int64_t)(lane_id() % LANES);
    double X[8], Y[8], Z[8], Mm[8], H[8];
    if (stage) {   // all loads first, then the LDS passes
        double rx[8], ry[8], rz[8], rm[8], rh[8];
        load8c(in.x, base, end, rx);
        load8c(in.y, base, end, ry);
        load8c(in.z, base, end, rz);
        load8c(in.m, base, end, rm);
        if constexpr (P == 1) load8c(in.h, base, end, rh);
        transpose8(rx, base, p0, end, stage, X);
        transpose8(ry, base, p0, end, stage, Y);
        transpose8(rz, base, p0, end, stage, Z);
        transpose8(rm, base, p0, end, stage, Mm);
        if constexpr (P == 1) transpose8(rh, base, p0, end, stage, H);
    } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int64_t i = p0 + t;
            const bool ok = i < end;
            X[t] = ok ? in.x[i] : 0.0;
            Y[t] = ok ? in.y[i] : 0.0;
            Z[t] = ok ? in.z[i] : 0.0;
            Mm[t] = ok ? in.m[i] : 0.0;
            if constexpr (P == 1) H[t] = ok ? in.h[i] : 0.0;
        }
    }
    chunk_sums_regs<P, LANES>(X, Y, Z, Mm, H, p0, end, g, c, sums, mx);
}

struct NodeOut {
    int32_t *nfirst, *ncount;
    double *nlo, *nhi, *ncom, *nM, *nhint, *nhnode, *nQ;
    int32_t *naxis;
    double *nplane;
    // median split only (else null): plane and caller index of the first
    // upper particle of each node, computed before the node's level pass
    const double *mplane;
    const int32_t *mtie;
};

// The side rule: a particle goes to the lower child iff (x, caller index)
// comes before (plane, tie). Splits through a centre use tie = INT32_MIN,
// i.e. x < plane; the median split's tie makes the halves exact.
__device__ __forceinline__ int32_t node_tie(const NodeOut &o, int64_t lab) {
    return o.mplane ? o.mtie[lab] : INT32_MIN;
}

__device__ __forceinline__ bool goes_left(double x, const int32_t *__restrict__ id, int64_t i,
                                          double plane, int32_t tie) {
    return x < plane || (tie != INT32_MIN && x == plane && id[i] < tie);
}

__device__ __forceinline__ void box_centre(const NodeOut &o, int64_t lab, double g[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] = 0.5 * (o.nlo[3 * lab + d] + o.nhi[3 * lab + d]);
}

// Payload-A result of a non-empty node: mass, centre of mass, h_node_int,
// and for an internal node the split axis/plane and the children's boxes.
// split = false (moments-only refresh): the node's box, split and children
// stay as built.
template <int LANES = kWave>
__device__ void finish_a(const NodeOut &o, int64_t lab, bool leaf, const double s[4], double mx,
                         bool split = true) {
    const double M = s[0] + 0.0;
    double com[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) com[d] = (s[1 + d] + 0.0) / M;
    const int l = lane_id() % LANES;
    if (l == 0) {
        o.nM[lab] = M;
#pragma unroll
        for (int d = 0; d < 3; ++d) o.ncom[3 * lab + d] = com[d];
        o.nhint[lab] = sqrt(mx);
        o.nhnode[lab] = -1.0;
    }
    if (leaf || !split) return;
    double lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = o.nlo[3 * lab + d];
        hi[d] = o.nhi[3 * lab + d];
    }
    int ax = 0;
    double best = hi[0] - lo[0];
    if (hi[1] - lo[1] > best) {
        best = hi[1] - lo[1];
        ax = 1;
    }
    if (hi[2] - lo[2] > best) ax = 2;
    const double plane = o.mplane ? o.mplane[lab] : (ax == 0 ? com[0] : (ax == 1 ? com[1] : com[2]));
    if (l == 0) {
        o.naxis[lab] = ax;
        o.nplane[lab] = plane;
    }
    if (l < 6) {   // children boxes: lanes 0-2 lower corners, 3-5 upper corners
        const int d = l % 3;
        const bool upper = l >= 3;
        const double vl = d == 0 ? lo[0] : (d == 1 ? lo[1] : lo[2]);   // no dynamic indexing
        const double vh = d == 0 ? hi[0] : (d == 1 ? hi[1] : hi[2]);
        const double v = upper ? vh : vl;
        const int64_t L = 2 * lab, R = 2 * lab + 1;
        double *dL = upper ? o.nhi : o.nlo;
        dL[3 * L + d] = (upper && d == ax) ? plane : v;
        dL[3 * R + d] = (!upper && d == ax) ? plane : v;
    }
}

template <int LANES = kWave>
__device__ void finish_b(const NodeOut &o, int64_t lab, const double s[6], double mx) {
    const int l = lane_id() % LANES;
    if (l < 6) o.nQ[6 * lab + l] = (l == 0 ? s[0] : l == 1 ? s[1] : l == 2 ? s[2] : l == 3 ? s[3] : l == 4 ? s[4] : s[5]) + 0.0;
    if (l == 0) o.nhnode[lab] = mx;
}

template <int LANES = kWave>
__device__ void finish_empty(const NodeOut &o, int64_t lab, bool leaf, int32_t first,
                             bool split = true) {
    const int l = lane_id() % LANES;
    double g[3];
    box_centre(o, lab, g);
    if (l == 0) {
        o.nM[lab] = 0.0;
        o.ncom[3 * lab] = g[0];
        o.ncom[3 * lab + 1] = g[1];
        o.ncom[3 * lab + 2] = g[2];
        o.nhint[lab] = -1.0;
        o.nhnode[lab] = -1.0;
        if (leaf) {
            for (int q = 0; q < 6; ++q) o.nQ[6 * lab + q] = 0.0;
        } else if (split) {
            o.naxis[lab] = -1;
            o.nfirst[2 * lab] = first;
            o.ncount[2 * lab] = 0;
            o.nfirst[2 * lab + 1] = first;
            o.ncount[2 * lab + 1] = 0;
        }
    }
    if (!leaf && split && l < 6) {
        const int d = l % 3;
        double *dst = l >= 3 ? o.nhi : o.nlo;
        const double v = dst[3 * lab + d];
        dst[3 * (2 * lab) + d] = v;
        dst[3 * (2 * lab + 1) + d] = v;
    }
}

struct PartOut {
    double *x, *y, *z, *m;
    int32_t *id;
};

// Stable partition of the elements [base, end): `lb` left and `rb` right
// elements of the node precede base. Elements are taken 64 at a time in
// order (lane l holds base + 64 t + l), ranks come from ballots, so the
// stores of a side are contiguous across lanes. All of the wave's loads are
// issued before its first store (the compiler cannot know that the output
// arrays do not alias the inputs).
__device__ __forceinline__ void scatter_chunk(const PartIn &in, const int32_t *__restrict__ id,
                                              const PartOut &out, int64_t base, int64_t end,
                                              int ax, double plane, int32_t tie, int64_t node_first,
                                              int64_t nleft_total, int64_t lb, int64_t rb) {
    const int l = lane_id();
    int64_t rl = lb, rr = rb;
    double vx[8], vy[8], vz[8], vm[8];
    int32_t vid[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int64_t i = base + 64 * t + l;
        const bool valid = i < end;
        vx[t] = valid ? in.x[i] : 0.0;
        vy[t] = valid ? in.y[i] : 0.0;
        vz[t] = valid ? in.z[i] : 0.0;
        vm[t] = valid ? in.m[i] : 0.0;
        vid[t] = valid ? id[i] : 0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int64_t i = base + 64 * t + l;
        const bool valid = i < end;
        const double xv = ax == 0 ? vx[t] : (ax == 1 ? vy[t] : vz[t]);
        // written out rather than through a helper: the helper form compiled
        // to a partition pass a third slower on gfx950 (measured)
        const bool left = valid && (xv < plane || (tie != INT32_MIN && xv == plane && vid[t] < tie));
        const uint64_t bl = ballot(left);
        const int nl = __popcll(bl);
        const int nv = (int)min<int64_t>(64, max<int64_t>(0, end - (base + 64 * t)));
        if (valid) {
            const int rk = rank_below(bl);
            const int64_t dst = left ? node_first + rl + rk : node_first + nleft_total + rr + (l - rk);
            out.x[dst] = vx[t];
            out.y[dst] = vy[t];
            out.z[dst] = vz[t];
            out.m[dst] = vm[t];
            out.id[dst] = vid[t];
        }
        rl += nl;
        rr += nv - nl;
    }
}

// ---------------------------------------------------------------------------
// one wave per node of the level: nodes of <= 512 particles are done here,
// larger ones are put on the big-node list.
// ---------------------------------------------------------------------------
struct BigCtl {
    int32_t *ctl;         // [0] big nodes, [1] items
    int32_t *big_node, *big_base, *item_big;
};

__device__ __forceinline__ void level_node(int64_t lab, bool leaf, bool split, const PartIn &in,
                                           const int32_t *__restrict__ id, const PartOut &out,
                                           const NodeOut &o, const BigCtl &bc, double *stage) {
    const int32_t s = o.nfirst[lab];
    const int32_t c = o.ncount[lab];
    if (c > kChunk) {
        int bi = 0, base = 0;
        const int nch = (c + kChunk - 1) / kChunk;
        if (lane_id() == 0) {
            bi = atomicAdd(&bc.ctl[0], 1);
            base = atomicAdd(&bc.ctl[1], nch);
            bc.big_node[bi] = (int32_t)lab;
            bc.big_base[bi] = base;
        }
        bi = __shfl(bi, 0, kWave);
        base = __shfl(base, 0, kWave);
        for (int j = lane_id(); j < nch; j += kWave) bc.item_big[base + j] = bi;
        return;
    }
    if (c == 0) {
        finish_empty(o, lab, leaf, s, split);
        return;
    }
    double g[3];
    box_centre(o, lab, g);
    double sa[4], mx;
    chunk_sums<0>(in, s, (int64_t)s + c, g, g, sa, mx, stage);
    finish_a(o, lab, leaf, sa, mx, split);
    if (leaf) {
        double com[3];
        const double M = sa[0] + 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) com[d] = (sa[1 + d] + 0.0) / M;
        double sb[6], hn;
        chunk_sums<1>(in, s, (int64_t)s + c, g, com, sb, hn, stage);
        finish_b(o, lab, sb, hn);
        return;
    }
    if (!split) return;
    // split: axis and plane as finish_a computed them (recomputed in-wave)
    double lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = o.nlo[3 * lab + d];
        hi[d] = o.nhi[3 * lab + d];
    }
    int ax = 0;
    double best = hi[0] - lo[0];
    if (hi[1] - lo[1] > best) {
        best = hi[1] - lo[1];
        ax = 1;
    }
    if (hi[2] - lo[2] > best) ax = 2;
    const double plane = o.mplane ? o.mplane[lab] : (sa[1 + ax] + 0.0) / (sa[0] + 0.0);
    const int32_t tie = node_tie(o, lab);
    // count the left side first (needed for the right side's base)
    const double *xa = ax == 0 ? in.x : (ax == 1 ? in.y : in.z);
    int nl = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int64_t i = (int64_t)s + 64 * t + lane_id();
        nl += (i < (int64_t)s + c) && goes_left(xa[i], id, i, plane, tie);
    }
    const int nleft = wave_sum_i(nl);
    scatter_chunk(in, id, out, s, (int64_t)s + c, ax, plane, tie, s, nleft, 0, 0);
    if (lane_id() == 0) {
        o.nfirst[2 * lab] = s;
        o.ncount[2 * lab] = nleft;
        o.nfirst[2 * lab + 1] = s + nleft;
        o.ncount[2 * lab + 1] = c - nleft;
    }
}

// One node per wave: every node of the level, or (packed levels) the nodes of
// the groups of npg nodes that k_level_packed left to it (group indices).
template <bool LEAF>
__global__ __launch_bounds__(kBlock) void k_level_small(int lvl, int split, PartIn in,
                                                        const int32_t *__restrict__ id,
                                                        PartOut out, NodeOut o, BigCtl bc,
                                                        const int32_t *__restrict__ groups, int npg) {
    const int64_t w = wave_index();
    const int64_t nodes = (int64_t)1 << lvl;
    int64_t j = w;
    if (groups) {
        if (w / npg >= bc.ctl[2]) return;
        j = (int64_t)groups[w / npg] * npg + w % npg;
    }
    if (j >= nodes) return;
    __shared__ double stage_all[kWavesPerBlock][kStage];
    level_node(nodes + j, LEAF, split != 0, in, id, out, o, bc, stage_all[threadIdx.x / kWave]);
}

// Deep levels: 64 / GW nodes per wave, one per GW-lane group, when all of
// them hold <= 8 GW particles (else the wave's nodes go on a list for
// k_level_small). Lane j of a group holds the node's elements [8 j, 8 j + 8);
// the stable partition ranks come from a scan of the lanes' left counts
// within the group.
template <int GW, bool LEAF>
__global__ __launch_bounds__(kBlock) void k_level_packed(int lvl, int split, PartIn in,
                                                         const int32_t *__restrict__ id,
                                                         PartOut out, NodeOut o, BigCtl bc,
                                                         int32_t *__restrict__ groups) {
    constexpr int kPack = kWave / GW;   // nodes per wave
    __shared__ double stage_all[kBlock / kWave][kStage];
    double *stage = stage_all[threadIdx.x / kWave];
    const int64_t w = wave_index();
    const int64_t nodes = (int64_t)1 << lvl;
    if (w * kPack >= nodes) return;
    const int lane = lane_id();
    const int gslot = lane / GW, gl = lane % GW;
    const int64_t j = w * kPack + gslot;
    const bool valid = j < nodes;
    const int64_t lab = nodes + (valid ? j : 0);
    const int32_t s = o.nfirst[lab];
    const int32_t c = valid ? o.ncount[lab] : 0;
    int cmax = c;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) cmax = max(cmax, __shfl_xor(cmax, off, kWave));
    if (cmax > GW * 8) {
        if (lane == 0) groups[atomicAdd(&bc.ctl[2], 1)] = (int32_t)w;
        return;
    }
    if constexpr (LEAF) {   // moments only: each lane loads its own 8 elements
        if (!valid) return;   // whole groups leave together
        if (c == 0) {
            finish_empty<GW>(o, lab, true, s, split != 0);
            return;
        }
        double g[3];
        box_centre(o, lab, g);
        double sa[4], mx;
        chunk_sums<0, GW>(in, s, (int64_t)s + c, g, g, sa, mx);
        finish_a<GW>(o, lab, true, sa, mx, split != 0);
        double com[3];
        const double M = sa[0] + 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) com[d] = (sa[1 + d] + 0.0) / M;
        double sb[6], hn;
        chunk_sums<1, GW>(in, s, (int64_t)s + c, g, com, sb, hn);
        finish_b<GW>(o, lab, sb, hn);
        return;
    }
    // the wave's nodes hold the contiguous range [w0, wend) (<= kChunk
    // elements), staged through LDS coalesced; every lane takes part, those of
    // absent or empty nodes with no elements
    const int64_t jl = (w * kPack + kPack < nodes ? w * kPack + kPack : nodes) - 1;
    const int64_t w0 = o.nfirst[nodes + w * kPack];
    const int64_t wend = (int64_t)o.nfirst[nodes + jl] + o.ncount[nodes + jl];
    const bool act = valid && c > 0;
    if (valid && c == 0) finish_empty<GW>(o, lab, false, s, split != 0);
    const int64_t e0 = (int64_t)s + 8 * gl, end = (int64_t)s + c;
    double X[8], Y[8], Z[8], Mm[8], H[8];
    {   // all loads first, then the LDS passes
        double rx[8], ry[8], rz[8], rm[8];
        load8c(in.x, w0, wend, rx);
        load8c(in.y, w0, wend, ry);
        load8c(in.z, w0, wend, rz);
        load8c(in.m, w0, wend, rm);
        transpose8(rx, w0, e0, end, stage, X);
        transpose8(ry, w0, e0, end, stage, Y);
        transpose8(rz, w0, e0, end, stage, Z);
        transpose8(rm, w0, e0, end, stage, Mm);
    }
    double g[3];
    box_centre(o, lab, g);
    double sa[4], mx;
    chunk_sums_regs<0, GW>(X, Y, Z, Mm, H, e0, end, g, g, sa, mx);
    if (act) finish_a<GW>(o, lab, false, sa, mx, split != 0);
    if (!split) return;
    int32_t I[8];
    {
        int32_t ri[8];
        load8c(id, w0, wend, ri);
        transpose8(ri, w0, e0, end, (int32_t *)stage, I);
    }
    double lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = o.nlo[3 * lab + d];
        hi[d] = o.nhi[3 * lab + d];
    }
    int ax = 0;
    double best = hi[0] - lo[0];
    if (hi[1] - lo[1] > best) {
        best = hi[1] - lo[1];
        ax = 1;
    }
    if (hi[2] - lo[2] > best) ax = 2;
    const double plane = o.mplane ? o.mplane[lab] : (sa[1 + ax] + 0.0) / (sa[0] + 0.0);
    const int32_t tie = node_tie(o, lab);
    uint32_t lb = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const double xv = ax == 0 ? X[t] : (ax == 1 ? Y[t] : Z[t]);
        if (act && e0 + t < end && (xv < plane || (tie != INT32_MIN && xv == plane && I[t] < tie)))
            lb |= 1u << t;
    }
    const int nl = __popc(lb);
    int incl = nl;   // inclusive scan of the left counts over the group
#pragma unroll
    for (int off = 1; off < GW; off <<= 1) {
        const int y = __shfl_up(incl, off, kWave);
        if (gl >= off) incl += y;
    }
    const int excl = incl - nl;
    const int nleft = __shfl(incl, gslot * GW + GW - 1, kWave);
    int dl[8];   // destination relative to w0, -1: none
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int lbefore = excl + __popc(lb & ((1u << t) - 1u));
        const int e = 8 * gl + t;
        const int64_t dst = (lb >> t) & 1u ? (int64_t)s + lbefore : (int64_t)s + nleft + (e - lbefore);
        dl[t] = act && e0 + t < end ? (int)(dst - w0) : -1;
    }
    scatter8w(out.x, w0, wend, dl, X, stage);
    scatter8w(out.y, w0, wend, dl, Y, stage);
    scatter8w(out.z, w0, wend, dl, Z, stage);
    scatter8w(out.m, w0, wend, dl, Mm, stage);
    scatter8w(out.id, w0, wend, dl, I, (int32_t *)stage);
    if (act && gl == 0) {
        o.nfirst[2 * lab] = s;
        o.ncount[2 * lab] = nleft;
        o.nfirst[2 * lab + 1] = s + nleft;
        o.ncount[2 * lab + 1] = c - nleft;
    }
}

// ---------------------------------------------------------------------------
// big nodes
// ---------------------------------------------------------------------------
// Level counts for the host: big nodes, chunks and the largest node's chunks
// of control block ctl into report[1..3], then the sequence number into
// report[0] (coherent host memory; the host polls it).
__device__ __forceinline__ void write_report(const int32_t *ctl, volatile int32_t *report, int32_t seq) {
    report[1] = ctl[0];
    report[2] = ctl[1];
    report[3] = ctl[3];
    __threadfence_system();
    report[0] = seq;
}

__global__ void k_report(const int32_t *ctl, volatile int32_t *report, int32_t seq) {
    write_report(ctl, report, seq);
}

// report (if given): the counts of bc, which the previous kernel completed
template <int P>
__global__ __launch_bounds__(kBlock) void k_chunk_reduce(PartIn in, NodeOut o, BigCtl bc,
                                                         double *__restrict__ part,
                                                         int32_t *__restrict__ clear_ctl = nullptr,
                                                         volatile int32_t *report = nullptr, int32_t seq = 0) {
    const int64_t w = wave_index();
    if (clear_ctl && blockIdx.x == 0 && threadIdx.x < 4) clear_ctl[threadIdx.x] = 0;
    if (report && blockIdx.x == 0 && threadIdx.x == 0) write_report(bc.ctl, report, seq);
    if (w >= bc.ctl[1]) return;
    const int bi = bc.item_big[w];
    const int64_t lab = bc.big_node[bi];
    const int64_t j = w - bc.big_base[bi];
    const int64_t s = o.nfirst[lab], c = o.ncount[lab];
    const int64_t base = s + j * kChunk;
    const int64_t end = min(base + kChunk, s + c);
    double g[3], com[3] = {0.0, 0.0, 0.0};
    box_centre(o, lab, g);
    if constexpr (P == 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) com[d] = o.ncom[3 * lab + d];
    }
    constexpr int NS = Pay<P>::NS;
    __shared__ double stage_all[kWavesPerBlock][kStage];
    double sums[NS], mx;
    chunk_sums<P>(in, base, end, g, com, sums, mx, stage_all[threadIdx.x / kWave]);
    const int l = lane_id();
    if (l < NS) {
        double v = sums[0];
#pragma unroll
        for (int q = 1; q < NS; ++q)
            if (l == q) v = sums[q];
        part[8 * w + l] = v;
    }
    if (l == 7) part[8 * w + 7] = mx;
}

// Canonical combination of a big node's chunk sums, one block of kFinWaves
// waves per big node. Groups of 64 chunks are summed across lanes (an
// adjacent-pair butterfly); the group count is padded with zero groups to a
// power of two gp, and wave w merges the aligned block of gp / kFinWaves
// groups it owns with a binary-counter stack (equal-size neighbours, left +
// right); the wave results are then merged pairwise. Every step combines
// aligned neighbours, so the result is the canonical pairwise sum.
constexpr int kFinWaves = 16;
constexpr int kFinOneMax = 4 * kWave;
constexpr int kReportSlots = 64;   // level reports, one per level (more than any depth)

// FW = kFinWaves, or 1 (one wave per node) on the levels whose big nodes are
// many and of at most a few groups.
template <int P, int FW = kFinWaves>
__global__ __launch_bounds__(FW * kWave) void k_big_finalize(int leaf_level, int split, NodeOut o,
                                                             BigCtl bc,
                                                             const double *__restrict__ part) {
    constexpr int NS = Pay<P>::NS;
    __shared__ double stk[FW][32][NS];
    __shared__ double res[FW][NS + 1];
    const int wv = threadIdx.x / kWave;
    const int64_t bi = blockIdx.x;
    if (bi >= bc.ctl[0]) return;
    const int64_t lab = bc.big_node[bi];
    const int64_t base = bc.big_base[bi];
    const int64_t c = o.ncount[lab];
    const int64_t nch = (c + kChunk - 1) / kChunk;
    const int64_t ngroups = (nch + kWave - 1) / kWave;
    int64_t gp = 1;
    while (gp < ngroups) gp <<= 1;
    const int64_t per = gp >= FW ? gp / FW : 1;   // groups per wave
    const int active = gp >= FW ? FW : (int)gp;
    if (wv < active) {
        double mx = -1.0;
        for (int64_t k = 0; k < per; ++k) {
            const int64_t gi = wv * per + k;
            const int64_t j = gi * kWave + lane_id();
            double v[NS];
            const bool ok = j < nch;
#pragma unroll
            for (int q = 0; q < NS; ++q) v[q] = ok ? part[8 * (base + j) + q] : 0.0;
            if (ok) mx = fmax(mx, part[8 * (base + j) + 7]);
#pragma unroll
            for (int q = 0; q < NS; ++q) v[q] = wave_sum(v[q]);
            int L = 0;
            while ((k >> L) & 1) {
#pragma unroll
                for (int q = 0; q < NS; ++q) v[q] = stk[wv][L][q] + v[q];
                ++L;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane_id() == 0) {
#pragma unroll
                for (int q = 0; q < NS; ++q) stk[wv][L][q] = v[q];
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        int top = 0;
        while ((1ll << top) < per) ++top;
        mx = wave_max(mx);
        if (lane_id() == 0) {
#pragma unroll
            for (int q = 0; q < NS; ++q) res[wv][q] = stk[wv][top][q];
            res[wv][NS] = mx;
        }
    }
    __syncthreads();
    if (wv != 0) return;
    // pairwise over the active waves' results (a power of two of them)
    double s[NS];
    double mx = -1.0;
    for (int w = 0; w < active; ++w) mx = fmax(mx, res[w][NS]);
    for (int width = 1; width < active; width <<= 1) {
        __builtin_amdgcn_wave_barrier();
        if (lane_id() == 0) {
            for (int w = 0; w + width < active; w += 2 * width)
#pragma unroll
                for (int q = 0; q < NS; ++q) res[w][q] = res[w][q] + res[w + width][q];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) s[q] = res[0][q];
    if constexpr (P == 0) {
        finish_a(o, lab, leaf_level != 0, s, mx, split != 0);
    } else {
        finish_b(o, lab, s, mx);
    }
}

// FIN (levels whose big nodes have at most 64 chunks): each wave first
// combines its node's chunk sums itself, as k_big_finalize<0, 1> does for a
// single group (one chunk per lane, the butterfly), and takes the split from
// them; the node's first chunk writes payload A. Otherwise the split comes
// from k_big_finalize.
template <bool FIN>
__global__ __launch_bounds__(kBlock) void k_part_count(PartIn in, const int32_t *__restrict__ id,
                                                       NodeOut o, BigCtl bc,
                                                       int32_t *__restrict__ part_left,
                                                       const double *__restrict__ part = nullptr) {
    const int64_t w = wave_index();
    if (w >= bc.ctl[1]) return;
    const int bi = bc.item_big[w];
    const int64_t lab = bc.big_node[bi];
    const int64_t j = w - bc.big_base[bi];
    const int64_t s = o.nfirst[lab], c = o.ncount[lab];
    const int64_t base = s + j * kChunk;
    const int64_t end = min(base + kChunk, s + c);
    int ax;
    double plane;
    if constexpr (FIN) {
        const int64_t nch = (c + kChunk - 1) / kChunk;   // <= kWave
        const int64_t p0 = bc.big_base[bi];
        const int l = lane_id();
        const bool ok = l < nch;
        double sv[4], mx = ok ? part[8 * (p0 + l) + 7] : -1.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) sv[q] = wave_sum(ok ? part[8 * (p0 + l) + q] : 0.0);
        mx = wave_max(mx);
        if (j == 0) finish_a(o, lab, false, sv, mx, true);
        double lo[3], hi[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = o.nlo[3 * lab + d];
            hi[d] = o.nhi[3 * lab + d];
        }
        ax = 0;
        double best = hi[0] - lo[0];
        if (hi[1] - lo[1] > best) {
            best = hi[1] - lo[1];
            ax = 1;
        }
        if (hi[2] - lo[2] > best) ax = 2;
        const double M = sv[0] + 0.0;
        const double sa = ax == 0 ? sv[1] : (ax == 1 ? sv[2] : sv[3]);
        plane = o.mplane ? o.mplane[lab] : (sa + 0.0) / M;   // as finish_a
    } else {
        ax = o.naxis[lab];
        plane = o.nplane[lab];
    }
    const int32_t tie = node_tie(o, lab);
    const double *xa = ax == 0 ? in.x : (ax == 1 ? in.y : in.z);
    int nl = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int64_t i = base + 64 * t + lane_id();
        nl += (i < end) && goes_left(xa[i], id, i, plane, tie);
    }
    nl = wave_sum_i(nl);
    if (lane_id() == 0) part_left[w] = nl;
}

// exclusive offsets of a big node's chunk left-counts, one block of
// kFinWaves waves per big node: each wave scans a contiguous run of chunks
// after an exclusive scan of the waves' totals
template <int FW = kFinWaves>
__global__ __launch_bounds__(FW * kWave) void k_part_scan(NodeOut o, BigCtl bc,
                                                          int32_t *__restrict__ part_left) {
    __shared__ int64_t tot[FW];
    const int wv = threadIdx.x / kWave;
    const int64_t bi = blockIdx.x;
    if (bi >= bc.ctl[0]) return;
    const int64_t lab = bc.big_node[bi];
    const int64_t base = bc.big_base[bi];
    const int64_t s = o.nfirst[lab], c = o.ncount[lab];
    const int64_t nch = (c + kChunk - 1) / kChunk;
    const int64_t seg = (nch + FW - 1) / FW;
    const int64_t c0 = wv * seg, c1 = min(nch, c0 + seg);
    int64_t mine = 0;
    for (int64_t g0 = c0; g0 < c1; g0 += kWave) {
        const int64_t j = g0 + lane_id();
        mine += wave_sum_i(j < c1 ? part_left[base + j] : 0);
    }
    if (lane_id() == 0) tot[wv] = mine;
    __syncthreads();
    int64_t run = 0;
    for (int w = 0; w < wv; ++w) run += tot[w];
    for (int64_t g0 = c0; g0 < c1; g0 += kWave) {
        const int64_t j = g0 + lane_id();
        const int v = j < c1 ? part_left[base + j] : 0;
        const int e = wave_excl_scan(v);
        if (j < c1) part_left[base + j] = (int32_t)(run + e);
        run += wave_sum_i(v);
    }
    if (wv == FW - 1 && lane_id() == 0) {
        int64_t all = 0;
        for (int w = 0; w < FW; ++w) all += tot[w];
        o.nfirst[2 * lab] = (int32_t)s;
        o.ncount[2 * lab] = (int32_t)all;
        o.nfirst[2 * lab + 1] = (int32_t)(s + all);
        o.ncount[2 * lab + 1] = (int32_t)(c - all);
    }
}

__device__ __forceinline__ void part_scatter(int64_t w, const PartIn &in, const int32_t *__restrict__ id,
                                             const PartOut &out, const NodeOut &o, const BigCtl &bc,
                                             const int32_t *__restrict__ part_left) {
    if (w >= bc.ctl[1]) return;
    const int bi = bc.item_big[w];
    const int64_t lab = bc.big_node[bi];
    const int64_t j = w - bc.big_base[bi];
    const int64_t s = o.nfirst[lab], c = o.ncount[lab];
    const int64_t base = s + j * kChunk;
    const int64_t end = min(base + kChunk, s + c);
    const int64_t lb = part_left[w];
    const int64_t rb = j * kChunk - lb;
    const int64_t nleft = o.ncount[2 * lab];
    scatter_chunk(in, id, out, base, end, o.naxis[lab], o.nplane[lab], node_tie(o, lab), s, nleft, lb, rb);
}

__global__ __launch_bounds__(kBlock) void k_part_scatter(PartIn in, const int32_t *__restrict__ id,
                                                         PartOut out, NodeOut o, BigCtl bc,
                                                         const int32_t *__restrict__ part_left) {
    part_scatter(wave_index(), in, id, out, o, bc, part_left);
}

constexpr int64_t kUpwardOne = 256;   // levels of at most this many nodes: Eq. 2 in one workgroup

// Eq. 2: parent quadrupole from the non-empty children, shifted by the
// offset between the centres of mass.
__global__ void k_upward(int lvl, NodeOut o) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nodes = (int64_t)1 << lvl;
    if (i >= nodes) return;
    const int64_t lab = nodes + i;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (o.ncount[lab] > 0) {
        const double pc[3] = {o.ncom[3 * lab], o.ncom[3 * lab + 1], o.ncom[3 * lab + 2]};
        for (int ch = 0; ch < 2; ++ch) {
            const int64_t C = 2 * lab + ch;
            if (o.ncount[C] == 0) continue;
            const double dx[3] = {o.ncom[3 * C] - pc[0], o.ncom[3 * C + 1] - pc[1],
                                  o.ncom[3 * C + 2] - pc[2]};
            const double r2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
            const double MC = o.nM[C];
            const double m3 = 3.0 * MC;
            const double mr2 = MC * r2;
            acc[0] += (o.nQ[6 * C + 0] + (m3 * dx[0]) * dx[0]) - mr2;
            acc[1] += o.nQ[6 * C + 1] + (m3 * dx[0]) * dx[1];
            acc[2] += o.nQ[6 * C + 2] + (m3 * dx[0]) * dx[2];
            acc[3] += (o.nQ[6 * C + 3] + (m3 * dx[1]) * dx[1]) - mr2;
            acc[4] += o.nQ[6 * C + 4] + (m3 * dx[1]) * dx[2];
            acc[5] += (o.nQ[6 * C + 5] + (m3 * dx[2]) * dx[2]) - mr2;
        }
    }
    for (int q = 0; q < 6; ++q) o.nQ[6 * lab + q] = acc[q];
}

// walk records: {box centre, h_node_int (-1 if empty)}, {centre of mass, H_B}
__global__ void k_records(int64_t nlab, NodeOut o, double4 *__restrict__ rec) {
    const int64_t lab = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (lab < 1 || lab >= nlab) return;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = o.nlo[3 * lab + d];
        hi[d] = o.nhi[3 * lab + d];
    }
    double hb = hi[0] - lo[0];
    if (hi[1] - lo[1] > hb) hb = hi[1] - lo[1];
    if (hi[2] - lo[2] > hb) hb = hi[2] - lo[2];
    const bool empty = o.ncount[lab] == 0;
    rec[2 * lab] = make_double4(0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2]),
                                empty ? -1.0 : o.nhint[lab]);
    rec[2 * lab + 1] = make_double4(o.ncom[3 * lab], o.ncom[3 * lab + 1], o.ncom[3 * lab + 2], hb);
}

// mixed form: FP32 offsets from the leaf centre of mass, FP32 m and h. One
// wave per 8 consecutive leaves (their particles are contiguous): a lane's
// leaf is the last of the 8 whose first position is <= its own.
__global__ void k_mixed_prep(int64_t nleaf, const int32_t *__restrict__ nfirst,
                             const int32_t *__restrict__ ncount, const double *__restrict__ ncom,
                             const double *__restrict__ px, const double *__restrict__ py,
                             const double *__restrict__ pz, const double *__restrict__ pm,
                             const double *__restrict__ ph, float *__restrict__ fdx,
                             float *__restrict__ fdy, float *__restrict__ fdz,
                             float *__restrict__ fm, float *__restrict__ fh) {
    const int64_t w = wave_index();
    const int64_t L0 = 8 * w;
    if (L0 >= nleaf) return;
    const int nl = nleaf - L0 < 8 ? (int)(nleaf - L0) : 8;
    int32_t f[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = j < nl ? nfirst[nleaf + L0 + j] : INT32_MAX;
    const int64_t s = f[0];
    const int64_t e = (int64_t)nfirst[nleaf + L0 + nl - 1] + ncount[nleaf + L0 + nl - 1];
    for (int64_t i = s + lane_id(); i < e; i += kWave) {
        int j = 0;
#pragma unroll
        for (int q = 1; q < 8; ++q) j += f[q] <= i;
        const int64_t lab = nleaf + L0 + j;
        fdx[i] = (float)(px[i] - ncom[3 * lab]);
        fdy[i] = (float)(py[i] - ncom[3 * lab + 1]);
        fdz[i] = (float)(pz[i] - ncom[3 * lab + 2]);
        fm[i] = (float)pm[i];
        fh[i] = (float)ph[i];
    }
}

// Sec. 2.1 "Updating the tree": has a particle left its lowest-level cell?
// The cell of tree position p is [lo, hi) on each axis (the split rule sends
// coordinate < plane to the lower child), closed at the root box's upper
// faces. Counts the particles whose new position is outside.
__global__ void k_outside(int64_t nleaf, const int32_t *__restrict__ nfirst,
                          const int32_t *__restrict__ ncount, const double *__restrict__ nlo,
                          const double *__restrict__ nhi, const int32_t *__restrict__ pid,
                          const double *__restrict__ x, const double *__restrict__ y,
                          const double *__restrict__ z, unsigned long long *__restrict__ out) {
    const int64_t w = wave_index();
    if (w >= nleaf) return;
    const int64_t lab = nleaf + w;
    const int64_t s = nfirst[lab], c = ncount[lab];
    double lo[3], hi[3], rhi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = nlo[3 * lab + d];
        hi[d] = nhi[3 * lab + d];
        rhi[d] = nhi[3 + d];   // root box (label 1)
    }
    int bad = 0;
    for (int64_t i = s + lane_id(); i < s + c; i += kWave) {
        const int32_t j = pid[i];
        const double r[3] = {x[j], y[j], z[j]};
        bool in = true;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            in = in && r[d] >= lo[d] && (r[d] < hi[d] || (hi[d] == rhi[d] && r[d] == hi[d]));
        bad += !in;
    }
    bad = wave_sum_i(bad);
    if (lane_id() == 0 && bad) atomicAdd(out, (unsigned long long)bad);
}

// ---------------------------------------------------------------------------
// Subtrees. A node is "big" while it holds more than kSubMax particles or
// lies more than kSubDepth levels above the lowest; big nodes go through the
// device-wide chunk passes above, one level per launch. Every node that is
// not big but whose parent is (or the root, if it is not big) is a subtree
// root: one wave finishes its whole subtree down to level k with everything
// in wave-private LDS -- the particles, and per node its range, box, mass,
// centre of mass and quadrupole. Each level's canonical sums, split and
// stable partition run there; node data, each level's particle order and
// the final particle arrays are written to global memory and never read
// back, and the quadrupoles are summed upwards (Eq. 2) from LDS. Roots come
// from a queue filled by the level passes; a persistent grid takes them one
// at a time, so every wave ends when the queue is empty.
// ---------------------------------------------------------------------------
constexpr int kSubMax = kChunk;                 // particles of a subtree root
constexpr int kSubDepth = 6;                    // levels below a subtree root
constexpr int kSubSlots = kSubMax + kSubMax / 8;
constexpr int kSubNodes = (2 << kSubDepth) - 1; // nodes of a subtree: level d, index j at 2^d - 1 + j

__device__ __forceinline__ bool is_big(int32_t c, int k, int lvl) {
    return c > 0 && (c > kSubMax || k - lvl > kSubDepth);
}

// One lane per node of the level (a wave per 64 nodes): the children of the
// previous level's big nodes are sorted into big nodes (registered for this
// level's chunk passes, as level_node does) and subtree roots (queued).
// Nodes below a subtree root are skipped: their parents' counts are still
// zero from the clear at the start of the build.
__global__ __launch_bounds__(kBlock) void k_level_classify(int lvl, int k, NodeOut o, BigCtl bc,
                                                           int32_t *__restrict__ roots,
                                                           int32_t *__restrict__ nroots, int max_big,
                                                           int max_items, int32_t *__restrict__ flag) {
    const int64_t w = wave_index();
    const int64_t nodes = (int64_t)1 << lvl;
    if (w * kWave >= nodes) return;
    const int lane = lane_id();
    const int64_t j = w * kWave + lane;
    const bool valid = j < nodes;
    const int64_t lab = nodes + (valid ? j : 0);
    bool consider = valid && (lvl == 0 || is_big(o.ncount[lab >> 1], k, lvl - 1));
    const int32_t c = consider ? o.ncount[lab] : 0;
    const bool big = consider && is_big(c, k, lvl);
    const bool root = consider && !big;
    const uint64_t br = ballot(root);
    int rbase = 0;
    if (lane == 0 && br) rbase = atomicAdd(nroots, __popcll(br));
    rbase = __shfl(rbase, 0, kWave);
    if (root) roots[rbase + rank_below(br)] = (int32_t)lab;
    int nch = 0, bi = 0, base = 0;
    bool big_ok = big;
    if (big) {
        nch = (c + kChunk - 1) / kChunk;
        bi = atomicAdd(&bc.ctl[0], 1);
        base = atomicAdd(&bc.ctl[1], nch);
        big_ok = bi < max_big && base + nch <= max_items;   // sized on the host; never exceeded
        if (big_ok) {
            bc.big_node[bi] = (int32_t)lab;
            bc.big_base[bi] = base;
        } else {
            atomicOr(flag, 1);
        }
    }
    // the chunk-to-node map of each big node, written by the whole wave
    uint64_t bb = ballot(big_ok);
    while (bb) {
        const int src = __ffsll((long long)bb) - 1;
        bb &= bb - 1;
        const int nc = __shfl(nch, src, kWave), b0 = __shfl(base, src, kWave), id = __shfl(bi, src, kWave);
        for (int q = lane; q < nc; q += kWave) bc.item_big[b0 + q] = id;
    }
}

// The children of the big nodes of level lvl - 1 (one lane each, from that
// level's list bp): sorted into big nodes of level lvl (registered in bn for
// its chunk passes) and subtree roots (queued). The last block to finish
// writes the level's totals (big nodes, chunks) to host memory `report`,
// then the sequence number `seq` that the host waits for.
struct ClassifyArgs {
    int lvl, k;
    BigCtl bp;
    int nparent;
    BigCtl bn;
    int32_t *roots, *nroots;
    int max_big, max_items;
    int32_t *flag;
};

// w: the wave's index among the nblocks workgroups that classify
__device__ __forceinline__ void classify_children(const ClassifyArgs &ca, const NodeOut &o, int64_t w) {
    const int lane = lane_id();
    const int lvl = ca.lvl, k = ca.k, nparent = ca.nparent, max_big = ca.max_big, max_items = ca.max_items;
    const BigCtl &bp = ca.bp, &bn = ca.bn;
    int32_t *__restrict__ roots = ca.roots;
    int32_t *nroots = ca.nroots;
    int32_t *flag = ca.flag;
    const int64_t t = w * kWave + lane;
    // nparent bounds the parents (the grid may be sized before their count is known)
    const int np = min(nparent, bp.ctl[0]);
    const bool valid = t < 2 * (int64_t)np;
    const int64_t lab = valid ? 2 * (int64_t)bp.big_node[t >> 1] + (t & 1) : 0;
    const int32_t c = valid ? o.ncount[lab] : 0;
    const bool big = valid && is_big(c, k, lvl);
    const bool root = valid && !big;
    const uint64_t br = ballot(root);
    // one atomic per wave and counter: the roots, the big nodes and their
    // chunks (ranks and offsets inside the wave from its ballot and scan)
    const uint64_t bg = ballot(big);
    const int nch = big ? (c + kChunk - 1) / kChunk : 0;
    const int cex = wave_excl_scan(nch);
    const int ctot = __shfl(cex + nch, kWave - 1, kWave);
    int mc = nch;   // the level's largest big node, in chunks
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) mc = max(mc, __shfl_xor(mc, off, kWave));
    int rbase = 0, bbase = 0, ibase = 0;
    if (lane == 0) {
        if (br) rbase = atomicAdd(nroots, __popcll(br));
        if (bg) {
            bbase = atomicAdd(&bn.ctl[0], __popcll(bg));
            ibase = atomicAdd(&bn.ctl[1], ctot);
            atomicMax(&bn.ctl[3], mc);
        }
    }
    rbase = __shfl(rbase, 0, kWave);
    if (root) roots[rbase + rank_below(br)] = (int32_t)lab;
    const int bi = __shfl(bbase, 0, kWave) + rank_below(bg);
    const int base = __shfl(ibase, 0, kWave) + cex;
    bool big_ok = big;
    if (big) {
        big_ok = bi < max_big && base + nch <= max_items;   // sized on the host; never exceeded
        if (big_ok) {
            bn.big_node[bi] = (int32_t)lab;
            bn.big_base[bi] = base;
        } else {
            atomicOr(flag, 1);
        }
    }
    uint64_t bb = ballot(big_ok);
    while (bb) {
        const int src = __ffsll((long long)bb) - 1;
        bb &= bb - 1;
        const int nc = __shfl(nch, src, kWave), b0 = __shfl(base, src, kWave), id = __shfl(bi, src, kWave);
        for (int q = lane; q < nc; q += kWave) bn.item_big[b0 + q] = id;
    }
}

// The children's classification and the partition of one level in one
// launch (both need only the scan): workgroups [0, ncls) classify, the
// others scatter, so the classification's atomics run under the scatter's
// memory traffic instead of between two launches. The level's counts reach
// the host from the next kernel in the stream (k_chunk_reduce of the next
// level, or k_report), which sees them complete.
__global__ __launch_bounds__(kBlock) void k_scatter_classify(PartIn in, const int32_t *__restrict__ id, PartOut out,
                                                             NodeOut o, BigCtl bc,
                                                             const int32_t *__restrict__ part_left, int ncls,
                                                             ClassifyArgs ca) {
    if ((int)blockIdx.x < ncls) {
        const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
        classify_children(ca, o, (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)w));
    } else {
        const int64_t w = (int64_t)(blockIdx.x - ncls) * kWavesPerBlock + threadIdx.x / kWave;
        part_scatter((int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)w), in, id, out, o, bc, part_left);
    }
}

struct SubArgs {
    int k;
    int64_t n;
    const int32_t *roots;
    const int32_t *qctl;     // [0] roots queued
    int32_t *qhead;          // next root to take
    double *bx[2], *by[2], *bz[2], *bm[2];   // particle buffers by level parity
    const double *x0, *y0, *z0, *m0;         // level 0: the caller's arrays
    int32_t *lvl_id;
    const double *h;         // the caller's smoothing lengths (caller order)
    double *ph;              // h in tree order, written for the subtree's particles
    NodeOut o;
};

struct SubLds {
    double x[kSubSlots], y[kSubSlots], z[kSubSlots], m[kSubSlots];
    int32_t id[kSubSlots];
    // per node of the subtree (slot 2^d - 1 + j for level l0 + d, label R0 2^d + j)
    int32_t first[kSubNodes], count[kSubNodes];   // first: subtree-relative
    double lo[kSubNodes][3], hi[kSubNodes][3];
    double mass[kSubNodes], com[kSubNodes][3], q[kSubNodes][6];
};

// All descendants of the empty node E (level lvl, first particle `first`,
// box lo/hi) down to level k: empty, with E's box; E's own range and box
// were written by its parent. The whole wave takes part.
__device__ __forceinline__ void fill_empty_subtree(const NodeOut o, int64_t E, int lvl, int k, int32_t first,
                                                  const double (&lo)[3], const double (&hi)[3]) {
    const int l = lane_id();
    double g[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] = 0.5 * (lo[d] + hi[d]);
    for (int j = 0; j <= k - lvl; ++j) {
        const int64_t b = E << j, cnt = (int64_t)1 << j;
        for (int64_t i = l; i < cnt; i += kWave) {
            const int64_t L = b + i;
            if (j > 0) {
                o.nfirst[L] = first;
                o.ncount[L] = 0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    o.nlo[3 * L + d] = lo[d];
                    o.nhi[3 * L + d] = hi[d];
                }
            }
            o.nM[L] = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) o.ncom[3 * L + d] = g[d];
            o.nhint[L] = -1.0;
            o.nhnode[L] = -1.0;
#pragma unroll
            for (int q = 0; q < 6; ++q) o.nQ[6 * L + q] = 0.0;
        }
    }
}

// One pass over up to 64 / GW nodes of subtree level d, GW lanes per node
// (each lane holds 8 consecutive elements of its node, the canonical
// pairwise tree padded to 8 GW): payload A and, for internal nodes, the
// split and the stable partition of the node's elements in LDS (in place:
// the pass's nodes are read completely before any element moves); the
// children's ranges and boxes go to their LDS slots.
// Sum and max over the GW lanes of this lane's group, GW a run-time power
// of two (the same xor butterfly as group_sum / group_max)
__device__ __forceinline__ double gsum(double v, int GW) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1)
        if (o < GW) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double gmax(double v, int GW) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1)
        if (o < GW) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ void sub_pass(const NodeOut o, int k, const double *__restrict__ hin,
                                         double *__restrict__ ph, SubLds &sh, int64_t R0, int d, int p,
                                         int lvl, int64_t s0, float *fdx, float *fdy, float *fdz, float *fm,
                                         float *fh, const int GW) {
    const bool leaf = lvl == k;
    const int lane = lane_id();
    const int gslot = lane / GW, gl = lane % GW;
    const int nd = 1 << d;
    const int j = p + gslot;
    const int slot = nd - 1 + (j < nd ? j : 0);
    const int c = j < nd ? sh.count[slot] : 0;
    const bool valid = c > 0;
    const int f = sh.first[slot];
    const int64_t lab = (R0 << d) + j;
    double lo[3], hi[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        lo[q] = sh.lo[slot][q];
        hi[q] = sh.hi[slot][q];
    }
    const double g[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
    double X[8], Y[8], Z[8], Mm[8], H[8];
    int32_t I[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = 8 * gl + t;
        const bool ok = valid && e < c;
        const int sl = stage_slot(ok ? f + e : 0);
        X[t] = ok ? sh.x[sl] : 0.0;
        Y[t] = ok ? sh.y[sl] : 0.0;
        Z[t] = ok ? sh.z[sl] : 0.0;
        Mm[t] = ok ? sh.m[sl] : 0.0;
        I[t] = ok ? sh.id[sl] : 0;
    }
    // the leaves' smoothing lengths: gathered first, used after payload A
    // (I is 0 past the node)
    if (leaf) {
#pragma unroll
        for (int t = 0; t < 8; ++t) H[t] = hin[I[t]];
    } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) H[t] = 0.0;
    }
    // payload A: m, m x, m y, m z summed by the canonical tree (8 in the
    // lane, then across the group), and max |r - g|^2 (as chunk_sums_regs<0>)
    double sa[4], mx;
    {
        double v[8][4];
        double ml = -1.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (valid && 8 * gl + t < c) {
                v[t][0] = Mm[t];
                v[t][1] = Mm[t] * X[t];
                v[t][2] = Mm[t] * Y[t];
                v[t][3] = Mm[t] * Z[t];
                ml = fmax(ml, dist2(X[t], Y[t], Z[t], g[0], g[1], g[2]));
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) v[t][q] = 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double a0 = (v[0][q] + v[1][q]) + (v[2][q] + v[3][q]);
            const double b0 = (v[4][q] + v[5][q]) + (v[6][q] + v[7][q]);
            sa[q] = gsum(a0 + b0, GW);
        }
        mx = gmax(ml, GW);
    }
    const double M = sa[0] + 0.0;
    double com[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) com[q] = (sa[1 + q] + 0.0) / M;
    const bool lead = valid && gl == 0;
    if (lead) {
        o.nM[lab] = M;
#pragma unroll
        for (int q = 0; q < 3; ++q) o.ncom[3 * lab + q] = com[q];
        o.nhint[lab] = sqrt(mx);
        o.nhnode[lab] = -1.0;
        sh.mass[slot] = M;
#pragma unroll
        for (int q = 0; q < 3; ++q) sh.com[slot][q] = com[q];
    }
    if (leaf) {
        // Eq. 1 about the leaf's centre of mass (each component summed by the
        // same tree as chunk_sums_regs<1>), and h_node
        double ml = -1.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const bool ok = valid && 8 * gl + t < c;
            if (ok) ml = fmax(ml, sqrt(dist2(X[t], Y[t], Z[t], g[0], g[1], g[2])) + 2.0 * H[t]);
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (valid && 8 * gl + t < c) ph[s0 + f + 8 * gl + t] = H[t];
        const double hn = gmax(ml, GW);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            double v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (valid && 8 * gl + t < c) {
                    const double d0 = X[t] - com[0], d1 = Y[t] - com[1], d2 = Z[t] - com[2];
                    const double r2 = (d0 * d0 + d1 * d1) + d2 * d2;
                    const double m3 = 3.0 * Mm[t];
                    const double mr2 = Mm[t] * r2;
                    v[t] = q == 0 ? (m3 * d0) * d0 - mr2 : q == 1 ? (m3 * d0) * d1 : q == 2 ? (m3 * d0) * d2
                         : q == 3 ? (m3 * d1) * d1 - mr2 : q == 4 ? (m3 * d1) * d2 : (m3 * d2) * d2 - mr2;
                } else {
                    v[t] = 0.0;
                }
            }
            const double sq = gsum(((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7])), GW) + 0.0;
            if (lead) {
                o.nQ[6 * lab + q] = sq;
                sh.q[slot][q] = sq;
            }
        }
        if (lead) o.nhnode[lab] = hn;
        if (fdx) {   // mixed form: FP32 offsets from the leaf's centre of mass
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int e = 8 * gl + t;
                if (valid && e < c) {
                    const int64_t i = s0 + f + e;
                    fdx[i] = (float)(X[t] - com[0]);
                    fdy[i] = (float)(Y[t] - com[1]);
                    fdz[i] = (float)(Z[t] - com[2]);
                    fm[i] = (float)Mm[t];
                    fh[i] = (float)H[t];
                }
            }
        }
        return;
    }
    // split through the centre of mass along the longest side
    int ax = 0;
    double best = hi[0] - lo[0];
    if (hi[1] - lo[1] > best) {
        best = hi[1] - lo[1];
        ax = 1;
    }
    if (hi[2] - lo[2] > best) ax = 2;
    const double plane = ax == 0 ? com[0] : (ax == 1 ? com[1] : com[2]);
    uint32_t lb = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const double xv = ax == 0 ? X[t] : (ax == 1 ? Y[t] : Z[t]);
        if (valid && 8 * gl + t < c && xv < plane) lb |= 1u << t;
    }
    const int nl = __popc(lb);
    int incl = nl;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        if (off < GW) {
            const int y = __shfl_up(incl, off, kWave);
            if (gl >= off) incl += y;
        }
    }
    const int excl = incl - nl;
    const int nleft = __shfl(incl, gslot * GW + GW - 1, kWave);
    int dst[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int e = 8 * gl + t;
        const int lbefore = excl + __popc(lb & ((1u << t) - 1u));
        dst[t] = valid && e < c ? ((lb >> t) & 1u ? f + lbefore : f + nleft + (e - lbefore)) : -1;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        if (dst[t] >= 0) {
            const int sl = stage_slot(dst[t]);
            sh.x[sl] = X[t];
            sh.y[sl] = Y[t];
            sh.z[sl] = Z[t];
            sh.m[sl] = Mm[t];
            sh.id[sl] = I[t];
        }
    }
    if (lead) {
        const int64_t L = 2 * lab, R = 2 * lab + 1;
        const int cs = 2 * nd - 1 + 2 * j;   // the children's slots
        o.nfirst[L] = (int32_t)(s0 + f);
        o.ncount[L] = nleft;
        o.nfirst[R] = (int32_t)(s0 + f + nleft);
        o.ncount[R] = c - nleft;
        sh.first[cs] = f;
        sh.count[cs] = nleft;
        sh.first[cs + 1] = f + nleft;
        sh.count[cs + 1] = c - nleft;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double lh = q == ax ? plane : hi[q], rl = q == ax ? plane : lo[q];
            o.nlo[3 * L + q] = lo[q];
            o.nhi[3 * L + q] = lh;
            o.nlo[3 * R + q] = rl;
            o.nhi[3 * R + q] = hi[q];
            sh.lo[cs][q] = lo[q];
            sh.hi[cs][q] = lh;
            sh.lo[cs + 1][q] = rl;
            sh.hi[cs + 1][q] = hi[q];
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// The next subtree root of a wave, fetched in four stages while the wave
// builds the current one, so that each stage's memory latency hides under a
// level of the current build: 0 takes a queue slot, 1 reads its label, 2 the
// root's range and box, 3 issues the loads of its particles (lane l holds
// elements l + 64 q), which the wave puts into LDS when it starts the root.
constexpr int kSubPer = kSubMax / kWave;
struct SubNext {
    int rv;          // lane 0: the queue slot from the atomic
    int r;           // the queue slot (uniform)
    int64_t R0, s0;
    int c0;
    double lo[3], hi[3];
    double vx[kSubPer], vy[kSubPer], vz[kSubPer], vm[kSubPer];
    int32_t vi[kSubPer];
};

__device__ __forceinline__ void next_root_stage(const SubArgs &a, int nq, int stage, SubNext &nx) {
    const int lane = lane_id();
    if (stage == 0) {
        nx.rv = 0;
        if (lane == 0) nx.rv = atomicAdd(a.qhead, 1);
    } else if (stage == 1) {
        nx.r = __builtin_amdgcn_readlane(nx.rv, 0);
        nx.R0 = nx.r < nq ? a.roots[nx.r] : 1;
    } else if (stage == 2) {
        if (nx.r >= nq) return;
        const int64_t R0 = nx.R0;
        nx.s0 = a.o.nfirst[R0];
        nx.c0 = a.o.ncount[R0];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            nx.lo[q] = a.o.nlo[3 * R0 + q];
            nx.hi[q] = a.o.nhi[3 * R0 + q];
        }
    } else {
        if (nx.r >= nq || nx.c0 == 0) return;
        const int l0 = 63 - __clzll((unsigned long long)nx.R0);
        const bool par = l0 & 1;   // buffers chosen by select, not by a dynamic index
        const bool top = l0 == 0;
        const double *ix = top ? a.x0 : (par ? a.bx[1] : a.bx[0]), *iy = top ? a.y0 : (par ? a.by[1] : a.by[0]);
        const double *iz = top ? a.z0 : (par ? a.bz[1] : a.bz[0]), *im = top ? a.m0 : (par ? a.bm[1] : a.bm[0]);
        const int32_t *idl = a.lvl_id + (int64_t)l0 * a.n;
#pragma unroll
        for (int q = 0; q < kSubPer; ++q) {
            const int i = lane + kWave * q;
            const int64_t src = nx.s0 + (i < nx.c0 ? i : 0);
            nx.vx[q] = ix[src];
            nx.vy[q] = iy[src];
            nx.vz[q] = iz[src];
            nx.vm[q] = im[src];
            nx.vi[q] = idl[src];
        }
    }
}

__global__ __launch_bounds__(kWave) void k_subtree(SubArgs a, float *fdx, float *fdy, float *fdz, float *fm,
                                                      float *fh) {
    __shared__ SubLds sh;
    const int lane = lane_id();
    const NodeOut o = a.o;
    const int k = a.k;
    const double *__restrict__ hin = a.h;
    double *__restrict__ ph = a.ph;
    const bool kp = k & 1;
    double *ox = kp ? a.bx[1] : a.bx[0], *oy = kp ? a.by[1] : a.by[0];
    double *oz = kp ? a.bz[1] : a.bz[0], *om = kp ? a.bm[1] : a.bm[0];
    const int nq = a.qctl[0];
    SubNext nx;
    for (int st = 0; st < 4; ++st) next_root_stage(a, nq, st, nx);   // the first root
    for (;;) {
        if (nx.r >= nq) break;
        const int64_t R0 = nx.R0;
        const int l0 = 63 - __clzll((unsigned long long)R0);
        const int64_t s0 = nx.s0;
        const int c0 = nx.c0;
        double rlo[3], rhi[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            rlo[q] = nx.lo[q];
            rhi[q] = nx.hi[q];
        }
        if (c0 == 0) {   // an empty root (at any depth): its whole subtree
            fill_empty_subtree(o, R0, l0, k, (int32_t)s0, rlo, rhi);
            for (int st = 0; st < 4; ++st) next_root_stage(a, nq, st, nx);
            continue;
        }
#pragma unroll
        for (int q = 0; q < kSubPer; ++q) {   // the root's particles, loaded while the last root was built
            const int i = lane + kWave * q;
            if (i < c0) {
                const int sl = stage_slot(i);
                sh.x[sl] = nx.vx[q];
                sh.y[sl] = nx.vy[q];
                sh.z[sl] = nx.vz[q];
                sh.m[sl] = nx.vm[q];
                sh.id[sl] = nx.vi[q];
            }
        }
        int nst = 0;   // the next root's fetch: one stage now, one after each level's passes
        next_root_stage(a, nq, nst++, nx);
        if (lane == 0) {
            sh.first[0] = 0;
            sh.count[0] = c0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                sh.lo[0][q] = rlo[q];
                sh.hi[0][q] = rhi[q];
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int D = k - l0;
        for (int d = 0; d <= D; ++d) {
            const int lvl = l0 + d, nd = 1 << d;
            // empty nodes of this level (their parent sent every element to
            // the other side): their subtrees are filled; nodes below them
            // carry count -1 and are skipped from here on
            const int cl = lane < nd ? sh.count[nd - 1 + lane] : 1;
            uint64_t emp = ballot(d > 0 && cl == 0);
            while (emp) {
                const int j = __ffsll((long long)emp) - 1;
                emp &= emp - 1;
                const int sl = nd - 1 + j;
                double clo[3], chi[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    clo[q] = sh.lo[sl][q];
                    chi[q] = sh.hi[sl][q];
                }
                fill_empty_subtree(o, (R0 << d) + j, lvl, k, (int32_t)(s0 + sh.first[sl]), clo, chi);
            }
            int cm = 0;
            for (int j = lane; j < nd; j += kWave) cm = max(cm, sh.count[nd - 1 + j]);
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) cm = max(cm, __shfl_xor(cm, off, kWave));
            const int gw = cm <= 8 ? 1 : cm <= 16 ? 2 : cm <= 32 ? 4 : cm <= 64 ? 8 : cm <= 128 ? 16
                         : cm <= 256 ? 32 : 64;
            const int npg = kWave / gw;
            float *f0 = lvl == k ? fdx : nullptr;
            if (lvl < k) {   // the next level's slots: -1 unless a non-empty parent sets them
                for (int i = lane; i < 2 * nd; i += kWave) sh.count[2 * nd - 1 + i] = -1;
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
            for (int p = 0; p < nd; p += npg)
                sub_pass(o, k, hin, ph, sh, R0, d, p, lvl, s0, f0, fdy, fdz, fm, fh, gw);
            if (nst < 4) next_root_stage(a, nq, nst++, nx);
            if (lvl == k) break;
            // this level's partition is complete: the next level's order
            for (int i = lane; i < c0; i += kWave)
                a.lvl_id[(int64_t)(lvl + 1) * a.n + s0 + i] = sh.id[stage_slot(i)];
        }
        while (nst < 4) next_root_stage(a, nq, nst++, nx);
        // final particle arrays (level k order)
        for (int i = lane; i < c0; i += kWave) {
            const int sl = stage_slot(i);
            ox[s0 + i] = sh.x[sl];
            oy[s0 + i] = sh.y[sl];
            oz[s0 + i] = sh.z[sl];
            om[s0 + i] = sh.m[sl];
        }
        // Eq. 2 upwards through the subtree's internal levels, from LDS
        for (int d = D - 1; d >= 0; --d) {
            const int nd = 1 << d;
            for (int j = lane; j < nd; j += kWave) {
                const int sl = nd - 1 + j;
                if (sh.count[sl] <= 0) continue;   // Q = 0, written with the empty subtree
                double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                const double pc[3] = {sh.com[sl][0], sh.com[sl][1], sh.com[sl][2]};
                for (int ch = 0; ch < 2; ++ch) {
                    const int cs = 2 * nd - 1 + 2 * j + ch;
                    if (sh.count[cs] <= 0) continue;
                    const double dx[3] = {sh.com[cs][0] - pc[0], sh.com[cs][1] - pc[1], sh.com[cs][2] - pc[2]};
                    const double r2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
                    const double MC = sh.mass[cs];
                    const double m3 = 3.0 * MC;
                    const double mr2 = MC * r2;
                    acc[0] += (sh.q[cs][0] + (m3 * dx[0]) * dx[0]) - mr2;
                    acc[1] += sh.q[cs][1] + (m3 * dx[0]) * dx[1];
                    acc[2] += sh.q[cs][2] + (m3 * dx[0]) * dx[2];
                    acc[3] += (sh.q[cs][3] + (m3 * dx[1]) * dx[1]) - mr2;
                    acc[4] += sh.q[cs][4] + (m3 * dx[1]) * dx[2];
                    acc[5] += (sh.q[cs][5] + (m3 * dx[2]) * dx[2]) - mr2;
                }
                const int64_t lab = (R0 << d) + j;
#pragma unroll
                for (int q6 = 0; q6 < 6; ++q6) {
                    sh.q[sl][q6] = acc[q6];
                    o.nQ[6 * lab + q6] = acc[q6];
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// Eq. 2 for the big nodes of one level (the others are done by their subtree's wave)
__global__ void k_upward_big(int lvl, int k, NodeOut o) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nodes = (int64_t)1 << lvl;
    if (i >= nodes) return;
    const int64_t lab = nodes + i;
    if (!is_big(o.ncount[lab], k, lvl)) return;
    const double pc[3] = {o.ncom[3 * lab], o.ncom[3 * lab + 1], o.ncom[3 * lab + 2]};
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int ch = 0; ch < 2; ++ch) {
        const int64_t C = 2 * lab + ch;
        if (o.ncount[C] == 0) continue;
        const double dx[3] = {o.ncom[3 * C] - pc[0], o.ncom[3 * C + 1] - pc[1], o.ncom[3 * C + 2] - pc[2]};
        const double r2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
        const double MC = o.nM[C];
        const double m3 = 3.0 * MC;
        const double mr2 = MC * r2;
        acc[0] += (o.nQ[6 * C + 0] + (m3 * dx[0]) * dx[0]) - mr2;
        acc[1] += o.nQ[6 * C + 1] + (m3 * dx[0]) * dx[1];
        acc[2] += o.nQ[6 * C + 2] + (m3 * dx[0]) * dx[2];
        acc[3] += (o.nQ[6 * C + 3] + (m3 * dx[1]) * dx[1]) - mr2;
        acc[4] += o.nQ[6 * C + 4] + (m3 * dx[1]) * dx[2];
        acc[5] += (o.nQ[6 * C + 5] + (m3 * dx[2]) * dx[2]) - mr2;
    }
    for (int q = 0; q < 6; ++q) o.nQ[6 * lab + q] = acc[q];
}

// k_upward_big for the levels top .. 0 in one launch: one workgroup, the
// levels in turn (a level reads only the one below it, written before the
// barrier by this workgroup)
__global__ __launch_bounds__(1024) void k_upward_levels(int top, int k, NodeOut o) {
    for (int lvl = top; lvl >= 0; --lvl) {
        const int64_t nodes = (int64_t)1 << lvl;
        for (int64_t i = threadIdx.x; i < nodes; i += blockDim.x) {
            const int64_t lab = nodes + i;
            if (!is_big(o.ncount[lab], k, lvl)) continue;
            const double pc[3] = {o.ncom[3 * lab], o.ncom[3 * lab + 1], o.ncom[3 * lab + 2]};
            double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int ch = 0; ch < 2; ++ch) {
                const int64_t C = 2 * lab + ch;
                if (o.ncount[C] == 0) continue;
                const double dx[3] = {o.ncom[3 * C] - pc[0], o.ncom[3 * C + 1] - pc[1], o.ncom[3 * C + 2] - pc[2]};
                const double r2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
                const double MC = o.nM[C];
                const double m3 = 3.0 * MC;
                const double mr2 = MC * r2;
                acc[0] += (o.nQ[6 * C + 0] + (m3 * dx[0]) * dx[0]) - mr2;
                acc[1] += o.nQ[6 * C + 1] + (m3 * dx[0]) * dx[1];
                acc[2] += o.nQ[6 * C + 2] + (m3 * dx[0]) * dx[2];
                acc[3] += (o.nQ[6 * C + 3] + (m3 * dx[1]) * dx[1]) - mr2;
                acc[4] += o.nQ[6 * C + 4] + (m3 * dx[1]) * dx[2];
                acc[5] += (o.nQ[6 * C + 5] + (m3 * dx[2]) * dx[2]) - mr2;
            }
            for (int q = 0; q < 6; ++q) o.nQ[6 * lab + q] = acc[q];
        }
        __syncthreads();
    }
}

// h in tree order for the big leaves (their order at level k is final);
// the subtree waves write it for their own particles
__global__ __launch_bounds__(kBlock) void k_gather_h_big(const double *__restrict__ h,
                                                         const int32_t *__restrict__ id, NodeOut o, BigCtl bc,
                                                         double *__restrict__ ph) {
    const int64_t w = wave_index();
    if (w >= bc.ctl[1]) return;
    const int bi = bc.item_big[w];
    const int64_t lab = bc.big_node[bi];
    const int64_t j = w - bc.big_base[bi];
    const int64_t s = o.nfirst[lab], c = o.ncount[lab];
    const int64_t base = s + j * kChunk;
    const int64_t end = min(base + kChunk, s + c);
    for (int64_t i = base + lane_id(); i < end; i += kWave) ph[i] = h[id[i]];
}

// k_mixed_prep for the big leaves only (the subtree waves write the FP32
// arrays of their own leaves), one wave per chunk of a big leaf
__global__ __launch_bounds__(kBlock) void k_mixed_big(NodeOut o, BigCtl bc, const double *__restrict__ px,
                                                      const double *__restrict__ py, const double *__restrict__ pz,
                                                      const double *__restrict__ pm, const double *__restrict__ ph,
                                                      float *__restrict__ fdx, float *__restrict__ fdy,
                                                      float *__restrict__ fdz, float *__restrict__ fm,
                                                      float *__restrict__ fh) {
    const int64_t w = wave_index();
    if (w >= bc.ctl[1]) return;
    const int bi = bc.item_big[w];
    const int64_t lab = bc.big_node[bi];
    const int64_t j = w - bc.big_base[bi];
    const int64_t s = o.nfirst[lab], c = o.ncount[lab];
    const int64_t base = s + j * kChunk;
    const int64_t end = min(base + kChunk, s + c);
    const double cx = o.ncom[3 * lab], cy = o.ncom[3 * lab + 1], cz = o.ncom[3 * lab + 2];
    for (int64_t i = base + lane_id(); i < end; i += kWave) {
        fdx[i] = (float)(px[i] - cx);
        fdy[i] = (float)(py[i] - cy);
        fdz[i] = (float)(pz[i] - cz);
        fm[i] = (float)pm[i];
        fh[i] = (float)ph[i];
    }
}


inline unsigned blocks_for_waves(int64_t waves) {
    return (unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
}

// ---------------------------------------------------------------------------
// median position split (Sec. 2.1 "Load balancing"): before a level's pass,
// the particle of rank floor(c/2) of every node in (coordinate, caller
// index) order along the node's split axis, i.e. the first particle of the
// upper child. With this split every node of level l holds floor(n / 2^l)
// or ceil(n / 2^l) particles, so a level is all small (one wave ranks each
// element by counting) or all big (radix select over the 12 bytes of a
// 96-bit key: order-preserving coordinate bits, then the caller index).
// ---------------------------------------------------------------------------
constexpr int kSelSmall = 1024;

__device__ __forceinline__ void tile_sync_build() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ int node_axis(const NodeOut &o, int64_t lab) {
    const double sx = o.nhi[3 * lab] - o.nlo[3 * lab];
    const double sy = o.nhi[3 * lab + 1] - o.nlo[3 * lab + 1];
    const double sz = o.nhi[3 * lab + 2] - o.nlo[3 * lab + 2];
    int ax = 0;
    double best = sx;
    if (sy > best) {
        best = sy;
        ax = 1;
    }
    if (sz > best) ax = 2;
    return ax;
}

// x + 0.0 turns -0 into +0, so numerically equal coordinates get equal keys
__device__ __forceinline__ uint64_t order_key(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x + 0.0);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ __forceinline__ double key_value(uint64_t k) {
    const uint64_t u = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
    return __longlong_as_double((long long)u);
}

// one wave (block) per node of <= kSelSmall particles
__global__ __launch_bounds__(kWave) void k_median_small(int lvl, PartIn in, const int32_t *__restrict__ id,
                                                        NodeOut o, double *__restrict__ mplane,
                                                        int32_t *__restrict__ mtie, int32_t *__restrict__ flag) {
    __shared__ double sx[kSelSmall];
    __shared__ int32_t sid[kSelSmall];
    const int64_t lab = ((int64_t)1 << lvl) + blockIdx.x;
    const int32_t s = o.nfirst[lab], c = o.ncount[lab];
    if (c == 0) return;
    if (c > kSelSmall) {   // cannot happen: node sizes follow from n and the level
        if (threadIdx.x == 0) atomicOr(flag, 1);
        return;
    }
    const int ax = node_axis(o, lab);
    const double *xa = ax == 0 ? in.x : (ax == 1 ? in.y : in.z);
    for (int i = threadIdx.x; i < c; i += kWave) {
        sx[i] = xa[s + i] + 0.0;
        sid[i] = id[s + i];
    }
    __syncthreads();
    const int target = c / 2;
    for (int i = threadIdx.x; i < c; i += kWave) {
        const double xi = sx[i];
        const int32_t ii = sid[i];
        int r = 0;
        for (int j = 0; j < c; ++j) {
            const double xj = sx[j];
            r += (xj < xi) || (xj == xi && sid[j] < ii);
        }
        if (r == target) {
            mplane[lab] = xi;
            mtie[lab] = ii;
        }
    }
}

struct MedSel {
    uint64_t *khi;    // per node of the level: coordinate key bytes found so far
    uint32_t *klo;    // caller-index bytes found so far
    int32_t *rank;    // rank still sought among the elements matching the prefix
    uint32_t *hist;   // 256 bins per node
};

__global__ void k_msel_init(int lvl, NodeOut o, MedSel m) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= ((int64_t)1 << lvl)) return;
    m.khi[j] = 0;
    m.klo[j] = 0;
    m.rank[j] = o.ncount[((int64_t)1 << lvl) + j] / 2;
}

// histogram of byte `pass` over the elements that match the prefix; one
// wave per kChunk elements of a node (cpn waves per node)
__global__ __launch_bounds__(kBlock) void k_msel_hist(int lvl, int cpn, int pass, PartIn in,
                                                      const int32_t *__restrict__ id, NodeOut o, MedSel m) {
    __shared__ uint32_t hist_all[kWavesPerBlock][256];
    uint32_t *hh = hist_all[threadIdx.x / kWave];
    const int64_t nodes = (int64_t)1 << lvl;
    const int64_t w = wave_index();
    if (w >= nodes * cpn) return;
    const int64_t j = w / cpn, ch = w % cpn;
    const int64_t lab = nodes + j;
    const int64_t s = o.nfirst[lab], c = o.ncount[lab];
    const int64_t b0 = s + ch * kChunk, e = min(b0 + kChunk, s + c);
    const int lane = lane_id();
    for (int q = lane; q < 256; q += kWave) hh[q] = 0;
    tile_sync_build();
    if (b0 < e) {
        const int ax = node_axis(o, lab);
        const double *xa = ax == 0 ? in.x : (ax == 1 ? in.y : in.z);
        const uint64_t phi = m.khi[j];
        const uint32_t plo = m.klo[j];
        for (int64_t i = b0 + lane; i < e; i += kWave) {
            const uint64_t kx = order_key(xa[i]);
            const uint32_t kid = (uint32_t)id[i];
            bool match;
            int digit;
            if (pass < 8) {
                match = pass == 0 || (kx >> (64 - 8 * pass)) == (phi >> (64 - 8 * pass));
                digit = (int)((kx >> (56 - 8 * pass)) & 0xffu);
            } else {
                const int p2 = pass - 8;
                match = kx == phi && (p2 == 0 || (kid >> (32 - 8 * p2)) == (plo >> (32 - 8 * p2)));
                digit = (int)((kid >> (24 - 8 * p2)) & 0xffu);
            }
            if (match) atomicAdd(&hh[digit], 1u);
        }
    }
    tile_sync_build();
    for (int q = lane; q < 256; q += kWave)
        if (hh[q]) atomicAdd(&m.hist[j * 256 + q], hh[q]);
}

// the byte of the sought element: the bin where the running count passes
// the rank; bins are cleared for the next pass
__global__ __launch_bounds__(kBlock) void k_msel_pick(int lvl, int pass, MedSel m, double *__restrict__ mplane,
                                                      int32_t *__restrict__ mtie) {
    const int64_t nodes = (int64_t)1 << lvl;
    const int64_t j = wave_index();
    if (j >= nodes) return;
    const int lane = lane_id();
    uint32_t v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = m.hist[j * 256 + 4 * lane + q];
        m.hist[j * 256 + 4 * lane + q] = 0;
    }
    const int tot = (int)(v[0] + v[1] + v[2] + v[3]);
    const int excl = wave_excl_scan(tot);
    const int r = m.rank[j];
    if (excl <= r && r < excl + tot) {
        int acc = excl, d = 4 * lane;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (r < acc + (int)v[q]) {
                d = 4 * lane + q;
                break;
            }
            acc += (int)v[q];
        }
        uint64_t khi = m.khi[j];
        uint32_t klo = m.klo[j];
        if (pass < 8)
            khi |= (uint64_t)d << (56 - 8 * pass);
        else
            klo |= (uint32_t)d << (24 - 8 * (pass - 8));
        m.khi[j] = khi;
        m.klo[j] = klo;
        m.rank[j] = r - acc;
        if (pass == 11) {
            mplane[nodes + j] = key_value(khi);
            mtie[nodes + j] = (int32_t)klo;
        }
    }
}

}  // namespace

static rcb_status big_chain(rcb_tree *t, BuildScratch &b, const NodeOut &o, const BigCtl &bc, int lvl,
                            bool split, const PartIn &in, const int32_t *id, const PartOut &out,
                            hipStream_t s);

// One level's node pass: payload A of every node (and B at the leaf level)
// by small-node, packed and big-node kernels; with split, the partition of
// the big nodes into `out` (the small ones partition themselves).
static rcb_status level_pass(rcb_tree *t, BuildScratch &b, const NodeOut &o, const BigCtl &bc, int lvl,
                             bool split, const PartIn &in, const int32_t *id, const PartOut &out,
                             hipStream_t s) {
    const int64_t n = t->n;
    const bool leaf = lvl == t->k;
    RCB_ZERO(b.ctl, sizeof(int32_t) * 4, s);
    const int64_t nodes = (int64_t)1 << lvl;
    // group width: 8, 16 or 32 lanes per node while the average node
    // holds at most 4 GW particles (capacity 8 GW)
    const int gw = n <= 32 * nodes ? 8 : (n <= 64 * nodes ? 16 : (n <= 128 * nodes ? 32 : 0));
    if (gw) {
        const int npg = kWave / gw;
        const int64_t ng = (nodes + npg - 1) / npg;
        // the leaf level's kernels carry the quadrupole payload; the others
        // are compiled without it (fewer registers)
        auto packed = [&](auto leaf_c) {
            constexpr bool L = decltype(leaf_c)::value;
            if (gw == 8)
                k_level_packed<8, L><<<blocks_for_waves(ng), kBlock, 0, s>>>(lvl, split, in, id, out, o, bc,
                                                                           b.pack_groups);
            else if (gw == 16)
                k_level_packed<16, L><<<blocks_for_waves(ng), kBlock, 0, s>>>(lvl, split, in, id, out, o, bc,
                                                                            b.pack_groups);
            else
                k_level_packed<32, L><<<blocks_for_waves(ng), kBlock, 0, s>>>(lvl, split, in, id, out, o, bc,
                                                                            b.pack_groups);
            k_level_small<L><<<blocks_for_waves(ng * npg), kBlock, 0, s>>>(lvl, split, in, id, out, o, bc,
                                                                         b.pack_groups, npg);
        };
        if (leaf) packed(std::true_type{});
        else packed(std::false_type{});
        RCB_LAUNCH_CHECK("k_level_packed + k_level_small<list>");
    } else {
        if (leaf)
            k_level_small<true><<<blocks_for_waves(nodes), kBlock, 0, s>>>(lvl, split, in, id, out, o, bc,
                                                                         nullptr, 1);
        else
            k_level_small<false><<<blocks_for_waves(nodes), kBlock, 0, s>>>(lvl, split, in, id, out, o, bc,
                                                                          nullptr, 1);
        RCB_LAUNCH_CHECK("k_level_small");
    }
    return big_chain(t, b, o, bc, lvl, split, in, id, out, s);
}

// The big nodes' passes of one level: chunk sums, their canonical
// combination (payload A, and B at the leaf level) and, when splitting, the
// left counts, their scan and the stable scatter.
static rcb_status big_chain(rcb_tree *t, BuildScratch &b, const NodeOut &o, const BigCtl &bc, int lvl,
                            bool split, const PartIn &in, const int32_t *id, const PartOut &out,
                            hipStream_t s) {
    const bool leaf = lvl == t->k;
    const int64_t item_waves = b.max_items;
    const int64_t nodes = (int64_t)1 << lvl;
    const int64_t bw = std::min<int64_t>(b.max_big, nodes);
    k_chunk_reduce<0><<<blocks_for_waves(item_waves), kBlock, 0, s>>>(in, o, bc, b.part);
    RCB_LAUNCH_CHECK("k_chunk_reduce<0>");
    k_big_finalize<0><<<(unsigned)bw, kFinWaves * kWave, 0, s>>>(leaf, split, o, bc, b.part);
    RCB_LAUNCH_CHECK("k_big_finalize<0>");
    if (leaf) {
        k_chunk_reduce<1><<<blocks_for_waves(item_waves), kBlock, 0, s>>>(in, o, bc, b.part);
        RCB_LAUNCH_CHECK("k_chunk_reduce<1>");
        k_big_finalize<1><<<(unsigned)bw, kFinWaves * kWave, 0, s>>>(leaf, split, o, bc, b.part);
        RCB_LAUNCH_CHECK("k_big_finalize<1>");
    } else if (split) {
        k_part_count<false><<<blocks_for_waves(item_waves), kBlock, 0, s>>>(in, id, o, bc, b.part_left);
        RCB_LAUNCH_CHECK("k_part_count");
        k_part_scan<><<<(unsigned)bw, kFinWaves * kWave, 0, s>>>(o, bc, b.part_left);
        RCB_LAUNCH_CHECK("k_part_scan");
        k_part_scatter<<<blocks_for_waves(item_waves), kBlock, 0, s>>>(in, id, out, o, bc,
                                                                       b.part_left);
        RCB_LAUNCH_CHECK("k_part_scatter");
    }
    return RCB_OK;
}

// Level counts written into pinned host memory by the first kernel after the
// classification of the level's nodes; the host polls the sequence number. A
// report that does not arrive within a few seconds, or a stream that has
// failed, ends the wait with an error.
static thread_local int32_t g_level_seq = 0;


static inline bool is_big_host(int64_t c, int k, int lvl) {
    return c > 0 && (c > kSubMax || k - lvl > kSubDepth);
}

static rcb_status finish_build(rcb_tree *t, BuildScratch &b, const NodeOut &o, Scratch &tmp, int cur,
                               hipStream_t s);

// The mixed form's FP32 particle arrays (tree-owned)
static rcb_status alloc_mixed(rcb_tree *t, hipStream_t s) {
    const size_t bytes = sizeof(float) * t->n;
    t->fdx = (float *)dalloc(t, bytes, s, t->allocs);
    t->fdy = (float *)dalloc(t, bytes, s, t->allocs);
    t->fdz = (float *)dalloc(t, bytes, s, t->allocs);
    t->fm = (float *)dalloc(t, bytes, s, t->allocs);
    t->fh = (float *)dalloc(t, bytes, s, t->allocs);
    if (!t->fdx || !t->fdy || !t->fdz || !t->fm || !t->fh) return RCB_ENOMEM;
    return RCB_OK;
}

rcb_status build_tree(rcb_tree *t, const double *x, const double *y, const double *z,
                      const double *m, const double *h, hipStream_t s) {
    const int64_t n = t->n;
    Scratch tmp(t, s);   // build scratch, released when the call returns
    auto A = [&](size_t bytes, std::vector<void *> &owner) { return dalloc(t, bytes, s, owner); };

    // tree-owned arrays
    t->nfirst = (int32_t *)A(sizeof(int32_t) * t->nlab, t->allocs);
    t->ncount = (int32_t *)A(sizeof(int32_t) * t->nlab, t->allocs);
    t->nlo = (double *)A(sizeof(double) * 3 * t->nlab, t->allocs);
    t->nhi = (double *)A(sizeof(double) * 3 * t->nlab, t->allocs);
    t->ncom = (double *)A(sizeof(double) * 3 * t->nlab, t->allocs);
    t->nM = (double *)A(sizeof(double) * t->nlab, t->allocs);
    t->nQ = (double *)A(sizeof(double) * 6 * t->nlab, t->allocs);
    t->nhint = (double *)A(sizeof(double) * t->nlab, t->allocs);
    t->nhnode = (double *)A(sizeof(double) * t->nlab, t->allocs);
    t->wrec = (double4 *)A(sizeof(double4) * 2 * t->nlab, t->allocs);
    t->ph = (double *)A(sizeof(double) * n, t->allocs);
    // particle order (caller indices) at every level; the last one is pid
    t->lvl_id = (int32_t *)A(sizeof(int32_t) * n * (t->k + 1), t->allocs);
    t->dflag = (int32_t *)A(sizeof(int32_t) * 8, t->allocs);
    BuildScratch b{};
    for (int i = 0; i < 2; ++i) {
        b.x[i] = (double *)A(sizeof(double) * n, tmp);
        b.y[i] = (double *)A(sizeof(double) * n, tmp);
        b.z[i] = (double *)A(sizeof(double) * n, tmp);
        b.m[i] = (double *)A(sizeof(double) * n, tmp);
    }
    // big nodes of one level: those of more than kChunk particles, and (fused
    // build) every non-empty node more than kSubDepth levels above the lowest
    const int64_t depth_big = t->k > kSubDepth ? (int64_t)1 << (t->k - kSubDepth - 1) : 0;
    b.max_big = std::min<int64_t>(t->nleaf, std::max<int64_t>(n / (kChunk + 1) + 1, depth_big));
    b.max_items = n / kChunk + b.max_big + 1;
    b.ctl = (int32_t *)A(sizeof(int32_t) * 4, tmp);
    b.big_node = (int32_t *)A(sizeof(int32_t) * b.max_big, tmp);
    b.big_base = (int32_t *)A(sizeof(int32_t) * b.max_big, tmp);
    b.item_big = (int32_t *)A(sizeof(int32_t) * b.max_items, tmp);
    b.part = (double *)A(sizeof(double) * 8 * b.max_items, tmp);
    b.part_left = (int32_t *)A(sizeof(int32_t) * b.max_items, tmp);
    b.pack_groups = (int32_t *)A(sizeof(int32_t) * (t->nleaf / 2 + 1), tmp);
    b.naxis = (int32_t *)A(sizeof(int32_t) * t->nlab, tmp);
    b.nplane = (double *)A(sizeof(double) * t->nlab, tmp);
    const int nbp = (int)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
    b.bounds = (double *)A(sizeof(double) * 6 * nbp, tmp);
    for (void *p : t->allocs)
        if (!p) return RCB_ENOMEM;
    for (void *p : tmp)
        if (!p) return RCB_ENOMEM;

    RCB_ZERO(t->dflag, sizeof(int32_t) * 8, s);
    if (t->p.validate) {
        k_validate<<<nbp, kBlock, 0, s>>>(x, y, z, m, h, n, t->dflag);
        RCB_LAUNCH_CHECK("k_validate");
        int32_t flag = 0;
        RCB_HIP(hipMemcpyAsync(&flag, t->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        RCB_HIP(hipStreamSynchronize(s));
        if (flag) {
            set_error("rcb_build: input has a non-finite coordinate, m <= 0 or h <= 0");
            return RCB_EINPUT;
        }
    }
    const unsigned gN = (unsigned)std::min<int64_t>(4096, (n + kBlock - 1) / kBlock);
    // median split: planes and ties per label, radix-select state for the
    // levels whose nodes exceed kSelSmall (at most n / kSelSmall nodes)
    const bool median = t->p.split == RCB_SPLIT_MEDIAN;
    // splits through a centre (mass or number): big nodes level by level,
    // then every subtree of at most kSubMax particles by one wave; level 0
    // reads the caller's arrays, whose order is the identity
    const bool fused = !median && getenv("RCB_BUILD_LEVELS") == nullptr;
    // control words cleared by k_bounds_final: the roots queue (2), and the
    // big-node control blocks of even and odd levels (4 each)
    int32_t *clr = (int32_t *)A(sizeof(int32_t) * 16, tmp);
    if (!clr) return RCB_ENOMEM;
    int32_t *qctl = clr;   // [0] roots queued, [1] next root to take
    int32_t *roots = nullptr, *bn2 = nullptr, *bb2 = nullptr, *ib2 = nullptr, *dcnt = nullptr;
    // the host learns each level's number of big nodes, chunks and largest
    // node from a report in the level's slot of coherent host memory (kept
    // for the thread's later builds), written by the first kernel after its
    // parent's classification; a level goes into the queue before its
    // report arrives, with grids sized by bounds, and the loop stops at the
    // first level without big nodes
    static thread_local int32_t *hcnt = nullptr;
    if (fused) {   // (everything allocated before the first launch)
        roots = (int32_t *)A(sizeof(int32_t) * t->nleaf, tmp);
        bn2 = (int32_t *)A(sizeof(int32_t) * b.max_big, tmp);
        bb2 = (int32_t *)A(sizeof(int32_t) * b.max_big, tmp);
        ib2 = (int32_t *)A(sizeof(int32_t) * b.max_items, tmp);
        if (!roots || !bn2 || !bb2 || !ib2) return RCB_ENOMEM;
        if (t->p.precision == RCB_MIXED) {   // written by the subtree waves
            rcb_status st = alloc_mixed(t, s);
            if (st != RCB_OK) return st;
        }
        if (!hcnt) {
            if (hipHostMalloc((void **)&hcnt, sizeof(int32_t) * 4 * kReportSlots,
                              hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
                hcnt = nullptr;
                return hip_fail(hipErrorOutOfMemory, "hipHostMalloc(level counts)");
            }
            for (int i = 0; i < 4 * kReportSlots; ++i) hcnt[i] = 0;
        }
        RCB_HIP(hipHostGetDevicePointer((void **)&dcnt, hcnt, 0));   // as seen by the device
    }
    if (!fused) {
        k_init<<<gN, kBlock, 0, s>>>(x, y, z, m, n, b.x[0], b.y[0], b.z[0], b.m[0], t->lvl_id);
        RCB_LAUNCH_CHECK("k_init");
    }
    k_bounds_partial<<<nbp, kBlock, 0, s>>>(x, y, z, n, b.bounds, fused ? t->lvl_id : nullptr);
    RCB_LAUNCH_CHECK("k_bounds_partial");
    k_bounds_final<<<1, 256, 0, s>>>(b.bounds, nbp, t->nlo, t->nhi, t->nfirst, t->ncount, (int32_t)n, clr, 16);
    RCB_LAUNCH_CHECK("k_bounds_final");
    double *mplane = nullptr;
    int32_t *mtie = nullptr;
    MedSel ms{};
    const int64_t max_sel = n / kSelSmall + 1;
    if (median) {
        mplane = (double *)A(sizeof(double) * t->nlab, tmp);
        mtie = (int32_t *)A(sizeof(int32_t) * t->nlab, tmp);
        ms.khi = (uint64_t *)A(sizeof(uint64_t) * max_sel, tmp);
        ms.klo = (uint32_t *)A(sizeof(uint32_t) * max_sel, tmp);
        ms.rank = (int32_t *)A(sizeof(int32_t) * max_sel, tmp);
        ms.hist = (uint32_t *)A(sizeof(uint32_t) * 256 * max_sel, tmp);
        for (void *p : {(void *)mplane, (void *)mtie, (void *)ms.khi, (void *)ms.klo, (void *)ms.rank,
                        (void *)ms.hist})
            if (!p) return RCB_ENOMEM;
        RCB_ZERO(ms.hist, sizeof(uint32_t) * 256 * max_sel, s);
    }
    NodeOut o{t->nfirst, t->ncount, t->nlo, t->nhi, t->ncom, t->nM, t->nhint, t->nhnode, t->nQ,
              b.naxis, b.nplane, mplane, mtie};
    BigCtl bc{b.ctl, b.big_node, b.big_base, b.item_big};
    if (fused) {
        // the control blocks and big-node lists alternate between levels: a
        // level's lists are read by its passes while the next level's are made
        const BigCtl bcs[2] = {BigCtl{clr + 2, b.big_node, b.big_base, b.item_big}, BigCtl{clr + 6, bn2, bb2, ib2}};
        k_level_classify<<<1, kBlock, 0, s>>>(0, t->k, o, bcs[0], roots, qctl, (int)b.max_big, (int)b.max_items,
                                              t->dflag + 5);
        RCB_LAUNCH_CHECK("k_level_classify");
        int64_t nbig = is_big_host((int64_t)n, t->k, 0) ? 1 : 0;
        int64_t nitems = nbig ? (n + kChunk - 1) / kChunk : 0;
        int64_t maxnch = nitems;   // chunks of the level's largest big node
        int cur = 0, last_big = -1;
        // one level's passes (not the lowest), with grids sized from the
        // counts or bounds given; with rseq, its first kernel reports the
        // level's counts into slot lvl (the previous launch completed them)
        auto level = [&](int lvl, int c, int64_t nb, int64_t ni, int64_t mc, int32_t rseq) -> rcb_status {
            const BigCtl &bl = bcs[lvl & 1], &bnx = bcs[(lvl + 1) & 1];
            // level 0 reads the caller's arrays (its order is the identity)
            const PartIn in = lvl == 0 ? PartIn{x, y, z, m, t->ph} : PartIn{b.x[c], b.y[c], b.z[c], b.m[c], t->ph};
            PartOut out{b.x[c ^ 1], b.y[c ^ 1], b.z[c ^ 1], b.m[c ^ 1], t->lvl_id + (int64_t)(lvl + 1) * n};
            const int32_t *id_cur = t->lvl_id + (int64_t)lvl * n;
            const unsigned gi = blocks_for_waves(ni), gb = (unsigned)nb;
            // one wave per node for the combination and the scan once no big
            // node has more than kFinOneMax chunks (else kFinWaves per node)
            const bool one = mc <= kFinOneMax;
            // the combination inside the count pass once no big node has more
            // than one group of chunks
            const bool fin = mc <= kWave;
            k_chunk_reduce<0><<<gi, kBlock, 0, s>>>(in, o, bl, b.part, bnx.ctl, rseq ? dcnt + 4 * lvl : nullptr,
                                                    rseq);
            RCB_LAUNCH_CHECK("k_chunk_reduce<0>");
            if (!fin) {
                if (one) k_big_finalize<0, 1><<<gb, kWave, 0, s>>>(0, 1, o, bl, b.part);
                else k_big_finalize<0><<<gb, kFinWaves * kWave, 0, s>>>(0, 1, o, bl, b.part);
                RCB_LAUNCH_CHECK("k_big_finalize<0>");
            }
            if (fin) k_part_count<true><<<gi, kBlock, 0, s>>>(in, id_cur, o, bl, b.part_left, b.part);
            else k_part_count<false><<<gi, kBlock, 0, s>>>(in, id_cur, o, bl, b.part_left);
            RCB_LAUNCH_CHECK("k_part_count");
            if (one) k_part_scan<1><<<gb, kWave, 0, s>>>(o, bl, b.part_left);
            else k_part_scan<><<<gb, kFinWaves * kWave, 0, s>>>(o, bl, b.part_left);
            RCB_LAUNCH_CHECK("k_part_scan");
            const int ncls = (int)blocks_for_waves((2 * nb + kWave - 1) / kWave);
            const ClassifyArgs ca{lvl + 1, t->k, bl, (int)nb, bnx, roots, qctl, (int)b.max_big, (int)b.max_items,
                                  t->dflag + 5};
            k_scatter_classify<<<ncls + gi, kBlock, 0, s>>>(in, id_cur, out, o, bl, b.part_left, ncls, ca);
            RCB_LAUNCH_CHECK("k_scatter_classify");
            return RCB_OK;
        };
        bool queued = false;   // the level is already in the queue (sized by bounds)
        for (int lvl = 0; lvl <= t->k && nbig > 0; ++lvl) {
            last_big = lvl;
            if (lvl == t->k) {   // the big leaves: their h, payloads A and B
                const BigCtl &bl = bcs[lvl & 1];
                const PartIn in{b.x[cur], b.y[cur], b.z[cur], b.m[cur], t->ph};
                const int32_t *id_cur = t->lvl_id + (int64_t)lvl * n;
                const unsigned gi = blocks_for_waves(nitems), gb = (unsigned)nbig;
                k_gather_h_big<<<gi, kBlock, 0, s>>>(h, id_cur, o, bl, t->ph);
                RCB_LAUNCH_CHECK("k_gather_h_big");
                k_chunk_reduce<0><<<gi, kBlock, 0, s>>>(in, o, bl, b.part);
                RCB_LAUNCH_CHECK("k_chunk_reduce<0>");
                k_big_finalize<0><<<gb, kFinWaves * kWave, 0, s>>>(1, 1, o, bl, b.part);
                RCB_LAUNCH_CHECK("k_big_finalize<0>");
                k_chunk_reduce<1><<<gi, kBlock, 0, s>>>(in, o, bl, b.part);
                RCB_LAUNCH_CHECK("k_chunk_reduce<1>");
                k_big_finalize<1><<<gb, kFinWaves * kWave, 0, s>>>(1, 1, o, bl, b.part);
                RCB_LAUNCH_CHECK("k_big_finalize<1>");
                break;
            }
            if (!queued) {
                rcb_status st = level(lvl, cur, nbig, nitems, maxnch, 0);
                if (st != RCB_OK) return st;
            }
            queued = false;
            cur ^= 1;
            const int32_t seq = ++g_level_seq;
            if (lvl + 1 < t->k) {
                // the next level goes into the queue before this one's counts
                // arrive, so the device does not wait for the host: its grids
                // are sized by bounds (at most two children per big node, one
                // more chunk per big node, no node larger than its parent),
                // and its first kernel reports its counts
                rcb_status st = level(lvl + 1, cur, 2 * nbig, nitems + nbig, maxnch, seq);
                if (st != RCB_OK) return st;
                queued = true;
            } else {
                k_report<<<1, 1, 0, s>>>(bcs[(lvl + 1) & 1].ctl, dcnt + 4 * (lvl + 1), seq);
                RCB_LAUNCH_CHECK("k_report");
            }
            int32_t *rep = hcnt + 4 * (lvl + 1);
            rcb_status ws = wait_host_word(rep, seq, s, "build: level pass");
            if (ws != RCB_OK) return ws;
            nbig = rep[1];
            nitems = rep[2];
            maxnch = rep[3];
            if (nbig > b.max_big || nitems > b.max_items) {
                set_error("rcb_build: internal capacity of the big-node lists exceeded");
                return RCB_EHIP;
            }
        }
        // the particle buffers of level k: every subtree writes its final
        // order there, as the last scatter of the big nodes did
        cur = t->k & 1;
        SubArgs sa{t->k, n, roots, qctl, qctl + 1, {b.x[0], b.x[1]}, {b.y[0], b.y[1]}, {b.z[0], b.z[1]},
                   {b.m[0], b.m[1]}, x, y, z, m, t->lvl_id, h, t->ph, o};
        // mixed form: the subtree waves write the FP32 leaf-frame arrays of
        // their leaves as they finish them, k_mixed_big those of big leaves
        const bool mixed = t->p.precision == RCB_MIXED;
        if (mixed) {
            if (last_big == t->k) {
                const BigCtl &bl = bcs[t->k & 1];
                k_mixed_big<<<blocks_for_waves(nitems), kBlock, 0, s>>>(o, bl, b.x[cur], b.y[cur], b.z[cur],
                                                                      b.m[cur], t->ph, t->fdx, t->fdy, t->fdz,
                                                                      t->fm, t->fh);
                RCB_LAUNCH_CHECK("k_mixed_big");
            }
        }
        const unsigned gsub = (unsigned)std::min<int64_t>(2048, t->nleaf);
        k_subtree<<<gsub, kWave, 0, s>>>(sa, t->fdx, t->fdy, t->fdz, t->fm, t->fh);
        RCB_LAUNCH_CHECK("k_subtree");
        // Eq. 2 for the big nodes: the wide levels one launch each, the
        // levels of at most kUpwardOne nodes in one workgroup
        int lvl = std::min(last_big, t->k - 1);
        for (; lvl >= 0 && ((int64_t)1 << lvl) > kUpwardOne; --lvl) {
            const int64_t nodes = (int64_t)1 << lvl;
            k_upward_big<<<(unsigned)((nodes + 255) / 256), 256, 0, s>>>(lvl, t->k, o);
            RCB_LAUNCH_CHECK("k_upward_big");
        }
        if (lvl >= 0) {
            k_upward_levels<<<1, 1024, 0, s>>>(lvl, t->k, o);
            RCB_LAUNCH_CHECK("k_upward_levels");
        }
        return finish_build(t, b, o, tmp, cur, s);
    }
    int cur = 0;
    for (int lvl = 0; lvl <= t->k; ++lvl) {
        const bool leaf = lvl == t->k;
        if (leaf) {
            k_gather_h<<<gN, kBlock, 0, s>>>(h, t->lvl_id + lvl * n, n, t->ph);
            RCB_LAUNCH_CHECK("k_gather_h");
        }
        PartIn in{b.x[cur], b.y[cur], b.z[cur], b.m[cur], t->ph};
        int32_t *id_next = leaf ? nullptr : t->lvl_id + (int64_t)(lvl + 1) * n;
        PartOut out{b.x[cur ^ 1], b.y[cur ^ 1], b.z[cur ^ 1], b.m[cur ^ 1], id_next};
        const int32_t *id_cur = t->lvl_id + (int64_t)lvl * n;
        if (median && !leaf) {
            const int64_t nodes = (int64_t)1 << lvl;
            const int64_t cmax = (n + nodes - 1) / nodes;   // ceil(n / 2^lvl): the largest node
            if (cmax <= kSelSmall) {
                k_median_small<<<(unsigned)nodes, kWave, 0, s>>>(lvl, in, id_cur, o, mplane, mtie, t->dflag + 5);
                RCB_LAUNCH_CHECK("k_median_small");
            } else {
                const int cpn = (int)((cmax + kChunk - 1) / kChunk);
                k_msel_init<<<(unsigned)((nodes + 255) / 256), 256, 0, s>>>(lvl, o, ms);
                RCB_LAUNCH_CHECK("k_msel_init");
                for (int pass = 0; pass < 12; ++pass) {
                    k_msel_hist<<<blocks_for_waves(nodes * cpn), kBlock, 0, s>>>(lvl, cpn, pass, in, id_cur, o, ms);
                    RCB_LAUNCH_CHECK("k_msel_hist");
                    k_msel_pick<<<blocks_for_waves(nodes), kBlock, 0, s>>>(lvl, pass, ms, mplane, mtie);
                    RCB_LAUNCH_CHECK("k_msel_pick");
                }
            }
        }
        rcb_status st = level_pass(t, b, o, bc, lvl, true, in, id_cur, out, s);
        if (st != RCB_OK) return st;
        if (!leaf) {
            cur ^= 1;
        }
    }
    for (int lvl = t->k - 1; lvl >= 0; --lvl) {
        const int64_t nodes = (int64_t)1 << lvl;
        k_upward<<<(unsigned)((nodes + 255) / 256), 256, 0, s>>>(lvl, o);
        RCB_LAUNCH_CHECK("k_upward");
    }
    return finish_build(t, b, o, tmp, cur, s);
}

// Walk records, the final particle buffers (the other half of the ping-pong
// is released) and the mixed form's FP32 arrays.
static rcb_status finish_build(rcb_tree *t, BuildScratch &b, const NodeOut &o, Scratch &tmp, int cur,
                               hipStream_t s) {
    const int64_t n = t->n;
    auto A = [&](size_t bytes, std::vector<void *> &owner) { return dalloc(t, bytes, s, owner); };
    k_records<<<(unsigned)((t->nlab + 255) / 256), 256, 0, s>>>(t->nlab, o, t->wrec);
    RCB_LAUNCH_CHECK("k_records");

    // keep the final particle buffers; release the other half of the ping-pong
    t->px = b.x[cur];
    t->py = b.y[cur];
    t->pz = b.z[cur];
    t->pm = b.m[cur];
    t->pid = t->lvl_id + (int64_t)t->k * n;
    for (void *p : {(void *)b.x[cur], (void *)b.y[cur], (void *)b.z[cur], (void *)b.m[cur]}) {
        t->allocs.push_back(p);
        tmp.keep(p);
    }
    if (t->p.precision == RCB_MIXED && !t->fdx) {   // (the fused build wrote them already)
        rcb_status st = alloc_mixed(t, s);
        if (st != RCB_OK) return st;
        k_mixed_prep<<<blocks_for_waves((t->nleaf + 7) / 8), kBlock, 0, s>>>(
            t->nleaf, t->nfirst, t->ncount, t->ncom, t->px, t->py, t->pz, t->pm, t->ph, t->fdx,
            t->fdy, t->fdz, t->fm, t->fh);
        RCB_LAUNCH_CHECK("k_mixed_prep");
    }
    return RCB_OK;
}

rcb_status count_outside(rcb_tree *t, const double *x, const double *y, const double *z,
                         int64_t *outside, hipStream_t s) {
    Scratch tmp(t, s);
    unsigned long long *cnt = (unsigned long long *)dalloc(t, sizeof(unsigned long long), s, tmp);
    if (!cnt) return RCB_ENOMEM;
    RCB_ZERO(cnt, sizeof(unsigned long long), s);
    k_outside<<<blocks_for_waves(t->nleaf), kBlock, 0, s>>>(t->nleaf, t->nfirst, t->ncount, t->nlo,
                                                            t->nhi, t->pid, x, y, z, cnt);
    RCB_LAUNCH_CHECK("k_outside");
    unsigned long long h = 0;
    RCB_HIP(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    RCB_HIP(hipStreamSynchronize(s));
    *outside = (int64_t)h;
    return RCB_OK;
}

// Scratch of a moments-only refresh, carved from one block: the gathered
// inputs of a level (4 FP64 per particle) and the big-node machinery of the
// level passes (no partition). Returns the bytes needed; with base != null
// also sets the pointers (each sub-buffer 256-byte aligned).
struct RefreshScratch {
    double *rx, *ry, *rz, *rm;
    BuildScratch b;
};

static size_t refresh_layout(const rcb_tree *t, char *base, RefreshScratch *r) {
    const int64_t n = t->n;
    const int64_t max_big = std::min<int64_t>(t->nleaf, n / (kChunk + 1) + 1);
    const int64_t max_items = n / kChunk + max_big + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? (void *)(base + off) : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    RefreshScratch z{};
    z.rx = (double *)take(sizeof(double) * n);
    z.ry = (double *)take(sizeof(double) * n);
    z.rz = (double *)take(sizeof(double) * n);
    z.rm = (double *)take(sizeof(double) * n);
    z.b.max_big = max_big;
    z.b.max_items = max_items;
    z.b.ctl = (int32_t *)take(sizeof(int32_t) * 4);
    z.b.big_node = (int32_t *)take(sizeof(int32_t) * max_big);
    z.b.big_base = (int32_t *)take(sizeof(int32_t) * max_big);
    z.b.item_big = (int32_t *)take(sizeof(int32_t) * max_items);
    z.b.part = (double *)take(sizeof(double) * 8 * max_items);
    z.b.pack_groups = (int32_t *)take(sizeof(int32_t) * (t->nleaf / 2 + 1));
    if (r) *r = z;
    return off;
}

// Moments-only refresh (the tree held fixed): new inputs in the built order,
// then every node's M, centre of mass, h_node_int, leaf Eq. 1 quadrupole and
// h_node by the same canonical sums as the build, Eq. 2 upwards, and the walk
// records; boxes, splits and ranges stay. The caller decides what happens to
// the interaction lists (rcb_refresh).
static rcb_status refresh_core(rcb_tree *t, const double *x, const double *y, const double *z,
                               const double *m, const double *h, RefreshScratch &r, hipStream_t s) {
    const int64_t n = t->n;
    t->farc_valid = false;   // the kept far coefficients belong to the old moments
    BuildScratch &b = r.b;
    if (t->p.validate) {
        const int nbp = (int)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
        RCB_ZERO(t->dflag, sizeof(int32_t), s);
        k_validate<<<nbp, kBlock, 0, s>>>(x, y, z, m, h, n, t->dflag);
        RCB_LAUNCH_CHECK("k_validate");
        int32_t flag = 0;
        RCB_HIP(hipMemcpyAsync(&flag, t->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        RCB_HIP(hipStreamSynchronize(s));
        if (flag) {
            set_error("rcb_refresh: input has a non-finite coordinate, m <= 0 or h <= 0");
            return RCB_EINPUT;
        }
    }
    const unsigned gN = (unsigned)std::min<int64_t>(4096, (n + kBlock - 1) / kBlock);
    NodeOut o{t->nfirst, t->ncount, t->nlo, t->nhi, t->ncom, t->nM, t->nhint, t->nhnode, t->nQ,
              nullptr, nullptr};
    BigCtl bc{b.ctl, b.big_node, b.big_base, b.item_big};
    const PartOut none{nullptr, nullptr, nullptr, nullptr, nullptr};
    // each level sums its nodes in that level's order of the build (ascending
    // caller index within every node), like the build itself
    for (int lvl = 0; lvl <= t->k; ++lvl) {
        const int32_t *idl = t->lvl_id + (int64_t)lvl * n;
        const bool leaf = lvl == t->k;
        PartIn in{r.rx, r.ry, r.rz, r.rm, nullptr};
        if (leaf) in = PartIn{t->px, t->py, t->pz, t->pm, t->ph};
        k_refresh_gather<<<gN, kBlock, 0, s>>>(x, y, z, m, h, idl, n, (double *)in.x, (double *)in.y,
                                               (double *)in.z, (double *)in.m, leaf ? t->ph : nullptr);
        RCB_LAUNCH_CHECK("k_refresh_gather");
        rcb_status st = level_pass(t, b, o, bc, lvl, false, in, idl, none, s);
        if (st != RCB_OK) return st;
    }
    for (int lvl = t->k - 1; lvl >= 0; --lvl) {
        const int64_t nodes = (int64_t)1 << lvl;
        k_upward<<<(unsigned)((nodes + 255) / 256), 256, 0, s>>>(lvl, o);
        RCB_LAUNCH_CHECK("k_upward");
    }
    k_records<<<(unsigned)((t->nlab + 255) / 256), 256, 0, s>>>(t->nlab, o, t->wrec);
    RCB_LAUNCH_CHECK("k_records");
    if (t->p.precision == RCB_MIXED) {
        k_mixed_prep<<<blocks_for_waves((t->nleaf + 7) / 8), kBlock, 0, s>>>(
            t->nleaf, t->nfirst, t->ncount, t->ncom, t->px, t->py, t->pz, t->pm, t->ph, t->fdx,
            t->fdy, t->fdz, t->fm, t->fh);
        RCB_LAUNCH_CHECK("k_mixed_prep");
    }
    t->nb_total = -1;   // neighbour counts belong to the old positions
    return RCB_OK;
}

rcb_status refresh_tree(rcb_tree *t, const double *x, const double *y, const double *z,
                        const double *m, const double *h, hipStream_t s) {
    Scratch tmp(t, s);
    const size_t bytes = refresh_layout(t, nullptr, nullptr);
    char *base = (char *)dalloc(t, bytes, s, tmp);
    if (!base) return RCB_ENOMEM;
    RefreshScratch r;
    refresh_layout(t, base, &r);
    return refresh_core(t, x, y, z, m, h, r, s);
}

// ---------------------------------------------------------------------------
// Refresh without allocation: the scratch lives in one static device array
// per GPU. Its name is only a host-side stand-in for the symbol; the device
// address is looked up once per device and used everywhere host code needs
// the memory. Calls on one device share the array, so calls that overlap
// race; every buffer that must start at zero is cleared by the level passes.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {nullptr};
}  // namespace

size_t refresh_noalloc_bytes(const rcb_tree *t) { return refresh_layout(t, nullptr, nullptr); }

size_t refresh_noalloc_capacity() { return kNoAllocScratchBytes; }

rcb_status refresh_tree_noalloc(rcb_tree *t, const double *x, const double *y, const double *z,
                                const double *m, const double *h, hipStream_t s) {
    const size_t bytes = refresh_layout(t, nullptr, nullptr);
    if (bytes > kNoAllocScratchBytes) {
        set_error("rcb_refresh_noalloc: the tree needs " + std::to_string(bytes) +
                  " bytes of scratch, more than the " + std::to_string(kNoAllocScratchBytes) +
                  " of the static array (about " + std::to_string(kNoAllocScratchBytes / 33) +
                  " particles); use rcb_refresh");
        return RCB_ECAPACITY;
    }
    int dev = 0;
    RCB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) {
        set_error("rcb_refresh_noalloc: device index out of range");
        return RCB_EINVAL;
    }
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *p = nullptr;
            hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e,
                                                        "hipGetSymbolAddress(scratch)");
            g_scratch_ptr[dev] = p;
        }
        ptr = g_scratch_ptr[dev];
    }
    RefreshScratch r;
    refresh_layout(t, (char *)ptr, &r);
    return refresh_core(t, x, y, z, m, h, r, s);
}

}  // namespace rcb
