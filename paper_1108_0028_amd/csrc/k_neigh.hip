// k_neigh.hip -- neighbour search from the walk's candidate cells
// (Sec. 2.3: "Neighbour walk" culled to the true neighbours, and the
// one-dimensional "Neighbour list").
//
// One wave per group of sibling leaves (k_walk.hip), taking the group's
// leaves in turn. Lanes are (sink slot s, slice j) over the leaf's particles
// (near_tile.h: S = min(c, 64) sinks, J = 64 / S slices). The candidate
// cells of the leaf (cells of the group's near list, ascending labels, whose
// candidate mask has the leaf) are staged through LDS 64 particles at a
// time; slice j of sink s tests tile entries j, j + J, .... A pair is a
// neighbour iff b != a and |r_a - r_b|^2 < (2 h_a)^2 in FP64 on the tree's
// copy of the inputs (the same predicate for every precision mode).
// Staging keeps only the sources inside the leaf's sphere (centre g_A,
// radius h_node(A) padded by 2^-32, Sec. 2.3.1): a neighbour b of a sink a
// has |r_b - g_A| <= |r_b - r_a| + |r_a - g_A| < 2 h_a + |r_a - g_A|
// <= h_node(A), so no neighbour is dropped, and the sources that stay are
// compacted in order. Ranks are taken by ballot within the sink's lane
// segment.
//
// The count call writes each particle's count into the caller's offsets
// array (scanned in place afterwards) and its first kNbCap ids into a slab
// row indexed by caller id (by tree position for very large N, see
// tree_rows), the next ones into chunks of a shared pool. The fill call
// streams the slab in caller order,
// sorts each list ascending (a 64-input sorting network held by 8 lanes) and
// stores it into the CSR. Lowest-level cells holding a particle with more
// neighbours than the slab takes (queued by the count call) are searched
// again, one wave each, writing only those particles' lists at their
// offsets; each such list is then sorted by one workgroup.
#include "near_tile.h"
#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
// The search takes one wave per workgroup: the work of a group of cells
// varies tenfold, and a wider workgroup would hold its LDS until its slowest
// wave ends.
constexpr int kSearchWaves = 1;
constexpr int kNbCap = 64;        // slab slots per particle (~50 neighbours expected)
constexpr int kNbChunk = 64;      // slots of an overflow chunk
constexpr int kNbChunks = 3;      // chunks a list may take: lists of up to 256 ids
constexpr int kLongLds = 4096;    // lists searched again: sorted in LDS up to this length
constexpr int kRingMask = 2 * kWave - 1;
constexpr int kRingBytes = 2 * kWave * 32;   // the ring of SrcN, in bytes
constexpr int kVmcnt0 = 0x0f70;   // s_waitcnt vmcnt(0), expcnt and lgkmcnt left free
constexpr int kIcmpUge = 35;      // unsigned >= for __builtin_amdgcn_uicmp

struct NeighArgs {
    int64_t nleaf;
    int gk;
    int64_t ngroup;
    const double4 *rec;       // walk records: rec[2 label] = (box centre, h_node_int)
    const double *hnode;
    const int32_t *nfirst, *ncount;
    const int64_t *gnear_beg, *gnear_end;
    const uint64_t *gnear;
    const double *px, *py, *pz, *ph;
    const int32_t *pid;
    int64_t *counts;          // slab mode: per-particle counts (caller order)
    const int64_t *offsets;   // fill mode: list starts (caller order)
    int32_t *ids;             // fill mode: final lists; slab mode: kNbCap slots per caller index
    int32_t *pool;            // slab mode: overflow chunks of kNbChunk slots
    int32_t *longc;           // slab mode: the kNbChunks chunks of each entry of longq
    int64_t pool_cap;         // chunks in pool
    int32_t *head;            // per caller index: its chunk, or -1 for a list searched again
    int32_t *ctl;             // [0] lists searched again, [1] leaves queued, [2] chunks taken,
                              // [3] lists in chunks (slab mode); [0] lists written (fill mode)
    int32_t *queue;           // leaves (index from 0) holding a list searched again: appended in
                              // slab mode, searched again (wave i: queue[i]) otherwise
    int32_t *longq;           // caller indices: lists in chunks (slab mode), lists written (fill)
    int64_t nq;               // fill mode: entries of queue
    bool tree_rows;           // slab mode: rows by tree position (else by caller index)
};

struct alignas(16) SrcN {
    double x, y, z;
    int32_t pb;   // tree position
    int32_t id;   // caller index
};

// tile: a ring of 128 sources; kept sources accumulate until at least 64 wait
// (at most 127), whole rows are taken and the rest waits; the last partial
// row is padded with sources that can never be neighbours (pb = -1 at
// infinite distance). cnt / chunk: per sink slot of the pass, the
// neighbours found so far (slots are handed out by LDS atomics, so a list is
// stored in no particular order; the fill call sorts it) and its chunk.
struct NeighShared {
    EntryChunk ec;
    SrcN tile[2 * kWave];
    int32_t cnt[kWave];
    int32_t chunk[kWave][kNbChunks];
};

// SLAB: ids go to slab row (caller index) while it has room, then to a chunk
// of the pool taken by the sink's 65th neighbour; lists longer than both, or
// whose chunk could not be had, are only counted, and their leaf is queued.
// Otherwise only the sinks queued that way are searched, their ids going to
// offsets[pid] + slot.
template <bool SLAB>
__global__ __launch_bounds__(kSearchWaves * kWave) void k_neigh(NeighArgs a) {
    __shared__ NeighShared sh_all[kSearchWaves];
    NeighShared &sh = sh_all[threadIdx.x / kWave];
    const int lane = lane_id();
    const int G = 1 << a.gk;
    int64_t gi;
    int li0, li1;   // the group's leaves to search
    if constexpr (SLAB) {
        gi = xcd_wave_index();
        if (gi >= a.ngroup) return;
        li0 = 0;
        li1 = G;
    } else {
        const int64_t q = wave_index();
        if (q >= a.nq) return;
        const int32_t l = a.queue[q];
        gi = l >> a.gk;
        li0 = l & (G - 1);
        li1 = li0 + 1;
    }
    const int64_t GL = (a.nleaf >> a.gk) + gi;
    if (a.ncount[GL] == 0) return;
    const int64_t n0 = a.gnear_beg[gi], n1 = a.gnear_end[gi];
    for (int li = li0; li < li1; ++li) {
        const int64_t A = a.nleaf + gi * G + li;
        const int32_t sA = a.nfirst[A], c = a.ncount[A];
        if (c == 0) continue;
        bool leaf_over = false;   // slab mode: a list of this leaf is searched again
        const LeafLanes L = leaf_lanes(c);
        const double4 gA = a.rec[2 * A];
        const double rA = a.hnode[A] * kReachPad;
        const double rA2 = rA * rA;
        for (int g0 = 0; g0 < c; g0 += L.S) {
            const int si = g0 + L.sslot;
            bool has_sink = L.sslot < L.S && si < c;
            const int32_t pa = sA + (has_sink ? si : 0);
            const int32_t oa = a.pid[pa];
            int64_t obase = (int64_t)(a.tree_rows ? pa : oa) * kNbCap;
            if constexpr (!SLAB) {   // the lists the count call could not keep
                const int64_t o0 = has_sink ? a.offsets[oa] : 0;
                has_sink = has_sink && a.offsets[oa + 1] - o0 > kNbCap && a.head[oa] < 0;
                obase = o0;
                if (ballot(has_sink) == 0ull) continue;
            }
            const double xa = a.px[pa], ya = a.py[pa], za = a.pz[pa];
            const double two_h = 2.0 * a.ph[pa];
            const double lim = has_sink ? two_h * two_h : -1.0;
            if (L.slice == 0) {
                sh.cnt[L.sslot] = 0;
#pragma unroll
                for (int q = 0; q < kNbChunks; ++q) sh.chunk[L.sslot][q] = -1;
            }
            tile_sync();
            int head = 0;   // ring position of the first waiting source
            int32_t *const row = a.ids + obase;
            // hit h with slot r (0 for lanes without a hit): into the slab row, or
            // (rare) one of the sink's chunks, each taken by the hit of its first slot
            auto put = [&](bool h, uint32_t r, int32_t id) {
                const bool low = !SLAB || r < (uint32_t)kNbCap;
                if (h & low) row[r] = id;
                if constexpr (SLAB) {
                    // lanes with r >= kNbCap, as the comparison's own lane mask
                    if (__builtin_amdgcn_uicmp(r, (uint32_t)kNbCap, kIcmpUge) != 0ull) {
                        const uint32_t q = (r - kNbCap) / kNbChunk, o = (r - kNbCap) % kNbChunk;
                        const bool kept = !low && q < (uint32_t)kNbChunks;
                        if (kept && o == 0) {
                            const int32_t ch = atomicAdd(a.ctl + 2, 1);
                            sh.chunk[L.sslot][q] = ch < a.pool_cap ? ch : -2;
                        }
                        tile_sync();
                        if (kept) {
                            const int32_t ch = sh.chunk[L.sslot][q];
                            if (ch >= 0) a.pool[(int64_t)ch * kNbChunk + o] = id;
                        }
                        tile_sync();
                    }
                }
            };
            auto test = [&](const SrcN &src) {
                return (src.pb != pa) & (dist2(xa, ya, za, src.x, src.y, src.z) < lim);
            };
            // the ring as byte offsets: (offset & kRingBytes - 1) wraps it
            auto at = [&](int b) -> const SrcN & {
                return *reinterpret_cast<const SrcN *>(reinterpret_cast<const char *>(sh.tile) +
                                                       (b & (kRingBytes - 1)));
            };
            // rows [0, np) of the waiting sources: slice j of a sink tests j, j + J,
            // ...; two rows per step, so that their LDS traffic overlaps
            auto rows = [&](int np) {
                const int b0 = (head + L.slice) * (int)sizeof(SrcN), bJ = L.J * (int)sizeof(SrcN);
                int u0 = 0;
                for (; u0 + L.J < np; u0 += 2 * L.J) {
                    const int b = b0 + u0 * (int)sizeof(SrcN);
                    const SrcN s0 = at(b), s1 = at(b + bJ);
                    const bool h0 = test(s0), h1 = test(s1);
                    uint32_t r0 = 0, r1 = 0;
                    if (h0) r0 = atomicAdd((uint32_t *)&sh.cnt[L.sslot], 1u);
                    if (h1) r1 = atomicAdd((uint32_t *)&sh.cnt[L.sslot], 1u);
                    put(h0, r0, s0.id);
                    put(h1, r1, s1.id);
                }
                if (u0 < np) {
                    const SrcN s0 = at(b0 + u0 * (int)sizeof(SrcN));
                    const bool h0 = test(s0);
                    uint32_t r0 = 0;
                    if (h0) r0 = atomicAdd((uint32_t *)&sh.cnt[L.sslot], 1u);
                    put(h0, r0, s0.id);
                }
                head = (head + np) & kRingMask;
            };
            int fill = 0;   // kept sources waiting in the ring from head
            for (int64_t e0 = n0; e0 < n1; e0 += kWave) {
                const int tot =
                    load_entry_chunk(a.gnear, a.nfirst, a.ncount, e0, n1, 1u << (8 + li), sh.ec);
                for (int t = 0; t < tot; t += kWave) {
                    const int q = t + lane;
                    double sx = 0.0, sy = 0.0, sz = 0.0;
                    int32_t spb = -1, sid = -1;
                    if (q < tot) {
                        const int k = entry_of(sh.ec, q);
                        const int32_t pb = sh.ec.fB[k] + (q - sh.ec.pos[k]);
                        sx = a.px[pb];
                        sy = a.py[pb];
                        sz = a.pz[pb];
                        spb = pb;
                        sid = a.pid[pb];
                    }
                    const bool keep = q < tot && dist2(gA.x, gA.y, gA.z, sx, sy, sz) < rA2;
                    const uint64_t kb = ballot(keep);
                    if (keep) {   // appended in order after the waiting ones
                        SrcN &dst = sh.tile[(head + fill + rank_below(kb)) & kRingMask];
                        dst.x = sx;
                        dst.y = sy;
                        dst.z = sz;
                        dst.pb = spb;
                        dst.id = sid;
                    }
                    // every gather has landed: otherwise the waits for them (which on
                    // this chip also wait for all earlier stores) are left to the rows
                    __builtin_amdgcn_s_waitcnt(kVmcnt0);
                    const int avail = fill + __popcll(kb);
                    tile_sync();
                    if (avail >= kWave) {   // whole rows only; the rest waits
                        const int np = avail - avail % L.J;
                        rows(np);
                        fill = avail - np;
                        tile_sync();
                    } else {
                        fill = avail;
                    }
                }
            }
            {   // pads the last partial row
                SrcN &dst = sh.tile[(head + fill + lane) & kRingMask];
                dst.x = dst.y = dst.z = __builtin_inf();
                dst.pb = -1;
                dst.id = -1;
            }
            tile_sync();
            rows(fill);
            tile_sync();
            if (SLAB && has_sink && L.slice == 0) {
                const int cnt = sh.cnt[L.sslot];
                a.counts[oa] = cnt;
                if (cnt > kNbCap) {
                    const int need = (cnt - kNbCap + kNbChunk - 1) / kNbChunk;
                    bool ok = need <= kNbChunks;
                    for (int q = 0; ok && q < need; ++q) ok = sh.chunk[L.sslot][q] >= 0;
                    if (ok) {   // at most one entry per chunk taken, so longq has room
                        const int32_t e = atomicAdd(a.ctl + 3, 1);
                        a.longq[e] = oa;
#pragma unroll
                        for (int q = 0; q < kNbChunks; ++q) a.longc[kNbChunks * e + q] = sh.chunk[L.sslot][q];
                        a.head[oa] = e;
                    } else {
                        a.head[oa] = -1;
                        atomicAdd(a.ctl, 1);
                        leaf_over = true;
                    }
                }
            }
            if (!SLAB && has_sink && L.slice == 0) a.longq[atomicAdd(a.ctl, 1)] = oa;
            tile_sync();   // cnt / chunk are reset by the next pass
        }
        if (SLAB && ballot(leaf_over) != 0ull && lane == 0) a.queue[atomicAdd(a.ctl + 1, 1)] = (int32_t)(A - a.nleaf);
    }
}

// caller index -> tree position (slab rows by tree position)
__global__ __launch_bounds__(kBlock) void k_inv(int64_t n, const int32_t *__restrict__ pid,
                                                int32_t *__restrict__ inv) {
    const int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (p < n) inv[pid[p]] = (int32_t)p;
}

// Sorting network on 64 keys, all comparators ascending: for k = 2, 4, ..., 64
// the first stage pairs i with i ^ (k - 1), the following ones i with i ^ d
// (d = k/4, ..., 1); the smaller key goes to the lower index. Key i sits in
// register i % 8 of lane i / 8 of an aligned group of 8 lanes, so strides
// below 8 are exchanges between registers and the others between lanes.
__device__ __forceinline__ void cex(uint32_t &lo, uint32_t &hi) {
    const uint32_t a = lo, b = hi;
    lo = a < b ? a : b;
    hi = a < b ? b : a;
}

// v of lane (lane ^ M) for M < 8, by DPP moves within rows (no LDS path):
// quad permutations give xor 1, 2 and 3, the half-row mirror xor 7, and the
// mirror followed by the quad reversal xor 4.
template <int M>
__device__ __forceinline__ uint32_t xor_lanes(uint32_t v) {
    constexpr int kQuadXor1 = 0xb1, kQuadXor2 = 0x4e, kQuadXor3 = 0x1b, kHalfMirror = 0x141;
    const int x = (int)v;
    if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_mov_dpp(x, kQuadXor1, 0xf, 0xf, true);
    if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_mov_dpp(x, kQuadXor2, 0xf, 0xf, true);
    if constexpr (M == 3) return (uint32_t)__builtin_amdgcn_mov_dpp(x, kQuadXor3, 0xf, 0xf, true);
    if constexpr (M == 7) return (uint32_t)__builtin_amdgcn_mov_dpp(x, kHalfMirror, 0xf, 0xf, true);
    if constexpr (M == 4)
        return (uint32_t)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(x, kHalfMirror, 0xf, 0xf, true),
                                                  kQuadXor3, 0xf, 0xf, true);
    static_assert(M == 1 || M == 2 || M == 3 || M == 4 || M == 7, "lane xor not provided");
    return v;
}

template <int K>
__device__ __forceinline__ void net64_flip(uint32_t (&v)[8], int j0) {
    if constexpr (K <= 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (u < (u ^ (K - 1))) cex(v[u], v[u ^ (K - 1)]);
    } else {
        // partner: lane j0 ^ (K / 8 - 1), register 7 - u
        const bool lower = (j0 & (K >> 4)) == 0;
        uint32_t w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = xor_lanes<(K >> 3) - 1>(v[7 - u]);
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = lower ? (v[u] < w[u] ? v[u] : w[u]) : (v[u] < w[u] ? w[u] : v[u]);
    }
}

template <int D>
__device__ __forceinline__ void net64_stride(uint32_t (&v)[8], int j0) {
    if constexpr (D < 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if ((u & D) == 0) cex(v[u], v[u | D]);
    } else {
        const bool lower = (j0 & (D >> 3)) == 0;   // partner: lane j0 ^ (D / 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t w = xor_lanes<(D >> 3)>(v[u]);
            v[u] = lower ? (v[u] < w ? v[u] : w) : (v[u] < w ? w : v[u]);
        }
    }
}

template <int K>
__device__ __forceinline__ void net64_merge(uint32_t (&v)[8], int j0) {
    net64_flip<K>(v, j0);
    if constexpr (K >= 4) net64_stride<K / 4>(v, j0);
    if constexpr (K >= 8) net64_stride<K / 8>(v, j0);
    if constexpr (K >= 16) net64_stride<K / 16>(v, j0);
    if constexpr (K >= 32) net64_stride<K / 32>(v, j0);
    if constexpr (K >= 64) net64_stride<K / 64>(v, j0);
}

// slab rows -> the caller's CSR, in caller order: 8 lanes per particle, each
// loading 8 consecutive slots of the row (keys past the count are 2^32 - 1,
// i.e. last); the lists are sorted ascending, staged in LDS and stored one
// particle at a time, each list by consecutive lanes. Lists longer than the
// row are the long-list kernels'.
__global__ __launch_bounds__(kBlock) void k_nb_compact(int64_t n, const int32_t *__restrict__ inv,
                                                       const int64_t *__restrict__ offsets,
                                                       const int32_t *__restrict__ slab,
                                                       int32_t *__restrict__ ids) {
    __shared__ uint32_t stage[kWaves][8 * kNbCap];
    uint32_t *st = stage[threadIdx.x / kWave];
    const int lane = lane_id();
    const int64_t a = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / 8;
    const int j0 = lane % 8, p = lane / 8;
    int64_t o = 0, c = 0;
    if (a < n) {
        o = offsets[a];
        c = offsets[a + 1] - o;
        if (c > kNbCap) c = 0;
    }
    uint32_t v[8];
    if (8 * j0 < c) {
        const int64_t r = inv ? (int64_t)inv[a] : a;   // the particle's slab row
        const int4 *src = reinterpret_cast<const int4 *>(slab + r * kNbCap + 8 * j0);
        const int4 x = src[0], y = src[1];
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (8 * j0 + u >= c) v[u] = 0xffffffffu;
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = 0xffffffffu;
    }
    if (ballot(c > 1) != 0ull) {   // wave-uniform: every lane takes part in the exchanges
        net64_merge<2>(v, j0);
        net64_merge<4>(v, j0);
        net64_merge<8>(v, j0);
        net64_merge<16>(v, j0);
        net64_merge<32>(v, j0);
        net64_merge<64>(v, j0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) st[p * kNbCap + 8 * j0 + u] = v[u];
    tile_sync();
#pragma unroll
    for (int q = 0; q < 8; ++q) {   // particle q of the wave: its list by lanes 0 .. c - 1
        const int64_t oq = ((int64_t)__builtin_amdgcn_readlane((int)(o >> 32), 8 * q) << 32) |
                           (uint32_t)__builtin_amdgcn_readlane((int)o, 8 * q);
        const int cq = __builtin_amdgcn_readlane((int)c, 8 * q);
        if (lane < cq) ids[oq + lane] = (int32_t)st[q * kNbCap + lane];
    }
}

// Network of the same kind over P = 2^logP keys in LDS (P <= kLongLds),
// comparators split over the nt threads of the caller (tid < nt); sync() is
// called after each stage.
template <typename Sync>
__device__ __forceinline__ void lds_network(uint32_t *key, int logP, int tid, int nt, Sync sync) {
    const int P = 1 << logP;
    for (int lk = 1; lk <= logP; ++lk) {
        for (int ld = lk - 1; ld >= 0; --ld) {
            const int d = 1 << ld;
            for (int t = tid; t < P / 2; t += nt) {
                const int i = ((t >> ld) << (ld + 1)) | (t & (d - 1));   // bit d of i is clear
                const int j = ld == lk - 1 ? (i ^ ((1 << lk) - 1)) : (i + d);
                const uint32_t x = key[i], y = key[j];
                if (y < x) {
                    key[i] = y;
                    key[j] = x;
                }
            }
            sync();
        }
    }
}

// The same all-ascending network over 64 U keys held U per lane (key i in
// register i % U of lane i / U): strides below U are exchanges between
// registers, the others between lanes (shuffles).
template <int U>
__device__ __forceinline__ void net_lanes(uint32_t (&v)[U], int lane) {
    for (int k = 2; k <= kWave * U; k <<= 1) {
        if (k <= U) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (u < (u ^ (k - 1))) cex(v[u], v[u ^ (k - 1)]);
        } else {   // partner: lane ^ (k / U - 1), register U - 1 - u
            const bool lower = (lane & (k / (2 * U))) == 0;
            uint32_t w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) w[u] = (uint32_t)__shfl_xor((int)v[U - 1 - u], k / U - 1, kWave);
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = lower ? (v[u] < w[u] ? v[u] : w[u]) : (v[u] < w[u] ? w[u] : v[u]);
        }
        for (int d = k / 4; d >= 1; d >>= 1) {
            if (d < U) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if ((u & d) == 0) cex(v[u], v[u | d]);
            } else {   // partner: lane ^ (d / U), same register
                const bool lower = (lane & (d / U)) == 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t w = (uint32_t)__shfl_xor((int)v[u], d / U, kWave);
                    v[u] = lower ? (v[u] < w ? v[u] : w) : (v[u] < w ? w : v[u]);
                }
            }
        }
    }
}

// Lists of kNbCap < c <= kNbCap + kNbChunks kNbChunk ids kept by the count
// call (row plus chunks): one wave per list, 4 keys per lane (16-byte loads:
// lanes 0-15 read the row, every further 16 lanes one chunk), sorted in
// registers.
__global__ __launch_bounds__(kBlock) void k_nb_compact_long(int32_t nlong, const int32_t *__restrict__ inv,
                                                            const int32_t *__restrict__ longq,
                                                            const int64_t *__restrict__ offsets,
                                                            const int32_t *__restrict__ slab,
                                                            const int32_t *__restrict__ longc,
                                                            const int32_t *__restrict__ pool,
                                                            int32_t *__restrict__ ids) {
    static_assert(kNbCap + kNbChunks * kNbChunk == 4 * kWave, "row + chunks = 4 keys per lane");
    const int64_t w = wave_index();
    if (w >= nlong) return;
    const int lane = lane_id();
    const int32_t a = longq[w];
    const int64_t o = offsets[a];
    const int c = (int)(offsets[a + 1] - o);
    const int i0 = 4 * lane;
    uint32_t v[4] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu};
    if (i0 < c) {
        const int32_t *src = i0 < kNbCap
                                 ? slab + (int64_t)(inv ? inv[a] : a) * kNbCap + i0
                                 : pool + (int64_t)longc[kNbChunks * w + (i0 - kNbCap) / kNbChunk] * kNbChunk +
                                       (i0 - kNbCap) % kNbChunk;
        const int4 q = *reinterpret_cast<const int4 *>(src);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u >= c) v[u] = 0xffffffffu;
    }
    net_lanes<4>(v, lane);
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (i0 + u < c) ids[o + i0 + u] = (int32_t)v[u];
}

// One workgroup per list searched again by the fill call: the same network
// over the list's length rounded up to a power of two P, in LDS (padded with
// 2^32 - 1) when P <= kLongLds, else in place in the CSR with the comparators
// that reach past the end left out (with every comparator ascending, keys of
// 2^32 - 1 past the end would never move).
__global__ __launch_bounds__(kBlock) void k_nb_sort_long(const int32_t *__restrict__ longq,
                                                         const int64_t *__restrict__ offsets,
                                                         int32_t *__restrict__ ids) {
    __shared__ uint32_t sm[kLongLds];
    const int32_t a = longq[blockIdx.x];
    const int64_t o = offsets[a], L = offsets[a + 1] - o;
    int logP = 0;
    while (((int64_t)1 << logP) < L) ++logP;
    const int64_t P = (int64_t)1 << logP;
    const int tid = threadIdx.x;
    if (P <= kLongLds) {
        for (int i = tid; i < P; i += kBlock) sm[i] = i < L ? (uint32_t)ids[o + i] : 0xffffffffu;
        __syncthreads();
        lds_network(sm, logP, tid, kBlock, [] { __syncthreads(); });
        for (int i = tid; i < L; i += kBlock) ids[o + i] = (int32_t)sm[i];
        return;
    }
    uint32_t *key = reinterpret_cast<uint32_t *>(ids + o);
    for (int lk = 1; lk <= logP; ++lk) {
        for (int ld = lk - 1; ld >= 0; --ld) {
            const int64_t d = (int64_t)1 << ld;
            for (int64_t t = tid; t < P / 2; t += kBlock) {
                const int64_t i = ((t >> ld) << (ld + 1)) | (t & (d - 1));
                const int64_t j = ld == lk - 1 ? (i ^ (((int64_t)1 << lk) - 1)) : (i + d);
                if (j < L) {
                    const uint32_t x = key[i], y = key[j];
                    if (y < x) {
                        key[i] = y;
                        key[j] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Slab rows go by caller index, so that the fill call streams them in the
// CSR's order; past 4 GiB of slab (16.7M particles) by tree position instead,
// where a wave's rows are contiguous: the search's scattered stores into a
// slab of tens of GB otherwise cost more than reading the rows back through
// the inverse permutation (1e8 particles: 83 -> 73 ms).
bool tree_rows(const rcb_tree *t) { return t->n * kNbCap * (int64_t)sizeof(int32_t) > ((int64_t)4 << 30); }

}  // namespace

// Count: one search that writes every particle's count into offsets (then
// scanned in place) and its ids into the slab row (and a chunk of the pool
// past the row); fill then compacts and sorts those, and searches again only
// the cells holding a list that did not fit.
rcb_status neighbours_count(rcb_tree *t, int64_t *offsets, int64_t *total, hipStream_t s) {
    if (t->lists_kept) {
        set_error("rcb_neighbours_count: the interaction lists were kept across rcb_refresh "
                  "(keep_lists = 1) and may miss neighbours of the new inputs; call rcb_walk first");
        return RCB_ESTATE;
    }
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    if (!t->nb_slab) {
        // one 64-slot chunk for every 8th particle: lists past 64 ids are 3% (Plummer)
        // to 8% (clumps) at ~50 neighbours on average; the rest is searched again by
        // the fill call
        t->nb_pool_cap = t->n / 8 + 1;
        t->nb_slab = (int32_t *)dalloc(t, sizeof(int32_t) * t->n * kNbCap, s, t->list_allocs);
        t->nb_pool = (int32_t *)dalloc(t, sizeof(int32_t) * t->nb_pool_cap * kNbChunk, s, t->list_allocs);
        t->nb_head = (int32_t *)dalloc(t, sizeof(int32_t) * t->n, s, t->list_allocs);
        t->nb_longq = (int32_t *)dalloc(t, sizeof(int32_t) * t->nb_pool_cap, s, t->list_allocs);
        t->nb_longc = (int32_t *)dalloc(t, sizeof(int32_t) * kNbChunks * t->nb_pool_cap, s, t->list_allocs);
        t->nb_queue = (int32_t *)dalloc(t, sizeof(int32_t) * t->nleaf, s, t->list_allocs);
        t->nb_ctl = (int32_t *)dalloc(t, sizeof(int32_t) * 4, s, t->list_allocs);
        if (!t->nb_slab || !t->nb_pool || !t->nb_head || !t->nb_longq || !t->nb_longc || !t->nb_queue ||
            !t->nb_ctl)
            return RCB_ENOMEM;
    }
    RCB_ZERO(t->nb_ctl, sizeof(int32_t) * 4, s);
    NeighArgs a{t->nleaf, t->gk, t->ngroup, t->wrec, t->nhnode, t->nfirst, t->ncount, t->gnear_beg,
                t->gnear_end, t->gnear, t->px, t->py, t->pz, t->ph, t->pid, offsets, nullptr, t->nb_slab,
                t->nb_pool, t->nb_longc, t->nb_pool_cap, t->nb_head, t->nb_ctl, t->nb_queue, t->nb_longq, 0,
                tree_rows(t)};
    const unsigned grid = (unsigned)((t->ngroup + kSearchWaves - 1) / kSearchWaves);
    k_neigh<true><<<grid, kSearchWaves * kWave, 0, s>>>(a);
    RCB_LAUNCH_CHECK("k_neigh<slab>");
    st = scan_i64(t, offsets, offsets, t->n, s);   // in place
    if (st != RCB_OK) return st;
    int32_t ctl[4] = {0, 0, 0, 0};
    const HostRead r[2] = {{offsets + t->n, total, (int)sizeof(int64_t)}, {t->nb_ctl, ctl, (int)sizeof(ctl)}};
    st = read_small(s, r, 2, "rcb_neighbours_count");
    if (st != RCB_OK) return st;
    t->nb_total = *total;
    t->nb_over = ctl[0];
    t->nb_nq = ctl[1];
    t->nb_long = ctl[3];
    return RCB_OK;
}

rcb_status neighbours_fill(rcb_tree *t, const int64_t *offsets, int32_t *ids, int64_t cap,
                           hipStream_t s) {
    if (t->nb_total < 0) {
        set_error("rcb_neighbours_fill: call rcb_neighbours_count on this tree first");
        return RCB_ESTATE;
    }
    if (t->nb_total > cap) {
        set_error("rcb_neighbours_fill: capacity " + std::to_string(cap) + " < total " +
                  std::to_string(t->nb_total));
        return RCB_ECAPACITY;
    }
    Scratch tmp(t, s);
    int32_t *inv = nullptr;   // caller index -> slab row, when rows go by tree position
    if (tree_rows(t)) {
        inv = (int32_t *)dalloc(t, sizeof(int32_t) * t->n, s, tmp);
        if (!inv) return RCB_ENOMEM;
        k_inv<<<(unsigned)((t->n + kBlock - 1) / kBlock), kBlock, 0, s>>>(t->n, t->pid, inv);
        RCB_LAUNCH_CHECK("k_inv");
    }
    const unsigned gridc = (unsigned)((t->n * 8 + kBlock - 1) / kBlock);
    k_nb_compact<<<gridc, kBlock, 0, s>>>(t->n, inv, offsets, t->nb_slab, ids);
    RCB_LAUNCH_CHECK("k_nb_compact");
    if (t->nb_long > 0) {
        const unsigned gl = (unsigned)((t->nb_long + kWaves - 1) / kWaves);
        k_nb_compact_long<<<gl, kBlock, 0, s>>>(t->nb_long, inv, t->nb_longq, offsets, t->nb_slab, t->nb_longc,
                                                t->nb_pool, ids);
        RCB_LAUNCH_CHECK("k_nb_compact_long");
    }
    if (t->nb_nq > 0) {
        int32_t *longq = (int32_t *)dalloc(t, sizeof(int32_t) * (size_t)t->nb_over, s, tmp);
        int32_t *ctl = (int32_t *)dalloc(t, sizeof(int32_t), s, tmp);
        if (!longq || !ctl) return RCB_ENOMEM;
        RCB_ZERO(ctl, sizeof(int32_t), s);
        NeighArgs a{t->nleaf, t->gk, t->ngroup, t->wrec, t->nhnode, t->nfirst, t->ncount, t->gnear_beg,
                    t->gnear_end, t->gnear, t->px, t->py, t->pz, t->ph, t->pid, nullptr, offsets, ids,
                    nullptr, nullptr, 0, t->nb_head, ctl, t->nb_queue, longq, t->nb_nq, false};
        const unsigned grid = (unsigned)((t->nb_nq + kSearchWaves - 1) / kSearchWaves);
        k_neigh<false><<<grid, kSearchWaves * kWave, 0, s>>>(a);
        RCB_LAUNCH_CHECK("k_neigh<fill>");
        // exactly the nb_over lists the count call could not keep append themselves
        k_nb_sort_long<<<(unsigned)t->nb_over, kBlock, 0, s>>>(longq, offsets, ids);
        RCB_LAUNCH_CHECK("k_nb_sort_long");
    }
    return RCB_OK;
}

}  // namespace rcb
