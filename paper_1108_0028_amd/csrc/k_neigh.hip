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
// compacted in order. Ranks
// are taken by ballot within the sink's lane segment, so each list keeps tree
// order. The count call writes the ids into a slab of kNbCap slots per
// particle as well as the counts; the fill call then compacts the slab into
// the caller's CSR; the lowest-level cells holding a particle with more
// neighbours than the slab takes (queued by the count call) are searched
// again, one wave each, writing at offsets[a] + rank.
#include "near_tile.h"
#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int64_t kNbCap = 192;   // slab slots per particle (~50 neighbours expected)

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
    int32_t *ids;             // fill mode: final lists; slab mode: kNbCap slots per particle
    int32_t *flag;            // slab mode: particles with more than kNbCap neighbours
    int32_t *queue;           // leaves (index from 0) holding such a particle: appended in slab
                              // mode, searched again (wave i: queue[i]) otherwise
    int32_t *nqueue;          // slab mode: entries appended
    int64_t nq;               // fill mode: entries to search
};

struct alignas(16) SrcN {
    double x, y, z;
    int32_t pb;   // tree position
    int32_t id;   // caller index
};

// tile: kept sources accumulate until at least 64 wait (at most 127); the
// last partial row is padded with sources that can never be neighbours
// (pb = -1 at infinite distance)
struct NeighShared {
    EntryChunk ec;
    SrcN tile[2 * kWave];
};

// SLAB: ids go to slot (tree position) * kNbCap + rank (ranks >= kNbCap are
// only counted), counts are stored in caller order. Otherwise ids go to
// offsets[pid] + rank.
template <bool SLAB>
__global__ __launch_bounds__(kBlock) void k_neigh(NeighArgs a) {
    __shared__ NeighShared sh_all[kWaves];
    NeighShared &sh = sh_all[threadIdx.x / kWave];
    const int lane = lane_id();
    const int G = 1 << a.gk;
    int64_t gi;
    int li0, li1;   // the group's leaves to search
    if constexpr (SLAB) {
        gi = wave_index();
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
        bool leaf_over = false;   // slab mode: a sink of this leaf outgrew the slab
        const LeafLanes L = leaf_lanes(c);
        const uint64_t segmask = seg_mask(L);
        const double4 gA = a.rec[2 * A];
        const double rA = a.hnode[A] * kReachPad;
        const double rA2 = rA * rA;
        for (int g0 = 0; g0 < c; g0 += L.S) {
            const int si = g0 + L.sslot;
            const bool has_sink = L.sslot < L.S && si < c;
            const int32_t pa = sA + (has_sink ? si : 0);
            const double xa = a.px[pa], ya = a.py[pa], za = a.pz[pa];
            const double two_h = 2.0 * a.ph[pa];
            const double lim = has_sink ? two_h * two_h : -1.0;
            int cnt = 0;
            const int32_t oa = a.pid[pa];
            const int64_t obase = SLAB ? (int64_t)pa * kNbCap : (has_sink ? a.offsets[oa] : 0);
            // rows [0, np) of the tile: slice j of a sink tests entries j, j + J, ...
            auto rows = [&](int np) {
                for (int u0 = 0; u0 < np; u0 += L.J) {
                    const SrcN s = sh.tile[u0 + L.slice];
                    const bool hit = s.pb != pa && dist2(xa, ya, za, s.x, s.y, s.z) < lim;
                    const uint64_t bal = ballot(hit) & segmask;
                    const int r = cnt + rank_below(bal);
                    if (hit && (!SLAB || r < kNbCap)) a.ids[obase + r] = s.id;
                    cnt += __popcll(bal);
                }
            };
            int fill = 0;   // kept sources waiting in tile[0, fill)
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
                        SrcN &dst = sh.tile[fill + rank_below(kb)];
                        dst.x = sx;
                        dst.y = sy;
                        dst.z = sz;
                        dst.pb = spb;
                        dst.id = sid;
                    }
                    const int avail = fill + __popcll(kb);
                    tile_sync();
                    if (avail >= kWave) {   // whole rows only; the rest waits
                        const int np = avail - avail % L.J;
                        rows(np);
                        fill = avail - np;
                        tile_sync();
                        double vx = 0.0, vy = 0.0, vz = 0.0;
                        int32_t vpb = -1, vid = -1;
                        if (lane < fill) {
                            const SrcN &src = sh.tile[np + lane];
                            vx = src.x;
                            vy = src.y;
                            vz = src.z;
                            vpb = src.pb;
                            vid = src.id;
                        }
                        tile_sync();
                        if (lane < fill) {
                            SrcN &dst = sh.tile[lane];
                            dst.x = vx;
                            dst.y = vy;
                            dst.z = vz;
                            dst.pb = vpb;
                            dst.id = vid;
                        }
                        tile_sync();
                    } else {
                        fill = avail;
                    }
                }
            }
            {   // pads the last partial row
                SrcN &dst = sh.tile[fill + lane];
                dst.x = dst.y = dst.z = __builtin_inf();
                dst.pb = -1;
                dst.id = -1;
            }
            tile_sync();
            rows(fill);
            tile_sync();
            if (SLAB && has_sink && L.slice == 0) {
                a.counts[oa] = cnt;
                if (cnt > kNbCap) {
                    atomicAdd(a.flag, 1);
                    leaf_over = true;
                }
            }
        }
        if (SLAB && ballot(leaf_over) != 0ull && lane == 0) a.queue[atomicAdd(a.nqueue, 1)] = (int32_t)(A - a.nleaf);
    }
}

// caller index -> tree position
__global__ __launch_bounds__(kBlock) void k_inv(int64_t n, const int32_t *__restrict__ pid,
                                                int32_t *__restrict__ inv) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) inv[pid[p]] = (int32_t)p;
}

// slab lists -> the caller's CSR, walked in caller order so that the list
// stores and offset loads are contiguous: 8 lanes per particle, each
// loading up to 8 slab entries before its first store
__global__ __launch_bounds__(kBlock) void k_nb_compact(int64_t n, const int32_t *__restrict__ inv,
                                                       const int64_t *__restrict__ offsets,
                                                       const int32_t *__restrict__ slab,
                                                       int32_t *__restrict__ ids) {
    const int64_t a = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / 8;
    const int j0 = threadIdx.x % 8;
    if (a >= n) return;
    const int64_t o = offsets[a], c = offsets[a + 1] - o;
    if (c > kNbCap) return;   // searched again by its group
    const int32_t *row = slab + (int64_t)inv[a] * kNbCap;
    for (int b = 0; b < (int)c; b += 64) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = b + 8 * u + j0;
            v[u] = j < c ? row[j] : 0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = b + 8 * u + j0;
            if (j < c) ids[o + j] = v[u];
        }
    }
}

}  // namespace

// Count: one search that also writes every particle's ids into a slab of
// kNbCap slots; fill then compacts the slab and searches again only the
// groups holding a particle with more neighbours than that.
rcb_status neighbours_count(rcb_tree *t, int64_t *offsets, int64_t *total, hipStream_t s) {
    if (t->lists_kept) {
        set_error("rcb_neighbours_count: the interaction lists were kept across rcb_refresh "
                  "(keep_lists = 1) and may miss neighbours of the new inputs; call rcb_walk first");
        return RCB_ESTATE;
    }
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    Scratch tmp(t, s);
    int64_t *counts = (int64_t *)dalloc(t, sizeof(int64_t) * t->n, s, tmp);
    if (!counts) return RCB_ENOMEM;
    if (!t->nb_slab) {
        t->nb_slab = (int32_t *)dalloc(t, sizeof(int32_t) * t->n * kNbCap, s, t->list_allocs);
        t->nb_queue = (int32_t *)dalloc(t, sizeof(int32_t) * t->nleaf, s, t->list_allocs);
        t->nb_inv = (int32_t *)dalloc(t, sizeof(int32_t) * t->n, s, t->list_allocs);
        if (!t->nb_slab || !t->nb_queue || !t->nb_inv) return RCB_ENOMEM;
    }
    RCB_HIP(hipMemsetAsync(t->dflag + 4, 0, sizeof(int32_t), s));
    RCB_HIP(hipMemsetAsync(t->dflag + 7, 0, sizeof(int32_t), s));
    NeighArgs a{t->nleaf, t->gk, t->ngroup, t->wrec, t->nhnode, t->nfirst, t->ncount, t->gnear_beg,
                t->gnear_end, t->gnear, t->px, t->py, t->pz, t->ph, t->pid, counts, nullptr, t->nb_slab,
                t->dflag + 4, t->nb_queue, t->dflag + 7, 0};
    const unsigned grid = (unsigned)((t->ngroup + kWaves - 1) / kWaves);
    k_neigh<true><<<grid, kBlock, 0, s>>>(a);
    RCB_LAUNCH_CHECK("k_neigh<slab>");
    st = scan_i64(t, counts, offsets, t->n, s);
    if (st != RCB_OK) return st;
    int32_t over[4] = {0, 0, 0, 0};   // dflag[4..7]: particles past the slab, ..., leaves queued
    RCB_HIP(hipMemcpyAsync(total, offsets + t->n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RCB_HIP(hipMemcpyAsync(over, t->dflag + 4, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, s));
    RCB_HIP(hipStreamSynchronize(s));
    t->nb_total = *total;
    t->nb_over = over[0];
    t->nb_nq = over[3];
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
    const unsigned gridc = (unsigned)((t->n * 8 + kBlock - 1) / kBlock);
    k_inv<<<(unsigned)((t->n + kBlock - 1) / kBlock), kBlock, 0, s>>>(t->n, t->pid, t->nb_inv);
    k_nb_compact<<<gridc, kBlock, 0, s>>>(t->n, t->nb_inv, offsets, t->nb_slab, ids);
    RCB_LAUNCH_CHECK("k_nb_compact");
    if (t->nb_nq > 0) {
        NeighArgs a{t->nleaf, t->gk, t->ngroup, t->wrec, t->nhnode, t->nfirst, t->ncount, t->gnear_beg,
                    t->gnear_end, t->gnear, t->px, t->py, t->pz, t->ph, t->pid, nullptr, offsets, ids, nullptr,
                    t->nb_queue, nullptr, t->nb_nq};
        const unsigned grid = (unsigned)((t->nb_nq + kWaves - 1) / kWaves);
        k_neigh<false><<<grid, kBlock, 0, s>>>(a);
        RCB_LAUNCH_CHECK("k_neigh<fill>");
    }
    return RCB_OK;
}

}  // namespace rcb
