// k_neigh.hip -- neighbour search from the walk's candidate cells
// (Sec. 2.3: "Neighbour walk" culled to the true neighbours, and the
// one-dimensional "Neighbour list").
//
// One wave per sink leaf A. Lanes are (sink slot s, slice j): S = the next
// power of two >= min(n_A, 64) sinks, J = 64 / S slices. The wave walks the
// candidate cells in ascending label order; for each cell, slice j of sink s
// tests the particles first_B + t J + j. A pair is a neighbour iff b != a and
// |r_a - r_b|^2 < (2 h_a)^2 in FP64 on the tree's copy of the inputs, the
// same predicate for every precision mode. Count mode writes per-particle
// counts; fill mode writes ids at offsets[a] + rank, ranks taken by ballot
// within the sink's lane segment so each list keeps tree order.
#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;

template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_neigh(int64_t nleaf, const int32_t *__restrict__ nfirst,
                                                  const int32_t *__restrict__ ncount,
                                                  const int64_t *__restrict__ near_off,
                                                  const int32_t *__restrict__ near_list,
                                                  const double *__restrict__ px,
                                                  const double *__restrict__ py,
                                                  const double *__restrict__ pz,
                                                  const double *__restrict__ ph,
                                                  const int32_t *__restrict__ pid,
                                                  int64_t *__restrict__ counts,
                                                  const int64_t *__restrict__ offsets,
                                                  int32_t *__restrict__ ids) {
    const int64_t li = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kWave;
    if (li >= nleaf) return;
    const int lane = lane_id();
    const int64_t A = nleaf + li;
    const int32_t sA = nfirst[A], nA = ncount[A];
    if (nA == 0) return;
    const int64_t l0 = near_off[li], l1 = near_off[li + 1];
    int S = 1;
    while (S < nA && S < kWave) S <<= 1;
    const int J = kWave / S;
    const int sslot = lane / J;   // sink slot
    const int slice = lane % J;
    const uint64_t segmask = (J == 64) ? ~0ull : (((1ull << J) - 1ull) << (sslot * J));
    for (int g0 = 0; g0 < nA; g0 += kWave) {
        const int si = g0 + sslot;
        const bool has_sink = si < nA;
        const int64_t pa = (int64_t)sA + (has_sink ? si : 0);
        const double xa = px[pa], ya = py[pa], za = pz[pa];
        const double two_h = 2.0 * ph[pa];
        const double lim = two_h * two_h;
        int64_t cnt = 0;
        int64_t obase = 0;
        if (FILL && has_sink) obase = offsets[pid[pa]];
        for (int64_t e = l0; e < l1; ++e) {
            const uint32_t ent = (uint32_t)near_list[e];
            if (!(ent >> 31)) continue;
            const int64_t B = ent & 0x7fffffffu;
            const int32_t fB = nfirst[B], cB = ncount[B];
            for (int32_t t0 = 0; t0 < cB; t0 += J) {
                const int32_t ob = t0 + slice;
                const int64_t pb = (int64_t)fB + ob;
                bool hit = false;
                if (has_sink && ob < cB && pb != pa) {
                    hit = dist2(xa, ya, za, px[pb], py[pb], pz[pb]) < lim;
                }
                if (FILL) {
                    const uint64_t bal = ballot(hit) & segmask;
                    if (hit) {
                        const int r = rank_below(bal);
                        ids[obase + cnt + r] = pid[pb];
                    }
                    cnt += __popcll(bal);
                } else {
                    cnt += hit;
                }
            }
        }
        if (!FILL) {
            // reduce the J slices of each sink
            for (int o = 1; o < J; o <<= 1) cnt += __shfl_xor(cnt, o, kWave);
            if (has_sink && slice == 0) counts[pid[pa]] = cnt;
        }
    }
}

}  // namespace

rcb_status neighbours_count(rcb_tree *t, int64_t *offsets, int64_t *total, hipStream_t s) {
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    std::vector<void *> tmp;
    int64_t *counts = (int64_t *)dalloc(t, sizeof(int64_t) * t->n, s, tmp);
    if (!counts) return RCB_ENOMEM;
    const unsigned grid = (unsigned)((t->nleaf + kWaves - 1) / kWaves);
    k_neigh<false><<<grid, kBlock, 0, s>>>(t->nleaf, t->nfirst, t->ncount, t->near_off, t->near_list,
                                           t->px, t->py, t->pz, t->ph, t->pid, counts, nullptr,
                                           nullptr);
    RCB_LAUNCH_CHECK("k_neigh<count>");
    st = scan_i64(t, counts, offsets, t->n, s);
    if (st != RCB_OK) return st;
    RCB_HIP(hipMemcpyAsync(total, offsets + t->n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RCB_HIP(hipFreeAsync(counts, s));
    RCB_HIP(hipStreamSynchronize(s));
    return RCB_OK;
}

rcb_status neighbours_fill(rcb_tree *t, const int64_t *offsets, int32_t *ids, int64_t cap,
                           hipStream_t s) {
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    int64_t total = 0;
    RCB_HIP(hipMemcpyAsync(&total, offsets + t->n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RCB_HIP(hipStreamSynchronize(s));
    if (total > cap) {
        set_error("rcb_neighbours_fill: capacity " + std::to_string(cap) + " < total " +
                  std::to_string(total));
        return RCB_ECAPACITY;
    }
    const unsigned grid = (unsigned)((t->nleaf + kWaves - 1) / kWaves);
    k_neigh<true><<<grid, kBlock, 0, s>>>(t->nleaf, t->nfirst, t->ncount, t->near_off, t->near_list,
                                          t->px, t->py, t->pz, t->ph, t->pid, nullptr, offsets, ids);
    RCB_LAUNCH_CHECK("k_neigh<fill>");
    return RCB_OK;
}

}  // namespace rcb
