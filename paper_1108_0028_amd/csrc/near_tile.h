// near_tile.h -- staging of a group's near-field sources through LDS.
//
// The sources of a group are the particles of the cells on its union near
// list (ascending labels; within a cell, tree order). A wave takes the list
// 64 entries at a time: lane j reads entry j, and an exclusive scan of the
// cell sizes gives each entry's first source index in the chunk. Sources are
// then staged 64 at a time: lane j loads source t + j (its entry found by a
// binary search over the chunk's prefix) into the LDS tile, and every sink
// lane reads the tile back as broadcasts. Entries that the caller does not
// need (for example cells with no candidate bit, for the neighbour search)
// are given zero sources.
#pragma once

#include "rcb_internal.h"

namespace rcb {

struct EntryChunk {
    int32_t fB[kWave];
    int32_t pos[kWave + 1];
    uint32_t mask[kWave];     // near mask (bits 0-7) | candidate mask (bits 8-15)
    int32_t label[kWave];
};

// Loads entries [e0, min(e0 + 64, n1)) into ec; returns the number of sources.
// keep_mask: entries whose (near|cand) mask has no bit of keep_mask count as
// empty.
__device__ __forceinline__ int load_entry_chunk(const uint64_t *__restrict__ gnear,
                                                const int32_t *__restrict__ nfirst,
                                                const int32_t *__restrict__ ncount, int64_t e0,
                                                int64_t n1, uint32_t keep_mask, EntryChunk &ec) {
    const int lane = lane_id();
    const int64_t e = e0 + lane;
    uint64_t ent = 0;
    int32_t cB = 0, fB = 0, lab = 0;
    uint32_t m = 0;
    if (e < n1) {
        ent = gnear[e];
        lab = (int32_t)((uint32_t)ent & 0x7fffffffu);
        m = (uint32_t)(ent >> 32) & 0xffffu;
        if (m & keep_mask) {
            fB = nfirst[lab];
            cB = ncount[lab];
        }
    }
    const int p = wave_excl_scan(cB);
    ec.fB[lane] = fB;
    ec.pos[lane] = p;
    ec.mask[lane] = m;
    ec.label[lane] = lab;
    if (lane == kWave - 1) ec.pos[kWave] = p + cB;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    return __builtin_amdgcn_readfirstlane(ec.pos[kWave]);   // the same on every lane
}

// entry k of the chunk holding source q (largest k with pos[k] <= q)
__device__ __forceinline__ int entry_of(const EntryChunk &ec, int q) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (ec.pos[lo + step] <= q) lo += step;
    return lo;
}

__device__ __forceinline__ void tile_sync() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Lanes of a wave over the sinks of one leaf of c > 0 particles: S = min(c, 64)
// sinks per pass, J = 64 / S slices per sink, lane = sslot * J + slice. Lanes
// with sslot >= S hold no sink. Slice j of a sink takes tile sources
// j, j + J, j + 2J, ...
struct LeafLanes {
    int S, J, sslot, slice;
};
__device__ __forceinline__ LeafLanes leaf_lanes(int c) {
    LeafLanes L;
    L.S = c < kWave ? c : kWave;
    L.J = kWave / L.S;
    L.sslot = lane_id() / L.J;
    L.slice = lane_id() - L.sslot * L.J;
    return L;
}

// Sum over the J consecutive lanes of each segment; the total lands on the
// segment's first lane (slice 0). After the step with offset o, lane i holds
// the sum of its segment's lanes [i, min(i + 2o, end)).
template <typename T>
__device__ __forceinline__ T seg_sum(T v, int slice, int J) {
    for (int o = 1; o < J; o <<= 1) {
        const T w = __shfl_down(v, o, kWave);
        if (slice + o < J) v += w;
    }
    return v;
}

// ballot bits of the lanes of this lane's segment
__device__ __forceinline__ uint64_t seg_mask(const LeafLanes &L) {
    return L.J == kWave ? ~0ull : (((1ull << L.J) - 1ull) << (L.sslot * L.J));
}

}  // namespace rcb
