// k_sort.hip -- stable sort of 64-bit items by their high 32 bits (a node
// label), one 8-bit digit per pass, least significant digit first.
//
// The deterministic VJP turns the per-group interaction lists into per-node
// lists of the groups that hold each node: the items enter in group order,
// and since every pass keeps equal digits in their input order, each node's
// groups come out ascending. Integer counting only; no floating point.
//
// A wave owns a tile of kTile consecutive items. Per pass:
//   (1) each wave counts the digits of its tile: hist[d * ntile + tile];
//   (2) an exclusive scan of hist (digit-major) gives every (digit, tile)
//       its first output slot;
//   (3) each wave walks its tile in order, 64 items per step: lanes holding
//       equal digits find each other with eight ballots, take consecutive
//       slots in lane order, and the lowest of them advances the digit's
//       slot for the next step.
#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesB = kBlock / kWave;
constexpr int kSteps = 64;
constexpr int64_t kTile = (int64_t)kWave * kSteps;   // items per wave
constexpr int kRadix = 256;

__device__ __forceinline__ uint32_t digit_of(uint64_t v, int shift) {
    return (uint32_t)(v >> (32 + shift)) & (kRadix - 1);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__global__ __launch_bounds__(kBlock) void k_sort_hist(const uint64_t *__restrict__ in, int64_t n,
                                                      int shift, int64_t ntile,
                                                      int64_t *__restrict__ hist) {
    __shared__ uint32_t cnt_all[kWavesB][kRadix];
    uint32_t *cnt = cnt_all[threadIdx.x / kWave];
    const int64_t tile = wave_index();
    if (tile >= ntile) return;
    const int lane = lane_id();
    for (int d = lane; d < kRadix; d += kWave) cnt[d] = 0;
    wave_sync();
    const int64_t t0 = tile * kTile;
    for (int st = 0; st < kSteps; ++st) {
        const int64_t i = t0 + st * kWave + lane;
        if (i < n) atomicAdd(&cnt[digit_of(in[i], shift)], 1u);
    }
    wave_sync();
    for (int d = lane; d < kRadix; d += kWave) hist[d * ntile + tile] = cnt[d];
}

__global__ __launch_bounds__(kBlock) void k_sort_scatter(const uint64_t *__restrict__ in,
                                                         uint64_t *__restrict__ out, int64_t n,
                                                         int shift, int64_t ntile,
                                                         const int64_t *__restrict__ off) {
    __shared__ int64_t base_all[kWavesB][kRadix];
    int64_t *base = base_all[threadIdx.x / kWave];
    const int64_t tile = wave_index();
    if (tile >= ntile) return;
    const int lane = lane_id();
    for (int d = lane; d < kRadix; d += kWave) base[d] = off[d * ntile + tile];
    wave_sync();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t t0 = tile * kTile;
    for (int st = 0; st < kSteps; ++st) {
        const int64_t i = t0 + st * kWave + lane;
        const bool ok = i < n;
        const uint64_t v = ok ? in[i] : 0ull;
        const uint32_t d = digit_of(v, shift);
        uint64_t peers = ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = ballot(ok && bit);
            peers &= bit ? bb : ~bb;
        }
        const int64_t pos = base[d] + __popcll(peers & below);
        wave_sync();
        if (ok) {
            out[pos] = v;
            if ((peers & below) == 0) base[d] += __popcll(peers);
        }
        wave_sync();
    }
}

}  // namespace

rcb_status sort_by_label(rcb_tree *t, uint64_t *a, uint64_t *b, int64_t n, int bits,
                         hipStream_t s, uint64_t **result) {
    *result = a;
    if (n <= 0 || bits <= 0) return RCB_OK;
    const int64_t ntile = (n + kTile - 1) / kTile;
    Scratch tmp(t, s);
    int64_t *hist = (int64_t *)dalloc(t, sizeof(int64_t) * (kRadix * ntile + 1), s, tmp);
    if (!hist) return RCB_ENOMEM;
    const unsigned grid = (unsigned)((ntile + kWavesB - 1) / kWavesB);
    uint64_t *src = a, *dst = b;
    for (int shift = 0; shift < bits; shift += 8) {
        k_sort_hist<<<grid, kBlock, 0, s>>>(src, n, shift, ntile, hist);
        RCB_LAUNCH_CHECK("k_sort_hist");
        rcb_status st = scan_i64(t, hist, hist, kRadix * ntile, s);
        if (st != RCB_OK) return st;
        k_sort_scatter<<<grid, kBlock, 0, s>>>(src, dst, n, shift, ntile, hist);
        RCB_LAUNCH_CHECK("k_sort_scatter");
        uint64_t *w = src;
        src = dst;
        dst = w;
    }
    *result = src;
    return RCB_OK;
}

}  // namespace rcb
