// k_scan.hip -- device exclusive prefix sum of int64 counts (neighbour
// offsets, per-leaf list offsets): out[0] = 0, out[i + 1] = out[i] + in[i];
// out may be in itself (in[n] is not read).
// Three passes over blocks of 2048 values: block sums, a one-block scan of
// the block sums, then the per-block scan with the block's carry.
#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kScanThreads = 256;
constexpr int kPer = 8;
constexpr int kTile = kScanThreads * kPer;

__device__ int64_t block_excl_scan(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kScanThreads / kWave];
    const int w = threadIdx.x / kWave;
    const int64_t e = wave_excl_scan64(v);
    if (lane_id() == kWave - 1) wsum[w] = e + v;
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        if (i < w) base += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return base + e;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int64_t *__restrict__ in,
                                                              int64_t n, int64_t *__restrict__ bsum) {
    const int64_t base = blockIdx.x * (int64_t)kTile + threadIdx.x * (int64_t)kPer;
    int64_t v = 0;
#pragma unroll
    for (int t = 0; t < kPer; ++t)
        if (base + t < n) v += in[base + t];
    int64_t tot;
    block_excl_scan(v, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(int64_t *__restrict__ bsum, int64_t nb) {
    int64_t carry = 0;
    for (int64_t off = 0; off < nb; off += kTile) {
        const int64_t base = off + threadIdx.x * (int64_t)kPer;
        int64_t v[kPer], s = 0;
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            v[t] = base + t < nb ? bsum[base + t] : 0;
            s += v[t];
        }
        int64_t tot;
        int64_t e = block_excl_scan(s, &tot) + carry;
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            if (base + t < nb) bsum[base + t] = e;
            e += v[t];
        }
        carry += tot;
    }
}

// in may equal out: each thread reads its own values before writing them
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int64_t *in, int64_t n,
                                                             const int64_t *__restrict__ bsum,
                                                             int64_t *out) {
    const int64_t base = blockIdx.x * (int64_t)kTile + threadIdx.x * (int64_t)kPer;
    int64_t v[kPer], s = 0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        v[t] = base + t < n ? in[base + t] : 0;
        s += v[t];
    }
    int64_t tot;
    int64_t e = block_excl_scan(s, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        if (base + t < n) out[base + t] = e;
        e += v[t];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) out[n] = e;
}

}  // namespace

rcb_status scan_i64(rcb_tree *t, const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    const int64_t nb = n > 0 ? (n + kTile - 1) / kTile : 1;
    Scratch tmp(t, s);
    int64_t *bsum = (int64_t *)dalloc(t, sizeof(int64_t) * nb, s, tmp);
    if (!bsum) return RCB_ENOMEM;
    k_scan_reduce<<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, bsum);
    RCB_LAUNCH_CHECK("k_scan_reduce");
    k_scan_top<<<1, kScanThreads, 0, s>>>(bsum, nb);
    RCB_LAUNCH_CHECK("k_scan_top");
    k_scan_apply<<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, bsum, out);
    RCB_LAUNCH_CHECK("k_scan_apply");
    return RCB_OK;
}

}  // namespace rcb
