// k_walk.hip -- per-leaf tree walk producing the interaction lists
// (Sec. 2.2 "Tree walk", Sec. 2.3.1 reachability, Sec. 2.4.1 MAC).
//
// One wave walks for one sink leaf A. The paper's walk is a depth-first
// traversal that starts at nodes 2 and 3 and either accepts, discards or
// opens each node. Here the wave keeps a LIFO stack of pending labels in LDS
// and tests up to 64 of them at once; opened nodes push both children
// (ballot + mbcnt compaction). The decisions per node B are exactly those of
// the serial walk, so the lists are the same sets:
//   empty B                             -> skipped (Sec. 2.1 "Load balancing")
//   reach(A,B): |g_A - g_B| < h_node(A) + h_node_int(B)
//       leaf -> near list, candidate bit set; else open
//   else H_B^2 < theta^2 |com_A - com_B|^2 -> far list
//   else leaf -> near list (no candidate bit); else open
// reach is evaluated squared with the radius sum padded by (1 + 2^-32).
// Near lists are then sorted by label, so candidate cells (and hence the
// neighbour lists) come out in tree order.
//
// Two launches: count (list sizes per leaf) and fill (after a scan of the
// sizes). The stack holds at most ~64 (k + 2) labels: each round pops the 64
// newest entries and pushes at most 128 children one level deeper.
#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr uint32_t kLabelMask = 0x7fffffffu;

template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_walk(const double4 *__restrict__ rec,
                                                 const double *__restrict__ hnode, int k,
                                                 int64_t nleaf, double theta2,
                                                 int64_t *__restrict__ near_cnt,
                                                 int64_t *__restrict__ far_cnt,
                                                 const int64_t *__restrict__ near_off,
                                                 const int64_t *__restrict__ far_off,
                                                 int32_t *__restrict__ near_list,
                                                 int32_t *__restrict__ far_list,
                                                 int32_t *__restrict__ flag) {
    __shared__ int32_t stk_all[kWaves][kStackCap];
    int32_t *stk = stk_all[threadIdx.x / kWave];
    const int64_t li = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kWave;
    if (li >= nleaf) return;
    const int lane = lane_id();
    const int64_t A = nleaf + li;
    const double4 ga = rec[2 * A], ca = rec[2 * A + 1];
    if (ga.w < 0.0) {   // empty leaf: no lists
        if (!FILL && lane == 0) {
            near_cnt[li] = 0;
            far_cnt[li] = 0;
        }
        return;
    }
    const double hA = hnode[A];
    int sp;
    if (k == 0) {
        if (lane == 0) stk[0] = 1;
        sp = 1;
    } else {
        if (lane == 0) {
            stk[0] = 3;
            stk[1] = 2;
        }
        sp = 2;
    }
    __builtin_amdgcn_wave_barrier();
    int64_t nn = 0, nf = 0;
    int64_t nbase = 0, fbase = 0;
    if (FILL) {
        nbase = near_off[li];
        fbase = far_off[li];
    }
    bool overflow = false;
    while (sp > 0) {
        const int b = sp < kWave ? sp : kWave;
        sp -= b;
        const bool act = lane < b;
        const int32_t node = act ? stk[sp + lane] : 0;
        double4 gb = make_double4(0.0, 0.0, 0.0, -1.0), cb = make_double4(0.0, 0.0, 0.0, 0.0);
        if (act) {
            gb = rec[2 * (int64_t)node];
            cb = rec[2 * (int64_t)node + 1];
        }
        const bool live = act && gb.w >= 0.0;
        const bool leafB = node >= nleaf;
        const double dg2 = dist2(ga.x, ga.y, ga.z, gb.x, gb.y, gb.z);
        const double rs = (hA + gb.w) * kReachPad;
        const bool reach = dg2 < rs * rs;
        const double R2 = dist2(ca.x, ca.y, ca.z, cb.x, cb.y, cb.z);
        const bool mac = cb.w * cb.w < theta2 * R2;
        const bool open = live && !leafB && (reach || !mac);
        const bool nearf = live && leafB && (reach || !mac);
        const bool farf = live && !reach && mac;
        const uint64_t bo = ballot(open);
        const int no = __popcll(bo);
        if (sp + 2 * no > kStackCap) {
            overflow = true;
            break;
        }
        __builtin_amdgcn_wave_barrier();
        if (open) {
            const int r = rank_below(bo);
            stk[sp + 2 * r] = 2 * node;
            stk[sp + 2 * r + 1] = 2 * node + 1;
        }
        __builtin_amdgcn_wave_barrier();
        sp += 2 * no;
        const uint64_t bn = ballot(nearf);
        const uint64_t bf = ballot(farf);
        if (FILL) {
            if (nearf)
                near_list[nbase + nn + rank_below(bn)] =
                    (int32_t)((uint32_t)node | ((uint32_t)reach << 31));
            if (farf) far_list[fbase + nf + rank_below(bf)] = node;
        }
        nn += __popcll(bn);
        nf += __popcll(bf);
    }
    if (overflow) {
        if (lane == 0) atomicOr(flag, 1);
        if (!FILL && lane == 0) {
            near_cnt[li] = 0;
            far_cnt[li] = 0;
        }
        return;
    }
    if (!FILL) {
        if (lane == 0) {
            near_cnt[li] = nn;
            far_cnt[li] = nf;
            if (nn > kStackCap) atomicAdd(&flag[1], 1);
        }
        return;
    }
}

// Sort each leaf's near list by label (bitonic network in LDS, one wave per
// leaf). Lists longer than the LDS tile are queued for k_sort_long.
__global__ __launch_bounds__(kBlock) void k_sort_near(int64_t nleaf, const int64_t *__restrict__ near_off,
                                                      int32_t *__restrict__ near_list,
                                                      int32_t *__restrict__ flag,
                                                      int32_t *__restrict__ long_q) {
    __shared__ int32_t buf_all[kWaves][kStackCap];
    int32_t *buf = buf_all[threadIdx.x / kWave];
    const int64_t li = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kWave;
    if (li >= nleaf) return;
    const int lane = lane_id();
    const int64_t nbase = near_off[li];
    const int64_t nn = near_off[li + 1] - nbase;
    if (nn <= 1) return;
    if (nn > kStackCap) {
        if (lane == 0) long_q[atomicAdd(&flag[2], 1)] = (int32_t)li;
        return;
    }
    int P = 1;
    while (P < nn) P <<= 1;
    for (int i = lane; i < P; i += kWave)
        buf[i] = i < nn ? near_list[nbase + i] : (int32_t)kLabelMask;
    __builtin_amdgcn_wave_barrier();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = lane; q < (P >> 1); q += kWave) {
                const int i = 2 * stride * (q / stride) + (q % stride);
                const int j = i + stride;
                const int32_t a = buf[i], c = buf[j];
                const bool up = (i & size) == 0;
                const uint32_t la = (uint32_t)a & kLabelMask, lc = (uint32_t)c & kLabelMask;
                if (up ? la > lc : la < lc) {
                    buf[i] = c;
                    buf[j] = a;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    for (int i = lane; i < nn; i += kWave) near_list[nbase + i] = buf[i];
}

// Sort of the queued long near lists, one block each, in global memory:
// bitonic network in its all-ascending form (the first merge step of each
// stage compares i with i ^ (size - 1)), so the virtual +inf padding past the
// list end never moves and pairs reaching past the end are simply skipped.
__global__ __launch_bounds__(1024) void k_sort_long(const int32_t *__restrict__ long_q,
                                                    const int64_t *__restrict__ near_off,
                                                    int32_t *__restrict__ near_list) {
    const int64_t li = long_q[blockIdx.x];
    int32_t *v = near_list + near_off[li];
    const int64_t nn = near_off[li + 1] - near_off[li];
    int64_t P = 1;
    while (P < nn) P <<= 1;
    for (int64_t size = 2; size <= P; size <<= 1) {
        for (int64_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int64_t q = threadIdx.x; q < (P >> 1); q += blockDim.x) {
                const int64_t i = 2 * stride * (q / stride) + (q % stride);
                const int64_t j = stride == (size >> 1) ? (i ^ (size - 1)) : i + stride;
                if (j < nn) {
                    const int32_t a = v[i], c = v[j];
                    if (((uint32_t)a & kLabelMask) > ((uint32_t)c & kLabelMask)) {
                        v[i] = c;
                        v[j] = a;
                    }
                }
            }
            __threadfence_block();
            __syncthreads();
        }
    }
}

}  // namespace

rcb_status ensure_walk(rcb_tree *t, hipStream_t s) {
    if (t->walked) return RCB_OK;
    const int64_t L = t->nleaf;
    std::vector<void *> tmp;
    int64_t *ncnt = (int64_t *)dalloc(t, sizeof(int64_t) * L, s, tmp);
    int64_t *fcnt = (int64_t *)dalloc(t, sizeof(int64_t) * L, s, tmp);
    t->near_off = (int64_t *)dalloc(t, sizeof(int64_t) * (L + 1), s, t->list_allocs);
    t->far_off = (int64_t *)dalloc(t, sizeof(int64_t) * (L + 1), s, t->list_allocs);
    if (!ncnt || !fcnt || !t->near_off || !t->far_off) return RCB_ENOMEM;
    const double theta2 = t->p.theta * t->p.theta;
    const unsigned grid = (unsigned)((L + kWaves - 1) / kWaves);
    RCB_HIP(hipMemsetAsync(t->dflag, 0, sizeof(int32_t) * 4, s));
    k_walk<false><<<grid, kBlock, 0, s>>>(t->wrec, t->nhnode, t->k, L, theta2, ncnt, fcnt, nullptr,
                                          nullptr, nullptr, nullptr, t->dflag);
    RCB_LAUNCH_CHECK("k_walk<count>");
    rcb_status st = scan_i64(t, ncnt, t->near_off, L, s);
    if (st != RCB_OK) return st;
    st = scan_i64(t, fcnt, t->far_off, L, s);
    if (st != RCB_OK) return st;
    int64_t tot[2] = {0, 0};
    int32_t flags[4] = {0, 0, 0, 0};
    RCB_HIP(hipMemcpyAsync(&tot[0], t->near_off + L, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RCB_HIP(hipMemcpyAsync(&tot[1], t->far_off + L, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RCB_HIP(hipMemcpyAsync(flags, t->dflag, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, s));
    RCB_HIP(hipStreamSynchronize(s));
    const int32_t nlong = flags[1];
    if (flags[0]) {
        set_error("walk: LIFO stack overflow (tree deeper than the stack supports)");
        return RCB_ECAPACITY;
    }
    t->near_list = (int32_t *)dalloc(t, sizeof(int32_t) * std::max<int64_t>(1, tot[0]), s, t->list_allocs);
    t->far_list = (int32_t *)dalloc(t, sizeof(int32_t) * std::max<int64_t>(1, tot[1]), s, t->list_allocs);
    if (!t->near_list || !t->far_list) return RCB_ENOMEM;
    k_walk<true><<<grid, kBlock, 0, s>>>(t->wrec, t->nhnode, t->k, L, theta2, nullptr, nullptr,
                                         t->near_off, t->far_off, t->near_list, t->far_list, t->dflag);
    RCB_LAUNCH_CHECK("k_walk<fill>");
    int32_t *long_q = nullptr;
    if (nlong > 0) {
        long_q = (int32_t *)dalloc(t, sizeof(int32_t) * nlong, s, tmp);
        if (!long_q) return RCB_ENOMEM;
    }
    k_sort_near<<<grid, kBlock, 0, s>>>(L, t->near_off, t->near_list, t->dflag, long_q);
    RCB_LAUNCH_CHECK("k_sort_near");
    if (nlong > 0) {
        k_sort_long<<<nlong, 1024, 0, s>>>(long_q, t->near_off, t->near_list);
        RCB_LAUNCH_CHECK("k_sort_long");
    }
    for (void *p : tmp) RCB_HIP(hipFreeAsync(p, s));
    t->near_total = tot[0];
    t->far_total = tot[1];
    t->walked = true;
    return RCB_OK;
}

}  // namespace rcb
