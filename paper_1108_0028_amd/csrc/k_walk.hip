// k_walk.hip -- tree walk producing the interaction lists
// (Sec. 2.2 "Tree walk", Sec. 2.3.1 reachability, Sec. 2.4.1 MAC).
//
// The paper walks the tree once per lowest-level cell. Here one wave walks
// for a GROUP of up to 8 sibling leaves (the leaves below one node of level
// k-3) at once: lanes are (pending entry e = lane/8, leaf slot i = lane%8),
// so every node record is loaded once for the whole group and tested
// against each leaf whose own walk reaches it. Stack entries carry the node
// label and the mask of leaves that visit it; per leaf the decisions are
// exactly those of the serial walk:
//   empty B                              -> skipped (Sec. 2.1 "Load balancing")
//   reach(A,B): |g_A - g_B| < h_node(A) + h_node_int(B)
//       leaf -> near, candidate; else open
//   else H_B^2 < theta^2 |com_A - com_B|^2 -> far
//   else leaf -> near (no candidate); else open
// reach is evaluated squared with the radius sum padded by (1 + 2^-32).
//
// Pure-MAC mode (the variant of Sec. 2.5: reachability does not override
// the MAC) runs two walks in one traversal. An entry carries two leaf
// masks: gravity (the MAC walk: accepted -> far unless B contains the leaf,
// else leaf -> near, internal -> open) and neighbour (the reachability
// walk: reachable -> leaf is a candidate, internal -> open; else dropped).
// A near entry then may be a candidate without being in a leaf's gravity
// near field (candidate bit set, near bit clear).
//
// Two kernels walk a group. k_walk_wide, the one normally run, gives each
// lane one popped stack entry (up to 64 per round) and tests it against all
// the group's leaves in turn, so a node costs one record load and one set
// of list/stack bookkeeping for 8 leaf tests; its LDS ring holds kWQueue
// entries, and a group that would outgrow it is queued and walked again by
// k_walk_group, whose lanes are (pending entry, leaf) and whose stack bound
// is proved below. Both make the same per-leaf decisions; their lists differ
// only in order (the wide walk's near lists are sorted by label, the 8-wide
// walk's are sorted afterwards).
//
// Output per group: a near list of (label, near mask, candidate mask) and a
// far list of (label, far mask) -- the union of the group's per-leaf lists.
// Near lists are sorted by label, so each leaf's candidates (and neighbour
// lists) come out in tree order. Two launches: count, then fill after a
// scan of the sizes. Per-leaf lists for inspection are expanded on demand.
#include <algorithm>
#include <cstdlib>

#include "rcb_internal.h"

namespace rcb {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
// (label, mask) entries per wave. Depth never decreases up the stack (children
// are pushed in the order of their parents), and a round that pops an entry of
// level d - 1 pops every entry above it, so at most 16 entries of each level
// are ever on the stack: <= 16 k <= 464 for k <= 29.
constexpr int kGStack = 512;
constexpr int kSortCap = 1024;       // near lists sorted in LDS up to this size
constexpr uint32_t kLabelMask = 0x7fffffffu;

// Lists are written at near_beg[g] / far_beg[g] if those are given, else at
// g * cap (fixed-capacity slabs); entries past the capacity are counted but
// not written, and such groups are counted in flag[3].
struct WalkArgs {
    const double4 *rec;
    const double *hnode;
    int k, gk;
    int64_t ngroup;
    double theta2;
    int64_t *near_cnt, *far_cnt;
    const int64_t *near_beg, *far_beg;
    int64_t near_cap, far_cap;
    uint64_t *near_list, *far_list;
    int32_t *flag;
    unsigned long long *stats;   // if given: [0] node records tested, [1] (node, leaf) tests
};

// bit 8 s set iff byte s of x is non-zero (the lead lane of entry s)
__device__ __forceinline__ uint64_t byte_any(uint64_t x) {
    x |= x >> 4;
    x |= x >> 2;
    x |= x >> 1;
    return x & 0x0101010101010101ull;
}

// stack entry: label | gravity mask << 32 | neighbour mask << 40
// only: if given, wave i walks group only[i] (i < nonly), else group i
template <bool PURE>
__global__ __launch_bounds__(kBlock) void k_walk_group(WalkArgs w, const int32_t *only, int64_t nonly) {
    __shared__ uint64_t stk_all[kWaves][kGStack];
    uint64_t *stk = stk_all[threadIdx.x / kWave];
    const int64_t wi = wave_index();
    if (wi >= (only ? nonly : w.ngroup)) return;
    const int64_t gi = only ? (int64_t)only[wi] : wi;
    const int lane = lane_id();
    const int G = 1 << w.gk;
    const int slot = lane >> 3;      // pending entry handled by this lane
    const int li = lane & 7;         // leaf slot within the group
    const int64_t nleaf = (int64_t)1 << w.k;
    const int64_t A = nleaf + gi * G + (li < G ? li : 0);
    const double4 ga = w.rec[2 * A], ca = w.rec[2 * A + 1];
    const double hA = w.hnode[A];
    const bool leaf_live = li < G && ga.w >= 0.0;
    const uint32_t live_mask = (uint32_t)(ballot(leaf_live) & 0xffull);
    int64_t nn = 0, nf = 0;
    const int64_t nbase = w.near_beg ? w.near_beg[gi] : gi * w.near_cap;
    const int64_t fbase = w.far_beg ? w.far_beg[gi] : gi * w.far_cap;
    if (live_mask == 0) {
        if (lane == 0) {
            w.near_cnt[gi] = 0;
            w.far_cnt[gi] = 0;
        }
        return;
    }
    const uint64_t root_masks = ((uint64_t)live_mask << 32) | (PURE ? (uint64_t)live_mask << 40 : 0ull);
    if (lane == 0) {
        if (w.k == 0) {
            stk[0] = 1ull | root_masks;
        } else {
            stk[0] = 3ull | root_masks;
            stk[1] = 2ull | root_masks;
        }
    }
    int sp = w.k == 0 ? 1 : 2;
    __builtin_amdgcn_wave_barrier();
    bool overflow = false;
    while (sp > 0) {
        const int b = sp < 8 ? sp : 8;
        sp -= b;
        const bool act = slot < b;
        // lanes past the popped entries read the top entry again and are masked
        const uint64_t ent = stk[sp + (act ? slot : 0)];
        const int32_t node = (int32_t)(ent & 0xffffffffull);
        const bool gbit = act && ((ent >> (32 + li)) & 1ull);
        const double4 gb = w.rec[2 * (int64_t)node];
        const double4 cb = w.rec[2 * (int64_t)node + 1];
        const bool nonempty = gb.w >= 0.0;
        const double dg2 = dist2(ga.x, ga.y, ga.z, gb.x, gb.y, gb.z);
        const double rs = (hA + gb.w) * kReachPad;
        const double R2 = dist2(ca.x, ca.y, ca.z, cb.x, cb.y, cb.z);
        // the per-lane tests as wave masks; the decisions are bit logic on them
        const uint64_t B_g = ballot(gbit && nonempty);          // gravity walk reaches B
        const uint64_t B_leaf = ballot(node >= nleaf);
        const uint64_t B_reach = ballot(dg2 < rs * rs);
        const uint64_t B_mac = ballot(cb.w * cb.w < w.theta2 * R2);
        uint64_t acc, B_n;
        if constexpr (PURE) {
            // B contains leaf A iff A's ancestor on B's level is B
            const int lvl = 31 - __builtin_clz((uint32_t)node);
            const uint64_t B_anc = ballot((A >> (w.k - lvl)) == (int64_t)node);
            acc = B_g & B_mac & ~B_anc;
            B_n = ballot(act && ((ent >> (40 + li)) & 1ull) && nonempty);
        } else {
            acc = B_g & B_mac & ~B_reach;
            B_n = B_g;
        }
        const uint64_t bf = acc;                                  // far
        const uint64_t grav = B_g & ~acc;                         // near or open for gravity
        const uint64_t bc = B_n & B_leaf & B_reach;               // neighbour candidate
        const uint64_t bn = (grav & B_leaf) | bc;                 // near entry
        const uint64_t bog = grav & ~B_leaf;                      // open for gravity
        const uint64_t bon = PURE ? (B_n & ~B_leaf & B_reach) : 0ull;   // open for neighbours
        const uint64_t bo = bog | bon;
        // one lane per entry (li == 0) turns the 8 decision bits into list entries
        const uint32_t ogm = (uint32_t)((bog >> (8 * slot)) & 0xffull);
        const uint32_t onm = (uint32_t)((bon >> (8 * slot)) & 0xffull);
        const uint32_t nm = (uint32_t)(((grav & B_leaf) >> (8 * slot)) & 0xffull);
        const uint32_t cm = (uint32_t)((bc >> (8 * slot)) & 0xffull);
        const uint32_t fm = (uint32_t)((bf >> (8 * slot)) & 0xffull);
        const bool lead = act && li == 0;
        const uint64_t b_open = byte_any(bo), b_near = byte_any(bn), b_far = byte_any(bf);
        const int no = __popcll(b_open);
        if (sp + 2 * no > kGStack) {
            overflow = true;
            break;
        }
        __builtin_amdgcn_wave_barrier();
        if (lead && (ogm | onm) != 0) {
            const int r = rank_below(b_open);
            const uint64_t masks = ((uint64_t)ogm << 32) | ((uint64_t)onm << 40);
            stk[sp + 2 * r] = (uint64_t)(2 * node) | masks;
            stk[sp + 2 * r + 1] = (uint64_t)(2 * node + 1) | masks;
        }
        __builtin_amdgcn_wave_barrier();
        sp += 2 * no;
        if (lead && (nm | cm) != 0) {
            const int64_t i = nn + rank_below(b_near);
            if (i < w.near_cap)
                w.near_list[nbase + i] =
                    (uint64_t)(uint32_t)node | ((uint64_t)nm << 32) | ((uint64_t)cm << 40);
        }
        if (lead && fm != 0) {
            const int64_t i = nf + rank_below(b_far);
            if (i < w.far_cap) w.far_list[fbase + i] = (uint64_t)(uint32_t)node | ((uint64_t)fm << 32);
        }
        nn += __popcll(b_near);
        nf += __popcll(b_far);
    }
    if (overflow) {
        if (lane == 0) {
            atomicOr(w.flag, 1);
            w.near_cnt[gi] = 0;
            w.far_cnt[gi] = 0;
        }
        return;
    }
    if (lane == 0) {
        w.near_cnt[gi] = nn;
        w.far_cnt[gi] = nf;
        if (nn > kSortCap) atomicAdd(&w.flag[1], 1);
        if (nn > w.near_cap || nf > w.far_cap) atomicAdd(&w.flag[3], 1);
    }
}

// Wide walk: lane j holds the j-th entry taken from the front of a FIFO ring
// in LDS; its node record is loaded once and tested against each leaf of the
// group (records in LDS), and the per-leaf decisions of the header become
// 8-bit masks per lane. Children are appended in the order of their parents,
// so nodes are visited level by level and, within a level, by increasing
// label: near entries (always lowest-level cells) come out sorted by label,
// as the neighbour lists' tree order needs, with no sort. At 4M particles
// the ring holds up to ~800 entries. A group whose appends would pass the
// ring stops: if queue is given its index is appended (flag[6] counts them)
// for the next tier to walk again, writing counts and lists over whatever
// this one wrote: the same kernel with a ring of kWQueue2 entries (one wave
// per block), then k_walk_group (and k_sort_lists for its near lists).
// only: if given, wave i walks group only[i] (i < nonly).
constexpr int kWQueue = 1024;    // powers of two
constexpr int kWQueue2 = 8192;

template <bool PURE, int QCAP, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_walk_wide(WalkArgs w, int32_t *queue, int32_t *nqueue,
                                                             const int32_t *only, int64_t nonly, int cap) {
    __shared__ uint32_t qlab_all[WAVES][QCAP];   // ring: node label
    __shared__ uint16_t qmsk_all[WAVES][QCAP];   // and gravity | neighbour << 8 masks
    __shared__ double4 leaf_all[WAVES][16];      // per leaf: (g, h_node), (com, -)
    uint32_t *qlab = qlab_all[threadIdx.x / kWave];
    uint16_t *qmsk = qmsk_all[threadIdx.x / kWave];
    double4 *lf = leaf_all[threadIdx.x / kWave];
    const int64_t wi = wave_index();
    if (wi >= (only ? nonly : w.ngroup)) return;
    const int64_t gi = only ? (int64_t)only[wi] : wi;
    const int lane = lane_id();
    const int G = 1 << w.gk;
    const int64_t nleaf = (int64_t)1 << w.k;
    const int64_t A0 = nleaf + gi * G;
    bool leaf_live = false;
    if (lane < 8) {
        const int64_t A = A0 + (lane < G ? lane : 0);
        const double4 ga = w.rec[2 * A];
        leaf_live = lane < G && ga.w >= 0.0;
        lf[lane] = make_double4(ga.x, ga.y, ga.z, w.hnode[A]);
        lf[8 + lane] = w.rec[2 * A + 1];
    }
    const uint32_t live_mask = (uint32_t)(ballot(leaf_live) & 0xffull);
    int64_t nn = 0, nf = 0;
    const int64_t nbase = w.near_beg ? w.near_beg[gi] : gi * w.near_cap;
    const int64_t fbase = w.far_beg ? w.far_beg[gi] : gi * w.far_cap;
    if (live_mask == 0) {
        if (lane == 0) {
            w.near_cnt[gi] = 0;
            w.far_cnt[gi] = 0;
        }
        return;
    }
    const uint16_t root_masks = (uint16_t)(live_mask | (PURE ? live_mask << 8 : 0u));
    if (lane == 0) {
        if (w.k == 0) {
            qlab[0] = 1u;
            qmsk[0] = root_masks;
        } else {
            qlab[0] = 2u;
            qlab[1] = 3u;
            qmsk[0] = qmsk[1] = root_masks;
        }
    }
    int head = 0, cnt = w.k == 0 ? 1 : 2;   // ring [head, head + cnt), indices mod kWQueue
    __builtin_amdgcn_wave_barrier();
    bool overflow = false;
    uint32_t n_nodes = 0, n_tests = 0;      // this lane's share of the walk statistics
    while (cnt > 0) {
        const int b = cnt < kWave ? cnt : kWave;
        const bool act = lane < b;
        const int slot = (head + (act ? lane : 0)) & (QCAP - 1);
        const uint32_t qm = qmsk[slot];
        const int32_t node = act ? (int32_t)qlab[slot] : 1;
        head = (head + b) & (QCAP - 1);
        cnt -= b;
        const int tail = (head + cnt) & (QCAP - 1);
        const double4 gb = w.rec[2 * (int64_t)node];
        const double4 cb = w.rec[2 * (int64_t)node + 1];
        const bool live = act && gb.w >= 0.0;   // taken and non-empty
        const bool isleaf = node >= nleaf;
        const uint32_t gmask = live ? qm & 0xffu : 0u;
        const uint32_t nmask = PURE && live ? (qm >> 8) & 0xffu : 0u;
        n_nodes += act;
        n_tests += __popc(gmask | nmask);
        const double H2 = cb.w * cb.w;
        const int lvl = 31 - __builtin_clz((uint32_t)node);
        // per leaf (last to first, shifted in): accepted were it visited, and
        // reachable; the visit masks are applied afterwards
        uint32_t acc_raw = 0, reach_raw = 0;
#pragma unroll
        for (int i = 7; i >= 0; --i) {
            const double4 ga = lf[i];
            const double4 ca = lf[8 + i];
            const double dg2 = dist2(ga.x, ga.y, ga.z, gb.x, gb.y, gb.z);
            const double rs = (ga.w + gb.w) * kReachPad;
            const bool reach = dg2 < rs * rs;
            const double R2 = dist2(ca.x, ca.y, ca.z, cb.x, cb.y, cb.z);
            const bool mac = H2 < w.theta2 * R2;
            bool acc;
            if constexpr (PURE) {
                const bool contains = ((A0 + i) >> (w.k - lvl)) == (int64_t)node;
                acc = mac && !contains;
            } else {
                acc = mac && !reach;
            }
            acc_raw = acc_raw + acc_raw + (uint32_t)acc;
            reach_raw = reach_raw + reach_raw + (uint32_t)reach;
        }
        const uint32_t far = acc_raw & gmask;
        const uint32_t keep = gmask & ~far;
        const uint32_t cand = reach_raw & (PURE ? nmask : gmask);
        const uint32_t ogm = isleaf ? 0u : keep;                    // open for gravity
        const uint32_t onm = PURE && !isleaf ? cand : 0u;           // open for neighbours
        const uint32_t nm = isleaf ? keep : 0u;                     // near field
        const uint32_t cm = isleaf ? cand : 0u;                     // neighbour candidate
        const bool op = (ogm | onm) != 0u;
        const uint64_t b_open = ballot(op);
        const int no = __popcll(b_open);
        if (cnt + 2 * no > cap) {
            overflow = true;
            break;
        }
        // the appended slots lie outside [head, head + cnt) (cnt + 2 no <=
        // cap <= QCAP); some are the ones just taken, read above
        __builtin_amdgcn_wave_barrier();
        if (op) {
            const int r = rank_below(b_open);
            const uint16_t masks = (uint16_t)(ogm | (onm << 8));
            const int s0 = (tail + 2 * r) & (QCAP - 1), s1 = (tail + 2 * r + 1) & (QCAP - 1);
            qlab[s0] = (uint32_t)(2 * node);
            qlab[s1] = (uint32_t)(2 * node + 1);
            qmsk[s0] = masks;
            qmsk[s1] = masks;
        }
        __builtin_amdgcn_wave_barrier();
        cnt += 2 * no;
        const bool hn = (nm | cm) != 0u;
        const uint64_t b_near = ballot(hn);
        if (hn) {
            const int64_t i = nn + rank_below(b_near);
            if (i < w.near_cap)
                w.near_list[nbase + i] = (uint64_t)(uint32_t)node | ((uint64_t)nm << 32) | ((uint64_t)cm << 40);
        }
        nn += __popcll(b_near);
        const bool hf = far != 0u;
        const uint64_t b_far = ballot(hf);
        if (hf) {
            const int64_t i = nf + rank_below(b_far);
            if (i < w.far_cap) w.far_list[fbase + i] = (uint64_t)(uint32_t)node | ((uint64_t)far << 32);
        }
        nf += __popcll(b_far);
    }
    if (w.stats) {
        const int sn = wave_sum_i((int)n_nodes), st = wave_sum_i((int)n_tests);
        if (lane == 0) {
            atomicAdd(&w.stats[0], (unsigned long long)sn);
            atomicAdd(&w.stats[1], (unsigned long long)st);
        }
    }
    if (overflow) {
        if (lane == 0 && queue) queue[atomicAdd(nqueue, 1)] = (int32_t)gi;
        return;
    }
    if (lane == 0) {
        w.near_cnt[gi] = nn;
        w.far_cnt[gi] = nf;
        if (nn > w.near_cap || nf > w.far_cap) atomicAdd(&w.flag[3], 1);
    }
}

// ends of the slab lists: [g cap, g cap + count)
__global__ __launch_bounds__(kBlock) void k_slab_ends(int64_t ngroup, int64_t near_cap, int64_t far_cap,
                                                      const int64_t *__restrict__ ncnt,
                                                      const int64_t *__restrict__ fcnt,
                                                      int64_t *__restrict__ nbeg, int64_t *__restrict__ nend,
                                                      int64_t *__restrict__ fbeg, int64_t *__restrict__ fend) {
    const int64_t g = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (g >= ngroup) return;
    nbeg[g] = g * near_cap;
    nend[g] = g * near_cap + ncnt[g];
    fbeg[g] = g * far_cap;
    fend[g] = g * far_cap + fcnt[g];
}

// Sort the near lists of the groups walked by k_walk_group by label (bitonic
// network in LDS, one wave per group, CAP entries at most): wave i takes group
// only[i]. Longer lists are queued for k_sort_long.
template <int CAP, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_sort_lists(int64_t nonly, const int32_t *__restrict__ only,
                                                              const int64_t *__restrict__ beg,
                                                              const int64_t *__restrict__ end,
                                                              uint64_t *__restrict__ list,
                                                              int32_t *__restrict__ nqueued,
                                                              int32_t *__restrict__ long_q) {
    __shared__ uint64_t buf_all[WAVES][CAP];
    uint64_t *buf = buf_all[threadIdx.x / kWave];
    const int64_t wi = wave_index();
    if (wi >= nonly) return;
    const int64_t gi = only[wi];
    const int lane = lane_id();
    const int64_t nbase = beg[gi];
    const int64_t nn = end[gi] - nbase;
    if (nn <= 1) return;
    if (nn > CAP) {
        if (lane == 0) long_q[atomicAdd(nqueued, 1)] = (int32_t)gi;
        return;
    }
    int P = 1;
    while (P < nn) P <<= 1;
    for (int i = lane; i < P; i += kWave) buf[i] = i < nn ? list[nbase + i] : (uint64_t)kLabelMask;
    __builtin_amdgcn_wave_barrier();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = lane; q < (P >> 1); q += kWave) {
                const int i = 2 * stride * (q / stride) + (q % stride);
                const int j = i + stride;
                const uint64_t a = buf[i], c = buf[j];
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
    for (int i = lane; i < nn; i += kWave) list[nbase + i] = buf[i];
}

// Sort of the queued long lists, one block each, in global memory:
// bitonic network in its all-ascending form (the first merge step of each
// stage compares i with i ^ (size - 1)), so the virtual +inf padding past the
// list end never moves and pairs reaching past the end are simply skipped.
__global__ __launch_bounds__(1024) void k_sort_long(const int32_t *__restrict__ long_q,
                                                    const int64_t *__restrict__ beg,
                                                    const int64_t *__restrict__ end,
                                                    uint64_t *__restrict__ list) {
    const int64_t gi = long_q[blockIdx.x];
    uint64_t *v = list + beg[gi];
    const int64_t nn = end[gi] - beg[gi];
    int64_t P = 1;
    while (P < nn) P <<= 1;
    for (int64_t size = 2; size <= P; size <<= 1) {
        for (int64_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int64_t q = threadIdx.x; q < (P >> 1); q += blockDim.x) {
                const int64_t i = 2 * stride * (q / stride) + (q % stride);
                const int64_t j = stride == (size >> 1) ? (i ^ (size - 1)) : i + stride;
                if (j < nn) {
                    const uint64_t a = v[i], c = v[j];
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

// Per-leaf lists from the group lists (inspection only): a leaf keeps the
// entries whose near or candidate mask has its bit; near entries become
// label | candidate << 31 | (candidate only, not in the near field) << 30.
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_expand(int64_t nleaf, int gk,
                                                   const int64_t *__restrict__ gnear_beg,
                                                   const int64_t *__restrict__ gnear_end,
                                                   const uint64_t *__restrict__ gnear,
                                                   const int64_t *__restrict__ gfar_beg,
                                                   const int64_t *__restrict__ gfar_end,
                                                   const uint64_t *__restrict__ gfar,
                                                   int64_t *__restrict__ ncnt, int64_t *__restrict__ fcnt,
                                                   const int64_t *__restrict__ noff,
                                                   const int64_t *__restrict__ foff,
                                                   int32_t *__restrict__ nlist,
                                                   int32_t *__restrict__ flist) {
    const int64_t li = wave_index();
    if (li >= nleaf) return;
    const int64_t gi = li >> gk;
    const int bit = (int)(li & ((1 << gk) - 1));
    const int lane = lane_id();
    int64_t nn = 0, nf = 0;
    const int64_t n0 = gnear_beg[gi], n1 = gnear_end[gi];
    for (int64_t e0 = n0; e0 < n1; e0 += kWave) {
        const int64_t e = e0 + lane;
        const uint64_t ent = e < n1 ? gnear[e] : 0ull;
        const uint32_t nb = (uint32_t)((ent >> (32 + bit)) & 1ull);
        const uint32_t cand = (uint32_t)((ent >> (40 + bit)) & 1ull);
        const bool has = (nb | cand) != 0;
        const uint64_t bl = ballot(has);
        if (FILL && has)
            nlist[noff[li] + nn + rank_below(bl)] =
                (int32_t)(((uint32_t)ent & kLabelMask) | (cand << 31) | ((nb ^ 1u) << 30));
        nn += __popcll(bl);
    }
    const int64_t f0 = gfar_beg[gi], f1 = gfar_end[gi];
    for (int64_t e0 = f0; e0 < f1; e0 += kWave) {
        const int64_t e = e0 + lane;
        const uint64_t ent = e < f1 ? gfar[e] : 0ull;
        const bool has = (ent >> (32 + bit)) & 1ull;
        const uint64_t bl = ballot(has);
        if (FILL && has) flist[foff[li] + nf + rank_below(bl)] = (int32_t)((uint32_t)ent & kLabelMask);
        nf += __popcll(bl);
    }
    if (!FILL && lane == 0) {
        ncnt[li] = nn;
        fcnt[li] = nf;
    }
}

}  // namespace

// Slab capacities: 1024 near and up to 16384 far entries per group, within
// a budget for both slabs of 8 GB or 480 bytes per particle, whichever is
// larger. At 4M particles and theta = 0.7 the group lists average ~170 near
// and ~2150 far entries; at depth 23 (67M-1e8 particles, 2^20 groups) the
// per-particle budget leaves 2816-4672 far entries per group, enough for the
// clustered test cloud's lists, so that the walk runs once. n = 0 gives the
// 8 GB budget alone (the fallback when the larger slabs cannot be had).
static void slab_caps(int64_t ngroup, int64_t n, int64_t &cn, int64_t &cf) {
    const int64_t budget = std::max<int64_t>((int64_t)8 << 30, 480 * n);
    cn = 1024;
    cf = budget / (8 * ngroup) - cn;
    cf = std::min<int64_t>(16384, std::max<int64_t>(1024, cf & ~(int64_t)63));
}

// One walk into fixed-capacity slabs; if any group's list is longer than its
// slab, the counts of that walk size exact lists and a second walk fills them.
rcb_status ensure_walk(rcb_tree *t, hipStream_t s) {
    if (t->walked) return RCB_OK;
    const int64_t NG = t->ngroup;
    Scratch tmp(t, s);
    // per-group counts, the later tiers' queues and the statistics: one block
    // kept by the tree for its later walks (no frees between the walk's
    // kernels and the next call's)
    const size_t ws_bytes = sizeof(int64_t) * 2 * NG + sizeof(int32_t) * 2 * NG + 2 * sizeof(unsigned long long) + 64;
    if (!t->walk_ws) {
        t->walk_ws = dalloc(t, ws_bytes, s, t->allocs);
        if (!t->walk_ws) return RCB_ENOMEM;
    }
    int64_t *ncnt = (int64_t *)t->walk_ws;
    int64_t *fcnt = ncnt + NG;
    unsigned long long *stats = (unsigned long long *)(fcnt + NG);
    int32_t *queue = (int32_t *)(stats + 2);    // groups for the 2nd tier
    int32_t *queue2 = queue + NG;               // and for k_walk_group
    int64_t cn = 0, cf = 0;
    std::vector<void *> slabs;
    uint64_t *nslab = nullptr, *fslab = nullptr;
    for (int attempt = 0; attempt < 2 && !(nslab && fslab); ++attempt) {
        for (void *p : slabs) dfree(t, p, s);
        slabs.clear();
        slab_caps(NG, attempt == 0 ? t->n : 0, cn, cf);
        nslab = (uint64_t *)dalloc(t, sizeof(uint64_t) * NG * cn, s, slabs);
        fslab = nslab ? (uint64_t *)dalloc(t, sizeof(uint64_t) * NG * cf, s, slabs) : nullptr;
    }
    for (void *p : slabs) tmp.push_back(p);   // freed at the end unless kept
    if (!nslab || !fslab) return RCB_ENOMEM;
    // RCB_WALK_WIDE_STACK (testing): smaller wide-walk rings, so that more
    // groups take the later tiers
    int cap1 = kWQueue, cap2 = kWQueue2;
    if (const char *e = getenv("RCB_WALK_WIDE_STACK")) {
        const int v = atoi(e);
        if (v >= 2) {
            cap1 = std::min(cap1, v);
            cap2 = std::min(cap2, v);
        }
    }
    WalkArgs w{t->wrec, t->nhnode, t->k, t->gk, NG, t->p.theta * t->p.theta, ncnt, fcnt,
               nullptr, nullptr, cn, cf, nslab, fslab, t->dflag, stats};
    const unsigned grid = (unsigned)((NG + kWaves - 1) / kWaves);
    const bool pure = t->p.pure_mac != 0;
    // the three tiers over all groups, then over the groups each one queued;
    // q1/q2 null: the queues are known (second pass) and are not appended to
    int64_t nq = 0, nq2 = 0;
    // the flags (errors, list counts, the tiers' queue lengths) and the
    // statistics, read once after each tier that runs
    int32_t flags[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long hstats[2] = {0, 0};
    auto read_flags = [&]() -> rcb_status {
        const HostRead r[2] = {{t->dflag, flags, (int)sizeof(flags)}, {stats, hstats, (int)sizeof(hstats)}};
        return read_small(s, r, 2, "rcb_walk");
    };
    // the slab lists' ends per group (in the common case, that no list
    // outgrew its slab); launched before the flags are read, again if the
    // later tiers rewrote some counts
    int64_t *ends = (int64_t *)dalloc(t, sizeof(int64_t) * 4 * NG, s, t->list_allocs);
    if (!ends) return RCB_ENOMEM;
    auto slab_ends = [&]() -> rcb_status {
        k_slab_ends<<<(unsigned)((NG + kBlock - 1) / kBlock), kBlock, 0, s>>>(NG, cn, cf, ncnt, fcnt, ends, ends + NG,
                                                                              ends + 2 * NG, ends + 3 * NG);
        RCB_LAUNCH_CHECK("k_slab_ends");
        return RCB_OK;
    };
    auto walk_tiers = [&](bool count_queues) -> rcb_status {
        int32_t *q1 = count_queues ? queue : nullptr, *q2 = count_queues ? queue2 : nullptr;
        if (pure) k_walk_wide<true, kWQueue, kWaves><<<grid, kBlock, 0, s>>>(w, q1, t->dflag + 6, nullptr, 0, cap1);
        else k_walk_wide<false, kWQueue, kWaves><<<grid, kBlock, 0, s>>>(w, q1, t->dflag + 6, nullptr, 0, cap1);
        RCB_LAUNCH_CHECK("k_walk_wide");
        if (count_queues) {
            rcb_status st = slab_ends();
            if (st != RCB_OK) return st;
            st = read_flags();
            if (st != RCB_OK) return st;
            nq = flags[6];
        }
        if (nq == 0) return RCB_OK;
        if (pure) k_walk_wide<true, kWQueue2, 1><<<(unsigned)nq, kWave, 0, s>>>(w, q2, t->dflag + 7, queue, nq, cap2);
        else k_walk_wide<false, kWQueue2, 1><<<(unsigned)nq, kWave, 0, s>>>(w, q2, t->dflag + 7, queue, nq, cap2);
        RCB_LAUNCH_CHECK("k_walk_wide<2nd tier>");
        if (count_queues) {
            rcb_status st = read_flags();
            if (st != RCB_OK) return st;
            nq2 = flags[7];
        }
        if (nq2 == 0) return RCB_OK;
        const unsigned gridq = (unsigned)((nq2 + kWaves - 1) / kWaves);
        if (pure) k_walk_group<true><<<gridq, kBlock, 0, s>>>(w, queue2, nq2);
        else k_walk_group<false><<<gridq, kBlock, 0, s>>>(w, queue2, nq2);
        RCB_LAUNCH_CHECK("k_walk_group");
        if (count_queues) return read_flags();
        return RCB_OK;
    };
    RCB_ZERO(t->dflag, sizeof(int32_t) * 4, s);
    RCB_ZERO(t->dflag + 6, sizeof(int32_t) * 2, s);
    RCB_ZERO(stats, sizeof(unsigned long long) * 2, s);
    rcb_status wst = walk_tiers(true);
    if (wst != RCB_OK) return wst;
    w.stats = nullptr;   // a second walk (exact lists) does not count again
    t->walk_requeued = nq;
    t->walk_nodes = (int64_t)hstats[0];
    t->walk_tests = (int64_t)hstats[1];
    if (flags[0]) {
        set_error("walk: stack overflow (tree deeper than the walk stack supports)");
        return RCB_ECAPACITY;
    }
    if (flags[5]) {   // set by the build's node bookkeeping, which is sized never to overflow
        set_error("walk: the build reported an internal capacity error (tree not valid)");
        return RCB_EHIP;
    }
    const int32_t nlong = flags[1];
    if (flags[3] == 0) {
        if (nq > 0) {   // the later tiers rewrote the counts of their groups
            rcb_status st = slab_ends();
            if (st != RCB_OK) return st;
        }
        t->gnear_beg = ends;
        t->gnear_end = ends + NG;
        t->gfar_beg = ends + 2 * NG;
        t->gfar_end = ends + 3 * NG;
        t->gnear = nslab;
        t->gfar = fslab;
        for (void *p : slabs) {
            tmp.keep(p);
            t->list_allocs.push_back(p);
        }
    } else {
        int64_t *noff = (int64_t *)dalloc(t, sizeof(int64_t) * (NG + 1), s, t->list_allocs);
        int64_t *foff = (int64_t *)dalloc(t, sizeof(int64_t) * (NG + 1), s, t->list_allocs);
        if (!noff || !foff) return RCB_ENOMEM;
        rcb_status st = scan_i64(t, ncnt, noff, NG, s);
        if (st != RCB_OK) return st;
        st = scan_i64(t, fcnt, foff, NG, s);
        if (st != RCB_OK) return st;
        int64_t tot[2] = {0, 0};
        const HostRead r[2] = {{noff + NG, &tot[0], (int)sizeof(int64_t)}, {foff + NG, &tot[1], (int)sizeof(int64_t)}};
        st = read_small(s, r, 2, "rcb_walk");
        if (st != RCB_OK) return st;
        t->gnear = (uint64_t *)dalloc(t, sizeof(uint64_t) * std::max<int64_t>(1, tot[0]), s, t->list_allocs);
        t->gfar = (uint64_t *)dalloc(t, sizeof(uint64_t) * std::max<int64_t>(1, tot[1]), s, t->list_allocs);
        if (!t->gnear || !t->gfar) return RCB_ENOMEM;
        t->gnear_beg = noff;
        t->gnear_end = noff + 1;
        t->gfar_beg = foff;
        t->gfar_end = foff + 1;
        w.near_beg = noff;
        w.far_beg = foff;
        w.near_cap = w.far_cap = INT64_MAX;
        w.near_list = t->gnear;
        w.far_list = t->gfar;
        wst = walk_tiers(false);
        if (wst != RCB_OK) return wst;
    }
    int32_t *long_q = nullptr;
    if (nlong > 0) {
        long_q = (int32_t *)dalloc(t, sizeof(int32_t) * nlong, s, tmp);
        if (!long_q) return RCB_ENOMEM;
    }
    if (nq2 > 0) {   // the wide walk's near lists are sorted already
        k_sort_lists<kSortCap, kWaves><<<(unsigned)((nq2 + kWaves - 1) / kWaves), kBlock, 0, s>>>(
            nq2, queue2, t->gnear_beg, t->gnear_end, t->gnear, t->dflag + 2, long_q);
        RCB_LAUNCH_CHECK("k_sort_lists<near>");
    }
    if (nlong > 0) {
        k_sort_long<<<nlong, 1024, 0, s>>>(long_q, t->gnear_beg, t->gnear_end, t->gnear);
        RCB_LAUNCH_CHECK("k_sort_long");
    }
    t->walked = true;
    t->lists_kept = false;
    return RCB_OK;
}

rcb_status ensure_leaf_lists(rcb_tree *t, hipStream_t s) {
    rcb_status st = ensure_walk(t, s);
    if (st != RCB_OK) return st;
    if (t->leaf_lists) return RCB_OK;
    const int64_t L = t->nleaf;
    Scratch tmp(t, s);
    int64_t *ncnt = (int64_t *)dalloc(t, sizeof(int64_t) * L, s, tmp);
    int64_t *fcnt = (int64_t *)dalloc(t, sizeof(int64_t) * L, s, tmp);
    t->near_off = (int64_t *)dalloc(t, sizeof(int64_t) * (L + 1), s, t->list_allocs);
    t->far_off = (int64_t *)dalloc(t, sizeof(int64_t) * (L + 1), s, t->list_allocs);
    if (!ncnt || !fcnt || !t->near_off || !t->far_off) return RCB_ENOMEM;
    const unsigned grid = (unsigned)((L + kWaves - 1) / kWaves);
    k_expand<false><<<grid, kBlock, 0, s>>>(L, t->gk, t->gnear_beg, t->gnear_end, t->gnear,
                                            t->gfar_beg, t->gfar_end, t->gfar,
                                            ncnt, fcnt, nullptr, nullptr, nullptr, nullptr);
    RCB_LAUNCH_CHECK("k_expand<count>");
    st = scan_i64(t, ncnt, t->near_off, L, s);
    if (st != RCB_OK) return st;
    st = scan_i64(t, fcnt, t->far_off, L, s);
    if (st != RCB_OK) return st;
    int64_t tot[2] = {0, 0};
    RCB_HIP(hipMemcpyAsync(&tot[0], t->near_off + L, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RCB_HIP(hipMemcpyAsync(&tot[1], t->far_off + L, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RCB_HIP(hipStreamSynchronize(s));
    t->near_list = (int32_t *)dalloc(t, sizeof(int32_t) * std::max<int64_t>(1, tot[0]), s, t->list_allocs);
    t->far_list = (int32_t *)dalloc(t, sizeof(int32_t) * std::max<int64_t>(1, tot[1]), s, t->list_allocs);
    if (!t->near_list || !t->far_list) return RCB_ENOMEM;
    k_expand<true><<<grid, kBlock, 0, s>>>(L, t->gk, t->gnear_beg, t->gnear_end, t->gnear,
                                           t->gfar_beg, t->gfar_end, t->gfar,
                                           nullptr, nullptr, t->near_off, t->far_off, t->near_list,
                                           t->far_list);
    RCB_LAUNCH_CHECK("k_expand<fill>");
    t->near_total = tot[0];
    t->far_total = tot[1];
    t->leaf_lists = true;
    return RCB_OK;
}

void drop_lists(rcb_tree *t, hipStream_t s) {
    for (void *p : t->list_allocs) dfree(t, p, s);
    t->list_allocs.clear();
    t->walked = false;
    t->lists_kept = false;
    t->gnear_beg = t->gnear_end = t->gfar_beg = t->gfar_end = nullptr;
    t->gnear = t->gfar = nullptr;
    t->leaf_lists = false;
    t->near_total = t->far_total = -1;
    t->near_off = t->far_off = nullptr;
    t->near_list = t->far_list = nullptr;
    t->nb_total = -1;
    t->nb_slab = t->nb_pool = t->nb_head = t->nb_longq = t->nb_longc = t->nb_queue = t->nb_ctl = nullptr;
    t->nb_pool_cap = 0;
    t->nb_over = t->nb_long = t->nb_nq = 0;
    t->walk_requeued = 0;
    t->walk_nodes = t->walk_tests = -1;
    t->farc = nullptr;
    t->farc_valid = false;
}

}  // namespace rcb
