// rcb_internal.h -- private declarations of the MI355X RCB-tree library.
//
// Layout in HBM (all arrays owned by the tree, allocated stream-ordered):
//   particles, tree order (a node's particles are contiguous, Sec. 2.1
//   "Particle sorting"): px py pz pm ph (FP64), pid (int32 caller index);
//   mixed form adds fdx fdy fdz (FP32 offset from the leaf centre of mass),
//   fm fh (FP32).
//   nodes, indexed by label (root 1, children 2n and 2n+1, Sec. 2.1 "Node
//   labelling"): nfirst ncount (int32), nlo nhi ncom (3 FP64 per label),
//   nM nhint nhnode (FP64), nQ (6 FP64 per label), nplane + naxis (split).
//   walk records: two double4 per label {g.xyz, h_int} {com.xyz, H_B};
//   an empty node has h_int = -1.
//   interaction lists: per leaf CSR, near entries = label | candidate << 31.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "rcb.h"

namespace rcb {

constexpr int kLeafC = 22;   // doubles per leaf in rcb_tree::farc

constexpr int kWave = 64;
constexpr int kChunk = 512;          // elements per wave item of the big-node passes
constexpr double kReachPad = 1.0 + 0x1p-32;

struct BuildScratch {
    // ping-pong particle buffers
    double *x[2], *y[2], *z[2], *m[2];
    // big-node machinery
    int32_t *ctl;          // [0] big-node count, [1] item count, [2] groups left by the packed pass
    int32_t *big_node;     // big-node list (labels)
    int32_t *big_base;     // first item of each big node
    int32_t *item_big;     // item -> big-node index
    double *part;          // item partial sums, 8 doubles per item
    int32_t *part_left;    // item left-flag counts, then exclusive offsets
    int32_t *naxis;        // split axis per label
    double *nplane;        // split coordinate per label
    double *bounds;        // per-block min/max partials (6 per block)
    int32_t *pack_groups;  // 8-node groups the packed pass leaves to k_level_small
    int64_t max_items;
    int64_t max_big;
};

}  // namespace rcb

struct rcb_tree {
    int64_t n = 0;
    int k = 0;
    int64_t nleaf = 0;
    int64_t nlab = 0;
    rcb_params p{};
    hipStream_t stream = nullptr;
    int device = 0;

    double *px = nullptr, *py = nullptr, *pz = nullptr, *pm = nullptr, *ph = nullptr;
    int32_t *pid = nullptr;            // tree position -> caller index (= lvl_id of level k)
    int32_t *lvl_id = nullptr;         // (k + 1) x n: the order at each level of the build
    float *fdx = nullptr, *fdy = nullptr, *fdz = nullptr, *fm = nullptr, *fh = nullptr;

    int32_t *nfirst = nullptr, *ncount = nullptr;
    double *nlo = nullptr, *nhi = nullptr, *ncom = nullptr, *nM = nullptr, *nQ = nullptr;
    double *nhint = nullptr, *nhnode = nullptr;
    double4 *wrec = nullptr;

    // interaction lists per group of 2^gk sibling leaves (gk = min(3, k)):
    // near entries label | near_mask << 32 | candidate_mask << 40 (sorted by
    // label), far entries label | far_mask << 32
    int gk = 0;
    int64_t ngroup = 0;
    bool walked = false;
    // the lists were kept across a refresh (the tree held fixed): gravity and
    // the VJP use them, the neighbour search needs a new walk
    bool lists_kept = false;
    // group list of group g: gnear[gnear_beg[g] .. gnear_end[g]) (likewise far)
    int64_t *gnear_beg = nullptr, *gnear_end = nullptr, *gfar_beg = nullptr, *gfar_end = nullptr;
    uint64_t *gnear = nullptr, *gfar = nullptr;
    // per-leaf lists, expanded from the group lists on demand (inspection)
    bool leaf_lists = false;
    int64_t near_total = -1, far_total = -1;
    int64_t *near_off = nullptr, *far_off = nullptr;
    void *walk_ws = nullptr;   // the walk's per-group counts, queues and statistics (kept for later walks)
    int32_t *near_list = nullptr, *far_list = nullptr;
    int64_t nb_total = -1;             // neighbour total of the last count call
    int32_t *nb_slab = nullptr;        // neighbour ids of the count call, kNbCap per particle
    int32_t *nb_pool = nullptr;        // overflow chunks of the slab rows
    int32_t *nb_head = nullptr;        // per particle: its chunk (lists past the row)
    int32_t *nb_longq = nullptr;       // particles whose list sits in row + chunks
    int32_t *nb_longc = nullptr;       // the chunks of each nb_longq entry
    int32_t *nb_queue = nullptr;       // leaves holding a list that the fill call searches again
    int32_t *nb_ctl = nullptr;         // device counters of the count call
    int64_t nb_pool_cap = 0;           // chunks in nb_pool
    int32_t nb_over = 0;               // lists the fill call searches again
    int32_t nb_long = 0;               // lists kept in row + chunk
    int32_t nb_nq = 0;                 // entries of nb_queue
    // device flags: [0] 8-wide walk stack overflow, [1] long near lists, [2] their
    // queue, [3] groups outgrowing the list slabs, [4] particles outgrowing
    // the neighbour slab, [5] median selection, [6] groups outgrowing the
    // first wide-walk FIFO, [7] groups outgrowing the second FIFO (walk) and
    // leaves queued for the neighbour re-search (neighbours)
    int32_t *dflag = nullptr;
    int64_t walk_requeued = 0;         // groups of the last walk that outgrew the first ring
    int64_t walk_nodes = -1;           // node records the first walk tier tested (per group)
    int64_t walk_tests = -1;           // (node, visiting leaf) tests of the first tier
    // per leaf: the 19 far-field coefficients of the current moments (written
    // by rcb_gravity, or by the VJP if no gravity call has) and 3 VJP scratch values
    double *farc = nullptr;
    bool farc_valid = false;

    std::vector<void *> allocs;        // everything to free on destroy
    std::vector<void *> list_allocs;
};

namespace rcb {

void set_error(const std::string &msg);
rcb_status hip_fail(hipError_t e, const char *what);
void *dalloc(rcb_tree *t, size_t bytes, hipStream_t s, std::vector<void *> &owner);
// Small device values read by the host once the work queued on s before them
// has run, without synchronising the stream: a one-thread kernel copies them
// into coherent pinned memory (one buffer per host thread) and writes a
// sequence number after them, which the host polls. Each item is a multiple
// of 4 bytes, 4-byte aligned; at most kReadItems items of kReadBytes in all.
constexpr int kReadItems = 8;
constexpr int kReadBytes = 128;
struct HostRead {
    const void *src;   // device
    void *dst;         // host
    int bytes;
};
rcb_status read_small(hipStream_t s, const HostRead *items, int n, const char *what);
// Zeroes `bytes` (a multiple of 4, 4-byte aligned) at p in stream order with a
// kernel of the library (hipMemsetAsync's fill left the device idle for tens
// of microseconds before it, and cannot go into a captured graph).
rcb_status zero_async(void *p, size_t bytes, hipStream_t s);
// Polls host word w until it equals seq (the stream is queried only once the
// wait is long, for errors); a report that does not come ends with an error.
rcb_status wait_host_word(volatile int32_t *w, int32_t seq, hipStream_t s, const char *what);
// releases a dalloc block in stream order (large blocks stay cached for reuse)
void dfree(rcb_tree *t, void *p, hipStream_t s);

// Scratch blocks of one call: every block still listed when the scope ends
// (on success and on every error return) is released in stream order. A
// block handed over to the tree is taken out with keep().
struct Scratch : std::vector<void *> {
    rcb_tree *t;
    hipStream_t s;
    Scratch(rcb_tree *t_, hipStream_t s_) : t(t_), s(s_) {}
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    void keep(void *p) {
        for (auto &q : *this)
            if (q == p) q = nullptr;
    }
    ~Scratch() {
        for (void *p : *this)
            if (p) dfree(t, p, s);
    }
};

// Forget the interaction lists and everything made from them (neighbour
// slab, kept far coefficients); the next call that needs lists walks again.
void drop_lists(rcb_tree *t, hipStream_t s);

// build (k_build.hip)
rcb_status build_tree(rcb_tree *t, const double *x, const double *y, const double *z,
                      const double *m, const double *h, hipStream_t s);
// particles whose new position lies outside their lowest-level cell (k_build.hip)
rcb_status count_outside(rcb_tree *t, const double *x, const double *y, const double *z,
                         int64_t *outside, hipStream_t s);
// moments-only refresh with new inputs, topology held fixed (k_build.hip)
rcb_status refresh_tree(rcb_tree *t, const double *x, const double *y, const double *z,
                        const double *m, const double *h, hipStream_t s);
// the same with its scratch in the library's static device array: no
// allocation; RCB_ECAPACITY if the tree needs more than the array holds
rcb_status refresh_tree_noalloc(rcb_tree *t, const double *x, const double *y, const double *z,
                                const double *m, const double *h, hipStream_t s);
size_t refresh_noalloc_bytes(const rcb_tree *t);
size_t refresh_noalloc_capacity();
// device exclusive scan of int64 counts in place-free form: out[0..n] (k_scan.hip)
rcb_status scan_i64(rcb_tree *t, const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
// stable sort of items by bits 32 .. 32 + bits - 1 (k_sort.hip); a and b hold n
// items each, the input in a; *result is a or b, whichever holds the output
rcb_status sort_by_label(rcb_tree *t, uint64_t *a, uint64_t *b, int64_t n, int bits,
                         hipStream_t s, uint64_t **result);
// walk (k_walk.hip)
rcb_status ensure_walk(rcb_tree *t, hipStream_t s);
rcb_status ensure_leaf_lists(rcb_tree *t, hipStream_t s);
// neighbours (k_neigh.hip)
rcb_status neighbours_count(rcb_tree *t, int64_t *offsets, int64_t *total, hipStream_t s);
rcb_status neighbours_fill(rcb_tree *t, const int64_t *offsets, int32_t *ids, int64_t cap,
                           hipStream_t s);
// gravity (k_grav.hip)
rcb_status gravity(rcb_tree *t, void *ax, void *ay, void *az, hipStream_t s);
// far-field coefficients f, J, H (19 per leaf, at stride) of every leaf
rcb_status far_coefficients(rcb_tree *t, double *out, int stride, hipStream_t s);
// vjp (k_vjp.hip)
rcb_status gravity_vjp(rcb_tree *t, const void *gx, const void *gy, const void *gz, void *dx,
                       void *dy, void *dz, void *dm, hipStream_t s);

// ---------------------------------------------------------------------------
// device helpers shared by the kernels of this library
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Index of this wave in the grid, passed through readfirstlane so that the
// compiler treats it, and everything derived from it, as wave-uniform
// (scalar registers and scalar loads).
__device__ __forceinline__ int64_t wave_index() {
    const uint32_t w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    return (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)w);
}

// Workgroups are handed to the 8 XCDs in turn (workgroup b to XCD b mod 8),
// and each XCD has its own L2. xcd_block() renumbers them so that XCD x takes
// one contiguous range of logical workgroups: neighbouring groups of cells,
// which share sources and tree nodes, then meet in the same L2. A bijection
// on [0, gridDim.x) for any grid size.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t b = blockIdx.x, nb = gridDim.x;
    const uint32_t q = nb / kXcds, r = nb % kXcds, x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}
__device__ __forceinline__ int64_t xcd_wave_index() {
    const uint32_t w = xcd_block() * (blockDim.x / kWave) + threadIdx.x / kWave;
    return (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)w);
}

// Canonical sum of the 64 lane values: adjacent lanes first, then pairs of
// pairs (xor butterfly; both partners of a pair get the same, commutative sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
// exclusive prefix sum over lanes
__device__ __forceinline__ int wave_excl_scan(int v) {
    int x = v;
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(x, o, kWave);
        if (l >= o) x += y;
    }
    return x - v;
}
__device__ __forceinline__ int64_t wave_excl_scan64(int64_t v) {
    int64_t x = v;
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int64_t y = __shfl_up(x, o, kWave);
        if (l >= o) x += y;
    }
    return x - v;
}
// A value known to be equal on every lane, moved to scalar registers.
__device__ __forceinline__ double uniform_f64(double v) {
    union {
        double d;
        int w[2];
    } u;
    u.d = v;
    u.w[0] = __builtin_amdgcn_readfirstlane(u.w[0]);
    u.w[1] = __builtin_amdgcn_readfirstlane(u.w[1]);
    return u.d;
}
// The value of the other lane of this lane's pair (2j, 2j + 1), by DPP.
__device__ __forceinline__ double swap_adjacent_lanes(double v) {
    union {
        double d;
        int w[2];
    } u, r;
    u.d = v;
    r.w[0] = __builtin_amdgcn_mov_dpp(u.w[0], 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    r.w[1] = __builtin_amdgcn_mov_dpp(u.w[1], 0xB1, 0xF, 0xF, false);
    return r.d;
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ int rank_below(uint64_t mask) {
    const int l = lane_id();
    uint64_t below = l ? (mask & ((~0ull) >> (64 - l))) : 0ull;
    return __popcll(below);
}
__device__ __forceinline__ double dist2(double ax, double ay, double az, double bx, double by,
                                        double bz) {
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return (dx * dx + dy * dy) + dz * dz;
}

}  // namespace rcb

#define RCB_HIP(expr)                                         \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return rcb::hip_fail(_e, #expr); \
    } while (0)

#define RCB_ZERO(p, bytes, stream)                                     \
    do {                                                               \
        rcb_status _z = rcb::zero_async((p), (bytes), (stream));       \
        if (_z != RCB_OK) return _z;                                   \
    } while (0)
#define RCB_LAUNCH_CHECK(name)                                   \
    do {                                                         \
        hipError_t _e = hipGetLastError();                       \
        if (_e != hipSuccess) return rcb::hip_fail(_e, name);    \
    } while (0)
