// rcb_api.hip -- the C ABI declared in include/rcb.h: argument checks on the
// host, tree lifetime, stream-ordered device memory.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "rcb_internal.h"

namespace rcb {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

__global__ void k_fill_f64(double *v, int64_t n, double value) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) v[i] = value;
}

rcb_status hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? RCB_ENOMEM : RCB_EHIP;
}

rcb_status wait_host_word(volatile int32_t *w, int32_t seq, hipStream_t s, const char *what) {
    const auto t0 = std::chrono::steady_clock::now();
    auto next_query = t0 + std::chrono::milliseconds(200);
    for (uint64_t spin = 0;; ++spin) {
        if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return RCB_OK;
        // the stream is queried (for a failed stream) only once the wait is
        // long, and then rarely: each query put a marker between the queued
        // kernels, which left the device idle for microseconds each time
        if ((spin & 1023) != 1023) continue;
        const auto now = std::chrono::steady_clock::now();
        if (now >= next_query) {
            next_query = now + std::chrono::milliseconds(50);
            const hipError_t q = hipStreamQuery(s);
            if (q != hipSuccess && q != hipErrorNotReady) return hip_fail(q, what);
            if (q == hipSuccess && __atomic_load_n(w, __ATOMIC_ACQUIRE) != seq) {
                set_error(std::string(what) + ": the device's report did not arrive");
                return RCB_EHIP;
            }
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(10)) {
                set_error(std::string(what) + ": timed out waiting for the device's report");
                return RCB_EHIP;
            }
        }
    }
}

namespace {
__global__ void k_zero(uint32_t *p, int64_t words) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}
}  // namespace

rcb_status zero_async(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return RCB_OK;
    if (bytes % 4 != 0 || ((uintptr_t)p & 3) != 0) {
        set_error("zero_async: unaligned block");
        return RCB_EINVAL;
    }
    const int64_t words = (int64_t)(bytes / 4);
    const unsigned grid = (unsigned)std::min<int64_t>(2048, (words + 255) / 256);
    k_zero<<<grid, 256, 0, s>>>((uint32_t *)p, words);
    RCB_LAUNCH_CHECK("k_zero");
    return RCB_OK;
}

namespace {
struct ReadArgs {
    const int32_t *src[kReadItems];
    int words[kReadItems];
    int n;
    volatile int32_t *box;   // [0] sequence number, data from [4]
    int32_t seq;
};

__global__ void k_read_small(ReadArgs r) {
    int o = 4;
    for (int i = 0; i < r.n; ++i)
        for (int w = 0; w < r.words[i]; ++w) r.box[o++] = r.src[i][w];
    __threadfence_system();
    r.box[0] = r.seq;
}
}  // namespace

rcb_status read_small(hipStream_t s, const HostRead *items, int n, const char *what) {
    static thread_local int32_t *box = nullptr, *dbox = nullptr;
    static thread_local int32_t seq = 0;
    if (n < 0 || n > kReadItems) {
        set_error(std::string(what) + ": too many values for one read");
        return RCB_EINVAL;
    }
    if (!box) {
        if (hipHostMalloc((void **)&box, sizeof(int32_t) * (4 + kReadBytes / 4),
                          hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
            box = nullptr;
            return hip_fail(hipErrorOutOfMemory, "hipHostMalloc(read buffer)");
        }
        box[0] = 0;
        if (hipHostGetDevicePointer((void **)&dbox, box, 0) != hipSuccess) {
            (void)hipHostFree(box);
            box = nullptr;
            return hip_fail(hipErrorInvalidValue, "hipHostGetDevicePointer(read buffer)");
        }
    }
    ReadArgs r{};
    int total = 0;
    for (int i = 0; i < n; ++i) {
        if (items[i].bytes % 4 != 0 || ((uintptr_t)items[i].src & 3) != 0) {
            set_error(std::string(what) + ": unaligned value");
            return RCB_EINVAL;
        }
        r.src[i] = (const int32_t *)items[i].src;
        r.words[i] = items[i].bytes / 4;
        total += items[i].bytes;
    }
    if (total > kReadBytes) {
        set_error(std::string(what) + ": values too large for one read");
        return RCB_EINVAL;
    }
    r.n = n;
    r.box = dbox;
    r.seq = ++seq;
    k_read_small<<<1, 1, 0, s>>>(r);
    RCB_LAUNCH_CHECK("k_read_small");
    rcb_status st = wait_host_word(box, r.seq, s, what);
    if (st != RCB_OK) return st;
    int o = 4;
    for (int i = 0; i < n; ++i) {
        memcpy(items[i].dst, box + o, items[i].bytes);
        o += items[i].bytes / 4;
    }
    return RCB_OK;
}

// Device memory of the library's own allocator. Blocks come from the
// device's default stream-ordered pool (its release threshold raised once per
// device, restored by rcb_release_cache) and, once freed, are kept by the
// library: a later request on the same device and the same stream that a
// kept block fits within a factor of two takes it back with no HIP call at
// all. Reuse on the stream that freed the block is safe in stream order with
// no event; a free therefore costs no HIP call either (each stream-ordered
// free put a marker into the stream that held the device for several
// microseconds between the kernels around it). A device keeps at most a
// quarter of its memory this way (past that, frees go to the pool). Kept
// blocks go back to the pool when an allocation fails and in
// rcb_release_cache, after the device has finished its work (the freeing
// streams are never used again, so they may have been destroyed by then).
namespace {
constexpr int kMaxDevices = 64;
struct KeptBlock {
    void *p;
    size_t bytes;
    int device;
    hipStream_t stream;   // freed on; compared, never used
};
std::mutex g_cache_mu;
std::vector<KeptBlock> g_kept;                         // free, kept for reuse
std::unordered_map<void *, size_t> g_live;             // the library's blocks in use: their size
bool g_pool_set[kMaxDevices] = {false};
uint64_t g_pool_thr[kMaxDevices] = {0};
size_t g_kept_bytes[kMaxDevices] = {0};
size_t g_kept_cap[kMaxDevices] = {0};

// Returns the kept blocks of `device` (all devices if < 0) to the pool once
// the device is idle, and trims the pool of every device concerned;
// g_cache_mu held.
void release_kept_locked(int device) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    bool touched[kMaxDevices] = {false};
    for (const KeptBlock &b : g_kept)
        if ((device < 0 || b.device == device) && b.device >= 0 && b.device < kMaxDevices) touched[b.device] = true;
    for (int d = 0; d < kMaxDevices; ++d) {
        if (!touched[d]) continue;
        (void)hipSetDevice(d);
        (void)hipDeviceSynchronize();   // every kept block's last use has finished
    }
    for (auto it = g_kept.begin(); it != g_kept.end();) {
        if (device >= 0 && it->device != device) {
            ++it;
            continue;
        }
        (void)hipSetDevice(it->device);
        (void)hipFreeAsync(it->p, nullptr);
        if (it->device >= 0 && it->device < kMaxDevices) g_kept_bytes[it->device] -= it->bytes;
        it = g_kept.erase(it);
    }
    for (int d = 0; d < kMaxDevices; ++d) {
        if (!touched[d]) continue;
        hipMemPool_t pool;
        (void)hipSetDevice(d);
        (void)hipDeviceSynchronize();
        if (hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
    }
    (void)hipSetDevice(cur);
    (void)hipGetLastError();
}
}  // namespace

void *dalloc(rcb_tree *t, size_t bytes, hipStream_t s, std::vector<void *> &owner) {
    if (t->p.alloc) {   // the caller's allocator
        void *q = t->p.alloc(bytes ? bytes : 16, (void *)s, t->p.alloc_ctx);
        if (!q) set_error("workspace allocator returned NULL for " + std::to_string(bytes) + " bytes");
        owner.push_back(q);
        return q;
    }
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (t->device >= 0 && t->device < kMaxDevices && !g_pool_set[t->device]) {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, t->device) == hipSuccess &&
            hipMemPoolGetAttribute(pool, hipMemPoolAttrReleaseThreshold, &g_pool_thr[t->device]) ==
                hipSuccess) {
            uint64_t thr = UINT64_MAX;
            hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
            g_pool_set[t->device] = true;
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) == hipSuccess) g_kept_cap[t->device] = tot / 4;
        }
        (void)hipGetLastError();
    }
    bytes = (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
    auto pick = g_kept.end();
    for (auto it = g_kept.begin(); it != g_kept.end(); ++it)
        if (it->device == t->device && it->stream == s && it->bytes >= bytes && it->bytes <= 2 * bytes &&
            (pick == g_kept.end() || it->bytes < pick->bytes))
            pick = it;
    void *p = nullptr;
    if (pick != g_kept.end()) {
        p = pick->p;
        g_live[p] = pick->bytes;
        g_kept_bytes[pick->device] -= pick->bytes;
        g_kept.erase(pick);
        owner.push_back(p);
        return p;
    }
    hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess && !g_kept.empty()) {
        (void)hipGetLastError();
        release_kept_locked(t->device);
        e = hipMallocAsync(&p, bytes, s);
    }
    if (e != hipSuccess) {
        set_error(std::string("hipMallocAsync(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
        (void)hipGetLastError();
        p = nullptr;
    } else {
        g_live[p] = bytes;
    }
    owner.push_back(p);
    return p;
}

void dfree(rcb_tree *t, void *p, hipStream_t s) {
    if (!p) return;
    if (t->p.free) {   // the caller's allocator
        t->p.free(p, (void *)s, t->p.alloc_ctx);
        return;
    }
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) {   // not the library's (never: every block is registered)
        (void)hipFreeAsync(p, s);
        (void)hipGetLastError();
        return;
    }
    const size_t bytes = it->second;
    g_live.erase(it);
    const int d = t->device;
    if (d < 0 || d >= kMaxDevices || g_kept_bytes[d] + bytes > g_kept_cap[d]) {
        (void)hipFreeAsync(p, s);   // past the cap: back to the pool
        (void)hipGetLastError();
        return;
    }
    g_kept.push_back(KeptBlock{p, bytes, d, s});
    g_kept_bytes[d] += bytes;
}

// frees every block in stream order on s (after the tree's last work on its
// own stream); the memory is reused only by work queued after the frees
static void free_all(rcb_tree *t, hipStream_t s) {
    if (s != t->stream) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
            (void)hipEventRecord(ev, t->stream);
            (void)hipStreamWaitEvent(s, ev, 0);
            (void)hipEventDestroy(ev);
        } else {
            (void)hipStreamSynchronize(t->stream);
        }
    }
    for (void *p : t->list_allocs) dfree(t, p, s);
    for (void *p : t->allocs) dfree(t, p, s);
    t->list_allocs.clear();
    t->allocs.clear();
}

}  // namespace rcb

using namespace rcb;

extern "C" {

void rcb_params_default(rcb_params *p) {
    if (!p) return;
    p->n_ll = 12;
    p->precision = RCB_FP64;
    p->theta = 0.7;
    p->validate = 0;
    p->pure_mac = 0;
    p->split = RCB_SPLIT_MASS;
    p->taylor_reading = RCB_READING_A;
    p->deterministic = 0;
    p->alloc = nullptr;
    p->free = nullptr;
    p->alloc_ctx = nullptr;
}

const char *rcb_last_error(void) { return g_last_error.c_str(); }

rcb_status rcb_build(const double *x, const double *y, const double *z, const double *m,
                     const double *h, int64_t n, const rcb_params *p, void *stream,
                     rcb_tree **out) {
    g_last_error.clear();
    if (!out) {
        set_error("rcb_build: out is NULL");
        return RCB_EINVAL;
    }
    *out = nullptr;
    if (!x || !y || !z || !m || !h || !p) {
        set_error("rcb_build: NULL input pointer or params");
        return RCB_EINVAL;
    }
    if (n < 1 || n > 0x7fffffffLL) {
        set_error("rcb_build: n must be in [1, 2^31 - 1]");
        return RCB_EINVAL;
    }
    if (p->n_ll < 1) {
        set_error("rcb_build: n_ll must be >= 1");
        return RCB_EINVAL;
    }
    if (!(p->theta >= 0.0) || !std::isfinite(p->theta)) {
        set_error("rcb_build: theta must be finite and >= 0");
        return RCB_EINVAL;
    }
    if (p->precision != RCB_FP64 && p->precision != RCB_MIXED) {
        set_error("rcb_build: unknown precision");
        return RCB_EINVAL;
    }
    if (p->pure_mac != 0 && p->pure_mac != 1) {
        set_error("rcb_build: pure_mac must be 0 or 1");
        return RCB_EINVAL;
    }
    if ((p->alloc == nullptr) != (p->free == nullptr)) {
        set_error("rcb_build: alloc and free must be given together");
        return RCB_EINVAL;
    }
    if (p->taylor_reading != RCB_READING_A && p->taylor_reading != RCB_READING_B) {
        set_error("rcb_build: taylor_reading must be RCB_READING_A or RCB_READING_B");
        return RCB_EINVAL;
    }
    if (p->deterministic != 0 && p->deterministic != 1) {
        set_error("rcb_build: deterministic must be 0 or 1");
        return RCB_EINVAL;
    }
    if (p->split != RCB_SPLIT_MASS && p->split != RCB_SPLIT_NUMBER && p->split != RCB_SPLIT_MEDIAN) {
        set_error("rcb_build: unknown split");
        return RCB_EINVAL;
    }
    int k = 0;
    while ((int64_t)p->n_ll * ((int64_t)1 << k) < n) ++k;
    if (k > 29) {
        set_error("rcb_build: tree deeper than 29 levels (n / n_ll too large)");
        return RCB_EINVAL;
    }
    rcb_tree *t = new rcb_tree();
    t->n = n;
    t->k = k;
    t->nleaf = (int64_t)1 << k;
    t->nlab = (int64_t)2 << k;
    t->gk = k < 3 ? k : 3;
    t->ngroup = (int64_t)1 << (k - t->gk);
    t->p = *p;
    t->stream = (hipStream_t)stream;
    if (hipGetDevice(&t->device) != hipSuccess) t->device = 0;
    rcb_status st;
    if (p->split == RCB_SPLIT_NUMBER) {
        // planes through the centre of number: build with unit weights (the
        // canonical sums then give sum(x) / count exactly), then recompute
        // every moment with the masses on the fixed tree
        Scratch tmp(t, t->stream);
        double *ones = (double *)dalloc(t, sizeof(double) * (size_t)n, t->stream, tmp);
        if (!ones) {
            st = RCB_ENOMEM;
        } else {
            k_fill_f64<<<(unsigned)((n + 255) / 256), 256, 0, t->stream>>>(ones, n, 1.0);
            st = hipGetLastError() == hipSuccess ? RCB_OK : RCB_EHIP;
            if (st == RCB_OK) st = build_tree(t, x, y, z, ones, h, t->stream);
            if (st == RCB_OK) st = refresh_tree(t, x, y, z, m, h, t->stream);
        }
    } else {
        st = build_tree(t, x, y, z, m, h, t->stream);
    }
    if (st != RCB_OK) {
        std::string msg = g_last_error;
        free_all(t, t->stream);
        delete t;
        g_last_error = msg;
        return st;
    }
    *out = t;
    return RCB_OK;
}

rcb_status rcb_check_cells(rcb_tree *t, const double *x, const double *y, const double *z,
                           int64_t n, int64_t *outside, void *stream) {
    g_last_error.clear();
    if (!t || !x || !y || !z || !outside) {
        set_error("rcb_check_cells: NULL argument");
        return RCB_EINVAL;
    }
    if (n != t->n) {
        set_error("rcb_check_cells: n = " + std::to_string(n) + " differs from the built n = " +
                  std::to_string(t->n));
        return RCB_ESTATE;
    }
    t->stream = (hipStream_t)stream;
    return count_outside(t, x, y, z, outside, t->stream);
}

rcb_status rcb_refresh(rcb_tree *t, const double *x, const double *y, const double *z,
                       const double *m, const double *h, int64_t n, int32_t keep_lists,
                       void *stream) {
    g_last_error.clear();
    if (!t || !x || !y || !z || !m || !h) {
        set_error("rcb_refresh: NULL argument");
        return RCB_EINVAL;
    }
    if (n != t->n) {
        set_error("rcb_refresh: n = " + std::to_string(n) + " differs from the built n = " +
                  std::to_string(t->n));
        return RCB_ESTATE;
    }
    if (keep_lists != 0 && keep_lists != 1) {
        set_error("rcb_refresh: keep_lists must be 0 or 1");
        return RCB_EINVAL;
    }
    t->stream = (hipStream_t)stream;
    rcb_status st = refresh_tree(t, x, y, z, m, h, t->stream);
    if (st != RCB_OK) return st;
    if (!keep_lists) drop_lists(t, t->stream);   // walked again by the next call that needs lists
    else if (t->walked) t->lists_kept = true;
    return RCB_OK;
}

rcb_status rcb_refresh_noalloc(rcb_tree *t, const double *x, const double *y, const double *z,
                               const double *m, const double *h, int64_t n, void *stream) {
    g_last_error.clear();
    if (!t || !x || !y || !z || !m || !h) {
        set_error("rcb_refresh_noalloc: NULL argument");
        return RCB_EINVAL;
    }
    if (n != t->n) {
        set_error("rcb_refresh_noalloc: n = " + std::to_string(n) + " differs from the built n = " +
                  std::to_string(t->n));
        return RCB_ESTATE;
    }
    t->stream = (hipStream_t)stream;
    rcb_status st = refresh_tree_noalloc(t, x, y, z, m, h, t->stream);
    if (st != RCB_OK) return st;
    if (t->walked) t->lists_kept = true;   // as rcb_refresh(keep_lists = 1): nothing is freed
    return RCB_OK;
}

size_t rcb_refresh_noalloc_scratch(const rcb_tree *t) {
    return t ? refresh_noalloc_bytes(t) : refresh_noalloc_capacity();
}

rcb_status rcb_walk(rcb_tree *t, void *stream) {
    g_last_error.clear();
    if (!t) {
        set_error("rcb_walk: NULL tree");
        return RCB_EINVAL;
    }
    t->stream = (hipStream_t)stream;
    if (t->lists_kept) drop_lists(t, t->stream);   // lists of older inputs: walk again
    return ensure_walk(t, t->stream);
}

rcb_status rcb_neighbours_count(rcb_tree *t, int64_t *offsets, int64_t *total, void *stream) {
    g_last_error.clear();
    if (!t || !offsets || !total) {
        set_error("rcb_neighbours_count: NULL argument");
        return RCB_EINVAL;
    }
    t->stream = (hipStream_t)stream;
    return neighbours_count(t, offsets, total, t->stream);
}

rcb_status rcb_neighbours_fill(rcb_tree *t, const int64_t *offsets, int32_t *ids, int64_t capacity,
                               void *stream) {
    g_last_error.clear();
    if (!t || !offsets || (!ids && capacity > 0)) {
        set_error("rcb_neighbours_fill: NULL argument");
        return RCB_EINVAL;
    }
    if (capacity < 0) {
        set_error("rcb_neighbours_fill: negative capacity");
        return RCB_EINVAL;
    }
    t->stream = (hipStream_t)stream;
    return neighbours_fill(t, offsets, ids, capacity, t->stream);
}

rcb_status rcb_gravity(rcb_tree *t, void *ax, void *ay, void *az, void *stream) {
    g_last_error.clear();
    if (!t || !ax || !ay || !az) {
        set_error("rcb_gravity: NULL argument");
        return RCB_EINVAL;
    }
    t->stream = (hipStream_t)stream;
    return gravity(t, ax, ay, az, t->stream);
}

rcb_status rcb_gravity_vjp(rcb_tree *t, const void *gx, const void *gy, const void *gz, void *dx,
                           void *dy, void *dz, void *dm, void *stream) {
    g_last_error.clear();
    if (!t || !gx || !gy || !gz || !dx || !dy || !dz || !dm) {
        set_error("rcb_gravity_vjp: NULL argument");
        return RCB_EINVAL;
    }
    if (t->p.taylor_reading != RCB_READING_A) {
        set_error("rcb_gravity_vjp: defined for Taylor reading A only");
        return RCB_EINVAL;
    }
    t->stream = (hipStream_t)stream;
    return gravity_vjp(t, gx, gy, gz, dx, dy, dz, dm, t->stream);
}

rcb_status rcb_get_info(const rcb_tree *t, rcb_tree_info *info) {
    if (!t || !info) {
        set_error("rcb_get_info: NULL argument");
        return RCB_EINVAL;
    }
    info->n = t->n;
    info->k = t->k;
    info->precision = t->p.precision;
    info->n_labels = t->nlab;
    info->near_total = t->leaf_lists ? t->near_total : -1;
    info->far_total = t->leaf_lists ? t->far_total : -1;
    info->theta = t->p.theta;
    info->walk_requeued = t->walked ? t->walk_requeued : -1;
    info->walk_nodes = t->walked ? t->walk_nodes : -1;
    info->walk_tests = t->walked ? t->walk_tests : -1;
    return RCB_OK;
}

rcb_status rcb_tree_export(rcb_tree *t, int32_t field, void *dst, size_t bytes, void *stream) {
    g_last_error.clear();
    if (!t || !dst) {
        set_error("rcb_tree_export: NULL argument");
        return RCB_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    t->stream = s;
    if (field >= RCB_FIELD_NEAR_OFF) {
        rcb_status st = ensure_leaf_lists(t, s);
        if (st != RCB_OK) return st;
    }
    const void *src = nullptr;
    size_t need = 0;
    const size_t L = (size_t)t->nlab;
    switch (field) {
        case RCB_FIELD_PERM: src = t->pid; need = sizeof(int32_t) * (size_t)t->n; break;
        case RCB_FIELD_FIRST: src = t->nfirst; need = sizeof(int32_t) * L; break;
        case RCB_FIELD_COUNT: src = t->ncount; need = sizeof(int32_t) * L; break;
        case RCB_FIELD_LO: src = t->nlo; need = sizeof(double) * 3 * L; break;
        case RCB_FIELD_HI: src = t->nhi; need = sizeof(double) * 3 * L; break;
        case RCB_FIELD_COM: src = t->ncom; need = sizeof(double) * 3 * L; break;
        case RCB_FIELD_MASS: src = t->nM; need = sizeof(double) * L; break;
        case RCB_FIELD_QUAD: src = t->nQ; need = sizeof(double) * 6 * L; break;
        case RCB_FIELD_HINT: src = t->nhint; need = sizeof(double) * L; break;
        case RCB_FIELD_HNODE: src = t->nhnode; need = sizeof(double) * L; break;
        case RCB_FIELD_NEAR_OFF: src = t->near_off; need = sizeof(int64_t) * ((size_t)t->nleaf + 1); break;
        case RCB_FIELD_FAR_OFF: src = t->far_off; need = sizeof(int64_t) * ((size_t)t->nleaf + 1); break;
        case RCB_FIELD_NEAR: src = t->near_list; need = sizeof(int32_t) * (size_t)t->near_total; break;
        case RCB_FIELD_FAR: src = t->far_list; need = sizeof(int32_t) * (size_t)t->far_total; break;
        default:
            set_error("rcb_tree_export: unknown field");
            return RCB_EINVAL;
    }
    if (bytes < need) {
        set_error("rcb_tree_export: buffer of " + std::to_string(bytes) + " bytes < " +
                  std::to_string(need));
        return RCB_ECAPACITY;
    }
    if (need) RCB_HIP(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToDevice, s));
    return RCB_OK;
}

void rcb_destroy(rcb_tree *t, void *stream) {
    if (!t) return;
    free_all(t, stream ? (hipStream_t)stream : t->stream);
    delete t;
}

void rcb_release_cache(void) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    release_kept_locked(-1);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (int d = 0; d < kMaxDevices; ++d) {
        if (!g_pool_set[d]) continue;
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess) {
            (void)hipSetDevice(d);
            (void)hipDeviceSynchronize();
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &g_pool_thr[d]);
            (void)hipMemPoolTrimTo(pool, 0);
        }
        g_pool_set[d] = false;
    }
    (void)hipSetDevice(cur);
    (void)hipGetLastError();
}

}  // extern "C"
