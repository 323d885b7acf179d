/*
 * rcb.h -- C ABI of the MI355X recursive coordinate bisection (RCB) tree:
 * neighbour search and self-gravity for N particles, after Gafton & Rosswog,
 * "A fast recursive coordinate bisection tree for neighbour search and
 * gravity", MNRAS 2011 (arXiv:1108.0028).
 *
 * Problem (Sec. 1-2): given positions, masses and smoothing lengths of N
 * particles, an average leaf population N_ll and an opening angle theta
 * (G = 1), return each particle's neighbours inside its kernel support 2h and
 * its gravitational acceleration: a kernel-softened direct sum over nearby
 * cells plus a quadrupole far field Taylor-expanded about each leaf's centre
 * of mass.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers (HIP global memory of the
 *    current device) unless a comment says "host". Arrays are plain
 *    structure-of-arrays, one element per particle, in the caller's particle
 *    order; every per-particle output is also in the caller's order.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    All work is enqueued on it; inputs must stay valid and outputs must not
 *    be read until the stream has passed the call. The calls that return
 *    host values or size device lists wait until the stream has passed the
 *    values they need: rcb_walk() (and the first call that runs the walk on
 *    demand) and rcb_neighbours_count() (by polling values the device writes
 *    into pinned host memory after the work before them), rcb_check_cells(),
 *    and rcb_build() / rcb_refresh() with validate = 1 (by synchronising the
 *    stream). rcb_build() (centre-of-mass and centre-of-number splits) also
 *    waits, level by level, for each level's count of large nodes while the
 *    device partitions the levels before it; it returns before the build has
 *    finished on the device. rcb_destroy() does not wait.
 *  - Inputs stay owned by the caller. rcb_build() copies what it needs, so
 *    the tree never aliases caller memory after the call returns.
 *  - Calls return rcb_status; nothing throws across the ABI. Argument errors
 *    are detected on the host before any launch. A failed call leaves its
 *    outputs unspecified; rcb_last_error() describes the last failure on
 *    the calling thread.
 *  - A tree may be used by one stream at a time; calls on one tree must not
 *    overlap.
 *  - Two environment variables select equivalent code paths, for tests:
 *    RCB_BUILD_LEVELS (any value) makes rcb_build() run every level as one
 *    device-wide pass instead of finishing small subtrees in one wave each
 *    (same tree, bit for bit); RCB_WALK_WIDE_STACK=n caps the walk's
 *    first-tier node queue at n entries, so that more groups go to the later
 *    tiers (same lists); RCB_VJP_DET_RECOMPUTE (any value) makes the
 *    deterministic rcb_gravity_vjp() recompute each node's adjoint per node
 *    instead of storing each far entry's (the path it takes when that array
 *    cannot be allocated; equal to rounding, each path repeats bit for bit).
 */
#ifndef RCB_H
#define RCB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rcb_tree rcb_tree;

typedef enum {
    RCB_OK = 0,
    RCB_EINVAL = 1,     /* invalid argument (null pointer, n < 1, n_ll < 1, theta < 0 or not finite, ...) */
    RCB_ENOMEM = 2,     /* device memory allocation failed */
    RCB_EHIP = 3,       /* HIP runtime error */
    RCB_ECAPACITY = 4,  /* caller buffer smaller than the result */
    RCB_ESTATE = 5,     /* call out of order for this tree */
    RCB_EINPUT = 6      /* validate = 1 found a non-finite coordinate, m <= 0 or h <= 0 */
} rcb_status;

typedef enum {
    RCB_FP64 = 0,       /* all interaction arithmetic in FP64 */
    RCB_MIXED = 1       /* FP32 leaf-relative interactions; FP64 moments and Taylor shift */
} rcb_precision;

typedef enum {
    RCB_SPLIT_MASS = 0,     /* split planes through the centre of mass (the paper's CMS) */
    RCB_SPLIT_NUMBER = 1,   /* through the centre of number: unit weights (Sec. 2.1 "Load balancing") */
    RCB_SPLIT_MEDIAN = 2    /* median position split (MPS, Sec. 2.1): the floor(c/2) particles first in
                               (coordinate, caller index) order go to the lower child, so the halves
                               are exact; the plane is the first upper particle's coordinate. Particles
                               tied with it may then sit on their cell's upper face, which
                               rcb_check_cells counts as outside (a rebuild is never missed) */
} rcb_split;

typedef enum {
    RCB_READING_A = 0,      /* J and H of Eq. 6 are the Jacobian and Hessian of the monopole +
                               quadrupole field f (Sec. 2.4.2 read literally; the default) */
    RCB_READING_B = 1       /* the quadrupole enters f only; J and H are those of the monopole
                               field (order-consistent alternative). rcb_gravity_vjp is defined
                               for reading A only */
} rcb_taylor_reading;

typedef struct {
    int32_t n_ll;       /* average particles per lowest-level cell, Sec. 3.2.1 (paper: 12) */
    int32_t precision;  /* rcb_precision */
    double theta;       /* opening angle of the geometric MAC, Sec. 2.4.1 (paper default 0.7) */
    int32_t validate;   /* 1: check inputs on the device first (one extra pass) */
    int32_t pure_mac;   /* 0: reachable cells are never accepted, whatever the MAC
                           (the paper's walk, Sec. 2.4.1); 1: the gravity lists follow
                           the MAC alone (the variant of Sec. 2.5) -- a cell is
                           accepted when the MAC holds unless it contains the sink
                           cell; neighbour candidates are then the leaves reached
                           through reachable cells only */
    int32_t split;      /* rcb_split: where a cell is cut; moments always use the masses */
    int32_t taylor_reading;   /* rcb_taylor_reading of the far-field sink coefficients */
    int32_t deterministic;    /* 0: rcb_gravity_vjp adds source-side near-field terms and node
                                 adjoints with atomics (fastest; reproducible to rounding);
                                 1: no atomics -- per-node and per-cell lists of the groups
                                 that hold each node or cell are made by a stable sort, and
                                 every sum runs in a fixed order, so repeated calls give the
                                 same bits (more time; device memory of 16 B per entry
                                 of the per-group lists and 72 B per far entry) */
    /* Optional workspace allocator, both or neither (NULL: the library
       allocates from the device's stream-ordered pool and keeps freed blocks
       for reuse on the stream that freed them). alloc(bytes, stream, ctx) returns device
       memory usable in stream order on `stream`, or NULL (the call then fails
       with RCB_ENOMEM); free(ptr, stream, ctx) releases it in stream order.
       Every block is freed by the call that allocated it or by
       rcb_destroy(). */
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *alloc_ctx;
} rcb_params;

/* Paper defaults: n_ll = 12, theta = 0.7, FP64, validate = 0, pure_mac = 0,
   split = RCB_SPLIT_MASS, taylor_reading = RCB_READING_A, deterministic = 0. */
void rcb_params_default(rcb_params *p);

/*
 * Build the tree top-down (Sec. 2.1): the root cell is the particles'
 * bounding box; each cell is split perpendicular to its longest side through
 * its centre of mass (or, with split = RCB_SPLIT_NUMBER, its centre of number:
 * the mean coordinate; with RCB_SPLIT_MEDIAN, its median), particles with
 * coordinate < plane going to the lower child 2n (stable), the rest to 2n+1,
 * until level k = min{k : n <= n_ll 2^k}.
 * Every node gets its mass, centre of mass (canonical pairwise sums over its
 * particles in ascending input index), traceless quadrupole (Eq. 1 at the
 * leaves, Eq. 2 upwards), h_node_int and, for leaves, h_node (Sec. 2.3.1).
 *  x, y, z, m, h: n FP64 values each (device). h > 0, m > 0.
 *  n >= 1 and n <= 2^31 - 1.  p: host pointer.  *out: new tree (host).
 * The interaction lists are made by the first call that needs them.
 */
rcb_status rcb_build(const double *x, const double *y, const double *z, const double *m,
                     const double *h, int64_t n, const rcb_params *p, void *stream,
                     rcb_tree **out);

/*
 * Integrity check of Sec. 2.1 "Updating the tree": how many particles, at
 * the new positions x, y, z (n FP64 each, device, caller order, n == the
 * built n), lie outside their lowest-level cell. A cell is its box with the
 * build's side rule: lo <= x < hi on each axis (closed at the root box's
 * upper faces), so 0 means the tree is still the tree these positions would
 * build with the same splits and rcb_refresh can replace a rebuild.
 *  outside: host int64, receives the count. Synchronises `stream`.
 * Errors: RCB_EINVAL (NULL pointer), RCB_ESTATE (n differs from the built n).
 */
rcb_status rcb_check_cells(rcb_tree *t, const double *x, const double *y, const double *z,
                           int64_t n, int64_t *outside, void *stream);

/*
 * Tree update of Sec. 2.1 "Updating the tree": when no particle has left its
 * lowest-level cell (rcb_check_cells() == 0) the tree is kept and only its
 * moments are recomputed. New positions, masses and smoothing lengths replace
 * the build's inputs, particle by particle in caller order; the topology
 * (cell ranges, boxes, splits) stays, and every node's mass, centre of mass,
 * h_node_int, the leaves' Eq. 1 quadrupole and h_node and the Eq. 2
 * quadrupoles above are recomputed by the same canonical sums as rcb_build.
 *  x, y, z, m, h: n FP64 values each (device), n == the built n.
 *  keep_lists: 0 -- the paper's step: the interaction lists (and neighbour
 *              counts, kept far coefficients) are dropped, and the next call
 *              that needs them walks the refreshed tree again, so neighbours
 *              and the reachability override follow the new h and positions.
 *              1 -- the tree held fixed for differentiation: rcb_gravity and
 *              rcb_gravity_vjp keep using the old lists (the map whose
 *              derivative rcb_gravity_vjp computes). Neighbour calls then
 *              return RCB_ESTATE, since the old lists may miss neighbours of
 *              the new inputs, until rcb_walk() has walked again.
 * Errors: RCB_EINVAL (NULL pointer, keep_lists not 0 or 1), RCB_ESTATE (n
 * differs from the built n), RCB_EINPUT (validate set and an input
 * non-finite or m, h <= 0).
 */
rcb_status rcb_refresh(rcb_tree *t, const double *x, const double *y, const double *z,
                       const double *m, const double *h, int64_t n, int32_t keep_lists,
                       void *stream);

/*
 * rcb_refresh(t, x, y, z, m, h, n, keep_lists = 1, stream) for callers that
 * cannot allocate device memory: code under HIP graph capture, tight
 * simulation or serving loops, harnesses that forbid hipMalloc. It allocates
 * and frees nothing: its scratch (the gathered inputs of each level, 32 bytes
 * per particle, and the level passes' bookkeeping, about 33 bytes per
 * particle in all) lives in one static device array of 64 MiB that every GPU
 * the library runs on holds until the process ends. The interaction lists
 * are kept, as with keep_lists = 1 (rcb_walk() makes new ones, and
 * allocates). Calls on one device share the array: calls that overlap in
 * time on one device, on any streams, race and must be serialised by the
 * caller. The tree itself must already exist (rcb_build allocates).
 *  Arguments, results and the other errors as rcb_refresh.
 * Errors: RCB_ECAPACITY if the tree needs more scratch than the array holds
 * (rcb_refresh_noalloc_scratch(t) > rcb_refresh_noalloc_scratch(NULL):
 * about 2 million particles).
 */
rcb_status rcb_refresh_noalloc(rcb_tree *t, const double *x, const double *y, const double *z,
                               const double *m, const double *h, int64_t n, void *stream);

/* Scratch bytes rcb_refresh_noalloc needs for tree t; with t == NULL the
   size of the static array (the maximum). */
size_t rcb_refresh_noalloc_scratch(const rcb_tree *t);

/*
 * Tree walk (Sec. 2.2, with the reachability test of Sec. 2.3.1 and the MAC
 * of Sec. 2.4.1): makes the near and far interaction lists of every
 * lowest-level cell and keeps them in the tree. The neighbour and gravity
 * calls run it themselves when it has not run yet; calling it first only
 * moves the work; after rcb_refresh(keep_lists = 1) it walks the refreshed
 * tree again. Waits until `stream` has passed the walk (the list sizes and
 * flags are read back through pinned host memory).
 * Errors: RCB_ECAPACITY if the last-resort walk's stack overflows (a tree
 * deeper than 29 levels), RCB_ENOMEM.
 * Environment (testing): RCB_WALK_WIDE_STACK=n caps the breadth-first
 * walk's node queues at n entries, so that more groups of cells are walked
 * again by the later tiers; the lists do not change.
 */
rcb_status rcb_walk(rcb_tree *t, void *stream);

/*
 * Neighbour search, step 1 (Sec. 2.3): for every particle a the number of
 * particles b != a with |r_a - r_b| < 2 h_a, found among the cells that the
 * reachability test of Sec. 2.3.1 keeps.
 *  offsets: device int64[n + 1], receives the exclusive prefix sum of the
 *           counts (offsets[0] = 0, offsets[n] = total).
 *  total:   host int64, receives offsets[n]. This call waits until `stream`
 *           has passed the count (the total is read back through pinned host
 *           memory).
 * Errors: RCB_ESTATE after rcb_refresh(keep_lists = 1) until rcb_walk().
 */
rcb_status rcb_neighbours_count(rcb_tree *t, int64_t *offsets, int64_t *total, void *stream);

/*
 * Neighbour search, step 2: writes the neighbour ids (caller indices) of
 * particle a to ids[offsets[a] .. offsets[a+1]) -- the one-dimensional list
 * of Sec. 2.3.2. Each list is ascending by caller index, so the output does
 * not depend on the tree (split rule, N_ll) that found it.
 *  offsets:  the array filled by rcb_neighbours_count() for this tree.
 *  ids:      device int32[capacity]; capacity >= total, else RCB_ECAPACITY.
 * The count call keeps each list in scratch owned by the tree (freed with
 * the interaction lists): a 64-slot row per particle (256 bytes) and, for
 * lists of up to 256, chunks of 64 slots from a pool of N/8 chunks (32 bytes
 * per particle); the cells holding a list that fit neither are searched
 * again here.
 */
rcb_status rcb_neighbours_fill(rcb_tree *t, const int64_t *offsets, int32_t *ids,
                               int64_t capacity, void *stream);

/*
 * Gravitational accelerations (Sec. 2.4), G = 1:
 *   a_a = -sum over particles b of near cells of m_b S(r_ab, h_ab) e_ab   (Eq. for f_ng)
 *         + f_A + J_A d_a + 1/2 d_a^T H_A d_a                             (Eq. 6)
 * with h_ab = (h_a + h_b)/2, d_a = r_a - COM_A, and f_A, J_A, H_A the field,
 * Jacobian and Hessian at COM_A of the quadrupole expansions (Eq. 5) of the
 * cells accepted by the MAC H_B / R_AB < theta (reachable cells are never
 * accepted unless pure_mac; with RCB_READING_B, J_A and H_A of the monopole
 * parts only). ax, ay, az: n values, FP64 for RCB_FP64, FP32 for RCB_MIXED.
 * The tree keeps f_A, J_A, H_A of every lowest-level cell (22 doubles per
 * cell, allocated on the first call) for a later rcb_gravity_vjp on the same
 * moments; rcb_refresh discards them.
 */
rcb_status rcb_gravity(rcb_tree *t, void *ax, void *ay, void *az, void *stream);

/*
 * Vector-Jacobian product of rcb_gravity with the tree held fixed (same
 * topology, particle-to-leaf map and interaction lists; masses, centres of
 * mass and quadrupoles vary with the inputs): for L = sum_a g_a . a_a,
 * writes dL/dx, dL/dy, dL/dz and dL/dm. h gets no gradient. Near-field pairs
 * are recomputed, not stored. g*: n values, d*: n values, FP64 for RCB_FP64
 * and FP32 for RCB_MIXED. Valid after rcb_build() (gravity need not have run).
 * Summation order: with deterministic = 0 the source-side near-field terms
 * and the node adjoints are added with atomics (FP64; FP32 in the mixed
 * form), so two calls agree to rounding, not bit for bit. With
 * deterministic = 1 nothing is added atomically: each node's adjoint is
 * summed over the groups that accepted it (ascending group, fixed chunks of
 * 512 entries, then the chunks in order; each group's part over its cells in
 * order) and each source particle's terms over the sink cells whose near
 * list holds its cell (sums in FP64 in both forms; a particle's pair with
 * itself, whose terms cancel, is left out); two calls on the same tree and
 * inputs give identical outputs. The lists of groups per node and per cell
 * are made on each call (stable label sort).
 * Errors: RCB_EINVAL (NULL argument, or a tree built with RCB_READING_B);
 * with deterministic = 1 also RCB_ENOMEM (the lists' sort buffers) and
 * RCB_ECAPACITY (more than 2^24 groups of 8 cells, k > 27).
 */
rcb_status rcb_gravity_vjp(rcb_tree *t, const void *gx, const void *gy, const void *gz,
                           void *dx, void *dy, void *dz, void *dm, void *stream);

typedef struct {
    int64_t n;            /* particles */
    int32_t k;            /* leaf level; leaves are labels 2^k .. 2^(k+1)-1 */
    int32_t precision;
    int64_t n_labels;     /* 2^(k+1); label 0 unused */
    int64_t near_total;   /* interaction-list sizes, -1 until the walk has run */
    int64_t far_total;
    double theta;
    int64_t walk_requeued; /* groups of 8 lowest-level cells whose walk outgrew the first
                              FIFO (1024 nodes) and was redone with a larger one or, past
                              8192 nodes, by the 8-wide walk (same lists); -1 before the walk */
    int64_t walk_nodes;    /* node records the breadth-first walk loaded: one per node per group
                              of 8 sibling cells (groups walked again by a later tier count only
                              their first attempt); -1 before the walk */
    int64_t walk_tests;    /* (node, lowest-level cell) pairs among those whose cell's own walk
                              reaches the node: the per-cell tests of Sec. 2.2; -1 before the walk */
} rcb_tree_info;

rcb_status rcb_get_info(const rcb_tree *t, rcb_tree_info *info /* host */);

/* Fields of rcb_tree_export(): the tree's own arrays, for inspection and tests. */
typedef enum {
    RCB_FIELD_PERM = 0,      /* int32[n]        tree position -> caller index */
    RCB_FIELD_FIRST = 1,     /* int32[n_labels] first tree position of each node */
    RCB_FIELD_COUNT = 2,     /* int32[n_labels] particles in each node */
    RCB_FIELD_LO = 3,        /* f64[3 n_labels] cell lower corner, (x,y,z) per label */
    RCB_FIELD_HI = 4,        /* f64[3 n_labels] cell upper corner */
    RCB_FIELD_COM = 5,       /* f64[3 n_labels] centre of mass */
    RCB_FIELD_MASS = 6,      /* f64[n_labels] */
    RCB_FIELD_QUAD = 7,      /* f64[6 n_labels] Q_xx Q_xy Q_xz Q_yy Q_yz Q_zz */
    RCB_FIELD_HINT = 8,      /* f64[n_labels] h_node_int (-1 for empty nodes) */
    RCB_FIELD_HNODE = 9,     /* f64[n_labels] h_node of leaves (-1 elsewhere) */
    RCB_FIELD_NEAR_OFF = 10, /* int64[2^k + 1] per-leaf offsets into NEAR (needs the walk) */
    RCB_FIELD_FAR_OFF = 11,  /* int64[2^k + 1] per-leaf offsets into FAR */
    RCB_FIELD_NEAR = 12,     /* int32[near_total] leaf label | candidate << 31 | (not in the
                                gravity near field, pure_mac only) << 30, ascending labels */
    RCB_FIELD_FAR = 13       /* int32[far_total] accepted node labels, unordered */
} rcb_field;

/*
 * Copy one of the tree's arrays into caller device memory `dst` of `bytes`
 * bytes (RCB_ECAPACITY if smaller than the field). List fields run the walk
 * first if it has not run yet.
 */
rcb_status rcb_tree_export(rcb_tree *t, int32_t field, void *dst, size_t bytes, void *stream);

/* Free the tree and its device memory, in stream order on `stream` (made to
   wait for the tree's last stream first; NULL = the tree's last stream), and
   return without waiting: the memory is reused only by work queued on that
   stream after the call (or, from the caller's allocator, as its free()
   allows). NULL t is a no-op. Blocks from the library's own allocator stay
   reserved for later requests on the same device and stream (up to a quarter
   of the device's memory; see rcb_release_cache). */
void rcb_destroy(rcb_tree *t, void *stream);

/* Give back the device memory the library keeps for reuse: its freed blocks,
   and the unused part of each device's default stream-ordered pool (its
   release threshold, raised by the library, is restored). Call it when no
   tree is in use, e.g. before another framework needs the memory. Waits for
   the devices concerned to finish their work; never fails. */
void rcb_release_cache(void);

/* Message of the last failed call on this thread ("" if none). */
const char *rcb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RCB_H */
