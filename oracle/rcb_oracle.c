/*
 * rcb_oracle.c -- plain, slow FP64 CPU oracle for the recursive coordinate
 * bisection (RCB) tree of Gafton & Rosswog, MNRAS 2011 ("A fast recursive
 * coordinate bisection tree for neighbour search and gravity").
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The product path (the
 * HIP library) shares no code, header, table or constant with it.
 *
 * Everything is FP64 with round-to-nearest; build with -ffp-contract=off so
 * that no multiply-add is fused. Each function names the passage it follows.
 * Where the paper leaves a detail open, the reading taken is stated inline:
 *   - depth: the smallest k >= 0 with N <= N_ll * 2^k (Sec. 2.1; Table 1's L).
 *   - a cell is its partition box; the root box is the particles' bounding box.
 *   - split axis = longest box side, ties to the lowest axis index.
 *   - a particle exactly on the split plane goes right (strict "<"); each side
 *     keeps the particles' relative order (stable partition).
 *   - node sums (mass, mass-weighted position, quadrupole) are canonical
 *     pairwise sums over the node's particles in ascending original index.
 *   - geometric centre = box centre; h_node_int exact over the particles.
 *   - reachability (Eq. of Sec. 2.3.1) is evaluated squared with a relative
 *     pad of 2^-32 on the radius sum; the MAC (Sec. 2.4.1) squared, strict.
 *   - neighbours of a: b != a with |r_a - r_b| < 2 h_a (gather form).
 *   - far-field J and H are the full Jacobian and Hessian of the truncated
 *     monopole + quadrupole field (Sec. 2.4.2).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REACH_PAD (1.0 + 0x1p-32)

/* ------------------------------------------------------------------------ */
/* Canonical pairwise sum: pad the values (in the given order) with +0.0 to  */
/* the next power of two, replace w[i] by w[2i] + w[2i+1] until one value is */
/* left, then add +0.0 (so that a -0.0 result reads +0.0).                   */
/* ------------------------------------------------------------------------ */
double orc_psum(const double *v, int64_t n)
{
    if (n <= 0) return 0.0;
    int64_t p = 1;
    while (p < n) p *= 2;
    double *w = (double *)malloc((size_t)p * sizeof(double));
    for (int64_t i = 0; i < n; ++i) w[i] = v[i];
    for (int64_t i = n; i < p; ++i) w[i] = 0.0;
    for (int64_t len = p; len > 1; len /= 2)
        for (int64_t i = 0; i < len / 2; ++i) w[i] = w[2 * i] + w[2 * i + 1];
    double s = w[0] + 0.0;
    free(w);
    return s;
}

static double dist2(double ax, double ay, double az, double bx, double by, double bz)
{
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return (dx * dx + dy * dy) + dz * dz;
}

/* ------------------------------------------------------------------------ */
/* Tree storage. Labels follow Sec. 2.1 "Node labelling": root = 1, children */
/* of n are 2n and 2n+1, level l holds labels 2^l .. 2^(l+1)-1.              */
/* ------------------------------------------------------------------------ */
/* Near-list entries: leaf label | flags. NEAR_NBONLY marks a leaf that only
   the neighbour search uses (set by the pure-MAC walk alone). */
#define NEAR_CAND 0x80000000u     /* neighbour candidate (reachable) */
#define NEAR_NBONLY 0x40000000u   /* not part of the gravity near field */
#define NEAR_LABEL 0x3fffffffu

typedef struct {
    int32_t *near;     /* leaf label | NEAR_CAND | NEAR_NBONLY */
    int64_t nnear;
    int64_t capnear;
    int32_t *far;      /* node label */
    int64_t nfar;
    int64_t capfar;
    int64_t visited;   /* non-empty nodes tested */
    int walked;
} leaf_lists;

typedef struct otree {
    int64_t n;
    int k;
    int n_ll;
    int64_t nlab;                  /* 2^(k+1); labels 1 .. nlab-1 */
    double *x, *y, *z, *m, *h;     /* inputs, original order */
    int64_t *perm;                 /* tree position -> original index */
    int64_t *first, *count;
    int32_t *axis;
    double *lo, *hi;               /* 3 per label */
    double *M, *com, *Q;           /* Q: xx xy xz yy yz zz per label */
    double *hint, *hnode;
    double theta;
    int split;                     /* 0: centre of mass, 1: centre of number, 2: median */
    int pure_mac;                  /* walk mode of the last orc_walk */
    int reading;                   /* Taylor coefficients: 0 = reading A, 1 = reading B */
    leaf_lists *lists;             /* one per leaf, index label - 2^k */
} otree;

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* The node's original indices in ascending order (a fresh array). */
static int64_t *node_members_sorted(const otree *t, int64_t lab)
{
    int64_t s = t->first[lab], c = t->count[lab];
    int64_t *ids = (int64_t *)malloc((size_t)(c > 0 ? c : 1) * sizeof(int64_t));
    memcpy(ids, t->perm + s, (size_t)c * sizeof(int64_t));
    int sorted = 1;
    for (int64_t i = 1; i < c; ++i)
        if (ids[i - 1] > ids[i]) { sorted = 0; break; }
    if (!sorted) qsort(ids, (size_t)c, sizeof(int64_t), cmp_i64);
    return ids;
}

/* Mass and centre of mass of a node (Sec. 2.1 "Multipole moments"). */
static void node_mass_com(const otree *t, int64_t lab, double *M, double com[3])
{
    int64_t c = t->count[lab];
    int64_t *ids = node_members_sorted(t, lab);
    double *v = (double *)malloc((size_t)(c > 0 ? c : 1) * sizeof(double));
    for (int64_t i = 0; i < c; ++i) v[i] = t->m[ids[i]];
    double mass = orc_psum(v, c);
    const double *xs[3] = {t->x, t->y, t->z};
    for (int d = 0; d < 3; ++d) {
        for (int64_t i = 0; i < c; ++i) v[i] = t->m[ids[i]] * xs[d][ids[i]];
        double s = orc_psum(v, c);
        com[d] = s / mass;
    }
    *M = mass;
    free(v);
    free(ids);
}

/* Centre of number of a node along one axis (Sec. 2.1 "Load balancing":   */
/* the centre of mass with every weight replaced by 1), i.e. the mean        */
/* coordinate, summed canonically in ascending original index.              */
static double node_mean(const otree *t, int64_t lab, const double *xa)
{
    int64_t c = t->count[lab];
    int64_t *ids = node_members_sorted(t, lab);
    double *v = (double *)malloc((size_t)(c > 0 ? c : 1) * sizeof(double));
    for (int64_t i = 0; i < c; ++i) v[i] = xa[ids[i]];
    double mean = orc_psum(v, c) / (double)c;
    free(v);
    free(ids);
    return mean;
}

/* Order of the median split: coordinate, then original index (numerical  */
/* comparison, so -0 and +0 tie and the index decides).                     */
static const double *g_sort_key;
static int cmp_by_key_then_index(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    double xi = g_sort_key[i], xj = g_sort_key[j];
    if (xi < xj) return -1;
    if (xi > xj) return 1;
    return (i > j) - (i < j);
}

/* Split one node perpendicular to its longest side through its centre of  */
/* mass, its centre of number, or its median (Sec. 2.1 "Load balancing",    */
/* "Particle sorting"). The median split (MPS) sends the floor(c/2)        */
/* particles that come first in (coordinate, original index) order to the  */
/* lower child; its plane is the coordinate of the first upper particle.    */
static void split_node(otree *t, int64_t lab)
{
    int64_t s = t->first[lab], c = t->count[lab];
    int64_t L = 2 * lab, R = 2 * lab + 1;
    for (int d = 0; d < 3; ++d) {
        t->lo[3 * L + d] = t->lo[3 * lab + d];
        t->hi[3 * L + d] = t->hi[3 * lab + d];
        t->lo[3 * R + d] = t->lo[3 * lab + d];
        t->hi[3 * R + d] = t->hi[3 * lab + d];
    }
    if (c == 0) {
        t->axis[lab] = -1;
        t->first[L] = s; t->count[L] = 0;
        t->first[R] = s; t->count[R] = 0;
        return;
    }
    double M, com[3];
    node_mass_com(t, lab, &M, com);
    int ax = 0;
    double best = t->hi[3 * lab] - t->lo[3 * lab];
    for (int d = 1; d < 3; ++d) {
        double side = t->hi[3 * lab + d] - t->lo[3 * lab + d];
        if (side > best) { best = side; ax = d; }
    }
    t->axis[lab] = ax;
    const double *xa = ax == 0 ? t->x : (ax == 1 ? t->y : t->z);
    double plane;
    int64_t tie = -1;          /* median split: (x, index) pairs below (plane, tie) go left */
    if (t->split == 2) {
        int64_t *ord = (int64_t *)malloc((size_t)c * sizeof(int64_t));
        memcpy(ord, t->perm + s, (size_t)c * sizeof(int64_t));
        g_sort_key = xa;
        qsort(ord, (size_t)c, sizeof(int64_t), cmp_by_key_then_index);
        plane = xa[ord[c / 2]] + 0.0;
        tie = ord[c / 2];
        free(ord);
    } else {
        plane = t->split == 1 ? node_mean(t, lab, xa) : com[ax];
    }
    int64_t *tmp = (int64_t *)malloc((size_t)c * sizeof(int64_t));
    int64_t nl = 0;
    for (int64_t i = 0; i < c; ++i) {
        int64_t b = t->perm[s + i];
        if (xa[b] < plane || (xa[b] == plane && b < tie)) tmp[nl++] = b;
    }
    int64_t j = nl;
    for (int64_t i = 0; i < c; ++i) {
        int64_t b = t->perm[s + i];
        if (!(xa[b] < plane || (xa[b] == plane && b < tie))) tmp[j++] = b;
    }
    memcpy(t->perm + s, tmp, (size_t)c * sizeof(int64_t));
    free(tmp);
    t->first[L] = s; t->count[L] = nl;
    t->first[R] = s + nl; t->count[R] = c - nl;
    t->hi[3 * L + ax] = plane;
    t->lo[3 * R + ax] = plane;
}

/* Node quantities for the current inputs on the fixed topology:            */
/* M, COM (all nodes), h_node_int (all), h_node and Eq. 1 quadrupole (leaves)*/
/* and Eq. 2 quadrupole shift (internal nodes, bottom-up).                  */
static void compute_moments(otree *t)
{
    int64_t leaf0 = (int64_t)1 << t->k;
    /* every label on its own: no node reads another's result here */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t lab = 1; lab < t->nlab; ++lab) {
        int64_t s = t->first[lab], c = t->count[lab];
        double g[3];
        for (int d = 0; d < 3; ++d) g[d] = 0.5 * (t->lo[3 * lab + d] + t->hi[3 * lab + d]);
        for (int q = 0; q < 6; ++q) t->Q[6 * lab + q] = 0.0;
        if (c == 0) {
            t->M[lab] = 0.0;
            for (int d = 0; d < 3; ++d) t->com[3 * lab + d] = g[d];
            t->hint[lab] = -1.0;
            t->hnode[lab] = -1.0;
            continue;
        }
        node_mass_com(t, lab, &t->M[lab], &t->com[3 * lab]);
        double hi_ = 0.0, hn = 0.0;
        for (int64_t i = 0; i < c; ++i) {
            int64_t b = t->perm[s + i];
            double r = sqrt(dist2(t->x[b], t->y[b], t->z[b], g[0], g[1], g[2]));
            if (r > hi_) hi_ = r;
            double rk = r + 2.0 * t->h[b];
            if (rk > hn) hn = rk;
        }
        t->hint[lab] = hi_;
        t->hnode[lab] = lab >= leaf0 ? hn : -1.0;
        if (lab >= leaf0) {
            /* Eq. 1 summed over the leaf's particles. */
            int64_t *ids = node_members_sorted(t, lab);
            double *v = (double *)malloc((size_t)c * sizeof(double));
            const double *cm = &t->com[3 * lab];
            for (int q = 0; q < 6; ++q) {
                static const int qi[6] = {0, 0, 0, 1, 1, 2}, qj[6] = {0, 1, 2, 1, 2, 2};
                for (int64_t i = 0; i < c; ++i) {
                    int64_t b = ids[i];
                    double d[3] = {t->x[b] - cm[0], t->y[b] - cm[1], t->z[b] - cm[2]};
                    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                    double val = 3.0 * t->m[b] * d[qi[q]] * d[qj[q]];
                    if (qi[q] == qj[q]) val -= t->m[b] * r2;
                    v[i] = val;
                }
                t->Q[6 * lab + q] = orc_psum(v, c);
            }
            free(v);
            free(ids);
        }
    }
    /* Eq. 2: shift child quadrupoles to the parent's centre of mass. */
    for (int lvl = t->k - 1; lvl >= 0; --lvl) {
        for (int64_t lab = (int64_t)1 << lvl; lab < ((int64_t)2 << lvl); ++lab) {
            if (t->count[lab] == 0) continue;
            static const int qi[6] = {0, 0, 0, 1, 1, 2}, qj[6] = {0, 1, 2, 1, 2, 2};
            double acc[6] = {0, 0, 0, 0, 0, 0};
            for (int ch = 0; ch < 2; ++ch) {
                int64_t C = 2 * lab + ch;
                if (t->count[C] == 0) continue;
                double dx[3];
                for (int d = 0; d < 3; ++d) dx[d] = t->com[3 * C + d] - t->com[3 * lab + d];
                double r2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2];
                for (int q = 0; q < 6; ++q) {
                    double term = t->Q[6 * C + q] + 3.0 * t->M[C] * dx[qi[q]] * dx[qj[q]];
                    if (qi[q] == qj[q]) term -= t->M[C] * r2;
                    acc[q] += term;
                }
            }
            for (int q = 0; q < 6; ++q) t->Q[6 * lab + q] = acc[q];
        }
    }
}

static void free_lists(otree *t)
{
    if (!t->lists) return;
    int64_t nleaf = (int64_t)1 << t->k;
    for (int64_t i = 0; i < nleaf; ++i) {
        free(t->lists[i].near);
        free(t->lists[i].far);
    }
    free(t->lists);
    t->lists = NULL;
}

void orc_free(otree *t)
{
    if (!t) return;
    free_lists(t);
    free(t->x); free(t->y); free(t->z); free(t->m); free(t->h);
    free(t->perm); free(t->first); free(t->count); free(t->axis);
    free(t->lo); free(t->hi); free(t->M); free(t->com); free(t->Q);
    free(t->hint); free(t->hnode);
    free(t);
}

static double *dup(const double *v, int64_t n)
{
    double *r = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    memcpy(r, v, (size_t)n * sizeof(double));
    return r;
}

/* Depth rule: the smallest k >= 0 with N <= N_ll * 2^k (Sec. 2.1; Table 1). */
int orc_depth_for(int64_t n, int n_ll)
{
    int k = 0;
    while ((int64_t)n_ll * ((int64_t)1 << k) < n) ++k;
    return k;
}

/* Top-down build (Sec. 2.1): root box = bounding box of all particles;   */
/* levels 0 .. k-1 are split in turn; then the node moments.             */
/* split: 0 = through the centre of mass, 1 = through the centre of number, */
/* 2 = median position split (equal halves).                                */
otree *orc_build(int64_t n, const double *x, const double *y, const double *z,
                 const double *m, const double *h, int n_ll, int split)
{
    if (n < 1 || n_ll < 1 || split < 0 || split > 2) return NULL;
    otree *t = (otree *)calloc(1, sizeof(otree));
    t->n = n;
    t->n_ll = n_ll;
    t->split = split;
    t->k = orc_depth_for(n, n_ll);
    t->nlab = (int64_t)2 << t->k;
    t->x = dup(x, n); t->y = dup(y, n); t->z = dup(z, n); t->m = dup(m, n); t->h = dup(h, n);
    t->perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) t->perm[i] = i;
    int64_t L = t->nlab;
    t->first = (int64_t *)calloc((size_t)L, sizeof(int64_t));
    t->count = (int64_t *)calloc((size_t)L, sizeof(int64_t));
    t->axis = (int32_t *)calloc((size_t)L, sizeof(int32_t));
    t->lo = (double *)calloc((size_t)(3 * L), sizeof(double));
    t->hi = (double *)calloc((size_t)(3 * L), sizeof(double));
    t->M = (double *)calloc((size_t)L, sizeof(double));
    t->com = (double *)calloc((size_t)(3 * L), sizeof(double));
    t->Q = (double *)calloc((size_t)(6 * L), sizeof(double));
    t->hint = (double *)calloc((size_t)L, sizeof(double));
    t->hnode = (double *)calloc((size_t)L, sizeof(double));
    const double *xs[3] = {x, y, z};
    for (int d = 0; d < 3; ++d) {
        double lo = xs[d][0], hi = xs[d][0];
        for (int64_t i = 1; i < n; ++i) {
            if (xs[d][i] < lo) lo = xs[d][i];
            if (xs[d][i] > hi) hi = xs[d][i];
        }
        t->lo[3 + d] = lo;
        t->hi[3 + d] = hi;
    }
    t->first[1] = 0;
    t->count[1] = n;
    t->axis[0] = -1;
    /* The nodes of one level are independent (each owns its particle range */
    /* and its two children), so a level is split in parallel, as the paper  */
    /* builds disjoint subtrees on separate processors (Sec. 2.1            */
    /* "Parallelisation"). The median split's sort uses a global comparator */
    /* key and stays serial.                                                 */
    for (int lvl = 0; lvl < t->k; ++lvl) {
        int64_t lab0 = (int64_t)1 << lvl, lab1 = (int64_t)2 << lvl;
#pragma omp parallel for schedule(dynamic, 1) if (split != 2)
        for (int64_t lab = lab0; lab < lab1; ++lab) split_node(t, lab);
    }
    for (int64_t lab = (int64_t)1 << t->k; lab < t->nlab; ++lab) t->axis[lab] = -1;
    compute_moments(t);
    return t;
}

/* Tree update with the topology held fixed (Sec. 2.1 "Updating the tree"): */
/* new inputs, same particle-to-leaf map, moments recomputed bottom-up.      */
void orc_refresh(otree *t, const double *x, const double *y, const double *z,
                 const double *m, const double *h)
{
    memcpy(t->x, x, (size_t)t->n * sizeof(double));
    memcpy(t->y, y, (size_t)t->n * sizeof(double));
    memcpy(t->z, z, (size_t)t->n * sizeof(double));
    memcpy(t->m, m, (size_t)t->n * sizeof(double));
    memcpy(t->h, h, (size_t)t->n * sizeof(double));
    compute_moments(t);
}

int orc_k(const otree *t) { return t->k; }

/* Threads of the OpenMP loops (walk, neighbours, gravity); the build is serial. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Taylor reading of the sink coefficients used by orc_gravity: 0 = A, 1 = B. */
void orc_set_reading(otree *t, int reading) { t->reading = reading; }
int64_t orc_n(const otree *t) { return t->n; }

void orc_topology(const otree *t, int64_t *perm, int64_t *first, int64_t *count, int32_t *axis)
{
    memcpy(perm, t->perm, (size_t)t->n * sizeof(int64_t));
    memcpy(first, t->first, (size_t)t->nlab * sizeof(int64_t));
    memcpy(count, t->count, (size_t)t->nlab * sizeof(int64_t));
    memcpy(axis, t->axis, (size_t)t->nlab * sizeof(int32_t));
}

void orc_nodes(const otree *t, double *lo, double *hi, double *com, double *M, double *Q,
               double *hint, double *hnode)
{
    int64_t L = t->nlab;
    memcpy(lo, t->lo, (size_t)(3 * L) * sizeof(double));
    memcpy(hi, t->hi, (size_t)(3 * L) * sizeof(double));
    memcpy(com, t->com, (size_t)(3 * L) * sizeof(double));
    memcpy(M, t->M, (size_t)L * sizeof(double));
    memcpy(Q, t->Q, (size_t)(6 * L) * sizeof(double));
    memcpy(hint, t->hint, (size_t)L * sizeof(double));
    memcpy(hnode, t->hnode, (size_t)L * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Walk (Sec. 2.2, 2.3.1, 2.4.1): depth-first from nodes 2 and 3.            */
/* ------------------------------------------------------------------------ */
static void push_near(leaf_lists *L, int64_t lab, uint32_t flags)
{
    if (L->nnear == L->capnear) {
        L->capnear = L->capnear ? 2 * L->capnear : 64;
        L->near = (int32_t *)realloc(L->near, (size_t)L->capnear * sizeof(int32_t));
    }
    L->near[L->nnear++] = (int32_t)((uint32_t)lab | flags);
}

static void push_far(leaf_lists *L, int64_t lab)
{
    if (L->nfar == L->capfar) {
        L->capfar = L->capfar ? 2 * L->capfar : 128;
        L->far = (int32_t *)realloc(L->far, (size_t)L->capfar * sizeof(int32_t));
    }
    L->far[L->nfar++] = (int32_t)lab;
}

/* Sec. 2.3.1: B is reachable from A if the spheres around the geometric     */
/* centres with radii h_node(A) and h_node_int(B) overlap.                   */
static int reachable(const otree *t, int64_t A, int64_t B)
{
    double gA[3], gB[3];
    for (int d = 0; d < 3; ++d) {
        gA[d] = 0.5 * (t->lo[3 * A + d] + t->hi[3 * A + d]);
        gB[d] = 0.5 * (t->lo[3 * B + d] + t->hi[3 * B + d]);
    }
    double dg2 = dist2(gA[0], gA[1], gA[2], gB[0], gB[1], gB[2]);
    double rs = (t->hnode[A] + t->hint[B]) * REACH_PAD;
    return dg2 < rs * rs;
}

/* Sec. 2.4.1, Eq. 4: H_B / R_AB < theta, H_B the longest side of B, R_AB   */
/* the distance of the centres of mass.                                      */
static int mac_accepts(const otree *t, int64_t A, int64_t B, double theta)
{
    double HB = t->hi[3 * B] - t->lo[3 * B];
    for (int d = 1; d < 3; ++d) {
        double side = t->hi[3 * B + d] - t->lo[3 * B + d];
        if (side > HB) HB = side;
    }
    const double *cA = &t->com[3 * A], *cB = &t->com[3 * B];
    double R2 = dist2(cA[0], cA[1], cA[2], cB[0], cB[1], cB[2]);
    return HB * HB < (theta * theta) * R2;
}

/* Combined walk of the paper (Sec. 2.4.1): a reachable cell is never       */
/* accepted; its leaves are neighbour candidates and belong to the near     */
/* field.                                                                   */
static void visit(const otree *t, int64_t A, int64_t B, double theta, leaf_lists *L)
{
    if (t->count[B] == 0) return;              /* empty cells are ignored */
    L->visited++;
    int is_leaf = B >= ((int64_t)1 << t->k);
    if (reachable(t, A, B)) {                  /* reachable: never accepted */
        if (is_leaf) push_near(L, B, NEAR_CAND);
        else { visit(t, A, 2 * B, theta, L); visit(t, A, 2 * B + 1, theta, L); }
        return;
    }
    if (mac_accepts(t, A, B, theta)) {         /* geometric MAC */
        push_far(L, B);
        return;
    }
    if (is_leaf) push_near(L, B, 0);
    else { visit(t, A, 2 * B, theta, L); visit(t, A, 2 * B + 1, theta, L); }
}

/* B is A or one of A's ancestors (labels of Sec. 2.1). */
static int contains(int64_t B, int64_t A)
{
    while (A > B) A >>= 1;
    return A == B;
}

/* Gravity walk with the geometric MAC alone (the variant of Sec. 2.5 where  */
/* reachability does not override the MAC). A cell that contains A itself   */
/* is never accepted: the combined walk never accepts one either, since a    */
/* particle of A lies in both cells and the triangle inequality then makes   */
/* the cell reachable.                                                       */
static void visit_mac(const otree *t, int64_t A, int64_t B, double theta, leaf_lists *L)
{
    if (t->count[B] == 0) return;
    L->visited++;
    if (!contains(B, A) && mac_accepts(t, A, B, theta)) {
        push_far(L, B);
        return;
    }
    if (B >= ((int64_t)1 << t->k)) push_near(L, B, 0);
    else { visit_mac(t, A, 2 * B, theta, L); visit_mac(t, A, 2 * B + 1, theta, L); }
}

/* Neighbour walk (Sec. 2.3): descend through reachable cells only; the     */
/* reachable leaves are the candidates.                                     */
static void visit_reach(const otree *t, int64_t A, int64_t B, leaf_lists *L)
{
    if (t->count[B] == 0) return;
    L->visited++;
    if (!reachable(t, A, B)) return;
    if (B >= ((int64_t)1 << t->k)) push_near(L, B, NEAR_CAND);
    else { visit_reach(t, A, 2 * B, L); visit_reach(t, A, 2 * B + 1, L); }
}

/* Pure-MAC lists of leaf A: the gravity walk's near leaves and the          */
/* neighbour walk's candidates merged into one list by ascending label       */
/* (both walks emit leaves in ascending order); a candidate outside the      */
/* gravity near field carries NEAR_NBONLY.                                   */
static void walk_leaf_pure(const otree *t, int64_t A, leaf_lists *L)
{
    leaf_lists cand = {0};
    int64_t r0 = t->k == 0 ? 1 : 2, r1 = t->k == 0 ? 1 : 3;
    for (int64_t B = r0; B <= r1; ++B) visit_mac(t, A, B, t->theta, L);
    for (int64_t B = r0; B <= r1; ++B) visit_reach(t, A, B, &cand);
    int32_t *grav = L->near;
    int64_t ng = L->nnear;
    L->near = NULL;
    L->nnear = L->capnear = 0;
    int64_t i = 0, j = 0;
    while (i < ng || j < cand.nnear) {
        uint32_t lg = i < ng ? (uint32_t)grav[i] & NEAR_LABEL : UINT32_MAX;
        uint32_t lc = j < cand.nnear ? (uint32_t)cand.near[j] & NEAR_LABEL : UINT32_MAX;
        if (lg == lc) { push_near(L, lg, NEAR_CAND); ++i; ++j; }
        else if (lg < lc) { push_near(L, lg, 0); ++i; }
        else { push_near(L, lc, NEAR_CAND | NEAR_NBONLY); ++j; }
    }
    L->visited += cand.visited;
    free(grav);
    free(cand.near);
}

static void walk_leaf(otree *t, int64_t A)
{
    leaf_lists *L = &t->lists[A - ((int64_t)1 << t->k)];
    L->nnear = L->nfar = L->visited = 0;
    L->walked = 1;
    if (t->count[A] == 0) return;
    if (t->pure_mac) {
        walk_leaf_pure(t, A, L);
    } else if (t->k == 0) {
        visit(t, A, 1, t->theta, L);
    } else {
        visit(t, A, 2, t->theta, L);
        visit(t, A, 3, t->theta, L);
    }
}

/* Walk the given leaves (labels); with leaves == NULL walk every leaf.      */
/* pure_mac = 0: the paper's walk (reachability overrides the MAC);          */
/* pure_mac = 1: gravity by the MAC alone, neighbours by reachability.       */
void orc_walk(otree *t, double theta, const int64_t *leaves, int64_t nleaves, int pure_mac)
{
    free_lists(t);
    t->pure_mac = pure_mac != 0;
    int64_t nleaf = (int64_t)1 << t->k;
    t->lists = (leaf_lists *)calloc((size_t)nleaf, sizeof(leaf_lists));
    t->theta = theta;
    if (leaves == NULL) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < nleaf; ++i) walk_leaf(t, nleaf + i);
    } else {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < nleaves; ++i) walk_leaf(t, leaves[i]);
    }
}

/* Per-leaf list sizes (0 for leaves not walked); stats[5*i..] =            */
/* {nodes tested, near leaves, far nodes, near-field particles, candidate   */
/* particles}; near leaves count every list entry.                          */
void orc_list_sizes(const otree *t, int64_t *nnear, int64_t *nfar, int64_t *stats)
{
    int64_t nleaf = (int64_t)1 << t->k;
    for (int64_t i = 0; i < nleaf; ++i) {
        const leaf_lists *L = &t->lists[i];
        nnear[i] = L->nnear;
        nfar[i] = L->nfar;
        if (stats) {
            int64_t P = 0, C = 0;
            for (int64_t j = 0; j < L->nnear; ++j) {
                uint32_t e = (uint32_t)L->near[j];
                int64_t lab = (int64_t)(e & NEAR_LABEL);
                if (!(e & NEAR_NBONLY)) P += t->count[lab];
                if (e & NEAR_CAND) C += t->count[lab];
            }
            stats[5 * i + 0] = L->visited;
            stats[5 * i + 1] = L->nnear;
            stats[5 * i + 2] = L->nfar;
            stats[5 * i + 3] = P;
            stats[5 * i + 4] = C;
        }
    }
}

/* Copy the lists of one leaf (label A). */
void orc_leaf_lists(const otree *t, int64_t A, int32_t *near, int32_t *far)
{
    const leaf_lists *L = &t->lists[A - ((int64_t)1 << t->k)];
    if (L->nnear) memcpy(near, L->near, (size_t)L->nnear * sizeof(int32_t));
    if (L->nfar) memcpy(far, L->far, (size_t)L->nfar * sizeof(int32_t));
}

/* ------------------------------------------------------------------------ */
/* Neighbours (Sec. 2.3): cull the candidate leaves to |r_ab| < 2 h_a.       */
/* Lists per particle, in original order. The culled list comes out in     */
/* tree order (candidate leaves by ascending label, leaf order inside); the */
/* one-dimensional list of Sec. 2.3.2 then holds it ascending by original   */
/* index, an order that does not depend on the tree.                        */
/* Particles whose leaf was not walked get count -1.                        */
/* ------------------------------------------------------------------------ */
static int64_t cull_particle(const otree *t, const leaf_lists *L, int64_t a, int32_t *out)
{
    int64_t cnt = 0;
    double two_h = 2.0 * t->h[a];
    double lim = two_h * two_h;
    for (int64_t j = 0; j < L->nnear; ++j) {
        if (!((uint32_t)L->near[j] & NEAR_CAND)) continue;
        int64_t B = (int64_t)((uint32_t)L->near[j] & NEAR_LABEL);
        for (int64_t p = t->first[B]; p < t->first[B] + t->count[B]; ++p) {
            int64_t b = t->perm[p];
            if (b == a) continue;
            if (dist2(t->x[a], t->y[a], t->z[a], t->x[b], t->y[b], t->z[b]) < lim) {
                if (out) out[cnt] = (int32_t)b;
                ++cnt;
            }
        }
    }
    return cnt;
}

static int cmp_i32(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    return (a > b) - (a < b);
}

void orc_neighbours_count(const otree *t, int64_t *counts)
{
    int64_t leaf0 = (int64_t)1 << t->k;
    for (int64_t i = 0; i < t->n; ++i) counts[i] = -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t A = leaf0; A < t->nlab; ++A) {
        const leaf_lists *L = &t->lists[A - leaf0];
        if (!L->walked) continue;
        for (int64_t p = t->first[A]; p < t->first[A] + t->count[A]; ++p) {
            int64_t a = t->perm[p];
            counts[a] = cull_particle(t, L, a, NULL);
        }
    }
}

void orc_neighbours_fill(const otree *t, const int64_t *offsets, int32_t *ids)
{
    int64_t leaf0 = (int64_t)1 << t->k;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t A = leaf0; A < t->nlab; ++A) {
        const leaf_lists *L = &t->lists[A - leaf0];
        if (!L->walked) continue;
        for (int64_t p = t->first[A]; p < t->first[A] + t->count[A]; ++p) {
            int64_t a = t->perm[p];
            int64_t c = cull_particle(t, L, a, ids + offsets[a]);
            qsort(ids + offsets[a], (size_t)c, sizeof(int32_t), cmp_i32);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Kernel softening (Sec. 2.4.3, Eq. for S(q)): F = S / r so that the pair   */
/* acceleration is -m_b F (r_a - r_b); q = r/h with h the mean of h_a, h_b.  */
/* dFr = (dF/dr)/r, used by the vector-Jacobian product.                     */
/* ------------------------------------------------------------------------ */
void orc_kernel_F(double r, double h, double *F, double *dFr)
{
    double q = r / h;
    double h3 = h * h * h;
    double h5 = h3 * h * h;
    if (q < 1.0) {
        *F = (4.0 / 3.0 - (6.0 / 5.0) * q * q + 0.5 * q * q * q) / h3;
        *dFr = (-12.0 / 5.0 + 1.5 * q) / h5;
    } else if (q < 2.0) {
        double q3 = q * q * q;
        *F = (8.0 / 3.0 - 3.0 * q + (6.0 / 5.0) * q * q - q3 / 6.0 - 1.0 / (15.0 * q3)) / h3;
        *dFr = (-3.0 / q + 12.0 / 5.0 - 0.5 * q + 1.0 / (5.0 * q3 * q * q)) / h5;
    } else {
        double r3 = r * r * r;
        *F = 1.0 / r3;
        *dFr = -3.0 / (r3 * r * r);
    }
}

/* ------------------------------------------------------------------------ */
/* Derivative tensors of 1/r (Sec. 2.4.2 needs them for the field of Eq. 5  */
/* and its Jacobian and Hessian). For an index tuple (i1..in):              */
/*   d^n (1/r) = sum over partial pairings P of the n slots in which paired */
/*   slots carry equal indices: D_{n-|P|} * prod over unpaired slots x_i,   */
/*   with D_m = (-1)^m (2m-1)!! / r^(2m+1).                                 */
/* The terms are tabulated once per order (monomial exponents + multiplicity)*/
/* ------------------------------------------------------------------------ */
#define MAXORD 6
typedef struct { int m, ex, ey, ez; double coeff; } dterm;
typedef struct { int nterm; dterm term[128]; } dentry;
static dentry *dtab[MAXORD + 1];

static void enum_pairings(int n, const int *idx, unsigned used, int npairs, int ex[3], dentry *e)
{
    int pos = -1;
    for (int i = 0; i < n; ++i)
        if (!(used & (1u << i))) { pos = i; break; }
    if (pos < 0) {
        int m = n - npairs;
        for (int j = 0; j < e->nterm; ++j) {
            dterm *d = &e->term[j];
            if (d->m == m && d->ex == ex[0] && d->ey == ex[1] && d->ez == ex[2]) { d->coeff += 1.0; return; }
        }
        dterm *d = &e->term[e->nterm++];
        d->m = m; d->ex = ex[0]; d->ey = ex[1]; d->ez = ex[2]; d->coeff = 1.0;
        return;
    }
    /* slot pos unpaired: contributes x_{idx[pos]} */
    ex[idx[pos]]++;
    enum_pairings(n, idx, used | (1u << pos), npairs, ex, e);
    ex[idx[pos]]--;
    /* slot pos paired with a later free slot carrying the same index */
    for (int q = pos + 1; q < n; ++q) {
        if (used & (1u << q)) continue;
        if (idx[q] != idx[pos]) continue;
        enum_pairings(n, idx, used | (1u << pos) | (1u << q), npairs + 1, ex, e);
    }
}

static void build_dtab(void)
{
    if (dtab[MAXORD]) return;
    for (int n = 0; n <= MAXORD; ++n) {
        int cnt = 1;
        for (int i = 0; i < n; ++i) cnt *= 3;
        dentry *tab = (dentry *)calloc((size_t)cnt, sizeof(dentry));
        for (int tup = 0; tup < cnt; ++tup) {
            int idx[MAXORD], v = tup;
            for (int i = n - 1; i >= 0; --i) { idx[i] = v % 3; v /= 3; }
            int ex[3] = {0, 0, 0};
            enum_pairings(n, idx, 0u, 0, ex, &tab[tup]);
        }
        dtab[n] = tab;
    }
}

void orc_init(void) { build_dtab(); }

/* out[3^n] = d^n(1/r) at R; index tuple (i1..in) at i1*3^(n-1) + ... + in. */
void orc_deriv_tensor(int n, const double *R, double *out)
{
    build_dtab();
    double r2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
    double r = sqrt(r2);
    double D[MAXORD + 1];
    double dfac = 1.0;                      /* (2m-1)!! */
    double rp = r;                          /* r^(2m+1) */
    for (int m = 0; m <= MAXORD; ++m) {
        if (m > 0) { dfac *= (double)(2 * m - 1); rp *= r2; }
        D[m] = ((m & 1) ? -dfac : dfac) / rp;
    }
    double px[MAXORD + 1], py[MAXORD + 1], pz[MAXORD + 1];
    px[0] = py[0] = pz[0] = 1.0;
    for (int i = 1; i <= MAXORD; ++i) {
        px[i] = px[i - 1] * R[0];
        py[i] = py[i - 1] * R[1];
        pz[i] = pz[i - 1] * R[2];
    }
    int cnt = 1;
    for (int i = 0; i < n; ++i) cnt *= 3;
    for (int tup = 0; tup < cnt; ++tup) {
        const dentry *e = &dtab[n][tup];
        double s = 0.0;
        for (int j = 0; j < e->nterm; ++j) {
            const dterm *d = &e->term[j];
            s += d->coeff * D[d->m] * px[d->ex] * py[d->ey] * pz[d->ez];
        }
        out[tup] = s;
    }
}

static void q_full(const double *q6, double Q[3][3])
{
    Q[0][0] = q6[0]; Q[0][1] = q6[1]; Q[0][2] = q6[2];
    Q[1][0] = q6[1]; Q[1][1] = q6[3]; Q[1][2] = q6[4];
    Q[2][0] = q6[2]; Q[2][1] = q6[4]; Q[2][2] = q6[5];
}

/* Field of one source node (mass M, traceless quadrupole Q about its COM) */
/* at R = r_sink - COM_B: Eq. 5 gives Phi = -M/r - (1/6) Q_jk d_jk(1/r), so */
/* f = -grad Phi: f_i = M g_i + Q_jk g_ijk / 6, J = grad f, H = grad J.     */
/* With T4 != NULL also T4 = grad H (needed by the vector-Jacobian product).*/
void orc_far_coeffs(double M, const double *q6, const double *R, double *f, double *J,
                    double *H, double *T4)
{
    double g1[3], g2[9], g3[27], g4[81], g5[243];
    static __thread double g6[729];
    double Q[3][3];
    q_full(q6, Q);
    orc_deriv_tensor(1, R, g1);
    orc_deriv_tensor(2, R, g2);
    orc_deriv_tensor(3, R, g3);
    orc_deriv_tensor(4, R, g4);
    orc_deriv_tensor(5, R, g5);
    if (T4) orc_deriv_tensor(6, R, g6);
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) s += Q[j][k] * g3[9 * i + 3 * j + k];
        f[i] = M * g1[i] + s / 6.0;
    }
    for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) s += Q[j][k] * g4[27 * i + 9 * j + 3 * k + l];
            J[3 * i + l] = M * g2[3 * i + l] + s / 6.0;
        }
    for (int i = 0; i < 3; ++i)
        for (int l = 0; l < 3; ++l)
            for (int mm = 0; mm < 3; ++mm) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j)
                    for (int k = 0; k < 3; ++k) s += Q[j][k] * g5[81 * i + 27 * j + 9 * k + 3 * l + mm];
                H[9 * i + 3 * l + mm] = M * g3[9 * i + 3 * l + mm] + s / 6.0;
            }
    if (T4) {
        for (int i = 0; i < 3; ++i)
            for (int l = 0; l < 3; ++l)
                for (int mm = 0; mm < 3; ++mm)
                    for (int nn = 0; nn < 3; ++nn) {
                        double s = 0.0;
                        for (int j = 0; j < 3; ++j)
                            for (int k = 0; k < 3; ++k)
                                s += Q[j][k] * g6[243 * i + 81 * j + 27 * k + 9 * l + 3 * mm + nn];
                        T4[27 * i + 9 * l + 3 * mm + nn] = M * g4[27 * i + 9 * l + 3 * mm + nn] + s / 6.0;
                    }
    }
}

/* Sink-leaf expansion coefficients: sums over the far list of leaf A. */
/* Sink coefficients of leaf A (Eq. 6). Reading A (default): J and H are the */
/* Jacobian and Hessian of the monopole + quadrupole field f. Reading B (the  */
/* order-consistent alternative): the quadrupole enters f only, J and H are  */
/* those of the monopole field.                                              */
static void leaf_far(const otree *t, int64_t A, const leaf_lists *L, double f[3], double J[9], double H[27])
{
    static const double no_quad[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    memset(f, 0, 3 * sizeof(double));
    memset(J, 0, 9 * sizeof(double));
    memset(H, 0, 27 * sizeof(double));
    for (int64_t j = 0; j < L->nfar; ++j) {
        int64_t B = L->far[j];
        double R[3], fb[3], Jb[9], Hb[27];
        for (int d = 0; d < 3; ++d) R[d] = t->com[3 * A + d] - t->com[3 * B + d];
        orc_far_coeffs(t->M[B], &t->Q[6 * B], R, fb, Jb, Hb, NULL);
        if (t->reading == 1) {
            double fm[3];
            orc_far_coeffs(t->M[B], no_quad, R, fm, Jb, Hb, NULL);
        }
        for (int i = 0; i < 3; ++i) f[i] += fb[i];
        for (int i = 0; i < 9; ++i) J[i] += Jb[i];
        for (int i = 0; i < 27; ++i) H[i] += Hb[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Gravity (Sec. 2.4): for each walked leaf A and particle a in A,          */
/*   a = -sum_{B in near(A)} sum_{b in B} m_b F(r_ab, h_ab) (r_a - r_b)     */
/*       + f_A + J_A d + (1/2) H_A[d, d],   d = r_a - COM_A  (Eq. 6).       */
/* Output in original order; particles in leaves not walked get NaN.        */
/* ------------------------------------------------------------------------ */
/* parts: 1 = the near field only, 2 = the far field only (with its Taylor */
/* evaluation, Eq. 6), 3 = both (orc_gravity). The parts exist to time the  */
/* near and far field separately, as Table 1's NG and FG columns do.        */
void orc_gravity_parts(const otree *t, double *ax, double *ay, double *az, int parts)
{
    int64_t leaf0 = (int64_t)1 << t->k;
    for (int64_t i = 0; i < t->n; ++i) ax[i] = ay[i] = az[i] = NAN;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t A = leaf0; A < t->nlab; ++A) {
        const leaf_lists *L = &t->lists[A - leaf0];
        if (!L->walked || t->count[A] == 0) continue;
        double f[3] = {0.0, 0.0, 0.0}, J[9] = {0.0}, H[27] = {0.0};
        if (parts & 2) leaf_far(t, A, L, f, J, H);
        for (int64_t p = t->first[A]; p < t->first[A] + t->count[A]; ++p) {
            int64_t a = t->perm[p];
            double acc[3] = {0.0, 0.0, 0.0};
            for (int64_t j = 0; j < ((parts & 1) ? L->nnear : 0); ++j) {
                if ((uint32_t)L->near[j] & NEAR_NBONLY) continue;   /* neighbour search only */
                int64_t B = (int64_t)((uint32_t)L->near[j] & NEAR_LABEL);
                for (int64_t q = t->first[B]; q < t->first[B] + t->count[B]; ++q) {
                    int64_t b = t->perm[q];
                    double v[3] = {t->x[a] - t->x[b], t->y[a] - t->y[b], t->z[a] - t->z[b]};
                    double r = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
                    double F, dFr;
                    orc_kernel_F(r, 0.5 * (t->h[a] + t->h[b]), &F, &dFr);
                    for (int d = 0; d < 3; ++d) acc[d] -= t->m[b] * F * v[d];
                }
            }
            double dl[3] = {t->x[a] - t->com[3 * A], t->y[a] - t->com[3 * A + 1], t->z[a] - t->com[3 * A + 2]};
            double out[3];
            for (int i = 0; i < 3; ++i) {
                double s = f[i];
                for (int l = 0; l < 3; ++l) s += J[3 * i + l] * dl[l];
                double s2 = 0.0;
                for (int l = 0; l < 3; ++l)
                    for (int mm = 0; mm < 3; ++mm) s2 += H[9 * i + 3 * l + mm] * dl[l] * dl[mm];
                out[i] = acc[i] + s + 0.5 * s2;
            }
            ax[a] = out[0];
            ay[a] = out[1];
            az[a] = out[2];
        }
    }
}

void orc_gravity(const otree *t, double *ax, double *ay, double *az)
{
    orc_gravity_parts(t, ax, ay, az, 3);
}

/* ------------------------------------------------------------------------ */
/* Vector-Jacobian product of the accelerations with the topology, the      */
/* particle-to-leaf map and the lists held fixed (every leaf must have been */
/* walked). L = sum_a g_a . a_a; outputs dL/dx, dL/dy, dL/dz, dL/dm.        */
/* M, COM and Q of every node are functions of the inputs:                  */
/*   M = sum m_b, COM = sum m_b r_b / M, Q = sum m_b (3 d d^T - |d|^2 I)    */
/* (Eq. 1 and Eq. 2 agree exactly for internal nodes: parallel-axis rule).  */
/* ------------------------------------------------------------------------ */
void orc_vjp(const otree *t, const double *gx, const double *gy, const double *gz,
             double *dx, double *dy, double *dz, double *dm)
{
    int64_t n = t->n, leaf0 = (int64_t)1 << t->k;
    const double *g[3] = {gx, gy, gz};
    double *dr[3] = {dx, dy, dz};
    if (t->reading != 0) {          /* defined for reading A only */
        for (int64_t i = 0; i < n; ++i) dx[i] = dy[i] = dz[i] = dm[i] = NAN;
        return;
    }
    for (int64_t i = 0; i < n; ++i) dx[i] = dy[i] = dz[i] = dm[i] = 0.0;
    int64_t L = t->nlab;
    double *adjM = (double *)calloc((size_t)L, sizeof(double));
    double *adjR = (double *)calloc((size_t)(3 * L), sizeof(double));
    double *adjQ = (double *)calloc((size_t)(9 * L), sizeof(double));
    for (int64_t A = leaf0; A < t->nlab; ++A) {
        const leaf_lists *LL = &t->lists[A - leaf0];
        if (t->count[A] == 0) continue;
        int64_t s = t->first[A], c = t->count[A];
        const double *cA = &t->com[3 * A];
        /* near field: K = F I + (dF/dr / r) v v^T, v = r_a - r_b */
        for (int64_t p = s; p < s + c; ++p) {
            int64_t a = t->perm[p];
            double ga[3] = {gx[a], gy[a], gz[a]};
            for (int64_t j = 0; j < LL->nnear; ++j) {
                if ((uint32_t)LL->near[j] & NEAR_NBONLY) continue;
                int64_t B = (int64_t)((uint32_t)LL->near[j] & NEAR_LABEL);
                for (int64_t q = t->first[B]; q < t->first[B] + t->count[B]; ++q) {
                    int64_t b = t->perm[q];
                    double v[3] = {t->x[a] - t->x[b], t->y[a] - t->y[b], t->z[a] - t->z[b]};
                    double r = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
                    double F, dFr;
                    orc_kernel_F(r, 0.5 * (t->h[a] + t->h[b]), &F, &dFr);
                    double vg = v[0] * ga[0] + v[1] * ga[1] + v[2] * ga[2];
                    for (int d = 0; d < 3; ++d) {
                        double Kg = F * ga[d] + dFr * v[d] * vg;
                        dr[d][a] -= t->m[b] * Kg;
                        dr[d][b] += t->m[b] * Kg;
                    }
                    dm[b] -= F * vg;
                }
            }
        }
        /* far field: per-leaf cotangent moments G0, G1, G2 */
        double G0[3] = {0, 0, 0}, G1[9], G2[27];
        memset(G1, 0, sizeof G1);
        memset(G2, 0, sizeof G2);
        double f[3], J[9], H[27];
        leaf_far(t, A, LL, f, J, H);
        for (int64_t p = s; p < s + c; ++p) {
            int64_t a = t->perm[p];
            double ga[3] = {gx[a], gy[a], gz[a]};
            double d[3] = {t->x[a] - cA[0], t->y[a] - cA[1], t->z[a] - cA[2]};
            for (int i = 0; i < 3; ++i) {
                G0[i] += ga[i];
                for (int l = 0; l < 3; ++l) {
                    G1[3 * i + l] += ga[i] * d[l];
                    for (int mm = 0; mm < 3; ++mm) G2[9 * i + 3 * l + mm] += ga[i] * d[l] * d[mm];
                }
            }
            /* direct dependence on r_a through d: J^T g + H[g, d] */
            for (int l = 0; l < 3; ++l) {
                double s1 = 0.0;
                for (int i = 0; i < 3; ++i) {
                    s1 += ga[i] * J[3 * i + l];
                    for (int mm = 0; mm < 3; ++mm) s1 += ga[i] * H[9 * i + 3 * l + mm] * d[mm];
                }
                dr[l][a] += s1;
            }
        }
        double cot[3] = {0, 0, 0};
        for (int64_t j = 0; j < LL->nfar; ++j) {
            int64_t B = LL->far[j];
            double R[3], fb[3], Jb[9], Hb[27], T4[81];
            for (int d = 0; d < 3; ++d) R[d] = cA[d] - t->com[3 * B + d];
            orc_far_coeffs(t->M[B], &t->Q[6 * B], R, fb, Jb, Hb, T4);
            double rho[3];
            for (int l = 0; l < 3; ++l) {
                double v1 = 0.0, v2 = 0.0, v3 = 0.0;
                for (int i = 0; i < 3; ++i) {
                    v1 += G0[i] * Jb[3 * i + l];
                    for (int mm = 0; mm < 3; ++mm) {
                        v2 += G1[3 * i + mm] * Hb[9 * i + 3 * mm + l];
                        for (int nn = 0; nn < 3; ++nn)
                            v3 += G2[9 * i + 3 * mm + nn] * T4[27 * i + 9 * mm + 3 * nn + l];
                    }
                }
                rho[l] = v1 + v2 + 0.5 * v3;
                cot[l] += 0.5 * v3;
                adjR[3 * B + l] -= rho[l];
            }
            /* d/dM and d/dQ_jk of G0.f + G1:J + G2:H/2 */
            double g1[3], g2[9], g3[27], g4[81], g5[243];
            orc_deriv_tensor(1, R, g1);
            orc_deriv_tensor(2, R, g2);
            orc_deriv_tensor(3, R, g3);
            orc_deriv_tensor(4, R, g4);
            orc_deriv_tensor(5, R, g5);
            double aM = 0.0;
            for (int i = 0; i < 3; ++i) {
                aM += g1[i] * G0[i];
                for (int l = 0; l < 3; ++l) {
                    aM += g2[3 * i + l] * G1[3 * i + l];
                    for (int mm = 0; mm < 3; ++mm) aM += 0.5 * g3[9 * i + 3 * l + mm] * G2[9 * i + 3 * l + mm];
                }
            }
            adjM[B] += aM;
            for (int jj = 0; jj < 3; ++jj)
                for (int kk = 0; kk < 3; ++kk) {
                    double aq = 0.0;
                    for (int i = 0; i < 3; ++i) {
                        aq += g3[9 * i + 3 * jj + kk] * G0[i];
                        for (int l = 0; l < 3; ++l) {
                            aq += g4[27 * i + 9 * jj + 3 * kk + l] * G1[3 * i + l];
                            for (int mm = 0; mm < 3; ++mm)
                                aq += 0.5 * g5[81 * i + 27 * jj + 9 * kk + 3 * l + mm] * G2[9 * i + 3 * l + mm];
                        }
                    }
                    adjQ[9 * B + 3 * jj + kk] += aq / 6.0;
                }
        }
        /* sink centre of mass: COM_A = sum m_a r_a / M_A */
        for (int64_t p = s; p < s + c; ++p) {
            int64_t a = t->perm[p];
            double d[3] = {t->x[a] - cA[0], t->y[a] - cA[1], t->z[a] - cA[2]};
            for (int l = 0; l < 3; ++l) dr[l][a] += t->m[a] / t->M[A] * cot[l];
            dm[a] += (cot[0] * d[0] + cot[1] * d[1] + cot[2] * d[2]) / t->M[A];
        }
    }
    /* push node adjoints to the particles of each source node */
    for (int64_t B = 1; B < t->nlab; ++B) {
        if (t->count[B] == 0) continue;
        const double *aR = &adjR[3 * B], *aQ = &adjQ[9 * B];
        if (adjM[B] == 0.0 && aR[0] == 0.0 && aR[1] == 0.0 && aR[2] == 0.0) {
            int any = 0;
            for (int q = 0; q < 9; ++q) any |= aQ[q] != 0.0;
            if (!any) continue;
        }
        const double *cB = &t->com[3 * B];
        double MB = t->M[B];
        for (int64_t p = t->first[B]; p < t->first[B] + t->count[B]; ++p) {
            int64_t b = t->perm[p];
            double d[3] = {t->x[b] - cB[0], t->y[b] - cB[1], t->z[b] - cB[2]};
            double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double mb = t->m[b];
            for (int l = 0; l < 3; ++l) {
                /* dQ_jk/dr_l = m (3 (delta_jl d_k + d_j delta_kl) - 2 d_l delta_jk) */
                double sq = 0.0;
                for (int jj = 0; jj < 3; ++jj)
                    for (int kk = 0; kk < 3; ++kk) {
                        double dq = 3.0 * ((jj == l ? d[kk] : 0.0) + (kk == l ? d[jj] : 0.0));
                        if (jj == kk) dq -= 2.0 * d[l];
                        sq += aQ[3 * jj + kk] * mb * dq;
                    }
                dr[l][b] += aR[l] * mb / MB + sq;
            }
            double sqm = 0.0;
            for (int jj = 0; jj < 3; ++jj)
                for (int kk = 0; kk < 3; ++kk) {
                    double qv = 3.0 * d[jj] * d[kk];
                    if (jj == kk) qv -= d2;
                    sqm += aQ[3 * jj + kk] * qv;
                }
            dm[b] += adjM[B] + (aR[0] * d[0] + aR[1] * d[1] + aR[2] * d[2]) / MB + sqm;
        }
    }
    (void)g;
    free(adjM);
    free(adjR);
    free(adjQ);
}
