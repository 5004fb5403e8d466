/*
 * askit_oracle.c -- reference oracle for the N log N hierarchical direct
 * solver of Yu, March & Biros, "An N log N Parallel Fast Direct Solver for
 * Kernel Matrices" (arXiv:1701.02324).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test-suite, by
 * the smoke check and by the CPU-baseline leg of the benchmark, and by
 * nothing else.  It shares no code, header, table or helper with the HIP
 * library; the two meet only through seeded input arrays.
 *
 * Plain FP64 C99: no BLAS, no blocking, textbook loops, OpenMP only across
 * the independent tree nodes of one level.  Every routine follows the
 * passage of the paper cited in its comment.  Where the paper leaves a
 * choice open (tree split rule, sampling, QR tie breaking, rank clamping,
 * LU pivot ties, ...) the reading taken is stated at the routine and listed
 * in the design notes of the repository.
 *
 * Notation follows the paper: X holds N points in d dimensions (stored
 * point-major, N x d row-major), m is the leaf size, s the skeleton rank,
 * alpha a tree node, l / r its children, alpha~ its skeleton, P_{a~ C} the
 * interpolative-decomposition projection, Phat = Ktilde^{-1} P (the "hat"
 * factor of Sec. 2.2), Z = I + V W the reduced system of eq. (8).
 *
 * Compile with -ffp-contract=off: the tree rules below fix the rounding of
 * every operation (explicit fma() where one is meant).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_ALLOC 2
#define ORC_ERR_STATE 4
#define ORC_ERR_SINGULAR 5

/* ------------------------------------------------------------------------ */
/* State                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    /* problem */
    int64_t N;
    int d, m, s, nsamp;     /* nsamp = sample cap (4s by default)          */
    uint64_t seed;
    int64_t problem;        /* problem index folded into the sampling seed */
    double h;
    double tol;             /* tau of the adaptive rank rule (0: fixed s)  */
    double *X;              /* N x d, original point order                 */
    /* tree */
    int D;                  /* depth; leaves at level D                    */
    int64_t nnodes;         /* 2^(D+1) - 1 heap-indexed nodes              */
    int64_t *perm;          /* perm[position] = original point index       */
    int64_t *nb, *ne;       /* node = positions [nb, ne)                   */
    int tree_built, skel_built, factored;
    /* skeletons (non-root nodes) */
    int *sr;                /* s_alpha, actual rank                        */
    int *nc;                /* |C|, number of candidate columns            */
    int *trunc;             /* 1 if the rank guard truncated s_alpha       */
    int64_t **skel;         /* s_alpha skeleton positions                  */
    double **P;             /* s_alpha x |C| row-major, P_{alpha~ C}       */
    /* factorization */
    double lambda;
    double **LU;            /* leaf: (lambda I + K_aa) LU; internal: Z LU  */
    int **piv;              /* row interchanges of the LU                  */
    double **Phat;          /* non-root: n_alpha x s_alpha row-major       */
    double *pivratio;       /* min|U_ii| / max|U_ii| per factored block    */
    /* kappa-nearest-neighbour sampling: 0 = uniform rows only            */
    int kappa;
    int64_t *knn;           /* N x kappa neighbour positions (-1 padded)   */
    int64_t **nbr, **nbrw;  /* per node: ranked neighbour list, weights    */
    int64_t *nnbr;          /* per node: its length (<= nsamp)             */
    /* level restriction (hybrid solver): 0 = none; L >= 1 = frontier level */
    int hybL;
    int64_t hM;             /* order of the reduced system I + V W          */
    int64_t *hoff;          /* row offset of each frontier node in it       */
    double *hLU;            /* its LU (row-major) and pivots                */
    int *hpiv;
    double hratio;
} orc_t;

static int level_of(int64_t id) {
    int l = 0;
    while (((int64_t)2 << l) - 1 <= id) l++;
    return l;
}
static int64_t first_at(int l) { return ((int64_t)1 << l) - 1; }
static int is_leaf(const orc_t *o, int64_t id) { return level_of(id) == o->D; }

/* ------------------------------------------------------------------------ */
/* Gaussian kernel, eq. (1)                                                 */
/* ------------------------------------------------------------------------ */

/* squared distance by direct differences, summed in increasing dimension */
static double sqdist(const double *x, const double *y, int d) {
    double r2 = 0.0;
    for (int k = 0; k < d; k++) {
        double t = x[k] - y[k];
        r2 = r2 + t * t;
    }
    return r2;
}

/* K(x,y) = exp(-|x-y|^2 / (2 h^2)), eq. (1) */
double orc_kernel(const double *x, const double *y, int d, double h) {
    return exp(-(sqdist(x, y, d) / (2.0 * h * h)));
}

/* dK/dh = K * r^2 / h^3 (derivative of eq. (1) in the bandwidth) */
static double kernel_dh(const double *x, const double *y, int d, double h) {
    double r2 = sqdist(x, y, d);
    return exp(-(r2 / (2.0 * h * h))) * r2 / (h * h * h);
}

static const double *pt(const orc_t *o, int64_t pos) { return o->X + o->perm[pos] * o->d; }

/* kernel entry between two tree positions; which=1 gives dK/dh */
static double kpos(const orc_t *o, int64_t a, int64_t b, int which) {
    return which ? kernel_dh(pt(o, a), pt(o, b), o->d, o->h) : orc_kernel(pt(o, a), pt(o, b), o->d, o->h);
}

/* ------------------------------------------------------------------------ */
/* Context                                                                  */
/* ------------------------------------------------------------------------ */

/* Tree depth (Sec. 2.1, "Partitioning the matrix"): the smallest D with
 * N <= m 2^D, so every leaf holds at most m and more than m/2 points. */
int orc_depth(int64_t N, int m) {
    int D = 0;
    while ((int64_t)m * ((int64_t)1 << D) < N) D++;
    return D;
}

orc_t *orc_new(const double *X, int64_t N, int d, int m, int s, int nsamp, uint64_t seed,
               int64_t problem, double h) {
    if (N < 1 || d < 1 || m < 2 || s < 1 || nsamp < 1 || !(h > 0.0)) return NULL;
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    if (!o) return NULL;
    o->N = N; o->d = d; o->m = m; o->s = s; o->nsamp = nsamp;
    o->seed = seed; o->problem = problem; o->h = h;
    o->X = (double *)malloc(sizeof(double) * N * d);
    o->D = orc_depth(N, m);
    o->nnodes = ((int64_t)2 << o->D) - 1;
    o->perm = (int64_t *)malloc(sizeof(int64_t) * N);
    o->nb = (int64_t *)malloc(sizeof(int64_t) * o->nnodes);
    o->ne = (int64_t *)malloc(sizeof(int64_t) * o->nnodes);
    o->sr = (int *)calloc(o->nnodes, sizeof(int));
    o->nc = (int *)calloc(o->nnodes, sizeof(int));
    o->trunc = (int *)calloc(o->nnodes, sizeof(int));
    o->skel = (int64_t **)calloc(o->nnodes, sizeof(int64_t *));
    o->P = (double **)calloc(o->nnodes, sizeof(double *));
    o->LU = (double **)calloc(o->nnodes, sizeof(double *));
    o->piv = (int **)calloc(o->nnodes, sizeof(int *));
    o->Phat = (double **)calloc(o->nnodes, sizeof(double *));
    o->pivratio = (double *)calloc(o->nnodes, sizeof(double));
    if (!o->X || !o->perm || !o->nb || !o->ne || !o->sr || !o->nc || !o->trunc || !o->skel ||
        !o->P || !o->LU || !o->piv || !o->Phat || !o->pivratio)
        return NULL;
    memcpy(o->X, X, sizeof(double) * N * d);
    /* node ranges: every split gives floor(n/2) points to the left child */
    o->nb[0] = 0; o->ne[0] = N;
    for (int64_t id = 0; id < first_at(o->D); id++) {
        int64_t b = o->nb[id], n = o->ne[id] - o->nb[id];
        o->nb[2 * id + 1] = b;          o->ne[2 * id + 1] = b + n / 2;
        o->nb[2 * id + 2] = b + n / 2;  o->ne[2 * id + 2] = o->ne[id];
    }
    for (int64_t i = 0; i < N; i++) o->perm[i] = i;
    return o;
}

static void free_factor(orc_t *o) {
    for (int64_t i = 0; i < o->nnodes; i++) {
        free(o->LU[i]); free(o->piv[i]); free(o->Phat[i]);
        o->LU[i] = NULL; o->piv[i] = NULL; o->Phat[i] = NULL;
    }
    free(o->hoff); free(o->hLU); free(o->hpiv);
    o->hoff = NULL; o->hLU = NULL; o->hpiv = NULL;
    o->factored = 0;
}

void orc_free(orc_t *o) {
    if (!o) return;
    free_factor(o);
    for (int64_t i = 0; i < o->nnodes; i++) { free(o->skel[i]); free(o->P[i]); }
    free(o->X); free(o->perm); free(o->nb); free(o->ne); free(o->sr); free(o->nc); free(o->trunc);
    free(o->skel); free(o->P); free(o->LU); free(o->piv); free(o->Phat); free(o->pivratio);
    if (o->nbr)
        for (int64_t i = 0; i < o->nnodes; i++) { free(o->nbr[i]); free(o->nbrw[i]); }
    free(o->knn); free(o->nbr); free(o->nbrw); free(o->nnbr);
    free(o);
}

int orc_get_depth(const orc_t *o) { return o->D; }

/* Adaptive rank (Sec. 2.1, "Computing low rank approximations"): the rank
 * of a node is the smallest s_alpha with sigma_{s_alpha+1} / sigma_1 < tau,
 * the singular values estimated by the diagonal of the pivoted QR, capped
 * at s (then s_max).  tau = 0 keeps the fixed rank s.  Takes effect at
 * the next skeletonization. */
int orc_set_tol(orc_t *o, double tau) {
    if (!(tau >= 0.0) || !(tau < 1.0)) return ORC_ERR_ARG;
    o->tol = tau;
    return ORC_OK;
}

/* Change the bandwidth while keeping the tree and the skeletons (the ID is
 * held fixed, as in the bandwidth derivative); the factorization is dropped. */
int orc_set_h(orc_t *o, double h) {
    if (!(h > 0.0)) return ORC_ERR_ARG;
    o->h = h;
    free_factor(o);
    return ORC_OK;
}
void orc_get_perm(const orc_t *o, int64_t *out) { memcpy(out, o->perm, sizeof(int64_t) * o->N); }
void orc_node_range(const orc_t *o, int64_t id, int64_t *b, int64_t *e) { *b = o->nb[id]; *e = o->ne[id]; }

/* ------------------------------------------------------------------------ */
/* Tree: ball-tree style equal split by a hyperplane (Sec. 2.1).            */
/* Reading: the hyperplane is normal to the principal axis of the node's    */
/* points and passes through their median.  Every reduction has a fixed     */
/* order so that any implementation of the same rules gets the same perm.   */
/* ------------------------------------------------------------------------ */

#define TREE_CHUNK 256
#define TREE_POWER_ITERS 50

/* sum of per-chunk partials by pairwise halving: p[i] = p[2i] + p[2i+1],
 * an odd tail element passes through unchanged */
static double pairwise_total(double *p, int64_t n) {
    while (n > 1) {
        int64_t h2 = (n + 1) / 2;
        for (int64_t i = 0; i < h2; i++) p[i] = (2 * i + 1 < n) ? p[2 * i] + p[2 * i + 1] : p[2 * i];
        n = h2;
    }
    return n ? p[0] : 0.0;
}

typedef struct { double key; int64_t id; int64_t pos; } keyed_t;

static int keyed_cmp(const void *a, const void *b) {
    const keyed_t *x = (const keyed_t *)a, *y = (const keyed_t *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id < y->id) ? -1 : (x->id > y->id);
}

/* principal axis of a d x d scatter matrix S: power iteration from the
 * normalised all-ones vector, then the entry of largest magnitude (lowest
 * index on ties) is made positive */
static void principal_axis(const double *S, int d, double *v) {
    double *w = (double *)malloc(sizeof(double) * d);
    double v0 = 1.0 / sqrt((double)d);
    for (int k = 0; k < d; k++) v[k] = v0;
    for (int it = 0; it < TREE_POWER_ITERS; it++) {
        for (int i = 0; i < d; i++) {
            double acc = 0.0;
            for (int j = 0; j < d; j++) acc = acc + S[i * d + j] * v[j];
            w[i] = acc;
        }
        double nn = 0.0;
        for (int i = 0; i < d; i++) nn = nn + w[i] * w[i];
        if (nn == 0.0) {
            for (int k = 0; k < d; k++) v[k] = 0.0;
            v[0] = 1.0;
            break;
        }
        double nrm = sqrt(nn);
        for (int i = 0; i < d; i++) v[i] = w[i] / nrm;
    }
    int kmax = 0;
    for (int k = 1; k < d; k++)
        if (fabs(v[k]) > fabs(v[kmax])) kmax = k;
    if (v[kmax] < 0.0)
        for (int k = 0; k < d; k++) v[k] = -v[k];
    free(w);
}

/* split one node: mean and scatter with chunked sums, axis, keys, sort */
static void split_node(orc_t *o, int64_t b, int64_t e) {
    const int d = o->d;
    const int64_t n = e - b, nch = (n + TREE_CHUNK - 1) / TREE_CHUNK;
    double *part = (double *)malloc(sizeof(double) * (nch ? nch : 1));
    double *mu = (double *)malloc(sizeof(double) * d);
    double *S = (double *)malloc(sizeof(double) * d * d);
    double *v = (double *)malloc(sizeof(double) * d);
    keyed_t *kv = (keyed_t *)malloc(sizeof(keyed_t) * n);
    /* pass 1: mean */
    for (int k = 0; k < d; k++) {
        for (int64_t c = 0; c < nch; c++) {
            double acc = 0.0;
            int64_t c0 = b + c * TREE_CHUNK, c1 = c0 + TREE_CHUNK < e ? c0 + TREE_CHUNK : e;
            for (int64_t i = c0; i < c1; i++) acc = acc + pt(o, i)[k];
            part[c] = acc;
        }
        mu[k] = pairwise_total(part, nch) / (double)n;
    }
    /* pass 2: scatter matrix of the centred points (upper triangle, mirrored) */
    for (int a = 0; a < d; a++)
        for (int c2 = a; c2 < d; c2++) {
            for (int64_t c = 0; c < nch; c++) {
                double acc = 0.0;
                int64_t c0 = b + c * TREE_CHUNK, c1 = c0 + TREE_CHUNK < e ? c0 + TREE_CHUNK : e;
                for (int64_t i = c0; i < c1; i++) {
                    const double *x = pt(o, i);
                    double t = (x[a] - mu[a]) * (x[c2] - mu[c2]);
                    acc = acc + t;
                }
                part[c] = acc;
            }
            S[a * d + c2] = S[c2 * d + a] = pairwise_total(part, nch);
        }
    principal_axis(S, d, v);
    /* projection keys: p = fma(x_k - mu_k, v_k, p) in increasing k */
    for (int64_t i = b; i < e; i++) {
        const double *x = pt(o, i);
        double p = 0.0;
        for (int k = 0; k < d; k++) p = fma(x[k] - mu[k], v[k], p);
        kv[i - b].key = p;
        kv[i - b].id = o->perm[i];
        kv[i - b].pos = i;
    }
    /* order by (key, original index); left child = first floor(n/2) */
    qsort(kv, (size_t)n, sizeof(keyed_t), keyed_cmp);
    for (int64_t i = 0; i < n; i++) o->perm[b + i] = kv[i].id;
    free(part); free(mu); free(S); free(v); free(kv);
}

int orc_set_knn(orc_t *o, int kappa);

int orc_build_tree(orc_t *o) {
    o->tree_built = 0;
    orc_set_knn(o, 0); /* neighbour lists belong to a tree */
    for (int64_t i = 0; i < o->N; i++) o->perm[i] = i;
    for (int l = 0; l < o->D; l++) {
        int64_t f = first_at(l), cnt = (int64_t)1 << l;
#pragma omp parallel for schedule(dynamic)
        for (int64_t j = 0; j < cnt; j++) split_node(o, o->nb[f + j], o->ne[f + j]);
    }
    o->tree_built = 1;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Row sampling S' of S = [N] \ alpha (Sec. 2.1, "Computing low rank        */
/* approximations").  Reading: uniform sampling without replacement, drawn */
/* with SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).                       */
/* ------------------------------------------------------------------------ */

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ULL

uint64_t orc_splitmix64(uint64_t *state) {
    uint64_t z = (*state += GOLDEN_GAMMA);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Starting state of a node's stream: output number k = id + 1 + problem 2^32
 * of the SplitMix64 generator started from `seed`, i.e. the generator's
 * output function applied to seed + k * gamma.  (Seeding sibling streams with
 * states that differ by multiples of gamma would make them shifted copies of
 * one another; passing the state through the output function does not.) */
uint64_t orc_node_seed(uint64_t seed, int64_t problem, int64_t id) {
    uint64_t k = (uint64_t)id + 1ULL + ((uint64_t)problem << 32);
    uint64_t st = seed + (k - 1ULL) * GOLDEN_GAMMA;
    return orc_splitmix64(&st);
}

/* floor(u * c / 2^64) */
static uint64_t scale_draw(uint64_t u, uint64_t c) {
    uint64_t ul = u & 0xffffffffULL, uh = u >> 32, cl = c & 0xffffffffULL, ch = c >> 32;
    uint64_t ll = ul * cl, lh = ul * ch, hl = uh * cl, hh = uh * ch;
    uint64_t mid = (ll >> 32) + (lh & 0xffffffffULL) + (hl & 0xffffffffULL);
    return hh + (lh >> 32) + (hl >> 32) + (mid >> 32);
}

/* Sample positions for the node [b,e), after the npre positions of pre[]
 * (distinct, outside the node, npre <= nsamp), which open the list: draws
 * that repeat any position already in the list are rejected.  When the
 * complement has at most nsamp positions it is taken whole, in increasing
 * order, and pre[] is not used.  Returns the number written to q. */
int64_t orc_sample_prefix(uint64_t seed, int64_t problem, int64_t id, int64_t N, int64_t b, int64_t e,
                          int nsamp, const int64_t *pre, int64_t npre, int64_t *q) {
    int64_t n = e - b, c = N - n;
    if (c <= 0) return 0;
    if (c <= nsamp) { /* the whole complement, increasing order */
        int64_t k = 0;
        for (int64_t i = 0; i < b; i++) q[k++] = i;
        for (int64_t i = e; i < N; i++) q[k++] = i;
        return k;
    }
    int64_t k = 0;
    for (int64_t t = 0; t < npre && k < nsamp; t++) q[k++] = pre[t];
    uint64_t st = orc_node_seed(seed, problem, id);
    while (k < nsamp) {
        int64_t r = (int64_t)scale_draw(orc_splitmix64(&st), (uint64_t)c);
        int64_t pos = r < b ? r : r + n;
        int dup = 0;
        for (int64_t t = 0; t < k; t++)
            if (q[t] == pos) { dup = 1; break; }
        if (!dup) q[k++] = pos;
    }
    return k;
}

/* uniform rows only */
int64_t orc_sample(uint64_t seed, int64_t problem, int64_t id, int64_t N, int64_t b, int64_t e,
                   int nsamp, int64_t *q) {
    return orc_sample_prefix(seed, problem, id, N, b, e, nsamp, NULL, 0, q);
}

/* ------------------------------------------------------------------------ */
/* kappa-nearest-neighbour importance sampling: the kappa of Sec. 4 (the    */
/* number of nearest neighbours the skeletonization sampling uses, Table    */
/* "speedup"), after the ASKIT library the paper builds on (Sec. 2.1 cites  */
/* it for the sampling).  Reading: a row is important for a node when it is */
/* among the kappa nearest neighbours of the node's points.                 */
/*  * neighbours: the kappa points nearest to each point (itself excluded), */
/*    ordered by (squared distance, position), the distance summed by       */
/*    direct differences in increasing dimension (nn_dist); -1 pads lists   */
/*    of N - 1 < kappa points;                                              */
/*  * a leaf's list: every neighbour of its points that lies outside it,    */
/*    weighted by the number of its points that have it as a neighbour; an  */
/*    internal node's list: its children's lists merged (weights of equal   */
/*    positions added) with the positions inside the node dropped;          */
/*    ranked by weight, largest first, lowest position on ties, and cut to  */
/*    the sample size;                                                      */
/*  * the sample S' of a node: its list first, in rank order, then uniform  */
/*    draws (orc_sample_prefix) up to the sample size.                      */
/* ------------------------------------------------------------------------ */

/* squared distance of the neighbour search: fma(t, t, r2) over
 * t = x_k - y_k in increasing dimension (one rounding per term) */
static double nn_dist(const double *x, const double *y, int d) {
    double r2 = 0.0;
    for (int k = 0; k < d; k++) {
        double t = x[k] - y[k];
        r2 = fma(t, t, r2);
    }
    return r2;
}

/* (d2, pos) before (d2', pos') */
static int nn_before(double da, int64_t pa, double db, int64_t pb) { return da < db || (da == db && pa < pb); }

/* the kappa nearest positions of position i, by brute force over all N */
static void knn_row(const orc_t *o, int64_t i, int kappa, int64_t *idx, double *dist) {
    int cnt = 0;
    const double *x = pt(o, i);
    for (int64_t j = 0; j < o->N; j++) {
        if (j == i) continue;
        double r2 = nn_dist(x, pt(o, j), o->d);
        if (cnt == kappa && !nn_before(r2, j, dist[kappa - 1], idx[kappa - 1])) continue;
        int p = cnt < kappa ? cnt++ : kappa - 1;
        while (p > 0 && nn_before(r2, j, dist[p - 1], idx[p - 1])) {
            dist[p] = dist[p - 1];
            idx[p] = idx[p - 1];
            p--;
        }
        dist[p] = r2;
        idx[p] = j;
    }
    for (int t = cnt; t < kappa; t++) idx[t] = -1;
}

typedef struct { int64_t pos, w; } nbr_t;
static int by_pos(const void *a, const void *b) {
    int64_t x = ((const nbr_t *)a)->pos, y = ((const nbr_t *)b)->pos;
    return x < y ? -1 : x > y;
}
static int by_rank(const void *a, const void *b) {
    const nbr_t *x = (const nbr_t *)a, *y = (const nbr_t *)b;
    if (x->w != y->w) return x->w > y->w ? -1 : 1;
    return x->pos < y->pos ? -1 : x->pos > y->pos;
}

/* entries E[0..n) (overwritten): drop positions in [b,e), add the weights of
 * equal positions, rank, keep the first cap; returns the length */
static int64_t rank_entries(nbr_t *E, int64_t n, int64_t b, int64_t e, int64_t cap, int64_t **pos, int64_t **w) {
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++)
        if (E[i].pos < b || E[i].pos >= e) E[k++] = E[i];
    qsort(E, (size_t)k, sizeof(nbr_t), by_pos);
    int64_t u = 0;
    for (int64_t i = 0; i < k;) {
        int64_t j = i, acc = 0;
        while (j < k && E[j].pos == E[i].pos) acc += E[j++].w;
        E[u].pos = E[i].pos;
        E[u].w = acc;
        u++;
        i = j;
    }
    qsort(E, (size_t)u, sizeof(nbr_t), by_rank);
    int64_t len = u < cap ? u : cap;
    *pos = (int64_t *)malloc(sizeof(int64_t) * (len > 0 ? len : 1));
    *w = (int64_t *)malloc(sizeof(int64_t) * (len > 0 ? len : 1));
    for (int64_t t = 0; t < len; t++) { (*pos)[t] = E[t].pos; (*w)[t] = E[t].w; }
    return len;
}

/* lists of every node of the subtree of `top`, bottom-up; rows[i - nb[top]]
 * holds the kappa neighbours of position i of that subtree */
static void subtree_lists(orc_t *o, int64_t top, const int64_t *rows, int kappa, int64_t **pos, int64_t **w,
                          int64_t *len) {
    int ltop = level_of(top);
    int64_t base = o->nb[top];
    for (int l = o->D; l >= ltop; l--) {
        int64_t span = (int64_t)1 << (l - ltop), f = first_at(l) + (top - first_at(ltop)) * span;
#pragma omp parallel for schedule(dynamic)
        for (int64_t j = 0; j < span; j++) {
            int64_t id = f + j, b = o->nb[id], e = o->ne[id];
            nbr_t *E;
            int64_t n = 0;
            if (l == o->D) {
                E = (nbr_t *)malloc(sizeof(nbr_t) * ((e - b) * kappa + 1));
                for (int64_t i = b; i < e; i++)
                    for (int t = 0; t < kappa; t++) {
                        int64_t q = rows[(i - base) * kappa + t];
                        if (q >= 0) { E[n].pos = q; E[n].w = 1; n++; }
                    }
            } else {
                int64_t cl = 2 * id + 1, cr = 2 * id + 2;
                E = (nbr_t *)malloc(sizeof(nbr_t) * (len[cl] + len[cr] + 1));
                for (int64_t t = 0; t < len[cl]; t++) { E[n].pos = pos[cl][t]; E[n].w = w[cl][t]; n++; }
                for (int64_t t = 0; t < len[cr]; t++) { E[n].pos = pos[cr][t]; E[n].w = w[cr][t]; n++; }
            }
            free(pos[id]); free(w[id]);
            len[id] = rank_entries(E, n, b, e, o->nsamp, &pos[id], &w[id]);
            free(E);
        }
    }
}

/* Neighbours of every point and the ranked list of every node (kappa >= 1);
 * kappa = 0 returns to uniform sampling.  Takes effect at the next
 * skeletonization. */
int orc_set_knn(orc_t *o, int kappa) {
    if (kappa < 0) return ORC_ERR_ARG;
    if (kappa > 0 && !o->tree_built) return ORC_ERR_STATE;
    if (o->nbr)
        for (int64_t i = 0; i < o->nnodes; i++) { free(o->nbr[i]); free(o->nbrw[i]); }
    free(o->knn); free(o->nbr); free(o->nbrw); free(o->nnbr);
    o->knn = NULL; o->nbr = NULL; o->nbrw = NULL; o->nnbr = NULL;
    o->kappa = kappa;
    if (kappa == 0) return ORC_OK;
    o->knn = (int64_t *)malloc(sizeof(int64_t) * o->N * kappa);
    o->nbr = (int64_t **)calloc(o->nnodes, sizeof(int64_t *));
    o->nbrw = (int64_t **)calloc(o->nnodes, sizeof(int64_t *));
    o->nnbr = (int64_t *)calloc(o->nnodes, sizeof(int64_t));
    if (!o->knn || !o->nbr || !o->nbrw || !o->nnbr) return ORC_ERR_ALLOC;
#pragma omp parallel
    {
        double *dist = (double *)malloc(sizeof(double) * kappa);
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < o->N; i++) knn_row(o, i, kappa, o->knn + i * kappa, dist);
        free(dist);
    }
    subtree_lists(o, 0, o->knn, kappa, o->nbr, o->nbrw, o->nnbr);
    return ORC_OK;
}

void orc_get_knn(const orc_t *o, int64_t *out) { memcpy(out, o->knn, sizeof(int64_t) * o->N * o->kappa); }

/* a node's list: returns its length, copies positions and weights */
int64_t orc_node_nbr(const orc_t *o, int64_t id, int64_t *pos, int64_t *w) {
    if (!o->nbr) return 0;
    memcpy(pos, o->nbr[id], sizeof(int64_t) * o->nnbr[id]);
    memcpy(w, o->nbrw[id], sizeof(int64_t) * o->nnbr[id]);
    return o->nnbr[id];
}

/* The neighbours of the positions [b, e) alone (brute force against all N),
 * for checks on problems too large for orc_set_knn. */
void orc_knn_rows(const orc_t *o, int64_t b, int64_t e, int kappa, int64_t *out) {
#pragma omp parallel
    {
        double *dist = (double *)malloc(sizeof(double) * kappa);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = b; i < e; i++) knn_row(o, i, kappa, out + (i - b) * kappa, dist);
        free(dist);
    }
}

/* The list and sample of node `id` computed from its subtree only (the
 * neighbours of its points by brute force, the lists of its descendants):
 * what orc_set_knn and the sampler give that node, at a cost of
 * n_id x N distances.  Returns the sample size; *nl = list length. */
int64_t orc_subtree_sample(orc_t *o, int64_t id, int kappa, int64_t *lpos, int64_t *lw, int64_t *nl, int64_t *q) {
    int64_t b = o->nb[id], e = o->ne[id];
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (e - b) * kappa);
    int64_t **pos = (int64_t **)calloc(o->nnodes, sizeof(int64_t *));
    int64_t **w = (int64_t **)calloc(o->nnodes, sizeof(int64_t *));
    int64_t *len = (int64_t *)calloc(o->nnodes, sizeof(int64_t));
    orc_knn_rows(o, b, e, kappa, rows);
    subtree_lists(o, id, rows, kappa, pos, w, len);
    *nl = len[id];
    memcpy(lpos, pos[id], sizeof(int64_t) * len[id]);
    memcpy(lw, w[id], sizeof(int64_t) * len[id]);
    int64_t ns = orc_sample_prefix(o->seed, o->problem, id, o->N, b, e, o->nsamp, pos[id], len[id], q);
    for (int64_t i = 0; i < o->nnodes; i++) { free(pos[i]); free(w[i]); }
    free(pos); free(w); free(len); free(rows);
    return ns;
}

/* The sample S' the skeletonization uses for node id (uniform, or with the
 * node's neighbour list first). */
int64_t orc_node_sample(const orc_t *o, int64_t id, int64_t *q) {
    const int64_t *pre = o->kappa > 0 ? o->nbr[id] : NULL;
    int64_t npre = o->kappa > 0 ? o->nnbr[id] : 0;
    return orc_sample_prefix(o->seed, o->problem, id, o->N, o->nb[id], o->ne[id], o->nsamp, pre, npre, q);
}

/* ------------------------------------------------------------------------ */
/* Interpolative decomposition by column-pivoted Householder QR             */
/* (Sec. 2.1, eq. (4)).  M is rows x cols, column-major, overwritten.       */
/* Reading: Businger-Golub pivoting with the trailing column norms          */
/* recomputed at every step, largest norm first, lowest column on ties;     */
/* LAPACK-style reflectors; stop after `steps` steps, or earlier at the     */
/* first step j > 0 with |R_jj| <= 1e-14 |R_00| (rank guard) or             */
/* |R_jj| < rtol |R_00| (the adaptive rank rule of Sec. 2.1 with tau =     */
/* rtol, the singular values estimated by R's diagonal; 0 disables it).     */
/* Returns the rank used.                                                   */
/* piv[j] = original column in position j; T = R11^{-1} R12 (rank x         */
/* (cols-rank), row-major) is written when T != NULL.                       */
/* ------------------------------------------------------------------------ */

#define RANK_GUARD 1e-14

int orc_qrcp_tol(double *M, int rows, int cols, int steps, double rtol, int *piv, double *Rdiag, double *T,
                 int *truncated) {
    double *nrm = (double *)malloc(sizeof(double) * cols);
    if (steps > cols) steps = cols;
    if (steps > rows) steps = rows;
    for (int k = 0; k < cols; k++) piv[k] = k;
    int rank = steps;
    double r00 = 0.0;
    if (truncated) *truncated = 0;
    for (int j = 0; j < steps; j++) {
        /* squared norms of the trailing columns, rows j..rows-1 in order */
        for (int k = j; k < cols; k++) {
            double acc = 0.0;
            for (int i = j; i < rows; i++) acc = acc + M[(int64_t)k * rows + i] * M[(int64_t)k * rows + i];
            nrm[k] = acc;
        }
        int p = j;
        for (int k = j + 1; k < cols; k++)
            if (nrm[k] > nrm[p]) p = k;
        if (p != j) {
            for (int i = 0; i < rows; i++) {
                double t = M[(int64_t)j * rows + i];
                M[(int64_t)j * rows + i] = M[(int64_t)p * rows + i];
                M[(int64_t)p * rows + i] = t;
            }
            int t = piv[j]; piv[j] = piv[p]; piv[p] = t;
        }
        /* reflector H = I - tau v v^T with v_j = 1 */
        double *col = M + (int64_t)j * rows;
        double alpha = col[j], xn = 0.0, beta, tau;
        for (int i = j + 1; i < rows; i++) xn = xn + col[i] * col[i];
        if (xn == 0.0) {
            beta = alpha; tau = 0.0;
        } else {
            beta = -copysign(sqrt(alpha * alpha + xn), alpha);
            tau = (beta - alpha) / beta;
            double sc = 1.0 / (alpha - beta);
            for (int i = j + 1; i < rows; i++) col[i] = col[i] * sc;
        }
        col[j] = beta;
        if (Rdiag) Rdiag[j] = beta;
        if (j == 0) r00 = fabs(beta);
        if (j > 0 && (fabs(beta) <= RANK_GUARD * r00 || fabs(beta) < rtol * r00)) {
            rank = j;
            if (truncated) *truncated = 1;
            break;
        }
        if (j == 0 && r00 == 0.0) { /* M == 0: one column, zero coefficients */
            rank = 1;
            if (truncated && steps > 1) *truncated = 1;
            break;
        }
        /* apply H to the columns right of j */
        for (int k = j + 1; k < cols; k++) {
            double *ck = M + (int64_t)k * rows;
            double w = ck[j];
            for (int i = j + 1; i < rows; i++) w = w + col[i] * ck[i];
            w = tau * w;
            ck[j] = ck[j] - w;
            for (int i = j + 1; i < rows; i++) ck[i] = ck[i] - col[i] * w;
        }
    }
    if (T) {
        int nr = cols - rank;
        if (r00 == 0.0) {
            for (int64_t t = 0; t < (int64_t)rank * nr; t++) T[t] = 0.0;
        } else {
            /* back substitution R11 T = R12 */
            for (int c = 0; c < nr; c++)
                for (int i = rank - 1; i >= 0; i--) {
                    double acc = M[(int64_t)(rank + c) * rows + i];
                    for (int k = i + 1; k < rank; k++)
                        acc = acc - M[(int64_t)k * rows + i] * T[(int64_t)k * nr + c];
                    T[(int64_t)i * nr + c] = acc / M[(int64_t)i * rows + i];
                }
        }
    }
    free(nrm);
    return rank;
}

/* fixed rank: the QR above with tau = 0 (only the rank guard) */
int orc_qrcp(double *M, int rows, int cols, int steps, int *piv, double *Rdiag, double *T, int *truncated) {
    return orc_qrcp_tol(M, rows, cols, steps, 0.0, piv, Rdiag, T, truncated);
}

/* ------------------------------------------------------------------------ */
/* Skeletonize (Alg. 1): bottom-up over the non-root nodes.  Leaf: ID of    */
/* K_{S' alpha}; internal: ID of K_{S' [l~ r~]}.  Reading: s_alpha =        */
/* min(s, |C|); if s >= |C| the skeleton is C itself and P = I.             */
/* ------------------------------------------------------------------------ */

static int skeletonize_node(orc_t *o, int64_t id) {
    int64_t b = o->nb[id], e = o->ne[id];
    int ncand;
    int64_t *cand;
    if (is_leaf(o, id)) {
        ncand = (int)(e - b);
        cand = (int64_t *)malloc(sizeof(int64_t) * ncand);
        for (int i = 0; i < ncand; i++) cand[i] = b + i;
    } else {
        int64_t l = 2 * id + 1, r = 2 * id + 2;
        ncand = o->sr[l] + o->sr[r];
        cand = (int64_t *)malloc(sizeof(int64_t) * ncand);
        for (int i = 0; i < o->sr[l]; i++) cand[i] = o->skel[l][i];
        for (int i = 0; i < o->sr[r]; i++) cand[o->sr[l] + i] = o->skel[r][i];
    }
    int srank = o->s < ncand ? o->s : ncand;
    free(o->skel[id]); free(o->P[id]);
    o->nc[id] = ncand;
    o->trunc[id] = 0;
    if (srank == ncand) { /* no compression possible: identity projection */
        o->sr[id] = ncand;
        o->skel[id] = cand;
        o->P[id] = (double *)calloc((size_t)ncand * ncand, sizeof(double));
        for (int i = 0; i < ncand; i++) o->P[id][(int64_t)i * ncand + i] = 1.0;
        return ORC_OK;
    }
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * o->nsamp);
    int64_t ns = orc_node_sample(o, id, q);
    double *M = (double *)malloc(sizeof(double) * ns * ncand);
    for (int c = 0; c < ncand; c++)
        for (int64_t i = 0; i < ns; i++) M[(int64_t)c * ns + i] = kpos(o, q[i], cand[c], 0);
    int *pv = (int *)malloc(sizeof(int) * ncand);
    double *T = (double *)malloc(sizeof(double) * (size_t)srank * ncand);
    int tr = 0;
    int rank = orc_qrcp_tol(M, (int)ns, ncand, srank, o->tol, pv, NULL, T, &tr);
    if (rank < srank) tr = 1;
    o->sr[id] = rank;
    o->trunc[id] = tr;
    o->skel[id] = (int64_t *)malloc(sizeof(int64_t) * rank);
    o->P[id] = (double *)calloc((size_t)rank * ncand, sizeof(double));
    for (int j = 0; j < rank; j++) o->skel[id][j] = cand[pv[j]];
    /* P[:, piv_j] = e_j (j < rank); P[:, piv_j] = T[:, j - rank] otherwise */
    int nr = ncand - rank;
    for (int j = 0; j < ncand; j++)
        for (int i = 0; i < rank; i++)
            o->P[id][(int64_t)i * ncand + pv[j]] = (j < rank) ? (i == j ? 1.0 : 0.0) : T[(int64_t)i * nr + (j - rank)];
    free(q); free(M); free(pv); free(T); free(cand);
    return ORC_OK;
}

int orc_skeletonize(orc_t *o) {
    if (!o->tree_built) return ORC_ERR_STATE;
    for (int l = o->D; l >= 1; l--) {
        int64_t f = first_at(l), cnt = (int64_t)1 << l;
#pragma omp parallel for schedule(dynamic)
        for (int64_t j = 0; j < cnt; j++) skeletonize_node(o, f + j);
    }
    o->skel_built = 1;
    free_factor(o);
    return ORC_OK;
}

/* skeleton access: ids are tree positions; P is s_alpha x |C| row-major */
void orc_skel_info(const orc_t *o, int64_t id, int *sr, int *nc, int *trunc) {
    *sr = o->sr[id]; *nc = o->nc[id]; *trunc = o->trunc[id];
}
void orc_skel_get(const orc_t *o, int64_t id, int64_t *skel_pos, double *P) {
    memcpy(skel_pos, o->skel[id], sizeof(int64_t) * o->sr[id]);
    memcpy(P, o->P[id], sizeof(double) * (size_t)o->sr[id] * o->nc[id]);
}
/* Replace one node's skeleton (used by tests that plant a mistake in the
 * oracle, and to build the identity case); the candidates stay as defined. */
int orc_skel_set(orc_t *o, int64_t id, int sr, const int64_t *skel_pos, const double *P) {
    if (id <= 0 || id >= o->nnodes) return ORC_ERR_ARG;
    /* the candidate set follows the children's current skeletons, which an
     * earlier import may have changed (imports go bottom-up) */
    o->nc[id] = is_leaf(o, id) ? (int)(o->ne[id] - o->nb[id]) : o->sr[2 * id + 1] + o->sr[2 * id + 2];
    if (sr < 1 || sr > o->nc[id]) return ORC_ERR_ARG;
    free(o->skel[id]); free(o->P[id]);
    o->sr[id] = sr;
    o->skel[id] = (int64_t *)malloc(sizeof(int64_t) * sr);
    o->P[id] = (double *)malloc(sizeof(double) * (size_t)sr * o->nc[id]);
    memcpy(o->skel[id], skel_pos, sizeof(int64_t) * sr);
    memcpy(o->P[id], P, sizeof(double) * (size_t)sr * o->nc[id]);
    free_factor(o);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Dense helpers (textbook loops)                                           */
/* ------------------------------------------------------------------------ */

/* C (m x n) = A (m x k) B (k x n), all row-major */
static void mm(const double *A, const double *B, double *C, int64_t m, int64_t k, int64_t n, int par) {
#pragma omp parallel for if (par) schedule(static)
    for (int64_t i = 0; i < m; i++) {
        for (int64_t j = 0; j < n; j++) C[i * n + j] = 0.0;
        for (int64_t t = 0; t < k; t++) {
            double a = A[i * k + t];
            for (int64_t j = 0; j < n; j++) C[i * n + j] = C[i * n + j] + a * B[t * n + j];
        }
    }
}

/* LU with partial pivoting (the GETRF of Sec. 2.2): row of largest |a| in
 * the column, lowest row on ties.  A = P L U, unit lower L.  piv[k] is the
 * row exchanged with row k.  Returns the ratio min|U_ii| / max|U_ii|. */
double orc_lu(double *A, int n, int *piv) {
    double umin = INFINITY, umax = 0.0;
    for (int k = 0; k < n; k++) {
        int p = k;
        for (int i = k + 1; i < n; i++)
            if (fabs(A[(int64_t)i * n + k]) > fabs(A[(int64_t)p * n + k])) p = i;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; j++) {
                double t = A[(int64_t)k * n + j];
                A[(int64_t)k * n + j] = A[(int64_t)p * n + j];
                A[(int64_t)p * n + j] = t;
            }
        double ukk = A[(int64_t)k * n + k];
        double au = fabs(ukk);
        if (au < umin) umin = au;
        if (au > umax) umax = au;
        if (ukk == 0.0) continue;
        for (int i = k + 1; i < n; i++) {
            double lik = A[(int64_t)i * n + k] / ukk;
            A[(int64_t)i * n + k] = lik;
            for (int j = k + 1; j < n; j++) A[(int64_t)i * n + j] = A[(int64_t)i * n + j] - lik * A[(int64_t)k * n + j];
        }
    }
    return n ? (umax > 0.0 ? umin / umax : 0.0) : 1.0;
}

/* solve A X = B in place; B is n x nrhs row-major */
void orc_lu_solve(const double *LU, const int *piv, int n, double *B, int nrhs) {
    for (int k = 0; k < n; k++)
        if (piv[k] != k)
            for (int c = 0; c < nrhs; c++) {
                double t = B[(int64_t)k * nrhs + c];
                B[(int64_t)k * nrhs + c] = B[(int64_t)piv[k] * nrhs + c];
                B[(int64_t)piv[k] * nrhs + c] = t;
            }
    for (int i = 0; i < n; i++) /* L y = b, unit diagonal */
        for (int k = 0; k < i; k++) {
            double l = LU[(int64_t)i * n + k];
            for (int c = 0; c < nrhs; c++) B[(int64_t)i * nrhs + c] = B[(int64_t)i * nrhs + c] - l * B[(int64_t)k * nrhs + c];
        }
    for (int i = n - 1; i >= 0; i--) { /* U x = y */
        for (int k = i + 1; k < n; k++) {
            double u = LU[(int64_t)i * n + k];
            for (int c = 0; c < nrhs; c++) B[(int64_t)i * nrhs + c] = B[(int64_t)i * nrhs + c] - u * B[(int64_t)k * nrhs + c];
        }
        double uii = LU[(int64_t)i * n + i];
        for (int c = 0; c < nrhs; c++) B[(int64_t)i * nrhs + c] = B[(int64_t)i * nrhs + c] / uii;
    }
}

/* solve A^T X = B in place: U^T z = b, L^T w = z, then undo the row swaps */
void orc_lu_solve_t(const double *LU, const int *piv, int n, double *B, int nrhs) {
    for (int i = 0; i < n; i++) {
        for (int k = 0; k < i; k++) {
            double u = LU[(int64_t)k * n + i];
            for (int c = 0; c < nrhs; c++) B[(int64_t)i * nrhs + c] = B[(int64_t)i * nrhs + c] - u * B[(int64_t)k * nrhs + c];
        }
        double uii = LU[(int64_t)i * n + i];
        for (int c = 0; c < nrhs; c++) B[(int64_t)i * nrhs + c] = B[(int64_t)i * nrhs + c] / uii;
    }
    for (int i = n - 1; i >= 0; i--)
        for (int k = i + 1; k < n; k++) {
            double l = LU[(int64_t)k * n + i];
            for (int c = 0; c < nrhs; c++) B[(int64_t)i * nrhs + c] = B[(int64_t)i * nrhs + c] - l * B[(int64_t)k * nrhs + c];
        }
    for (int k = n - 1; k >= 0; k--)
        if (piv[k] != k)
            for (int c = 0; c < nrhs; c++) {
                double t = B[(int64_t)k * nrhs + c];
                B[(int64_t)k * nrhs + c] = B[(int64_t)piv[k] * nrhs + c];
                B[(int64_t)piv[k] * nrhs + c] = t;
            }
}

/* ------------------------------------------------------------------------ */
/* Kernel blocks between skeletons and node points                          */
/* ------------------------------------------------------------------------ */

/* out (s_src x n) = K(X_{skel}, X_{[b,e)}) */
static double *kblock_skel(const orc_t *o, int64_t skel_node, int64_t b, int64_t e, int which, int par) {
    int sr = o->sr[skel_node];
    int64_t n = e - b;
    double *K = (double *)malloc(sizeof(double) * sr * n);
#pragma omp parallel for if (par) schedule(static)
    for (int a = 0; a < sr; a++)
        for (int64_t j = 0; j < n; j++) K[a * n + j] = kpos(o, o->skel[skel_node][a], b + j, which);
    return K;
}

/* P_c = P_{[l~ r~] alpha~} = (P_{alpha~ [l~ r~]})^T, (s_l+s_r) x s_alpha */
static double *pc_of(const orc_t *o, int64_t id) {
    int sr = o->sr[id], nc = o->nc[id];
    double *Pc = (double *)malloc(sizeof(double) * sr * nc);
    for (int i = 0; i < nc; i++)
        for (int k = 0; k < sr; k++) Pc[(int64_t)i * sr + k] = o->P[id][(int64_t)k * nc + i];
    return Pc;
}

/* ------------------------------------------------------------------------ */
/* Factorize (Alg. 2) and Solve (Alg. 3)                                    */
/* ------------------------------------------------------------------------ */

/* Solve(alpha, u, do_recur) of Alg. 3 on the rows of node alpha.  u is
 * n_alpha x nrhs row-major, in tree-position order, overwritten by w.
 * With do_recur the children are solved first (v = D^{-1} u); in both
 * cases the node step is w = v - W Z^{-1} V v of eq. (8). */
static void solve_node(const orc_t *o, int64_t id, double *u, int nrhs, int do_recur, int par) {
    int64_t b = o->nb[id], n = o->ne[id] - b;
    if (is_leaf(o, id)) {
        orc_lu_solve(o->LU[id], o->piv[id], (int)n, u, nrhs);
        return;
    }
    int64_t l = 2 * id + 1, r = 2 * id + 2;
    int64_t nl = o->ne[l] - o->nb[l], nr = o->ne[r] - o->nb[r];
    int sl = o->sr[l], srr = o->sr[r], ns = sl + srr;
    double *ul = u, *ur = u + nl * nrhs;
    if (do_recur) {
        solve_node(o, l, ul, nrhs, 1, par);
        solve_node(o, r, ur, nrhs, 1, par);
    }
    /* t = V v = [K_{l~ r} v_r ; K_{r~ l} v_l] */
    double *K1 = kblock_skel(o, l, o->nb[r], o->ne[r], 0, par);
    double *K2 = kblock_skel(o, r, o->nb[l], o->ne[l], 0, par);
    double *t = (double *)malloc(sizeof(double) * ns * nrhs);
    mm(K1, ur, t, sl, nr, nrhs, par);
    mm(K2, ul, t + (int64_t)sl * nrhs, srr, nl, nrhs, par);
    /* y = Z^{-1} t */
    orc_lu_solve(o->LU[id], o->piv[id], ns, t, nrhs);
    /* w = v - W y, W = blockdiag(Phat_l, Phat_r) */
    double *wl = (double *)malloc(sizeof(double) * nl * nrhs);
    double *wr = (double *)malloc(sizeof(double) * nr * nrhs);
    mm(o->Phat[l], t, wl, nl, sl, nrhs, par);
    mm(o->Phat[r], t + (int64_t)sl * nrhs, wr, nr, srr, nrhs, par);
    for (int64_t i = 0; i < nl * nrhs; i++) ul[i] = ul[i] - wl[i];
    for (int64_t i = 0; i < nr * nrhs; i++) ur[i] = ur[i] - wr[i];
    free(K1); free(K2); free(t); free(wl); free(wr);
    (void)b;
}

/* telescoped projection P_{alpha alpha~} (n_alpha x s_alpha), eq. (9):
 * leaf: P_{alpha~ alpha}^T; internal: blockdiag(P_{l l~}, P_{r r~}) P_c */
static double *telescoped_P(const orc_t *o, int64_t id) {
    int64_t n = o->ne[id] - o->nb[id];
    int sr = o->sr[id];
    if (is_leaf(o, id)) {
        double *Pt = (double *)malloc(sizeof(double) * n * sr);
        for (int64_t i = 0; i < n; i++)
            for (int k = 0; k < sr; k++) Pt[i * sr + k] = o->P[id][(int64_t)k * n + i];
        return Pt;
    }
    int64_t l = 2 * id + 1, r = 2 * id + 2;
    int64_t nl = o->ne[l] - o->nb[l], nr = o->ne[r] - o->nb[r];
    double *Pl = telescoped_P(o, l), *Pr = telescoped_P(o, r), *Pc = pc_of(o, id);
    double *out = (double *)malloc(sizeof(double) * n * sr);
    mm(Pl, Pc, out, nl, o->sr[l], sr, 0);
    mm(Pr, Pc + (int64_t)o->sr[l] * sr, out + nl * sr, nr, o->sr[r], sr, 0);
    free(Pl); free(Pr); free(Pc);
    return out;
}

static int factor_leaf(orc_t *o, int64_t id) {
    int64_t b = o->nb[id], n = o->ne[id] - b;
    double *A = (double *)malloc(sizeof(double) * n * n);
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < n; j++) A[i * n + j] = kpos(o, b + i, b + j, 0) + (i == j ? o->lambda : 0.0);
    o->piv[id] = (int *)malloc(sizeof(int) * (n ? n : 1));
    o->pivratio[id] = orc_lu(A, (int)n, o->piv[id]);
    o->LU[id] = A;
    if (id > 0) { /* Phat = (lambda I + K_aa)^{-1} P_{alpha alpha~} */
        double *Ph = telescoped_P(o, id);
        orc_lu_solve(A, o->piv[id], (int)n, Ph, o->sr[id]);
        o->Phat[id] = Ph;
    }
    return ORC_OK;
}

/* variant 0: paper form, Phat = Solve(alpha, W P_c, false) of Alg. 2
 *            (= (I + W V)^{-1} W P_c, eq. (10));
 * variant 1: subtree traversal, Phat = Ktilde_aa^{-1} P_{alpha alpha~}
 *            by a full recursive Solve (the N log^2 N scheme of Sec. 2.2);
 * variant 2: push-through identity (I + W V)^{-1} W = W (I + V W)^{-1},
 *            Phat = W Z^{-1} P_c. */
static int factor_internal(orc_t *o, int64_t id, int variant, int par) {
    int64_t l = 2 * id + 1, r = 2 * id + 2;
    int64_t nl = o->ne[l] - o->nb[l], nr = o->ne[r] - o->nb[r], n = nl + nr;
    int sl = o->sr[l], srr = o->sr[r], ns = sl + srr;
    /* Z = [[I, K_{l~ r} Phat_r], [K_{r~ l} Phat_l, I]], eq. (8) */
    double *K1 = kblock_skel(o, l, o->nb[r], o->ne[r], 0, par);
    double *K2 = kblock_skel(o, r, o->nb[l], o->ne[l], 0, par);
    double *B1 = (double *)malloc(sizeof(double) * sl * srr);
    double *B2 = (double *)malloc(sizeof(double) * srr * sl);
    mm(K1, o->Phat[r], B1, sl, nr, srr, par);
    mm(K2, o->Phat[l], B2, srr, nl, sl, par);
    double *Z = (double *)calloc((size_t)ns * ns, sizeof(double));
    for (int i = 0; i < ns; i++) Z[(int64_t)i * ns + i] = 1.0;
    for (int i = 0; i < sl; i++)
        for (int j = 0; j < srr; j++) Z[(int64_t)i * ns + sl + j] = B1[(int64_t)i * srr + j];
    for (int i = 0; i < srr; i++)
        for (int j = 0; j < sl; j++) Z[(int64_t)(sl + i) * ns + j] = B2[(int64_t)i * sl + j];
    o->piv[id] = (int *)malloc(sizeof(int) * ns);
    o->pivratio[id] = orc_lu(Z, ns, o->piv[id]);
    o->LU[id] = Z;
    free(K1); free(K2); free(B1); free(B2);
    if (id == 0) return ORC_OK; /* the root has no skeleton and no Phat */
    int sa = o->sr[id];
    double *Ph = (double *)malloc(sizeof(double) * n * sa);
    if (variant == 1) {
        double *Pt = telescoped_P(o, id);
        memcpy(Ph, Pt, sizeof(double) * n * sa);
        free(Pt);
        solve_node(o, id, Ph, sa, 1, par);
    } else {
        double *Pc = pc_of(o, id);
        if (variant == 0) {
            /* u = W P_c, then the node step of Solve without recursion */
            mm(o->Phat[l], Pc, Ph, nl, sl, sa, par);
            mm(o->Phat[r], Pc + (int64_t)sl * sa, Ph + nl * sa, nr, srr, sa, par);
            solve_node(o, id, Ph, sa, 0, par);
        } else {
            orc_lu_solve(Z, o->piv[id], ns, Pc, sa);
            mm(o->Phat[l], Pc, Ph, nl, sl, sa, par);
            mm(o->Phat[r], Pc + (int64_t)sl * sa, Ph + nl * sa, nr, srr, sa, par);
        }
        free(Pc);
    }
    o->Phat[id] = Ph;
    return ORC_OK;
}

/* Reduced system of the hybrid solver (Sec. 2.3, "Fast hybrid solver").
 * With the frontier A at level L, D = blockdiag(lambda I + Ktilde_aa),
 * U = blockdiag(P_{a a~}) and V_{ab} = K_{a~ b} (a != b, zero on the
 * diagonal), so that lambda I + Ktilde = D + U V = D (I + W V), W = D^{-1} U
 * = blockdiag(Phat_a).  Z = I + V W has the blocks K_{a~ b} Phat_b (a != b)
 * and the identity on the diagonal; the oracle assembles and LU-factors it
 * (the method solves it iteratively). */
static int factor_reduced(orc_t *o) {
    int L = o->hybL;
    int64_t f = first_at(L), cnt = (int64_t)1 << L;
    o->hoff = (int64_t *)malloc(sizeof(int64_t) * (cnt + 1));
    o->hoff[0] = 0;
    for (int64_t j = 0; j < cnt; j++) o->hoff[j + 1] = o->hoff[j] + o->sr[f + j];
    int64_t M = o->hM = o->hoff[cnt];
    double *Z = (double *)calloc((size_t)M * M, sizeof(double));
    for (int64_t i = 0; i < M; i++) Z[i * M + i] = 1.0;
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int64_t a = 0; a < cnt; a++)
        for (int64_t b = 0; b < cnt; b++) {
            if (a == b) continue;
            int64_t ia = f + a, ib = f + b, nb = o->ne[ib] - o->nb[ib];
            int sa = o->sr[ia], sb = o->sr[ib];
            double *Kab = kblock_skel(o, ia, o->nb[ib], o->ne[ib], 0, 0);
            double *blk = (double *)malloc(sizeof(double) * sa * sb);
            mm(Kab, o->Phat[ib], blk, sa, nb, sb, 0);
            for (int i = 0; i < sa; i++)
                for (int k = 0; k < sb; k++) Z[(o->hoff[a] + i) * M + o->hoff[b] + k] = blk[(int64_t)i * sb + k];
            free(Kab); free(blk);
        }
    o->hpiv = (int *)malloc(sizeof(int) * (M ? M : 1));
    o->hratio = orc_lu(Z, (int)M, o->hpiv);
    o->hLU = Z;
    return ORC_OK;
}

int orc_factorize(orc_t *o, double lambda, int variant) {
    if (!o->skel_built) return ORC_ERR_STATE;
    if (!(lambda >= 0.0) || variant < 0 || variant > 2) return ORC_ERR_ARG;
    free_factor(o);
    o->lambda = lambda;
    /* with a level restriction only the frontier's subtrees are factored */
    int top = o->hybL > 0 ? o->hybL : 0;
    for (int l = o->D; l >= top; l--) {
        int64_t f = first_at(l), cnt = (int64_t)1 << l;
        int inner = cnt < 8; /* few nodes: parallelise inside the node */
#pragma omp parallel for schedule(dynamic) if (!inner)
        for (int64_t j = 0; j < cnt; j++) {
            if (l == o->D) factor_leaf(o, f + j);
            else factor_internal(o, f + j, variant, inner);
        }
    }
    if (o->hybL > 0) factor_reduced(o);
    o->factored = 1;
    return ORC_OK;
}

/* Level restriction (Sec. 2.3): L = 0 keeps the full method; 1 <= L <= D
 * puts the skeletonization frontier at level L.  Nodes above it are not
 * compressed: for frontier nodes a != b, Ktilde_ab = P_{a a~} K_{a~ b}.
 * L = 1 gives the full method's matrix (the root has no skeleton).  The
 * factorization is dropped. */
int orc_set_level(orc_t *o, int L) {
    if (L < 0 || L > o->D || (L > 0 && o->D < 1)) return ORC_ERR_ARG;
    free_factor(o);
    o->hybL = L;
    return ORC_OK;
}
double orc_reduced_ratio(const orc_t *o) { return o->hLU ? o->hratio : 1.0; }
int64_t orc_reduced_order(const orc_t *o) { return o->hLU ? o->hM : 0; }

void orc_get_phat(const orc_t *o, int64_t id, double *out) {
    memcpy(out, o->Phat[id], sizeof(double) * (o->ne[id] - o->nb[id]) * o->sr[id]);
}
/* Z LU of an internal node (or leaf LU), n x n row-major, and its pivots */
int orc_block_size(const orc_t *o, int64_t id) {
    return is_leaf(o, id) ? (int)(o->ne[id] - o->nb[id]) : o->sr[2 * id + 1] + o->sr[2 * id + 2];
}
void orc_get_lu(const orc_t *o, int64_t id, double *out, int *piv) {
    int n = orc_block_size(o, id);
    memcpy(out, o->LU[id], sizeof(double) * n * n);
    memcpy(piv, o->piv[id], sizeof(int) * n);
}
double orc_pivratio(const orc_t *o, int64_t id) { return o->pivratio[id]; }

/* column-major N x nrhs (original order) <-> row-major position order */
static double *to_pos(const orc_t *o, const double *B, int64_t ldb, int nrhs) {
    double *u = (double *)malloc(sizeof(double) * o->N * nrhs);
    for (int64_t i = 0; i < o->N; i++)
        for (int c = 0; c < nrhs; c++) u[i * nrhs + c] = B[(int64_t)c * ldb + o->perm[i]];
    return u;
}
static void from_pos(const orc_t *o, const double *u, double *Xo, int64_t ldx, int nrhs) {
    for (int64_t i = 0; i < o->N; i++)
        for (int c = 0; c < nrhs; c++) Xo[(int64_t)c * ldx + o->perm[i]] = u[i * nrhs + c];
}

/* x = (lambda I + Ktilde)^{-1} b: leaf LU solves, then one node step per
 * level from the leaves up (Alg. 3 with do_recur on the root, level by level).
 * With a level restriction (Alg. HybridSolve): v = D^{-1} u by the node
 * steps up to the frontier, t = V v (MatVecV: t_a = sum_{b != a} K_{a~ b}
 * v_b), y = Z^{-1} t, x = v - W y (MatVecW: x_b -= Phat_b y_b). */
int orc_solve(const orc_t *o, const double *B, int64_t ldb, int nrhs, double *Xo, int64_t ldx) {
    if (!o->factored) return ORC_ERR_STATE;
    double *u = to_pos(o, B, ldb, nrhs);
    int top = o->hybL > 0 ? o->hybL : 0;
    for (int l = o->D; l >= top; l--) {
        int64_t f = first_at(l), cnt = (int64_t)1 << l;
        int inner = cnt < 8;
#pragma omp parallel for schedule(dynamic) if (!inner)
        for (int64_t j = 0; j < cnt; j++) solve_node(o, f + j, u + o->nb[f + j] * nrhs, nrhs, 0, inner);
    }
    if (o->hybL > 0) {
        int64_t f = first_at(o->hybL), cnt = (int64_t)1 << o->hybL, M = o->hM;
        double *t = (double *)calloc((size_t)M * nrhs, sizeof(double));
#pragma omp parallel for schedule(dynamic)
        for (int64_t a = 0; a < cnt; a++)
            for (int64_t b = 0; b < cnt; b++) {
                if (a == b) continue;
                int64_t ia = f + a, ib = f + b, nb = o->ne[ib] - o->nb[ib];
                double *Kab = kblock_skel(o, ia, o->nb[ib], o->ne[ib], 0, 0);
                double *tb = (double *)malloc(sizeof(double) * o->sr[ia] * nrhs);
                mm(Kab, u + o->nb[ib] * nrhs, tb, o->sr[ia], nb, nrhs, 0);
                for (int64_t i = 0; i < (int64_t)o->sr[ia] * nrhs; i++) t[o->hoff[a] * nrhs + i] += tb[i];
                free(Kab); free(tb);
            }
        orc_lu_solve(o->hLU, o->hpiv, (int)M, t, nrhs);
#pragma omp parallel for schedule(dynamic)
        for (int64_t b = 0; b < cnt; b++) {
            int64_t ib = f + b, nb = o->ne[ib] - o->nb[ib];
            double *w = (double *)malloc(sizeof(double) * nb * nrhs);
            mm(o->Phat[ib], t + o->hoff[b] * nrhs, w, nb, o->sr[ib], nrhs, 0);
            double *ub = u + o->nb[ib] * nrhs;
            for (int64_t i = 0; i < nb * nrhs; i++) ub[i] = ub[i] - w[i];
            free(w);
        }
        free(t);
    }
    from_pos(o, u, Xo, ldx, nrhs);
    free(u);
    return ORC_OK;
}

/* x = (lambda I + Ktilde)^{-T} g.  With Ktilde_aa = D (I + W V) (eq. (7))
 * and (I + W V)^{-1} = I - W Z^{-1} V (eq. (3)):
 *   Ktilde_aa^{-T} = D^{-T} (I - V^T Z^{-T} W^T),
 * applied from the root down, then the transposed leaf solves. */
int orc_solve_t(const orc_t *o, const double *B, int64_t ldb, int nrhs, double *Xo, int64_t ldx) {
    if (!o->factored || o->hybL > 0) return ORC_ERR_STATE;
    double *g = to_pos(o, B, ldb, nrhs);
    for (int lv = 0; lv <= o->D; lv++) {
        int64_t f = first_at(lv), cnt = (int64_t)1 << lv;
        int inner = cnt < 8;
#pragma omp parallel for schedule(dynamic) if (!inner)
        for (int64_t j = 0; j < cnt; j++) {
            int64_t id = f + j;
            double *gn = g + o->nb[id] * nrhs;
            if (lv == o->D) {
                orc_lu_solve_t(o->LU[id], o->piv[id], (int)(o->ne[id] - o->nb[id]), gn, nrhs);
                continue;
            }
            int64_t l = 2 * id + 1, r = 2 * id + 2;
            int64_t nl = o->ne[l] - o->nb[l], nr = o->ne[r] - o->nb[r];
            int sl = o->sr[l], srr = o->sr[r], ns = sl + srr;
            double *gl = gn, *gr = gn + nl * nrhs;
            /* gt = W^T g = [Phat_l^T g_l ; Phat_r^T g_r] */
            double *gt = (double *)calloc((size_t)ns * nrhs, sizeof(double));
            for (int64_t i = 0; i < nl; i++)
                for (int k = 0; k < sl; k++)
                    for (int c = 0; c < nrhs; c++) gt[(int64_t)k * nrhs + c] += o->Phat[l][i * sl + k] * gl[i * nrhs + c];
            for (int64_t i = 0; i < nr; i++)
                for (int k = 0; k < srr; k++)
                    for (int c = 0; c < nrhs; c++)
                        gt[(int64_t)(sl + k) * nrhs + c] += o->Phat[r][i * srr + k] * gr[i * nrhs + c];
            orc_lu_solve_t(o->LU[id], o->piv[id], ns, gt, nrhs); /* y = Z^{-T} gt */
            /* g -= V^T y: g_l -= K_{r~ l}^T y_bot, g_r -= K_{l~ r}^T y_top */
            double *K1 = kblock_skel(o, l, o->nb[r], o->ne[r], 0, inner);
            double *K2 = kblock_skel(o, r, o->nb[l], o->ne[l], 0, inner);
            for (int64_t i = 0; i < nl; i++)
                for (int k = 0; k < srr; k++)
                    for (int c = 0; c < nrhs; c++) gl[i * nrhs + c] -= K2[(int64_t)k * nl + i] * gt[(int64_t)(sl + k) * nrhs + c];
            for (int64_t i = 0; i < nr; i++)
                for (int k = 0; k < sl; k++)
                    for (int c = 0; c < nrhs; c++) gr[i * nrhs + c] -= K1[(int64_t)k * nr + i] * gt[(int64_t)k * nrhs + c];
            free(gt); free(K1); free(K2);
        }
    }
    from_pos(o, g, Xo, ldx, nrhs);
    free(g);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Hierarchical matvec with the approximate matrix (Sec. 2.1, last          */
/* paragraph before Alg. 1, in the left-projection form of eq. (6)):        */
/*   leaves: (lambda I + K_aa) x_a;                                         */
/*   every internal alpha: c_l += K_{l~ r} x_r, c_r += K_{r~ l} x_l;        */
/*   push c down: [c_l~; c_r~] += P_c c_beta (telescoping, eq. (9));        */
/*   leaves: y_a += P_{alpha~ alpha}^T c_a.                                  */
/* which = 0: lambda I + Ktilde; which = 1: dKtilde/dh with the skeletons   */
/* and projections held fixed (no lambda).  With a level restriction at L   */
/* (Sec. 2.3) the nodes above the frontier add no potentials; instead each  */
/* frontier node a gets c_a = sum_{b != a} K_{a~ b} x_b, pushed down from L. */
/* ------------------------------------------------------------------------ */

int orc_matvec(const orc_t *o, int which, const double *Xin, int64_t ldx, int nrhs, double *Y, int64_t ldy) {
    if (!o->skel_built) return ORC_ERR_STATE;
    double *x = to_pos(o, Xin, ldx, nrhs);
    double *y = (double *)calloc((size_t)o->N * nrhs, sizeof(double));
    double **c = (double **)calloc(o->nnodes, sizeof(double *));
    for (int64_t id = 1; id < o->nnodes; id++) c[id] = (double *)calloc((size_t)o->sr[id] * nrhs, sizeof(double));
    /* leaves */
    int64_t fl = first_at(o->D), nleaf = (int64_t)1 << o->D;
#pragma omp parallel for schedule(dynamic)
    for (int64_t j = 0; j < nleaf; j++) {
        int64_t id = fl + j, b = o->nb[id], e = o->ne[id];
        for (int64_t i = b; i < e; i++)
            for (int64_t k = b; k < e; k++) {
                double a = kpos(o, i, k, which) + ((i == k && !which) ? o->lambda : 0.0);
                for (int q = 0; q < nrhs; q++) y[i * nrhs + q] += a * x[k * nrhs + q];
            }
    }
    /* skeleton potentials (with a level restriction: below the frontier,
     * plus every frontier node's potential from all other frontier nodes) */
    int top = o->hybL > 0 ? o->hybL : 0;
    if (top > 0) {
        int64_t f = first_at(top), cnt = (int64_t)1 << top;
#pragma omp parallel for schedule(dynamic)
        for (int64_t a = 0; a < cnt; a++)
            for (int k = 0; k < o->sr[f + a]; k++)
                for (int64_t i = 0; i < o->N; i++) {
                    if (i >= o->nb[f + a] && i < o->ne[f + a]) continue;
                    double kv = kpos(o, o->skel[f + a][k], i, which);
                    for (int q = 0; q < nrhs; q++) c[f + a][(int64_t)k * nrhs + q] += kv * x[i * nrhs + q];
                }
    }
    for (int lv = top; lv < o->D; lv++) {
        int64_t f = first_at(lv), cnt = (int64_t)1 << lv;
#pragma omp parallel for schedule(dynamic)
        for (int64_t j = 0; j < cnt; j++) {
            int64_t id = f + j, l = 2 * id + 1, r = 2 * id + 2;
            for (int a = 0; a < o->sr[l]; a++)
                for (int64_t k = o->nb[r]; k < o->ne[r]; k++) {
                    double kv = kpos(o, o->skel[l][a], k, which);
                    for (int q = 0; q < nrhs; q++) c[l][(int64_t)a * nrhs + q] += kv * x[k * nrhs + q];
                }
            for (int a = 0; a < o->sr[r]; a++)
                for (int64_t k = o->nb[l]; k < o->ne[l]; k++) {
                    double kv = kpos(o, o->skel[r][a], k, which);
                    for (int q = 0; q < nrhs; q++) c[r][(int64_t)a * nrhs + q] += kv * x[k * nrhs + q];
                }
        }
    }
    /* push down through the internal projections */
    for (int lv = top > 1 ? top : 1; lv < o->D; lv++) {
        int64_t f = first_at(lv), cnt = (int64_t)1 << lv;
#pragma omp parallel for schedule(dynamic)
        for (int64_t j = 0; j < cnt; j++) {
            int64_t id = f + j, l = 2 * id + 1, r = 2 * id + 2;
            int nc = o->nc[id], sa = o->sr[id], sl = o->sr[l];
            for (int i = 0; i < nc; i++) {
                double *dst = (i < sl) ? c[l] + (int64_t)i * nrhs : c[r] + (int64_t)(i - sl) * nrhs;
                for (int k = 0; k < sa; k++) {
                    double p = o->P[id][(int64_t)k * nc + i];
                    for (int q = 0; q < nrhs; q++) dst[q] += p * c[id][(int64_t)k * nrhs + q];
                }
            }
        }
    }
    if (o->D > 0) {
#pragma omp parallel for schedule(dynamic)
        for (int64_t j = 0; j < nleaf; j++) {
            int64_t id = fl + j, b = o->nb[id], n = o->ne[id] - b;
            for (int64_t i = 0; i < n; i++)
                for (int k = 0; k < o->sr[id]; k++) {
                    double p = o->P[id][(int64_t)k * n + i];
                    for (int q = 0; q < nrhs; q++) y[(b + i) * nrhs + q] += p * c[id][(int64_t)k * nrhs + q];
                }
        }
    }
    from_pos(o, y, Y, ldy, nrhs);
    for (int64_t id = 1; id < o->nnodes; id++) free(c[id]);
    free(c); free(x); free(y);
    return ORC_OK;
}

/* Dense N x N assembly (row-major, original point order) of
 * lambda I + Ktilde (which = 0) or dKtilde/dh (which = 1), block by block:
 * leaf diagonal blocks exact; for every internal alpha the off-diagonal
 * blocks P_{l l~} K_{l~ r} and P_{r r~} K_{r~ l} of eq. (6), with the
 * telescoped projections of eq. (9).  With a level restriction at L, the
 * internal nodes above the frontier are replaced by the blocks
 * P_{a a~} K_{a~ b} between every two frontier nodes a != b. */
int orc_dense(const orc_t *o, int which, double *A) {
    if (!o->skel_built) return ORC_ERR_STATE;
    int64_t N = o->N;
    for (int64_t i = 0; i < N * N; i++) A[i] = 0.0;
    int64_t fl = first_at(o->D), nleaf = (int64_t)1 << o->D;
    for (int64_t j = 0; j < nleaf; j++) {
        int64_t id = fl + j, b = o->nb[id], e = o->ne[id];
        for (int64_t i = b; i < e; i++)
            for (int64_t k = b; k < e; k++)
                A[o->perm[i] * N + o->perm[k]] = kpos(o, i, k, which) + ((i == k && !which) ? o->lambda : 0.0);
    }
    int top = o->hybL > 0 ? o->hybL : 0;
    if (top > 0) { /* frontier pairs: P_{a a~} K_{a~ b} */
        int64_t f = first_at(top), cnt = (int64_t)1 << top;
        for (int64_t a = f; a < f + cnt; a++)
            for (int64_t bb = f; bb < f + cnt; bb++) {
                if (a == bb) continue;
                int64_t na = o->ne[a] - o->nb[a], nbb = o->ne[bb] - o->nb[bb];
                double *Pa = telescoped_P(o, a);
                double *Kb = kblock_skel(o, a, o->nb[bb], o->ne[bb], which, 1);
                double *blk = (double *)malloc(sizeof(double) * na * nbb);
                mm(Pa, Kb, blk, na, o->sr[a], nbb, 1);
                for (int64_t i = 0; i < na; i++)
                    for (int64_t k = 0; k < nbb; k++)
                        A[o->perm[o->nb[a] + i] * N + o->perm[o->nb[bb] + k]] = blk[i * nbb + k];
                free(Pa); free(Kb); free(blk);
            }
    }
    for (int64_t id = top > 0 ? first_at(top) : 0; id < fl; id++) {
        int64_t l = 2 * id + 1, r = 2 * id + 2;
        for (int side = 0; side < 2; side++) {
            int64_t a = side ? r : l, bb = side ? l : r; /* rows of a, columns of bb */
            int64_t na = o->ne[a] - o->nb[a], nbb = o->ne[bb] - o->nb[bb];
            double *Pa = telescoped_P(o, a);
            double *Kb = kblock_skel(o, a, o->nb[bb], o->ne[bb], which, 1);
            double *blk = (double *)malloc(sizeof(double) * na * nbb);
            mm(Pa, Kb, blk, na, o->sr[a], nbb, 1);
            for (int64_t i = 0; i < na; i++)
                for (int64_t k = 0; k < nbb; k++) A[o->perm[o->nb[a] + i] * N + o->perm[o->nb[bb] + k]] = blk[i * nbb + k];
            free(Pa); free(Kb); free(blk);
        }
    }
    return ORC_OK;
}

/* dense kernel matrix K(X_I, X_J) (row-major) for arbitrary original indices */
void orc_kernel_matrix(const double *X, int d, double h, const int64_t *I, int64_t ni, const int64_t *J,
                       int64_t nj, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < ni; a++)
        for (int64_t b = 0; b < nj; b++) out[a * nj + b] = orc_kernel(X + I[a] * d, X + J[b] * d, d, h);
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
