/*
 * askit.h -- C ABI of libaskit, a gfx950 (MI355X) implementation of the
 * hierarchical direct solver for regularized kernel systems of
 *   Yu, March & Biros, "An N log N Parallel Fast Direct Solver for Kernel
 *   Matrices", arXiv:1701.02324.
 *
 * Problem (Sec. 1): given N points x_i in R^d, the Gaussian kernel of eq. (1)
 * K_ij = exp(-|x_i - x_j|^2 / (2 h^2)) and lambda >= 0, solve
 * (lambda I + Ktilde) x = b, where Ktilde is the hierarchical (ASKIT)
 * approximation of K built from a binary tree and skeletons (Sec. 2.1).
 * The pipeline is build_tree -> skeletonize (Alg. 1) -> factorize (Alg. 2)
 * -> solve (Alg. 3).
 *
 * Conventions for every entry point:
 *  - Array arguments are owned by the caller; the library never frees them
 *    and never keeps them after the call returns (inputs are copied when
 *    retained).  They are DEVICE pointers (memory of the current HIP
 *    device), except where an entry point says otherwise; the points of
 *    askit_build_tree, the permutation of askit_tree_perm and the arrays of
 *    askit_solve, askit_solve_transpose, askit_matvec and
 *    askit_adjoint_scalars may also be HOST pointers (pageable or pinned,
 *    told apart by hipPointerGetAttributes).  Host arrays are staged through
 *    device buffers of the call, which then synchronizes `stream` before it
 *    returns.
 *  - Points are N x d row-major (point-major; the paper's d x N matrix X).
 *  - Right-hand sides and solutions are N x nrhs column-major with leading
 *    dimension ld >= N, in the caller's original point order.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *    and runs asynchronously unless stated otherwise.  Argument validation is
 *    synchronous.  Calls on one handle must not overlap.
 *  - Every call returns an askit_status; askit_last_error() gives the
 *    message of the last failure on the calling thread.
 *  - Handles own all device workspace and are released only by *_destroy.
 *    A factor keeps a reference to its tree: destroy factors first.
 */
#ifndef ASKIT_H
#define ASKIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ASKIT_OK = 0,
    ASKIT_ERR_ARG = 1,       /* invalid argument; nothing was enqueued        */
    ASKIT_ERR_ALLOC = 2,     /* device allocation failed                       */
    ASKIT_ERR_HIP = 3,       /* a HIP runtime call failed                      */
    ASKIT_ERR_STATE = 4,     /* call out of order (e.g. solve before factor)   */
    ASKIT_ERR_SINGULAR = 5,  /* an exactly zero pivot was met                  */
    ASKIT_WARN_ILLCOND = 6   /* result written, but a block's pivot ratio fell
                                below 1e-12 (instability of Sec. 3 detected)   */
} askit_status;

typedef enum { ASKIT_FP64 = 0, ASKIT_MIXED = 1 } askit_precision;

typedef struct askit_tree_s *askit_tree;
typedef struct askit_factor_s *askit_factor;

/* Method parameters.  leaf_size = m (>= 2), rank = s (>= 1; fixed rank,
 * clamped per node to the number of candidates), n_samples = rows sampled
 * per node for the ID (0 -> 4 s), seed = sampling seed, problem = index
 * folded into the sampling streams, h = kernel bandwidth (> 0).
 * tol = tau of the adaptive rank of Sec. 2.1 ("Computing low rank
 * approximations"): a node's rank is the smallest s_alpha with
 * |R_{s_alpha s_alpha}| < tau |R_00| on the diagonal of its pivoted QR
 * (the estimate of sigma_{s_alpha+1} / sigma_1), at most rank (then s_max);
 * 0 keeps the fixed rank.  In [0, 1).  Every QR also stops at the rank
 * guard |R_jj| <= 1e-14 |R_00|.
 * qr_split_levels chooses the launch shape of the pivoted QR, not its
 * result: nodes at tree levels 1 .. L are factored by several workgroups
 * each, one launch per pivot step, the deeper ones by one workgroup each
 * (0 -> L = D - 1, every internal level, in askit_skeletonize and
 * L = min(D - 1, 9), the levels with fewer than 1024 nodes, in
 * askit_skeletonize_factorize; -1 -> none).  Both shapes give bit-identical
 * skeletons.
 * knn = kappa of the nearest-neighbour importance sampling (the number of
 * neighbours the skeletonization sampling uses, Sec. 4, Table "speedup"); 0
 * samples uniform rows only.  With kappa > 0 the tree build also finds the
 * kappa nearest points of every point (exact, by squared distance summed
 * as fma(t, t, r2) over t = x_k - y_k in increasing k, ties to the lower
 * tree position) and ranks, for every node, the neighbours of its points
 * that lie outside it: a leaf weighs each by the number of its points that
 * have it as a neighbour, an internal node merges its children's lists
 * (weights added) and drops its own points; largest weight first, lowest
 * position on ties, cut to n_samples.  A node's sampled rows are its list,
 * then uniform draws as with knn = 0 (repeats of listed rows rejected).
 * In [0, 64] ([0, 32] for d > 32), knn * N < 2^31. */
typedef struct {
    int32_t leaf_size;
    int32_t rank;
    int32_t n_samples;
    int32_t qr_split_levels;
    uint64_t seed;
    int64_t problem;
    double h;
    double tol;
    int32_t knn;
    int32_t reserved;  /* 0 */
} askit_options;

/* Tree build (Sec. 2.1, "Partitioning the matrix"): complete binary tree of
 * depth D = ceil(log2(N / m)); each node's points are split in two halves
 * (floor(n/2) to the left) by the hyperplane through their median along
 * their principal axis.  X: device or host, N x d row-major FP64, copied.
 * Blocks until the tree is built.  Errors: ASKIT_ERR_ARG for N < 1 or
 * N >= 2^31, d < 1 or d > 64, m < 2, s < 1, h <= 0 or not finite, tol
 * outside [0, 1), non-finite coordinates, n_samples < 0 or > 4096,
 * qr_split_levels < -1, knn outside its range, a largest leaf ceil(N / 2^D)
 * above 512 points or 2 s above 512 (the kernels hold a leaf block and a
 * reduced system of order s_l + s_r in one workgroup). */
askit_status askit_build_tree(const double *X, int64_t N, int32_t d, const askit_options *opt, void *stream,
                              askit_tree *out);

/* The kappa nearest neighbours of every point found by the tree build
 * (knn > 0): idx[i * kappa + t] = tree position of the t-th nearest point
 * of tree position i (t = 0 nearest; -1 where N - 1 < kappa).  idx: device
 * or host, N x kappa int32.  Errors: ASKIT_ERR_STATE if knn = 0. */
askit_status askit_tree_knn(askit_tree t, int32_t *idx);

/* The ranked neighbour lists of the nodes (knn > 0; see askit_options):
 * node id's list is pos[id * n_samples + k], weight[id * n_samples + k] for
 * k < len[id] (the root's is empty).  pos, weight: nnodes x n_samples int32;
 * len: nnodes int32; device or host.  Errors: ASKIT_ERR_STATE if knn = 0. */
askit_status askit_tree_neighbor_lists(askit_tree t, int32_t *pos, int32_t *weight, int32_t *len);

/* Tree depth D and the permutation (perm[position] = original index). */
askit_status askit_tree_depth(askit_tree t, int32_t *D);
askit_status askit_tree_perm(askit_tree t, int64_t *perm /* device or host, N */);

/* Skeletonize (Alg. 1; ID of eq. (4)): bottom-up over all non-root nodes,
 * sample min(n_samples, N - n_alpha) rows outside the node, form the kernel
 * block against the candidates (the node's points for a leaf, [l~ r~] for an
 * internal node) and select s columns by column-pivoted QR in FP64.
 * Blocks until done. */
askit_status askit_skeletonize(askit_tree t, void *stream);

/* Skeleton exchange (positions in the tree order; P = P_{alpha~ C}, row-major
 * s_alpha x |C|).  sizes[2*i] = s_alpha, sizes[2*i+1] = |C| for heap node i
 * (i = 1 .. 2^(D+1)-2; entry 0 is the root and stays 0).  ids holds
 * nnodes * rank int32 and P nnodes * rank * cmax doubles with
 * cmax = max(leaf_size, 2 rank), node i at offset i * rank (ids) and
 * i * rank * cmax (P).  All three are HOST pointers.  Export with ids and P
 * both NULL fills only sizes.  Import replaces the skeletons of a built tree
 * (used to factor on a given set of skeletons).  The ranks fix the shapes of
 * every later step: Z of node alpha has order s_l + s_r, Phat_alpha has
 * s_alpha columns. */
askit_status askit_skeletons_export(askit_tree t, int32_t *ids, double *P, int32_t *sizes);

/* Rows of the sampled block that the last skeletonization's pivoted QR
 * factored, per heap node (device or host array of 2^(D+1) - 1 int32): the
 * sampled rows min(n_samples, N - n_alpha) less those dropped as numerically
 * zero (squared norm at most 1e-44 of the block's squared Frobenius norm);
 * 0 for the root and for nodes with at most `rank` candidates (P = I, no
 * QR).  For work accounting.  ASKIT_ERR_STATE before a skeletonization;
 * imported skeletons keep the counts of the last skeletonization. */
askit_status askit_tree_qr_rows(askit_tree t, int32_t *rows);

/* Sampled rows S' of the last skeletonization (Sec. 2.1: the rows outside the
 * node that stand in for its complement in the ID), as tree positions in
 * draw order: n_samples int32 per heap node at offset node * n_samples
 * (device or host array of (2^(D+1) - 1) * n_samples).  A node's first
 * min(n_samples, N - n_alpha) entries are its sample, in the order of the
 * rows of its sampled block; the entries of the root and of nodes with at
 * most `rank` candidates (no QR) are unspecified.  ASKIT_ERR_STATE before a
 * skeletonization. */
askit_status askit_tree_samples(askit_tree t, int32_t *samples);
askit_status askit_skeletons_import(askit_tree t, const int32_t *ids, const double *P, const int32_t *sizes);

/* Factorize (Alg. 2, eqs. (7)-(10)): leaf LU of lambda I + K_aa; for every
 * internal node the reduced system Z = I + V W of eq. (8) formed from fused
 * kernel-block x Phat products and LU-factored in FP64; Phat telescoped by
 * eq. (10).  precision: ASKIT_FP64, or ASKIT_MIXED (FP32 kernel blocks, Phat
 * and level products; FP64 LUs).  Blocks until done.  Returns
 * ASKIT_WARN_ILLCOND (with a valid factor) when a pivot ratio min|U_ii| /
 * max|U_ii| of some block is below 1e-12. */
askit_status askit_factorize(askit_tree t, double lambda, int32_t precision, void *stream, askit_factor *out);

/* Tile autotuning of the level-batched factorization (the level schedule of
 * Sec. 2.2 as one launch per kernel and tree height): times the FP64
 * factorization's level products of t at every tree height -- the blocks
 * K_{l~ r} Phat_r of the reduced systems Z (eq. (8)) and the telescoped
 * Phat (eq. (10)) -- in each tile configuration: 64, 128 or 256 output
 * columns per tile (at most twice the built-in choice for the rank) and
 * contraction chunks of 2048, 4096 or 8192 points, and keeps the fastest
 * per height in the tree.  Later factorizations of t (askit_factorize,
 * askit_skeletonize_factorize; FP64, and mixed with tiles of at most 128
 * columns) use it; the batched entry points keep the built-in choice.  The
 * chunk changes the grouping of the split sums, so results change by
 * rounding only.  Blocks until done.  Errors: ASKIT_ERR_STATE before
 * askit_skeletonize, ASKIT_ERR_ARG for a bad lambda. */
askit_status askit_tune_factorization(askit_tree t, double lambda, void *stream);

/* The factorization's tile configuration, set by the caller (to restore one
 * that askit_tune_factorization chose earlier, e.g. from the "tune" entry of
 * askit_get_stats, or to fix one).  table is a host array of 3 * heights
 * int32 values; for tree height h = 1 .. heights, table[3 (h - 1)] is the
 * output columns per k_kmm tile (64, 128 or 256), table[3 (h - 1) + 1] the
 * contraction points per split chunk (2048, 4096 or 8192) and
 * table[3 (h - 1) + 2] the output columns per k_gmm tile (64, 128 or 256).
 * heights must equal the tree depth; heights = 0 (table may be NULL)
 * returns to the built-in choice.  Applies to later factorizations as for
 * askit_tune_factorization; the tile widths change no result, the chunk
 * changes results by rounding only.  Errors: ASKIT_ERR_ARG for a NULL tree
 * or table, a wrong height count or a size not listed. */
askit_status askit_tree_set_tiling(askit_tree t, const int32_t *table, int32_t heights);

/* Launch shape of the factorization's LU with partial pivoting (Sec. 2.2:
 * the reduced systems Z of eq. (8), and the leaf blocks when lambda = 0).
 * A batch of LUs whose largest matrix has more than n rows runs one panel
 * of 32 columns at a time over the whole batch: one workgroup per matrix
 * factors the panel and its block row of U, then the trailing update is
 * spread over one workgroup per 64 x 64 tile, so that a few large matrices
 * occupy more than a few compute units.  Smaller batches keep one
 * workgroup per matrix for the whole factorization.  Default 256; n >= 512
 * never splits; n = 0 splits every batch.  The factors are the same bit
 * for bit either way.  Applies to later factorizations of the tree; a
 * batch (askit_batch_create, askit_factorize_batched) takes the smallest n
 * of its trees.  Errors: ASKIT_ERR_ARG for a NULL tree or n < 0. */
askit_status askit_tree_set_lu_split(askit_tree t, int32_t n);

/* Hybrid solver (Sec. 2.3, "Fast hybrid solver"; Alg. HybridSolve, MatVecW,
 * MatVecV) with the skeletonization frontier at tree level `level`
 * (1 .. D): the frontier's nodes and their subtrees are factored as by
 * askit_factorize (FP64); above the frontier nothing is compressed, so the
 * matrix is lambda I + Ktilde with Ktilde_ab = P_{a a~} K_{a~ b} for any two
 * frontier nodes a != b (level 1 gives askit_factorize's matrix, the root
 * having no skeleton).  askit_solve on this factor runs HybridSolve:
 * v = D^{-1} u up to the frontier, t = V v, the reduced system
 * (I + V W) y = t of order sum_a s_a (at most 2^level * rank) by restarted
 * GMRES with V (kernel summations) and W (the frontier's Phat) applied
 * matrix-free, then x = v - W y.  askit_set_refinement sets that GMRES's
 * iteration cap (default 2000; restarts every 1024) and relative residual target (default
 * 1e-12); askit_last_solve_info reports it.  askit_matvec (which 0 and 1)
 * applies the same restricted matrix; the transpose solve and which = 2 are
 * not available (ASKIT_ERR_STATE).  Errors: ASKIT_ERR_STATE before
 * askit_skeletonize, ASKIT_ERR_ARG for level outside [1, D] or a bad
 * lambda; pivot ratios as for askit_factorize (frontier subtrees only). */
askit_status askit_factorize_hybrid(askit_tree t, double lambda, int32_t level, void *stream, askit_factor *out);

/* askit_skeletonize followed by askit_factorize (Alg. 1 then Alg. 2) as one
 * call, with the same results bit for bit.  The factorization of height h
 * needs only the skeletons of heights <= h, so it runs on a library-owned
 * non-blocking stream one height behind the skeletonization, which runs on
 * `stream`; the leaf LUs start at once.  The call returns when both are done
 * (`stream` is ordered after the factorization).  Errors as for the two
 * calls; ASKIT_ERR_STATE if factors of this tree still exist. */
askit_status askit_skeletonize_factorize(askit_tree t, double lambda, int32_t precision, void *stream,
                                         askit_factor *out);

/* X = (lambda I + Ktilde)^{-1} B (Alg. 3).  B, X: device, N x nrhs
 * column-major (ldb, ldx >= N); B and X may alias.  With refinement enabled
 * (the default for a MIXED factor, see askit_set_refinement) the result is
 * refined against the FP64 operator of askit_matvec by restarted GMRES
 * preconditioned with the stored factorization, until the relative residual
 * |b - A x| / |b| of every column is below refine_tol or max_refine operator
 * applications; see askit_last_solve_info.  Without refinement the call is
 * asynchronous on `stream`; with it, `stream` is synchronized at every
 * iteration. */
askit_status askit_solve(askit_factor f, const double *B, int64_t ldb, int32_t nrhs, double *X, int64_t ldx,
                         void *stream);

/* X = (lambda I + Ktilde)^{-T} B: the transpose of the same factorization
 * (Ktilde is not symmetric in the form of eq. (6)), applied from the root
 * down: Ktilde_aa^{-T} = D^{-T} (I - V^T Z^{-T} W^T).  Same conventions,
 * including refinement (GMRES on the transposed operator, askit_matvec with
 * which = 2, preconditioned by the transposed factors). */
askit_status askit_solve_transpose(askit_factor f, const double *B, int64_t ldb, int32_t nrhs, double *X,
                                   int64_t ldx, void *stream);

/* Y = (lambda I + Ktilde) X (which = 0), Y = dKtilde/dh X (which = 1,
 * skeletons held fixed) or Y = (lambda I + Ktilde)^T X (which = 2), the
 * hierarchical matvec of Sec. 2.1 in the form of eq. (6), FP64, kernel blocks
 * recomputed.  The transpose evaluates skeleton charges P_{a a~}^T x_a,
 * gathered upward through the projections, at the sibling's points.  Same
 * layout conventions. */
askit_status askit_matvec(askit_factor f, int32_t which, const double *X, int64_t ldx, int32_t nrhs, double *Y,
                          int64_t ldy, void *stream);

/* Refinement controls: max_refine = largest number of preconditioned
 * operator applications (0 = plain direct solve; defaults: MIXED 100, FP64 0),
 * refine_tol = target relative residual (default 1e-11).  The refinement
 * also stops when it stagnates: a restart cycle ends once four Arnoldi steps
 * gain less than 5% in the estimated residual, and the refinement ends once
 * a cycle fails to halve the true residual (askit_last_solve_info then
 * reports converged = 0 with the residual reached). */
askit_status askit_set_refinement(askit_factor f, int32_t max_refine, double refine_tol);

typedef struct {
    int32_t iterations;        /* preconditioned operator applications       */
    int32_t converged;         /* 1 if the residual reached refine_tol       */
    double initial_residual;   /* max over columns of |b - A x0| / |b|, x0 =
                                  the direct solve with the stored factors   */
    double residual;           /* same for the returned x                    */
} askit_solve_info;

askit_status askit_last_solve_info(askit_factor f, askit_solve_info *info);

/* Bandwidth of the factorizations made after this call, with the tree's
 * skeletons and projections held fixed (the ID is not differentiated).  Used
 * for derivatives in h and finite differences; a tree starts with options.h. */
askit_status askit_tree_set_bandwidth(askit_tree t, double h);

/* Adjoint scalars of the differentiation of x = A^{-1} b, A = lambda I +
 * Ktilde(h): given x and z = A^{-T} g (both N x nrhs column-major, leading
 * dimension ld, device), returns
 *   dlambda = -sum_j z_j . x_j                   (dA/dlambda = I)
 *   dh      = -sum_j z_j . (dKtilde/dh x_j)     (kernel blocks recomputed
 *                                                 with dk/dh = k r^2 / h^3)
 * so that dL/dlambda and dL/dh follow for a loss L with dL/dx = g.
 * Synchronizes `stream`; outputs are HOST scalars. */
askit_status askit_adjoint_scalars(askit_factor f, const double *X, const double *Z, int64_t ld, int32_t nrhs,
                                   double *dlambda, double *dh, void *stream);

/* Factor diagnostics: the smallest pivot ratio min|U_ii|/max|U_ii| over all
 * leaf and reduced-system LUs, and its node. */
askit_status askit_factor_pivot_ratio(askit_factor f, double *ratio, int32_t *node);

/* Batches of independent problems (level-batched execution).  Trees of a
 * batch share rank, dimension and sample count; sizes, leaf sizes, depths,
 * bandwidths and lambdas may differ.
 *  - askit_skeletonize_batched: Alg. 1 on all trees, one launch per kernel
 *    and tree height (distance from the leaves) over the nodes of all trees.
 *  - askit_batch_create: allocates one factor per tree, builds the
 *    factorization and solve plans over all trees (one launch per kernel and
 *    height) and captures each in a hipGraph; nothing is computed yet.
 *    lambdas: HOST array of count values; nrhs = right-hand sides per solve.
 *  - askit_batch_factorize: replays the factorization graph on `stream`.
 *  - askit_factorize_batched: askit_batch_create, then one
 *    askit_batch_factorize on `stream`; on failure nothing is returned.
 *  - askit_batch_check: pivot ratios of all factors (synchronizes).
 *  - askit_batch_solve: B[i], X[i] (HOST arrays of count DEVICE pointers, each
 *    N_i x nrhs column-major with ld = N_i) -> X[i] = A_i^{-1} B[i]; replays
 *    the solve graph and synchronizes `stream` before returning.
 *  - askit_batch_factor: borrowed handle of problem i (for matvec, transpose
 *    solve, refinement); it is released by askit_batch_destroy. */
typedef struct askit_batch_s *askit_batch;
askit_status askit_skeletonize_batched(askit_tree *trees, int32_t count, void *stream);
askit_status askit_batch_create(askit_tree *trees, int32_t count, const double *lambdas, int32_t precision,
                                int32_t nrhs, askit_batch *out);
askit_status askit_batch_factorize(askit_batch b, void *stream);
askit_status askit_factorize_batched(askit_tree *trees, int32_t count, const double *lambdas, int32_t precision,
                                     int32_t nrhs, void *stream, askit_batch *out);
askit_status askit_batch_check(askit_batch b, double *min_ratio, int32_t *problem, void *stream);
askit_status askit_batch_solve(askit_batch b, const double *const *B, double *const *X, void *stream);
askit_status askit_batch_factor(askit_batch b, int32_t i, askit_factor *f);
void askit_batch_destroy(askit_batch b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * permutation of askit_build_tree / askit_tree_perm (the same tree rules,
 * the same kernels, bit-identical result) without building a tree handle.
 * X: device, N x d row-major FP64 (finite; not checked here), perm: device,
 * N int64 (perm[position] = original index).  Every temporary (node ranges,
 * level partial sums, means, scatter matrices, axes, sort keys and their
 * merge buffers) lives in one library-owned static device array of 64 MiB
 * per device, kept until the process ends; no device memory is allocated or
 * freed.  The temporaries of N points in d dimensions with leaf size m
 * take about N (32 + 32 / m + 8 max(d, d (d + 1) / 2) / 256) bytes: N up to
 * about 1.8M at d = 16, m = 512; larger inputs return ASKIT_ERR_ARG and
 * enqueue nothing.
 * Asynchronous on `stream`.  Calls that overlap on one device (other
 * streams, other threads) race on the array: serialize them. */
askit_status askit_tree_permutation_noalloc(const double *X, int64_t N, int32_t d, int32_t leaf_size,
                                            int64_t *perm, void *stream);

/* Per-phase timings (ms) and sizes of the last calls on a handle, as JSON. */
askit_status askit_get_stats(askit_tree t, askit_factor f, char *json, size_t cap);

/* Per-kernel timing (process-wide state: meant for runs where one thread
 * calls the library): with profiling on, every launch of the library is
 * bracketed by HIP events on its stream; askit_profile_report writes
 * {"phase:kernel": [total_ms, launches], ...} (it synchronizes on the pending
 * events).  Enabling resets the totals.  on = 2 keeps the totals per tree
 * height for the skeletonization and factorization launches, named
 * "phase:kernel@h<height>" (height 0 = leaves); plans built while it is on
 * keep those names.  on = 3 also records every launch's start and end (ms
 * from the first profiled launch, across streams), reported as
 * "@timeline": [[name, start, end], ...]. */
askit_status askit_profile_enable(int32_t on);
askit_status askit_profile_report(char *json, size_t cap);

/* Device memory cache.  Released device blocks of 64 MiB or more (a
 * factorization's arenas, the refinement's Krylov basis) are kept by the
 * library, per device, and reused by later allocations of about the same
 * size; a block enters the cache only after its device has been synchronized.
 * This call frees every cached block of every device (hipFree) and writes the
 * number of bytes freed to *bytes_released when that pointer is not NULL.
 * Buffers of live trees and factors are not touched.  Allocation failures
 * empty the cache of the failing device by themselves before they are
 * reported. */
askit_status askit_release_cached_memory(uint64_t *bytes_released);

const char *askit_last_error(void);
void askit_tree_destroy(askit_tree t);
void askit_factor_destroy(askit_factor f);

#ifdef __cplusplus
}
#endif

#endif /* ASKIT_H */
