// askit_kernels.h -- declarations of the library's kernels for the host-side
// orchestrator (definitions live in the k_*.hip translation units).
#pragma once
#include "askit_dev.h"

namespace askit {

// tree (k_tree.hip)
__global__ void k_tree_chunk_mean(const double *X, const int64_t *perm, int d, const int64_t *nb, const int64_t *ne,
                                  int64_t first, int cnt, int maxch, double *part);
__global__ void k_tree_mean(const int64_t *nb, const int64_t *ne, int64_t first, int cnt, int maxch, int d,
                            double *part, double *mu);
__global__ void k_tree_chunk_scatter(const double *X, const int64_t *perm, int d, const int64_t *nb,
                                     const int64_t *ne, int64_t first, int cnt, int maxch, const double *mu,
                                     const int16_t *pa, const int16_t *pc, int npair, double *part);
__global__ void k_tree_scatter(const int64_t *nb, const int64_t *ne, int64_t first, int cnt, int maxch, int d,
                               const int16_t *pa, const int16_t *pc, int npair, double *part, double *S);
__global__ void k_tree_axis(int cnt, int d, const double *S, double *axis);
__global__ void k_tree_keys(const double *X, const int64_t *perm, int d, const int64_t *nb, const int64_t *ne,
                            int64_t first, int blocks_per_node, const double *mu, const double *axis, double *key,
                            int64_t *kid);
__global__ void k_tree_sort_tiles(const int64_t *nb, const int64_t *ne, int64_t first, int tiles_per_node,
                                  double *key, int64_t *kid);
__global__ void k_tree_merge(const int64_t *nb, const int64_t *ne, int64_t first, int blocks_per_node, int64_t w,
                             const double *ki, const int64_t *ii, double *ko, int64_t *io);
__global__ void k_copy_ids(const int64_t *src, int64_t *dst, int64_t n);
__global__ void k_gather_points(const double *X, const int64_t *perm, int d, int64_t N, double *Xp);
__global__ void k_iota(int64_t *p, int64_t n);
__global__ void k_node_ranges(int64_t *nb, int64_t *ne, int64_t N, int D);
__global__ void k_pair_index(int16_t *pa, int16_t *pc, int d);
__global__ void k_check_finite(const double *X, int64_t n, int32_t *bad);

// skeletons (k_skel.hip)
__global__ void k_sample(const SampTask *tasks, int nsamp, int32_t *err);
__global__ void k_sample_block(const SkelTask *tasks, int rowtiles, int ldm, int d, int coltiles);
__global__ void k_sample_rownorm(const SkelTask *tasks, int rowtiles, int ldm, int d, int coltiles);
__global__ void k_qrcp(const SkelTask *tasks, int s, int ldm, int d);
__global__ void k_qs_rows(const SkelTask *tasks, QrWork w, int ldm);
__global__ void k_qs_rowmap(const SkelTask *tasks, QrWork w);
__global__ void k_qs_init(const SkelTask *tasks, QrWork w, int s, int ldm);
__global__ void k_qs_step(const SkelTask *tasks, QrWork w, int j, int s0);
__global__ void k_qs_finish(const SkelTask *tasks, QrWork w, int s, int ldm);

// kappa-NN sampling (k_knn.hip)
__global__ void k_knn_boxes(const double *Xp, int64_t N, int d, int dpad, float *lo, float *hi);
__global__ void k_knn_box_up(float *lo, float *hi, int64_t below, int64_t nbelow, int64_t at, int64_t nat, int dpad);
template <int K, int DIM>
__global__ void k_knn(const double *Xp, int64_t N, int d, const float *lo, const float *hi, const int64_t *levoff,
                      int top, int kappa, int32_t *out, unsigned long long *visits);
__global__ void k_nbr_rank(NbrTask t, int64_t first, int64_t pmax, uint64_t *scratch);

// LU (k_lu.hip)
__global__ void k_lu(const LuTask *tasks);
__global__ void k_lup_panel(const LuTask *tasks, LuSplit w, int kb);
__global__ void k_lup_update(const LuTask *tasks, LuSplit w, const TileItem *items, int kb);
__global__ void k_lup_finish(const LuTask *tasks, LuSplit w, const TileItem *items);
__global__ void k_lu_nopiv(const LuTask *tasks);
__global__ void k_lu_diaginv(const LuTask *tasks);
template <typename T, int NR, bool TRANS>
__global__ void k_lusolve(const LuTask *tasks, int ntask, int nrhs, int panels);

// products (k_prod.hip)
template <typename T, typename TB, typename TO, int TC, bool XR, int CG>
__global__ void k_kmm(const KmmTask *tasks, const TileItem *items, int ncol, int d);
template <typename T, int TC> __global__ void k_gmm(const GmmTask *tasks, const TileItem *items, int ncol, int kchunk);
template <typename T, typename TO> __global__ void k_reduce(const RedTask *tasks, int ncol, int blocks_per_task);

// misc (k_misc.hip)
template <typename T>
__global__ void k_gather_rhs_t(const double *B, int64_t ldb, const int64_t *iperm, int64_t N, int nrhs, T *W,
                               int64_t ldw);
template <typename T>
__global__ void k_scatter_rhs_t(const T *W, int64_t ldw, const int64_t *iperm, int64_t N, int nrhs, double *X,
                                int64_t ldx, int add);
__global__ void k_invert_perm(const int64_t *perm, int64_t N, int64_t *iperm);
__global__ void k_leaf_block(const LeafTask *tasks, int tiles, int d);
template <typename T>
__global__ void k_gather_multi(const GatherTask *tasks, const double *const *B, int nrhs, int bpt);
template <typename T>
__global__ void k_scatter_multi(const GatherTask *tasks, double *const *X, int nrhs, int bpt);
__global__ void k_identity(const IdTask *tasks, int bpm);
template <typename TS, typename TD> __global__ void k_copy(const CopyTask *tasks, int rowblocks);
template <typename T> __global__ void k_axpy(T *Y, const T *X, int64_t ld, int64_t n, int nrhs, double a);
__global__ void k_residual(const double *B, int64_t ldb, double *R, int64_t ldr, int64_t N, int nrhs);
__global__ void k_update(double *X, int64_t ldx, const double *D, int64_t ldd, int64_t N, int nrhs);
__global__ void k_zero(double *p, int64_t n);
__global__ void k_mdot_part(const double *V, const double *W, int64_t N, int nrhs, int64_t chunk, double *part);
__global__ void k_mdot_finish(const double *part, int nchunk, int njc, double *out);
__global__ void k_maxpy(double *W, const double *V, const double *h, int nv, int64_t N, int nrhs);
__global__ void k_lincomb(double *U, const double *V, const double *y, int nv, int64_t N, int nrhs);
__global__ void k_scale_cols(double *D, const double *W, const double *sc, int64_t N, int nrhs);
__global__ void k_sub_from(const double *B, int64_t ldb, double *R, int64_t N, int nrhs);

}  // namespace askit
