// k_misc.hip -- data movement around the level kernels: permutation of the
// right-hand sides into tree order and back, leaf-block assembly, identity
// blocks of the reduced systems, strided copies / precision casts and the
// small reductions of the refinement loop.
#include "askit_dev.h"

namespace askit {

// Permutation of right-hand sides between the caller's point order and tree
// order (W row-major in tree order, row stride ldw), by tiles of 64 points x
// 64 columns through LDS, over the caller's point order i (iperm[i] = tree
// position of point i): the caller's column-major block is read and written
// by whole columns, the tree-order block by whole rows, both coalesced.  256
// threads; grid = (ceil(N / 64), ceil(nrhs / 64)).
// W(iperm[i], c) = B[i + c * ldb]
template <typename T>
__global__ __launch_bounds__(256) void k_gather_rhs_t(const double *__restrict__ B, int64_t ldb,
                                                      const int64_t *__restrict__ iperm, int64_t N, int nrhs,
                                                      T *__restrict__ W, int64_t ldw) {
    __shared__ double tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64, lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const GLB double *Bg = glb(B);
    for (int cc = wave; cc < 64; cc += 4)
        tile[lane][cc] = (i0 + lane < N && c0 + cc < nrhs) ? Bg[(i0 + lane) + (int64_t)(c0 + cc) * ldb] : 0.0;
    __syncthreads();
    GLB T *Wg = glb(W);
    for (int r = wave; r < 64; r += 4) {
        if (i0 + r >= N) break;
        const int64_t row = glb(iperm)[i0 + r];
        if (c0 + lane < nrhs) Wg[row * ldw + c0 + lane] = (T)tile[r][lane];
    }
}

// X[i + c * ldx] (op)= W(iperm[i], c); op 0: store, 1: add
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_rhs_t(const T *__restrict__ W, int64_t ldw,
                                                       const int64_t *__restrict__ iperm, int64_t N, int nrhs,
                                                       double *__restrict__ X, int64_t ldx, int add) {
    __shared__ double tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64, lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const GLB T *Wg = glb(W);
    for (int r = wave; r < 64; r += 4) {
        const bool live = i0 + r < N;
        const int64_t row = live ? glb(iperm)[i0 + r] : 0;
        tile[r][lane] = (live && c0 + lane < nrhs) ? (double)Wg[row * ldw + c0 + lane] : 0.0;
    }
    __syncthreads();
    GLB double *Xg = glb(X);
    for (int cc = wave; cc < 64; cc += 4) {
        if (c0 + cc >= nrhs) break;
        if (i0 + lane < N) {
            GLB double *dst = Xg + (i0 + lane) + (int64_t)(c0 + cc) * ldx;
            if (add) *dst += tile[lane][cc];
            else *dst = tile[lane][cc];
        }
    }
}

// iperm[perm[p]] = p
__global__ void k_invert_perm(const int64_t *__restrict__ perm, int64_t N, int64_t *__restrict__ iperm) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) glb(iperm)[glb(perm)[p]] = p;
}

// batched permutation of right-hand sides (pointer table on the device);
// grid = problem * blocks_per_task
template <typename T>
__global__ void k_gather_multi(const GatherTask *__restrict__ tasks, const double *const *__restrict__ B, int nrhs,
                               int bpt) {
    const int p = blockIdx.x / bpt;
    const GatherTask t = tasks[p];
    const int64_t e = (int64_t)(blockIdx.x % bpt) * blockDim.x + threadIdx.x;
    if (e >= t.N * nrhs) return;
    const int64_t pos = e / nrhs;
    const int c = (int)(e % nrhs);
    ((T *)t.W)[pos * t.ldw + c] = (T)B[p][t.perm[pos] + (int64_t)c * t.N];
}

template <typename T>
__global__ void k_scatter_multi(const GatherTask *__restrict__ tasks, double *const *__restrict__ X, int nrhs,
                                int bpt) {
    const int p = blockIdx.x / bpt;
    const GatherTask t = tasks[p];
    const int64_t e = (int64_t)(blockIdx.x % bpt) * blockDim.x + threadIdx.x;
    if (e >= t.N * nrhs) return;
    const int64_t pos = e / nrhs;
    const int c = (int)(e % nrhs);
    X[p][t.perm[pos] + (int64_t)c * t.N] = (double)((const T *)t.W)[pos * t.ldw + c];
}

template __global__ void k_gather_multi<double>(const GatherTask *, const double *const *, int, int);
template __global__ void k_gather_multi<float>(const GatherTask *, const double *const *, int, int);
template __global__ void k_scatter_multi<double>(const GatherTask *, double *const *, int, int);
template __global__ void k_scatter_multi<float>(const GatherTask *, double *const *, int, int);

// lambda I + K(X_a, X_a) in column-major, 64 x 64 tiles with both point
// sets staged in LDS; grid = task * tiles^2 + tile
__global__ __launch_bounds__(256) void k_leaf_block(const LeafTask *__restrict__ tasks, int tiles, int d) {
    // row points at an odd stride (lanes read different points: no bank
    // conflicts), column points (one point per wave: broadcast) at stride d,
    // or zero padded to kXrDim coordinates for d <= kXrDim, when each
    // thread reads its row point into registers once (the padded terms add
    // exact zeros: the same entries bit for bit)
    extern __shared__ double dyn_lds[];  // 64 (d | 1) + 64 max(d, kXrDim) doubles
    const int dp = d | 1, xw = d <= kXrDim ? kXrDim : d;
    double *ys = dyn_lds, *xs = dyn_lds + 64 * dp;
    const int per = tiles * tiles;
    const LeafTask t = tasks[blockIdx.x / per];
    const int rt = (blockIdx.x % per) % tiles, ct = (blockIdx.x % per) / tiles;
    const int r0 = rt * 64, c0 = ct * 64;
    if (r0 >= t.n || c0 >= t.n) return;
    const int nr = min(64, t.n - r0), nc = min(64, t.n - c0);
    for (int i = threadIdx.x; i < 64 * d; i += blockDim.x) {
        const int a = i / d, k = i % d;
        ys[a * dp + k] = a < nr ? glb(t.X)[(t.b + r0 + a) * d + k] : 0.0;
    }
    for (int i = threadIdx.x; i < 64 * xw; i += blockDim.x) {
        const int a = i / xw, k = i % xw;
        xs[i] = (a < nc && k < d) ? glb(t.X)[(t.b + c0 + a) * d + k] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x % 64;
    if (r >= nr) return;
    const double *y = ys + r * dp;
    double yr[kXrDim];
#pragma unroll
    for (int k = 0; k < kXrDim; k++) yr[k] = (d <= kXrDim && k < d) ? y[k] : 0.0;
    for (int c = threadIdx.x / 64; c < nc; c += 4) {
        const double *x = xs + c * xw;
        double r2 = 0.0;
        if (d <= kXrDim) {
#pragma unroll
            for (int k = 0; k < kXrDim; k++) {
                const double df = yr[k] - x[k];
                r2 = fma(df, df, r2);
            }
        } else {
            for (int k = 0; k < d; k++) {
                const double df = y[k] - x[k];
                r2 = fma(df, df, r2);
            }
        }
        double v = exp(r2 * t.scale);
        if (r0 + r == c0 + c) v += t.lambda;
        glb(t.A)[(r0 + r) + (int64_t)(c0 + c) * t.lda] = v;
    }
}

// n x n identity blocks (column-major, ld = n); grid = task * blocks_per_matrix,
// one wave per column (block b: columns 4 b .. 4 b + 3), lanes over the rows
__global__ void k_identity(const IdTask *__restrict__ tasks, int bpm) {
    const IdTask t = tasks[blockIdx.x / bpm];
    const int c = (blockIdx.x % bpm) * 4 + (int)threadIdx.x / kWave;
    if (c >= t.n) return;
    GLB double *col = glb(t.Z) + (int64_t)c * t.n;
    for (int r = (int)threadIdx.x % kWave; r < t.n; r += kWave) col[r] = r == c ? 1.0 : 0.0;
}

// dst(r, c) = src(r, c) with precision conversion; grid = task * rowblocks
template <typename TS, typename TD>
__global__ void k_copy(const CopyTask *__restrict__ tasks, int rowblocks) {
    // one wave per row (block b of a task: rows 4 b .. 4 b + 3), lanes over
    // the columns: no index division per element
    const CopyTask t = tasks[blockIdx.x / rowblocks];
    const int r = (blockIdx.x % rowblocks) * 4 + (int)threadIdx.x / kWave;
    if (r >= t.rows) return;
    const GLB TS *src = glb((const TS *)t.src) + (int64_t)r * t.sld;
    GLB TD *dst = glb((TD *)t.dst) + (int64_t)r * t.dld;
    for (int c = (int)threadIdx.x % kWave; c < t.cols; c += kWave) dst[c] = (TD)src[c];
}

// Y(r, c) += a * X(r, c) over n rows x nrhs columns (row-major, stride ld)
template <typename T>
__global__ void k_axpy(T *__restrict__ Y, const T *__restrict__ X, int64_t ld, int64_t n, int nrhs, double a) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    int64_t r = t / nrhs;
    int c = (int)(t % nrhs);
    Y[r * ld + c] += (T)(a * (double)X[r * ld + c]);
}

// refinement helpers on column-major N x nrhs arrays (ld):
//   R = B - R;  X += D;  per-column sums of squares into acc[3 * nrhs]
__global__ void k_residual(const double *__restrict__ B, int64_t ldb, double *__restrict__ R, int64_t ldr, int64_t N,
                           int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    int64_t i = t % N;
    int c = (int)(t / N);
    R[i + c * ldr] = B[i + c * ldb] - R[i + c * ldr];
}

__global__ void k_update(double *__restrict__ X, int64_t ldx, const double *__restrict__ D, int64_t ldd, int64_t N,
                         int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    int64_t i = t % N;
    int c = (int)(t / N);
    X[i + c * ldx] += D[i + c * ldd];
}

// --- batched Krylov helpers on column-major N x nrhs blocks (ld = N) ------
// vectors V_j are stored back to back: V + j * N * nrhs

// partial[(j * nrhs + c) * nchunk + chunk] = sum over the chunk of V_j(:,c) W(:,c)
// grid: x = j * nrhs + c, y = chunk; rows of a chunk summed in a fixed order
__global__ void k_mdot_part(const double *__restrict__ V, const double *__restrict__ W, int64_t N, int nrhs,
                            int64_t chunk, double *__restrict__ part) {
    __shared__ double sh[256];
    const int jc = blockIdx.x, c = jc % nrhs, j = jc / nrhs;
    const double *v = V + (int64_t)j * N * nrhs + (int64_t)c * N, *w = W + (int64_t)c * N;
    const int64_t r0 = (int64_t)blockIdx.y * chunk, r1 = min(N, r0 + chunk);
    double acc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) acc = fma(v[i], w[i], acc);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)jc * gridDim.y + blockIdx.y] = sh[0];
}

// out[jc] = sum of the nchunk partials of jc, in chunk order
__global__ void k_mdot_finish(const double *__restrict__ part, int nchunk, int njc, double *__restrict__ out) {
    int jc = blockIdx.x * blockDim.x + threadIdx.x;
    if (jc >= njc) return;
    double acc = 0.0;
    for (int k = 0; k < nchunk; k++) acc += part[(int64_t)jc * nchunk + k];
    out[jc] = acc;
}

// W(:,c) -= sum_{j < nv} h[j * nrhs + c] V_j(:,c)
__global__ void k_maxpy(double *__restrict__ W, const double *__restrict__ V, const double *__restrict__ h, int nv,
                        int64_t N, int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const int c = (int)(t / N);
    double acc = W[t];
    for (int j = 0; j < nv; j++) acc = fma(-h[j * nrhs + c], V[(int64_t)j * N * nrhs + t], acc);
    W[t] = acc;
}

// U(:,c) = sum_{j < nv} y[j * nrhs + c] V_j(:,c)
__global__ void k_lincomb(double *__restrict__ U, const double *__restrict__ V, const double *__restrict__ y, int nv,
                          int64_t N, int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    const int c = (int)(t / N);
    double acc = 0.0;
    for (int j = 0; j < nv; j++) acc = fma(y[j * nrhs + c], V[(int64_t)j * N * nrhs + t], acc);
    U[t] = acc;
}

// D(:,c) = W(:,c) * sc[c]
__global__ void k_scale_cols(double *__restrict__ D, const double *__restrict__ W, const double *__restrict__ sc,
                             int64_t N, int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    D[t] = W[t] * sc[t / N];
}

// R = B - R (column-major, R with ld N, B with ldb); X += D (X with ldx)
__global__ void k_sub_from(const double *__restrict__ B, int64_t ldb, double *__restrict__ R, int64_t N, int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    int64_t i = t % N, c = t / N;
    R[t] = B[i + c * ldb] - R[t];
}

__global__ void k_zero(double *__restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template __global__ void k_gather_rhs_t<double>(const double *, int64_t, const int64_t *, int64_t, int, double *, int64_t);
template __global__ void k_gather_rhs_t<float>(const double *, int64_t, const int64_t *, int64_t, int, float *, int64_t);
template __global__ void k_scatter_rhs_t<double>(const double *, int64_t, const int64_t *, int64_t, int, double *, int64_t, int);
template __global__ void k_scatter_rhs_t<float>(const float *, int64_t, const int64_t *, int64_t, int, double *, int64_t, int);
template __global__ void k_copy<double, double>(const CopyTask *, int);
template __global__ void k_copy<double, float>(const CopyTask *, int);
template __global__ void k_copy<float, double>(const CopyTask *, int);
template __global__ void k_axpy<double>(double *, const double *, int64_t, int64_t, int, double);
template __global__ void k_axpy<float>(float *, const float *, int64_t, int64_t, int, double);

}  // namespace askit
