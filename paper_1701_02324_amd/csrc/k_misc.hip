// k_misc.hip -- data movement around the level kernels: permutation of the
// right-hand sides into tree order and back, leaf-block assembly, identity
// blocks of the reduced systems, strided copies / precision casts and the
// small reductions of the refinement loop.
#include "askit_dev.h"

namespace askit {

// W(pos, c) = B[perm[pos] + c * ldb]   (W row-major, row stride ldw)
template <typename T>
__global__ void k_gather_rhs(const double *__restrict__ B, int64_t ldb, const int64_t *__restrict__ perm, int64_t N,
                             int nrhs, T *__restrict__ W, int64_t ldw) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    int64_t pos = t / nrhs;
    int c = (int)(t % nrhs);
    W[pos * ldw + c] = (T)B[perm[pos] + (int64_t)c * ldb];
}

// X[perm[pos] + c * ldx] (op)= W(pos, c); op 0: store, 1: add
template <typename T>
__global__ void k_scatter_rhs(const T *__restrict__ W, int64_t ldw, const int64_t *__restrict__ perm, int64_t N,
                              int nrhs, double *__restrict__ X, int64_t ldx, int add) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * nrhs) return;
    int64_t pos = t / nrhs;
    int c = (int)(t % nrhs);
    double v = (double)W[pos * ldw + c];
    double *dst = X + perm[pos] + (int64_t)c * ldx;
    if (add) *dst += v;
    else *dst = v;
}

// lambda I + K(X_a, X_a) in column-major; grid = task * n_max + column
__global__ void k_leaf_block(const LeafTask *__restrict__ tasks, int nmax, int d) {
    const LeafTask t = tasks[blockIdx.x / nmax];
    const int j = blockIdx.x % nmax;
    if (j >= t.n) return;
    const double *y = t.X + (t.b + j) * d;
    double yc[kMaxDim];
    for (int k = 0; k < d; k++) yc[k] = y[k];
    for (int i = threadIdx.x; i < t.n; i += blockDim.x) {
        const double *x = t.X + (t.b + i) * d;
        double r2 = 0.0;
        for (int k = 0; k < d; k++) {
            double df = x[k] - yc[k];
            r2 = fma(df, df, r2);
        }
        double v = exp(r2 * t.scale);
        if (i == j) v += t.lambda;
        t.A[i + (int64_t)j * t.lda] = v;
    }
}

// n x n identity blocks (column-major, ld = n), one block per matrix
__global__ void k_identity(double *__restrict__ Z, int n, int64_t stride, int count) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t per = (int64_t)n * n;
    if (t >= per * count) return;
    int64_t m = t / per, e = t % per;
    Z[m * stride + e] = (e % n == e / n) ? 1.0 : 0.0;
}

// dst(r, c) = src(r, c) with precision conversion; grid = task * rowblocks + rb
template <typename TS, typename TD>
__global__ void k_copy(const CopyTask *__restrict__ tasks, int rowblocks) {
    const CopyTask t = tasks[blockIdx.x / rowblocks];
    const int64_t e = (int64_t)(blockIdx.x % rowblocks) * blockDim.x + threadIdx.x;
    if (e >= (int64_t)t.rows * t.cols) return;
    const int64_t r = e / t.cols, c = e % t.cols;
    ((TD *)t.dst)[r * t.dld + c] = (TD)((const TS *)t.src)[r * t.sld + c];
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

// per column: acc[c] += |u|^2, acc[nrhs + c] += |v|^2 (block partials, fixed order
// per block, blocks combined with atomics: the values only steer the loop)
__global__ void k_colnorms(const double *__restrict__ U, int64_t ldu, const double *__restrict__ V, int64_t ldv,
                           int64_t N, int nrhs, double *__restrict__ acc) {
    __shared__ double su[256], sv[256];
    const int c = blockIdx.y;
    double pu = 0.0, pv = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double u = U[i + c * ldu], v = V[i + c * ldv];
        pu = fma(u, u, pu);
        pv = fma(v, v, pv);
    }
    su[threadIdx.x] = pu;
    sv[threadIdx.x] = pv;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            su[threadIdx.x] += su[threadIdx.x + o];
            sv[threadIdx.x] += sv[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(acc + c, su[0]);
        atomicAdd(acc + nrhs + c, sv[0]);
    }
}

__global__ void k_zero(double *__restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template __global__ void k_gather_rhs<double>(const double *, int64_t, const int64_t *, int64_t, int, double *, int64_t);
template __global__ void k_gather_rhs<float>(const double *, int64_t, const int64_t *, int64_t, int, float *, int64_t);
template __global__ void k_scatter_rhs<double>(const double *, int64_t, const int64_t *, int64_t, int, double *, int64_t, int);
template __global__ void k_scatter_rhs<float>(const float *, int64_t, const int64_t *, int64_t, int, double *, int64_t, int);
template __global__ void k_copy<double, double>(const CopyTask *, int);
template __global__ void k_copy<double, float>(const CopyTask *, int);
template __global__ void k_copy<float, double>(const CopyTask *, int);
template __global__ void k_axpy<double>(double *, const double *, int64_t, int64_t, int, double);
template __global__ void k_axpy<float>(float *, const float *, int64_t, int64_t, int, double);

}  // namespace askit
