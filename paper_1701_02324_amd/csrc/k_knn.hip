// k_knn.hip -- kappa-nearest-neighbour importance sampling for the
// skeletonization (the kappa of the sampling in Sec. 4, Table "speedup":
// the neighbours of a node's points that lie outside it are sampled first).
//
//  * k_knn_boxes: the bounding box of every run of kKnnRun consecutive tree
//    positions (the tree keeps such runs spatially compact).
//  * k_knn: exact all-kappa-nearest neighbours, one wave per 64 query
//    points.  The wave visits the runs outward from its own (own run, next,
//    previous, ...); a run is skipped when, for every lane, the distance
//    from its query to the run's box is above the lane's current kappa-th
//    distance (with a 1e-12 relative margin that covers the rounding of
//    both distances), otherwise its points are compared one by one, their
//    coordinates read by wave-uniform loads.  Each lane keeps its sorted
//    list (squared distance, position) in registers and inserts by a fixed
//    compare-exchange pass, so the result does not depend on the visiting
//    order: the kappa smallest pairs in lexicographic order.  Distances are
//    fma(t, t, r2) over t = x_k - y_k in increasing k; the padded
//    coordinates (zero on both sides) add exact zeros.
//  * k_nbr_rank: a node's ranked neighbour list, one workgroup per node of
//    a level (bottom-up): the entries (leaf: the neighbours of its points,
//    weight 1 each; internal: its children's lists with their weights)
//    outside the node are sorted by position (bitonic, keys position << 32 |
//    weight), equal positions merged with their weights added, re-keyed
//    (2^32 - 1 - weight) << 32 | position and sorted again: the list, the
//    largest weight first, lowest position on ties, is cut to the sample
//    size.  Entries are sorted in LDS up to kNbrLds keys, in a global scratch
//    slot beyond.
//
// This file is compiled with FP contraction off: the distances' rounding is
// the explicit fma above.
#include "askit_dev.h"

namespace askit {

constexpr int kKnnRun = 64;  // positions per bounding box

__device__ inline bool nn_before(double da, int ia, double db, int ib) { return da < db || (da == db && ia < ib); }

// thread -> (run, dimension): min and max of the run's coordinates
__global__ void k_knn_boxes(const double *__restrict__ Xp, int64_t N, int d, int dpad, double *__restrict__ lo,
                            double *__restrict__ hi) {
    const int64_t nrun = (N + kKnnRun - 1) / kKnnRun;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nrun * dpad) return;
    const int64_t r = g / dpad;
    const int k = (int)(g % dpad);
    double a = 0.0, b = 0.0;
    if (k < d) {
        const int64_t j0 = r * kKnnRun, j1 = j0 + kKnnRun < N ? j0 + kKnnRun : N;
        a = b = Xp[j0 * d + k];
        for (int64_t j = j0 + 1; j < j1; j++) {
            const double v = Xp[j * d + k];
            a = fmin(a, v);
            b = fmax(b, v);
        }
    }
    lo[g] = a;
    hi[g] = b;
}

// K: list length kept in registers (>= kappa); DIM: coordinates per point
// held (>= d, zero padded).  Points are read from Xp at stride d; boxes at
// stride DIM.
template <int K, int DIM>
__global__ __launch_bounds__(64) void k_knn(const double *__restrict__ Xp, int64_t N, int d,
                                            const double *__restrict__ lo, const double *__restrict__ hi, int kappa,
                                            int32_t *__restrict__ out) {
    const int lane = threadIdx.x;
    const int64_t q0 = (int64_t)blockIdx.x * kWave, q = q0 + lane;
    const bool live = q < N;
    double x[DIM];
#pragma unroll
    for (int k = 0; k < DIM; k++) x[k] = (live && k < d) ? Xp[q * d + k] : 0.0;
    double ld[K];
    int li[K];
#pragma unroll
    for (int t = 0; t < K; t++) {
        ld[t] = INFINITY;
        li[t] = 0x7fffffff;
    }
    const int64_t nrun = (N + kKnnRun - 1) / kKnnRun, r0 = q0 / kKnnRun;
    for (int64_t u = 0; u < nrun; u++) {
        // outward from the wave's own run: 0, +1, -1, +2, -2, ...
        const int64_t off = (u & 1) ? (u + 1) / 2 : -(u / 2);
        int64_t r = r0 + off;
        r = r < 0 ? r + nrun : (r >= nrun ? r - nrun : r);
        // lower bound of the squared distance from the query to the box
        double lb = 0.0;
        const double *bl = lo + r * DIM, *bh = hi + r * DIM;
#pragma unroll
        for (int k = 0; k < DIM; k++) {
            const double g = fmax(fmax(bl[k] - x[k], x[k] - bh[k]), 0.0);
            lb = fma(g, g, lb);
        }
        const bool skip = !live || lb * (1.0 - 1e-12) > ld[K - 1];
        if (__all(skip)) continue;
        const int64_t j0 = r * kKnnRun, j1 = j0 + kKnnRun < N ? j0 + kKnnRun : N;
        for (int64_t j = j0; j < j1; j++) {
            const double *y = Xp + j * d;
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; k++) {
                const double t = x[k] - (k < d ? y[k] : 0.0);
                r2 = fma(t, t, r2);
            }
            const int jj = (int)j;
            if (live && jj != (int)q && nn_before(r2, jj, ld[K - 1], li[K - 1])) {
                // fixed compare-exchange pass: the new pair sinks to its place
                double cd = r2;
                int ci = jj;
#pragma unroll
                for (int t = 0; t < K; t++) {
                    const bool b = nn_before(cd, ci, ld[t], li[t]);
                    const double td = ld[t];
                    const int ti = li[t];
                    ld[t] = b ? cd : td;
                    li[t] = b ? ci : ti;
                    cd = b ? td : cd;
                    ci = b ? ti : ci;
                }
            }
        }
    }
    if (live) {
#pragma unroll
        for (int t = 0; t < K; t++)
            if (t < kappa) out[q * kappa + t] = li[t] == 0x7fffffff ? -1 : li[t];
    }
}

template __global__ void k_knn<8, 16>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<16, 16>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<32, 16>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<64, 16>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<8, 32>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<16, 32>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<32, 32>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<64, 32>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<8, 64>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<16, 64>(const double *, int64_t, int, const double *, const double *, int, int32_t *);
template __global__ void k_knn<32, 64>(const double *, int64_t, int, const double *, const double *, int, int32_t *);

// ascending bitonic sort of the P keys at a (P a power of two), all threads
template <typename PK>
__device__ inline void bitonic(PK a, int P) {
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += kNbrThreads) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t x = a[i], y = a[l];
                    if ((x > y) == ((i & k) == 0)) {
                        a[i] = y;
                        a[l] = x;
                    }
                }
            }
            __syncthreads();
        }
}

// key of entry i of node id (position << 32 | weight), or kNone for an entry
// inside the node or a missing neighbour; entries: leaf (e - b) kappa, else
// the two children's list lengths
constexpr uint64_t kNone = ~0ULL;
__device__ inline uint64_t nbr_entry(const NbrTask &t, int64_t id, int64_t b, int64_t e, int64_t i) {
    int32_t p, w;
    if (t.leaf) {
        p = t.knn[b * t.kappa + i];
        w = 1;
        if (p < 0) return kNone;
    } else {
        const int64_t cl = 2 * id + 1, nl = t.len[cl];
        const int64_t c = i < nl ? cl : cl + 1, k = i < nl ? i : i - nl;
        p = t.pos[c * t.cap + k];
        w = t.w[c * t.cap + k];
    }
    if (p >= b && p < e) return kNone;
    return ((uint64_t)(uint32_t)p << 32) | (uint32_t)w;
}

template <typename PK>
__device__ inline void rank_node(PK A, PK B, int P, const NbrTask &t, int64_t id, int64_t nent, int *slot) {
    const int tid = threadIdx.x;
    const int64_t b = t.nb[id], e = t.ne[id];
    // the entries outside the node, in any order (equal keys are equal), then padding
    for (int64_t i = tid; i < nent; i += kNbrThreads) {
        const uint64_t key = nbr_entry(t, id, b, e, i);
        if (key != kNone) A[atomicAdd(slot, 1)] = key;
    }
    __syncthreads();
    for (int i = *slot + tid; i < P; i += kNbrThreads) A[i] = kNone;
    __syncthreads();
    bitonic(A, P);
    // runs of equal positions: the head adds the run's weights
    for (int i = tid; i < P; i += kNbrThreads) {
        const uint64_t key = A[i];
        uint64_t out = kNone;
        if (key != kNone && (i == 0 || (A[i - 1] >> 32) != (key >> 32))) {
            uint64_t acc = 0;
            for (int j = i; j < P && (A[j] >> 32) == (key >> 32); j++) acc += A[j] & 0xffffffffULL;
            out = ((0xffffffffULL - acc) << 32) | (key >> 32);
        }
        B[i] = out;
    }
    __syncthreads();
    bitonic(B, P);
    const int cap = t.cap;
    for (int i = tid; i < cap && i < P; i += kNbrThreads) {
        const uint64_t key = B[i];
        if (key == kNone) break;
        t.pos[id * cap + i] = (int32_t)(key & 0xffffffffULL);
        t.w[id * cap + i] = (int32_t)(0xffffffffULL - (key >> 32));
        // the list ends at the first padding key, or at the cut
        if (i + 1 == cap || i + 1 == P || B[i + 1] == kNone) t.len[id] = i + 1;
    }
    if (tid == 0 && B[0] == kNone) t.len[id] = 0;
}

// One workgroup per node first + blockIdx.x.  The node's entries outside it
// are counted first; up to kNbrLds of them are sorted in LDS, more in the
// workgroup's scratch slot (2 pmax keys, pmax a power of two >= every
// node's entry count).
__global__ __launch_bounds__(kNbrThreads) void k_nbr_rank(NbrTask t, int64_t first, int64_t pmax,
                                                          uint64_t *scratch) {
    __shared__ uint64_t A[kNbrLds], B[kNbrLds];
    __shared__ int cnt;
    const int64_t id = first + blockIdx.x, b = t.nb[id], e = t.ne[id];
    const int64_t nent = t.leaf ? (e - b) * t.kappa : (int64_t)t.len[2 * id + 1] + t.len[2 * id + 2];
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int local = 0;
    for (int64_t i = threadIdx.x; i < nent; i += kNbrThreads) local += nbr_entry(t, id, b, e, i) != kNone;
    atomicAdd(&cnt, local);
    __syncthreads();
    int P = 2;
    while (P < cnt) P <<= 1;
    __syncthreads();
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    if (P <= kNbrLds) {
        rank_node(A, B, P, t, id, nent, &cnt);
    } else {
        GLB uint64_t *g = glb(scratch) + (int64_t)blockIdx.x * 2 * pmax;
        rank_node(g, g + P, P, t, id, nent, &cnt);
    }
}

}  // namespace askit
