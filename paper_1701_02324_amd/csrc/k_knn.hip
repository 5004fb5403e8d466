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
//    both distances), otherwise its points are staged in LDS and compared
//    one by one (the number of points compared, per wave, is counted in
//    `visits`).  Each lane keeps its sorted
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
// stride DIM.  The wave takes the runs in batches of kKnnBatch (in the
// outward order): the batch's boxes are staged in LDS and tested against
// every lane's query (a run is kept if any lane may find a neighbour in
// it), then each kept run is tested again with the lanes' current
// thresholds and, if still kept, its points are staged in LDS and compared.
constexpr int kKnnBatch = 32;
// points compared together (independent distance chains): four for short
// lists of points of at most 16 coordinates; one otherwise, where the
// registers leave no room for four (measured at 2^20 points in 16-D: kappa =
// 8 168 against 185 ms, kappa = 32 246 against 366 ms)
template <int K, int DIM> constexpr int knn_group() { return K <= 16 && DIM <= 16 ? 4 : 1; }
__device__ inline int64_t knn_run_of(int64_t u, int64_t r0, int64_t nrun) {
    // outward from the wave's own run: 0, +1, -1, +2, -2, ...
    const int64_t r = r0 + ((u & 1) ? (u + 1) / 2 : -(u / 2));
    return r < 0 ? r + nrun : (r >= nrun ? r - nrun : r);
}

template <int K, int DIM>
__global__ __launch_bounds__(64) void k_knn(const double *__restrict__ Xp, int64_t N, int d,
                                            const double *__restrict__ lo, const double *__restrict__ hi, int kappa,
                                            int32_t *__restrict__ out, unsigned long long *__restrict__ visits) {
    __shared__ double sp[kKnnRun * DIM];          // points of the run being compared
    __shared__ double sb[kKnnBatch * 2 * DIM];    // boxes of the batch: lo then hi per run
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
    // lower bound of the squared distance from this lane's query to box i
    // of the batch
    auto bound = [&](int i) {
        const double *bl = sb + i * 2 * DIM, *bh = bl + DIM;
        double lb = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; k++) {
            const double g = fmax(fmax(bl[k] - x[k], x[k] - bh[k]), 0.0);
            lb = fma(g, g, lb);
        }
        return lb;
    };
    // a run may hold a neighbour of a lane unless its bound exceeds the
    // lane's kappa-th distance by the 1e-12 margin
    auto may = [&](double lb) { return live && !(lb * (1.0 - 1e-12) > ld[K - 1]); };
    const int64_t nrun = (N + kKnnRun - 1) / kKnnRun, r0 = q0 / kKnnRun;
    for (int64_t u0 = 0; u0 < nrun; u0 += kKnnBatch) {
        const int nb = nrun - u0 < kKnnBatch ? (int)(nrun - u0) : kKnnBatch;
        __syncthreads();
        for (int e = lane; e < nb * 2 * DIM; e += kWave) {
            const int i = e / (2 * DIM), k = e % (2 * DIM);
            const int64_t r = knn_run_of(u0 + i, r0, nrun);
            sb[e] = k < DIM ? lo[r * DIM + k] : hi[r * DIM + k - DIM];
        }
        __syncthreads();
        uint64_t mask = 0;
        for (int i = 0; i < nb; i++)
            if (__any(may(bound(i)))) mask |= 1ull << i;
        while (mask) {
            const int i = __builtin_ctzll(mask);
            mask &= mask - 1;
            if (!__any(may(bound(i)))) continue;  // thresholds fell since the batch test
            const int64_t r = knn_run_of(u0 + i, r0, nrun);
            const int64_t j0 = r * kKnnRun;
            const int nj = N - j0 < kKnnRun ? (int)(N - j0) : kKnnRun;
            __syncthreads();
            if (lane < nj) {
#pragma unroll
                for (int k = 0; k < DIM; k++) sp[lane * DIM + k] = k < d ? Xp[(j0 + lane) * d + k] : 0.0;
            }
            __syncthreads();
            if (lane == 0) atomicAdd(visits, (unsigned long long)nj);  // points compared by this wave
            constexpr int kKnnGroup = knn_group<K, DIM>();
            for (int j4 = 0; j4 < nj; j4 += kKnnGroup) {
                double r2[kKnnGroup];
#pragma unroll
                for (int p = 0; p < kKnnGroup; p++) r2[p] = 0.0;
#pragma unroll
                for (int k = 0; k < DIM; k++)
#pragma unroll
                    for (int p = 0; p < kKnnGroup; p++) {
                        const double t = x[k] - sp[((j4 + p) & (kKnnRun - 1)) * DIM + k];
                        r2[p] = fma(t, t, r2[p]);
                    }
#pragma unroll
                for (int p = 0; p < kKnnGroup; p++) {
                    const int j = (int)(j0 + j4 + p);
                    if (live && j4 + p < nj && j != (int)q && nn_before(r2[p], j, ld[K - 1], li[K - 1])) {
                        // fixed compare-exchange pass: the new pair sinks to its place
                        double cd = r2[p];
                        int ci = j;
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
        }
    }
    if (live) {
#pragma unroll
        for (int t = 0; t < K; t++)
            if (t < kappa) out[q * kappa + t] = li[t] == 0x7fffffff ? -1 : li[t];
    }
}

template __global__ void k_knn<8, 16>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<16, 16>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<32, 16>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<64, 16>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<8, 32>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<16, 32>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<32, 32>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<64, 32>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<8, 64>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<16, 64>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);
template __global__ void k_knn<32, 64>(const double *, int64_t, int, const double *, const double *, int,
                                             int32_t *, unsigned long long *);

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
