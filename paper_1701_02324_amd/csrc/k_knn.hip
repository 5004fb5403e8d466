// k_knn.hip -- kappa-nearest-neighbour importance sampling for the
// skeletonization (the kappa of the sampling in Sec. 4, Table "speedup":
// the neighbours of a node's points that lie outside it are sampled first).
//
//  * k_knn_boxes, k_knn_box_up: the bounding box of every run of kKnnRun
//    consecutive tree positions (the tree keeps such runs spatially
//    compact), and a binary tree of boxes over the runs.
//  * k_knn: exact all-kappa-nearest neighbours, one wave per 64 query
//    points.  The wave walks the box tree depth first, nearer child first;
//    a subtree is skipped when, for every lane, the distance from its query
//    to the subtree's box is above the lane's current kappa-th distance
//    (with a 1e-12 relative margin that covers the rounding of both
//    distances); the points of the runs reached are staged in LDS and
//    compared one by one (the number of points compared, per wave, is
//    counted in `visits`).  Each lane keeps its sorted
//    list (squared distance, position) in registers and inserts by a fixed,
//    branch-free pass over it, so the result does not depend on the visiting
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

__device__ inline bool nn_before(double da, int ia, double db, int ib) { return (da < db) | ((da == db) & (ia < ib)); }

// thread -> (run, dimension): min and max of the run's coordinates, stored
// in FP32 rounded outward (the box can only grow, so the distance bounds
// stay lower bounds)
__device__ inline float round_down_f(double v) {
    float f = (float)v;
    return (double)f > v ? nextafterf(f, -INFINITY) : f;
}
__device__ inline float round_up_f(double v) {
    float f = (float)v;
    return (double)f < v ? nextafterf(f, INFINITY) : f;
}
__global__ void k_knn_boxes(const double *__restrict__ Xp, int64_t N, int d, int dpad, float *__restrict__ lo,
                            float *__restrict__ hi) {
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
    lo[g] = round_down_f(a);
    hi[g] = round_up_f(b);
}

// box of node i of a level of the box tree: the union of its children 2i
// and 2i + 1 (when it exists) on the level below; boxes at stride dpad
__global__ void k_knn_box_up(float *__restrict__ lo, float *__restrict__ hi, int64_t below, int64_t nbelow,
                             int64_t at, int64_t nat, int dpad) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nat * dpad) return;
    const int64_t i = g / dpad;
    const int k = (int)(g % dpad);
    const int64_t c0 = below + 2 * i, c1 = 2 * i + 1 < nbelow ? c0 + 1 : c0;
    lo[(at + i) * dpad + k] = fmin(lo[c0 * dpad + k], lo[c1 * dpad + k]);
    hi[(at + i) * dpad + k] = fmax(hi[c0 * dpad + k], hi[c1 * dpad + k]);
}

// K: list length kept in registers (>= kappa); DIM: coordinates per point
// held (>= d, zero padded).  Points are read from Xp at stride d.  The runs'
// boxes form a binary tree (level 0: the runs; node i of level l covers runs
// i 2^l .. (i + 1) 2^l - 1; boxes at stride DIM, level l from levoff[l]).
// The wave walks it depth first from the root, the child nearer to its own
// run first: a node is skipped when every lane's query is farther from its
// box than the lane's current kappa-th distance (with the 1e-12 margin); a
// run that is not skipped has its points staged in LDS and compared.  The
// stack (node = level << 26 | index) lives in the lanes' registers.
// points compared together (independent distance chains): four for short
// lists of points of at most 16 coordinates; one otherwise, where four (or
// two) leave one wave per SIMD or spill the list
template <int K, int DIM> constexpr int knn_group() { return K <= 16 && DIM <= 16 ? 4 : 1; }

template <int K, int DIM>
__global__ __launch_bounds__(64) void k_knn(const double *__restrict__ Xp, int64_t N, int d,
                                            const float *__restrict__ lo, const float *__restrict__ hi,
                                            const int64_t *__restrict__ levoff, int top, int kappa,
                                            int32_t *__restrict__ out, unsigned long long *__restrict__ visits) {
    __shared__ double sp[kKnnRun * DIM];  // points of the run being compared
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
    constexpr int kIdxBits = 26;
    int stk = 0, nst = 0;  // lane t holds stack entry t; nst is uniform
    auto push = [&](int lvl, int64_t idx) {
        if (lane == nst) stk = (lvl << kIdxBits) | (int)idx;
        nst++;
    };
    push(top, 0);
    while (nst > 0) {
        nst--;
        const int node = __builtin_amdgcn_readlane(stk, nst);
        const int lvl = node >> kIdxBits;
        const int64_t idx = node & ((1 << kIdxBits) - 1);
        // lower bound of the squared distance from this lane's query to the box
        const float *bl = lo + (levoff[lvl] + idx) * DIM, *bh = hi + (levoff[lvl] + idx) * DIM;
        double lb = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; k++) {
            const double g = fmax(fmax((double)bl[k] - x[k], x[k] - (double)bh[k]), 0.0);
            lb = fma(g, g, lb);
        }
        if (!__any(live && !(lb * (1.0 - 1e-12) > ld[K - 1]))) continue;
        if (lvl > 0) {
            // children on the level below: the one nearer to this wave's own
            // run goes on top of the stack
            const int64_t c0 = 2 * idx, c1 = 2 * idx + 1;
            const int64_t nbelow = levoff[lvl] - levoff[lvl - 1];
            const bool right_near = (r0 >> (lvl - 1)) > c0;
            if (c1 < nbelow) {
                if (right_near) {
                    push(lvl - 1, c0);
                    push(lvl - 1, c1);
                } else {
                    push(lvl - 1, c1);
                    push(lvl - 1, c0);
                }
            } else {
                push(lvl - 1, c0);
            }
            continue;
        }
        const int64_t j0 = idx * kKnnRun;
        const int nj = nrun - 1 == idx ? (int)(N - j0) : kKnnRun;
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
                    // in place, from the end: entry t takes entry t - 1 when
                    // the new pair goes before both, the new pair when it
                    // goes before entry t only
                    const double cd = r2[p];
                    bool bt = true;
#pragma unroll
                    for (int t = K - 1; t > 0; t--) {
                        const bool bp = nn_before(cd, j, ld[t - 1], li[t - 1]);
                        const double nd = bp ? ld[t - 1] : cd;
                        const int ni = bp ? li[t - 1] : j;
                        ld[t] = bt ? nd : ld[t];
                        li[t] = bt ? ni : li[t];
                        bt = bp;
                    }
                    ld[0] = bt ? cd : ld[0];
                    li[0] = bt ? j : li[0];
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

template __global__ void k_knn<8, 16>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<16, 16>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<32, 16>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<64, 16>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<8, 32>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<16, 32>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<32, 32>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<64, 32>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<8, 64>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<16, 64>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);
template __global__ void k_knn<32, 64>(const double *, int64_t, int, const float *, const float *,
                                             const int64_t *, int, int, int32_t *, unsigned long long *);

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
