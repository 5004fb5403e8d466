// k_tree.hip -- level-by-level tree build on the GPU (Sec. 2.1, "Partitioning
// the matrix": binary tree, equal halves split by a hyperplane).
//
// Split rule of every node [b, e): the hyperplane through the median of the
// node's points along their principal axis.  Each reduction has a fixed
// order so that the permutation is a deterministic function of the input:
//   * sums over positions run left to right inside chunks of 256 positions;
//     chunk partials are combined by pairwise halving (p[i] = p[2i] + p[2i+1],
//     an odd tail passes through);
//   * the mean comes first, then the scatter matrix of the centred points;
//   * the axis is 50 power iterations from the normalised all-ones vector
//     (products summed in increasing index), made unique in sign by making
//     its entry of largest magnitude (lowest index on ties) positive;
//   * projection keys p = fma(x_k - mu_k, v_k, p) over k = 0..d-1;
//   * points are ordered by (key, original index); the left child takes the
//     first floor(n/2).
// This file is compiled with FP contraction off: every rounding is explicit.
#include "askit_dev.h"

namespace askit {

// --- chunk sums of the coordinates -------------------------------------------
// thread -> (node, chunk, dim); nodes of one level: ranges nb/ne[first + j]
__global__ void k_tree_chunk_mean(const double *__restrict__ X, const int64_t *__restrict__ perm, int d,
                                  const int64_t *__restrict__ nb, const int64_t *__restrict__ ne, int64_t first,
                                  int cnt, int maxch, double *__restrict__ part) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)cnt * maxch * d) return;
    int k = (int)(t % d);
    int64_t r = t / d;
    int c = (int)(r % maxch);
    int node = (int)(r / maxch);
    int64_t b = nb[first + node], e = ne[first + node];
    int64_t c0 = b + (int64_t)c * kTreeChunk;
    if (c0 >= e) return;
    int64_t c1 = c0 + kTreeChunk < e ? c0 + kTreeChunk : e;
    double acc = 0.0;
    for (int64_t i = c0; i < c1; i++) acc = acc + X[perm[i] * d + k];
    part[((int64_t)node * maxch + c) * d + k] = acc;
}

// pairwise halving of nch partials (stride `stride` apart), in place
__device__ double pairwise_total(double *p, int64_t nch, int stride) {
    while (nch > 1) {
        int64_t h = (nch + 1) / 2;
        for (int64_t i = 0; i < h; i++)
            p[i * stride] = (2 * i + 1 < nch) ? p[2 * i * stride] + p[(2 * i + 1) * stride] : p[2 * i * stride];
        nch = h;
    }
    return p[0];
}

// thread -> (node, dim): mean of the node's points
__global__ void k_tree_mean(const int64_t *__restrict__ nb, const int64_t *__restrict__ ne, int64_t first, int cnt,
                            int maxch, int d, double *__restrict__ part, double *__restrict__ mu) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt * d) return;
    int node = t / d, k = t % d;
    int64_t n = ne[first + node] - nb[first + node];
    int64_t nch = (n + kTreeChunk - 1) / kTreeChunk;
    double tot = pairwise_total(part + (int64_t)node * maxch * d + k, nch, d);
    mu[t] = tot / (double)n;
}

// thread -> (node, chunk, pair a <= c): chunk sums of centred products
__global__ void k_tree_chunk_scatter(const double *__restrict__ X, const int64_t *__restrict__ perm, int d,
                                     const int64_t *__restrict__ nb, const int64_t *__restrict__ ne, int64_t first,
                                     int cnt, int maxch, const double *__restrict__ mu, const int16_t *__restrict__ pa,
                                     const int16_t *__restrict__ pc, int npair, double *__restrict__ part) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)cnt * maxch * npair) return;
    int q = (int)(t % npair);
    int64_t r = t / npair;
    int c = (int)(r % maxch);
    int node = (int)(r / maxch);
    int64_t b = nb[first + node], e = ne[first + node];
    int64_t c0 = b + (int64_t)c * kTreeChunk;
    if (c0 >= e) return;
    int64_t c1 = c0 + kTreeChunk < e ? c0 + kTreeChunk : e;
    int a = pa[q], cc = pc[q];
    double ma = mu[node * d + a], mc = mu[node * d + cc];
    double acc = 0.0;
    for (int64_t i = c0; i < c1; i++) {
        const double *x = X + perm[i] * d;
        double prod = (x[a] - ma) * (x[cc] - mc);
        acc = acc + prod;
    }
    part[((int64_t)node * maxch + c) * npair + q] = acc;
}

// thread -> (node, pair): scatter matrix entry by pairwise halving
__global__ void k_tree_scatter(const int64_t *__restrict__ nb, const int64_t *__restrict__ ne, int64_t first, int cnt,
                               int maxch, int d, const int16_t *__restrict__ pa, const int16_t *__restrict__ pc,
                               int npair, double *__restrict__ part, double *__restrict__ S) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt * npair) return;
    int node = t / npair, q = t % npair;
    int64_t n = ne[first + node] - nb[first + node];
    int64_t nch = (n + kTreeChunk - 1) / kTreeChunk;
    double v = pairwise_total(part + (int64_t)node * maxch * npair + q, nch, npair);
    double *Sn = S + (int64_t)node * d * d;
    Sn[pa[q] * d + pc[q]] = v;
    Sn[pc[q] * d + pa[q]] = v;
}

// thread -> node: power iteration, sign rule -> axis v
__global__ void k_tree_axis(int cnt, int d, const double *__restrict__ S, double *__restrict__ axis) {
    int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= cnt) return;
    const double *Sn = S + (int64_t)node * d * d;
    double v[kMaxDim], w[kMaxDim];
    double v0 = 1.0 / sqrt((double)d);
    for (int k = 0; k < d; k++) v[k] = v0;
    for (int it = 0; it < kPowerIters; it++) {
        for (int i = 0; i < d; i++) {
            double acc = 0.0;
            for (int j = 0; j < d; j++) acc = acc + Sn[i * d + j] * v[j];
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
    double sg = v[kmax] < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < d; k++) axis[node * d + k] = sg * v[k];
}

// block (x: positions of a node, y-linear: node) -> keys and original ids
__global__ void k_tree_keys(const double *__restrict__ X, const int64_t *__restrict__ perm, int d,
                            const int64_t *__restrict__ nb, const int64_t *__restrict__ ne, int64_t first,
                            int blocks_per_node, const double *__restrict__ mu, const double *__restrict__ axis,
                            double *__restrict__ key, int64_t *__restrict__ kid) {
    int node = blockIdx.x / blocks_per_node;
    int64_t i = nb[first + node] + (int64_t)(blockIdx.x % blocks_per_node) * blockDim.x + threadIdx.x;
    if (i >= ne[first + node]) return;
    int64_t id = perm[i];
    const double *x = X + id * d;
    const double *m = mu + node * d, *v = axis + node * d;
    double p = 0.0;
    for (int k = 0; k < d; k++) p = __builtin_fma(x[k] - m[k], v[k], p);
    key[i] = p;
    kid[i] = id;
}

__device__ inline bool kless(double ka, int64_t ia, double kb, int64_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// bitonic sort of tiles of up to 1024 positions inside each node
constexpr int kSortTile = 1024;

__global__ __launch_bounds__(512) void k_tree_sort_tiles(const int64_t *__restrict__ nb, const int64_t *__restrict__ ne,
                                                         int64_t first, int tiles_per_node, double *__restrict__ key,
                                                         int64_t *__restrict__ kid) {
    __shared__ double sk[kSortTile];
    __shared__ int64_t si[kSortTile];
    int node = blockIdx.x / tiles_per_node;
    int64_t b = nb[first + node], e = ne[first + node];
    int64_t t0 = b + (int64_t)(blockIdx.x % tiles_per_node) * kSortTile;
    if (t0 >= e) return;
    int len = (int)((e - t0) < kSortTile ? (e - t0) : kSortTile);
    for (int i = threadIdx.x; i < kSortTile; i += blockDim.x) {
        if (i < len) {
            sk[i] = key[t0 + i];
            si[i] = kid[t0 + i];
        } else {
            sk[i] = INFINITY;
            si[i] = INT64_MAX;
        }
    }
    __syncthreads();
    for (int k = 2; k <= kSortTile; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < kSortTile; i += blockDim.x) {
                int l = i ^ j;
                if (l > i) {
                    bool up = (i & k) == 0;
                    bool gt = kless(sk[l], si[l], sk[i], si[i]);
                    if (gt == up) {
                        double tk = sk[i]; sk[i] = sk[l]; sk[l] = tk;
                        int64_t ti = si[i]; si[i] = si[l]; si[l] = ti;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < len; i += blockDim.x) {
        key[t0 + i] = sk[i];
        kid[t0 + i] = si[i];
    }
}

// merge pass: runs of width w (relative to the node start) are merged in
// pairs; every element finds its output slot by a binary search in the
// other run (keys are unique thanks to the index tie-break)
__global__ void k_tree_merge(const int64_t *__restrict__ nb, const int64_t *__restrict__ ne, int64_t first,
                             int blocks_per_node, int64_t w, const double *__restrict__ ki,
                             const int64_t *__restrict__ ii, double *__restrict__ ko, int64_t *__restrict__ io) {
    int node = blockIdx.x / blocks_per_node;
    int64_t b = nb[first + node], e = ne[first + node];
    int64_t li = (int64_t)(blockIdx.x % blocks_per_node) * blockDim.x + threadIdx.x;
    int64_t n = e - b;
    if (li >= n) return;
    int64_t pb = (li / (2 * w)) * (2 * w);
    int64_t aend = pb + w < n ? pb + w : n;
    int64_t bend = pb + 2 * w < n ? pb + 2 * w : n;
    double k = ki[b + li];
    int64_t id = ii[b + li];
    int64_t out;
    if (li < aend) {  // in run A: count elements of B smaller
        int64_t lo = aend, hi = bend;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (kless(ki[b + mid], ii[b + mid], k, id)) lo = mid + 1;
            else hi = mid;
        }
        out = li + (lo - aend);
    } else {  // in run B: count elements of A smaller
        int64_t lo = pb, hi = aend;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (kless(ki[b + mid], ii[b + mid], k, id)) lo = mid + 1;
            else hi = mid;
        }
        out = pb + (li - aend) + (lo - pb);
    }
    ko[b + out] = k;
    io[b + out] = id;
}

__global__ void k_copy_ids(const int64_t *__restrict__ src, int64_t *__restrict__ dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Xp[pos] = X[perm[pos]]
__global__ void k_gather_points(const double *__restrict__ X, const int64_t *__restrict__ perm, int d, int64_t N,
                                double *__restrict__ Xp) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * d) return;
    int64_t i = t / d;
    int k = (int)(t % d);
    Xp[t] = X[perm[i] * d + k];
}

// node ranges of the complete tree of depth D over N positions (heap order):
// from the root down, the left child takes floor(n / 2); one thread per node
__global__ void k_node_ranges(int64_t *__restrict__ nb, int64_t *__restrict__ ne, int64_t N, int D) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= ((int64_t)2 << D) - 1) return;
    int l = 0;
    while ((((int64_t)2 << l) - 1) <= id) l++;
    const int64_t j = id - (((int64_t)1 << l) - 1);
    int64_t b = 0, n = N;
    for (int k = l - 1; k >= 0; k--) {
        if ((j >> k) & 1) {
            b += n / 2;
            n -= n / 2;
        } else {
            n /= 2;
        }
    }
    nb[id] = b;
    ne[id] = b + n;
}

// index pairs (a, c), a <= c, of the scatter matrix's upper triangle, row by
// row: pair i -> (pa[i], pc[i])
__global__ void k_pair_index(int16_t *__restrict__ pa, int16_t *__restrict__ pc, int d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d * (d + 1) / 2) return;
    int a = 0, first = 0;
    while (first + (d - a) <= i) {
        first += d - a;
        a++;
    }
    pa[i] = (int16_t)a;
    pc[i] = (int16_t)(a + (i - first));
}

__global__ void k_iota(int64_t *__restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

// finite-ness check of the input coordinates
__global__ void k_check_finite(const double *__restrict__ X, int64_t n, int32_t *__restrict__ bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(X[i])) atomicOr(bad, 1);
}

}  // namespace askit
