// k_skel.hip -- skeletonization kernels (Sec. 2.1, "Computing low rank
// approximations"; Alg. 1; the ID of eq. (4)).
//
//  * k_sample: the sampled rows S' of a node: min(nsamp, N - n) distinct
//    positions outside the node, drawn uniformly with SplitMix64 (Steele, Lea
//    & Flood 2014) from the node's own stream, duplicates rejected; when the
//    complement has at most nsamp positions it is taken whole, in order.
//  * k_sample_block: the kernel block K(X_S', X_C) in FP64, column-major
//    (levels factored by the split QR).
//  * k_sample_rownorm: for the levels factored by k_qrcp, only the squared
//    row norms of that block in groups of kQsCols columns; k_qrcp generates
//    the rows it keeps itself.
//  * k_qrcp: column-pivoted Householder QR of that block, truncated at the
//    rank s (trailing column norms recomputed at every step, largest norm
//    first, lowest column on ties), the rank guard |R_jj| <= 1e-14 |R_00|,
//    the adaptive rank rule |R_jj| < tol |R_00| when tol > 0 (the ratio of
//    singular values of Sec. 2.1, estimated by R's diagonal),
//    T = R11^{-1} R12 and the projection P = [I T] Pi^T, written transposed.
#include "askit_dev.h"

#include <type_traits>

namespace askit {

// ---------------------------------------------------------------------------
// sampling: one wave per node.  The node's neighbour list (kappa-NN
// sampling), if any, opens the sample.  Draw i (i = 1, 2, ..) of the node's stream is
// the SplitMix64 output of state + i * gamma, so the 64 lanes take 64
// consecutive draws per round.  A draw is kept when its point was drawn
// neither in an earlier round (open-addressing set in LDS) nor by a lower
// lane of this round; kept draws go out in draw order until nsamp are held.
// ---------------------------------------------------------------------------
constexpr int kSampHashBits = 13;  // 8192 slots: nsamp <= 4096
constexpr uint64_t kSplitMixGamma = 0x9E3779B97F4A7C15ULL;

__device__ inline uint64_t splitmix_at(uint64_t state, uint64_t i) {
    uint64_t z = state + i * kSplitMixGamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(64) void k_sample(const SampTask *__restrict__ tasks, int nsamp, int32_t *__restrict__ err) {
    __shared__ int32_t table[1 << kSampHashBits];
    constexpr uint32_t mask = (1u << kSampHashBits) - 1u;
    const SampTask t = tasks[blockIdx.x];
    const int64_t n = t.e - t.b, c = t.N - n;
    const int lane = threadIdx.x;
    if (c <= nsamp) {
        for (int64_t i = lane; i < c; i += kWave) t.out[i] = (int32_t)(i < t.b ? i : i + n);
        return;
    }
    for (int i = lane; i < (1 << kSampHashBits); i += kWave) table[i] = 0;
    __syncthreads();
    // the neighbour list opens the sample (distinct positions outside the
    // node); its positions join the set, so draws that repeat them are
    // rejected like repeated draws
    const int npre = t.npre < nsamp ? t.npre : nsamp;
    for (int i = lane; i < npre; i += kWave) {
        const int32_t pos = t.pre[i];
        t.out[i] = pos;
        const uint32_t key = (uint32_t)pos + 1u;
        for (uint32_t sl = (uint32_t)(((uint64_t)pos * kSplitMixGamma) >> (64 - kSampHashBits));; sl = (sl + 1) & mask)
            if (atomicCAS(&table[sl], 0, (int32_t)key) == 0) break;
    }
    __syncthreads();
    // at most cap draws (a stream that cannot fill the sample is an error)
    const uint64_t cap = 64ULL * (uint64_t)(c + nsamp);
    int k = npre;
    for (uint64_t base = 0; k < nsamp; base += kWave) {
        const uint64_t i = base + (uint64_t)lane + 1;
        const bool valid = i <= cap;
        const uint64_t r = __umul64hi(splitmix_at(t.state, i), (uint64_t)c);
        const int64_t pos = (int64_t)r < t.b ? (int64_t)r : (int64_t)r + n;
        const uint32_t key = (uint32_t)pos + 1u;
        const uint32_t slot = (uint32_t)(((uint64_t)pos * kSplitMixGamma) >> (64 - kSampHashBits));
        bool fresh = valid;
        if (valid) {
            for (uint32_t sl = slot;; sl = (sl + 1) & mask) {
                const int32_t v = table[sl];
                if (v == 0) break;
                if ((uint32_t)v == key) {
                    fresh = false;
                    break;
                }
            }
        }
        for (int u = 0; u < kWave - 1; u++) {
            const uint32_t ku = (uint32_t)__builtin_amdgcn_readlane((int)key, u);
            if (u < lane && ku == key) fresh = false;
        }
        const unsigned long long bal = __ballot(fresh);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        const int need = nsamp - k;
        if (fresh && before < need) {
            t.out[k + before] = (int32_t)pos;
            // the keys of a round are distinct and absent from the set
            for (uint32_t sl = slot;; sl = (sl + 1) & mask)
                if (atomicCAS(&table[sl], 0, (int32_t)key) == 0) break;
        }
        __syncthreads();
        const int got = __popcll(bal);
        k += got < need ? got : need;
        if (k < nsamp && base + kWave >= cap) {
            if (lane == 0) atomicOr(err, 1);
            break;
        }
    }
}

// ---------------------------------------------------------------------------
// sampled kernel block M = K(X_S', X_C), column-major (ldm rows)
// ---------------------------------------------------------------------------
__device__ inline int32_t cand_pos(const SkelTask &t, int c, int sl) {
    if (t.leaf) return (int32_t)(t.b + c);
    return c < sl ? glb(t.skl)[c] : glb(t.skr)[c - sl];
}

__device__ inline double sqdist(const double *x, const double *y, int d) {
    double r2 = 0.0;
    for (int k = 0; k < d; k++) {
        double df = x[k] - y[k];
        r2 = fma(df, df, r2);
    }
    return r2;
}

// the same sum over kXrDim coordinates, the row point y in registers and the
// column point x in LDS, both zero padded beyond d (the padded terms add
// exact zeros, so the value is sqdist's bit for bit)
__device__ inline double sqdist_xr(const double *x, const double (&y)[kXrDim]) {
    double r2 = 0.0;
#pragma unroll
    for (int k = 0; k < kXrDim; k++) {
        const double df = x[k] - y[k];
        r2 = fma(df, df, r2);
    }
    return r2;
}

// tile staging of the sampled-block kernels: row points at an odd stride
// (lanes read different points: no bank conflicts), column points at
// stride xs_stride(d) (one point per wave: broadcast), zero padded to
// kXrDim coordinates for d <= kXrDim, when the row point is then read into
// registers once per thread
__device__ inline int xs_stride(int d) { return d <= kXrDim ? kXrDim : d; }

// block: 256 threads on a 64 x 64 tile (sampled rows x candidate columns);
// both point sets are staged in LDS, each thread writes 16 entries of one
// column (consecutive rows across lanes: coalesced column-major stores)
__global__ __launch_bounds__(256) void k_sample_block(const SkelTask *__restrict__ tasks, int rowtiles, int ldm, int d,
                                                      int coltiles) {
    extern __shared__ double dyn_lds[];  // 64 (d | 1) + 64 xs_stride(d) doubles
    const int dp = d | 1, xw = xs_stride(d);
    double *ys = dyn_lds, *xs = dyn_lds + 64 * dp;
    const int per = rowtiles * coltiles;
    const int task = blockIdx.x / per, rt = (blockIdx.x % per) % rowtiles, ct = (blockIdx.x % per) / rowtiles;
    const SkelTask t = tasks[task];
    const int r0 = rt * 64, c0 = ct * 64;
    const int sl = t.leaf ? 0 : *glb(t.srl);
    const int ncand = t.leaf ? t.n : sl + *glb(t.srr);
    const GLB double *X = glb(t.X);
    const GLB int32_t *q = glb(t.q);
    if (r0 >= t.nq || c0 >= ncand) return;
    const int nr = min(64, t.nq - r0), nc = min(64, ncand - c0);
    for (int i = threadIdx.x; i < 64 * d; i += blockDim.x) {
        const int a = i / d, k = i % d;
        ys[a * dp + k] = a < nr ? X[(int64_t)q[r0 + a] * d + k] : 0.0;
    }
    for (int i = threadIdx.x; i < 64 * xw; i += blockDim.x) {
        const int a = i / xw, k = i % xw;
        xs[i] = (a < nc && k < d) ? X[(int64_t)cand_pos(t, c0 + a, sl) * d + k] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x % 64;
    if (r >= nr) return;
    const double *y = ys + r * dp;
    if (d <= kXrDim) {
        double yr[kXrDim];
#pragma unroll
        for (int k = 0; k < kXrDim; k++) yr[k] = k < d ? y[k] : 0.0;
        for (int c = threadIdx.x / 64; c < nc; c += 4)
            glb(t.M)[(int64_t)(c0 + c) * ldm + r0 + r] = exp(sqdist_xr(xs + c * kXrDim, yr) * t.scale);
    } else {
        for (int c = threadIdx.x / 64; c < nc; c += 4)
            glb(t.M)[(int64_t)(c0 + c) * ldm + r0 + r] = exp(sqdist(xs + c * d, y, d) * t.scale);
    }
}

// The one-workgroup QR's input: instead of the block, the squared norm of
// each row over each group of kQsCols columns (g = 0, kQsCols, ...; the sums
// row_part forms, in the same order), written as entry (row i, column
// g / kQsCols) of the node's block.  Same tiling, staging and entries as
// k_sample_block; a thread forms the group sums of one row.  The block itself
// is never stored: k_qrcp generates the rows that carry weight (gen_rows).
__global__ __launch_bounds__(256) void k_sample_rownorm(const SkelTask *__restrict__ tasks, int rowtiles, int ldm,
                                                        int d, int coltiles) {
    extern __shared__ double dyn_lds[];  // 64 (d | 1) + 64 xs_stride(d) doubles
    const int dp = d | 1, xw = xs_stride(d);
    double *ys = dyn_lds, *xs = dyn_lds + 64 * dp;
    const int per = rowtiles * coltiles;
    const int task = blockIdx.x / per, rt = (blockIdx.x % per) % rowtiles, ct = (blockIdx.x % per) / rowtiles;
    const SkelTask t = tasks[task];
    const int r0 = rt * 64, c0 = ct * 64;
    const int sl = t.leaf ? 0 : *glb(t.srl);
    const int ncand = t.leaf ? t.n : sl + *glb(t.srr);
    const GLB double *X = glb(t.X);
    const GLB int32_t *q = glb(t.q);
    if (r0 >= t.nq || c0 >= ncand) return;
    const int nr = min(64, t.nq - r0), nc = min(64, ncand - c0);
    for (int i = threadIdx.x; i < 64 * d; i += blockDim.x) {
        const int a = i / d, k = i % d;
        ys[a * dp + k] = a < nr ? X[(int64_t)q[r0 + a] * d + k] : 0.0;
    }
    for (int i = threadIdx.x; i < 64 * xw; i += blockDim.x) {
        const int a = i / xw, k = i % xw;
        xs[i] = (a < nc && k < d) ? X[(int64_t)cand_pos(t, c0 + a, sl) * d + k] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x % 64;
    if (r >= nr) return;
    const double *y = ys + r * dp;
    double yr[kXrDim];
#pragma unroll
    for (int k = 0; k < kXrDim; k++) yr[k] = (d <= kXrDim && k < d) ? y[k] : 0.0;
    for (int cg = (threadIdx.x / 64) * kQsCols; cg < nc; cg += 4 * kQsCols) {
        double v[kQsCols];
        if (d <= kXrDim) {
#pragma unroll
            for (int u = 0; u < kQsCols; u++)
                v[u] = cg + u < nc ? exp(sqdist_xr(xs + (cg + u) * kXrDim, yr) * t.scale) : 0.0;
        } else {
#pragma unroll
            for (int u = 0; u < kQsCols; u++) v[u] = cg + u < nc ? exp(sqdist(xs + (cg + u) * d, y, d) * t.scale) : 0.0;
        }
        double p = 0.0;
#pragma unroll
        for (int u = 0; u < kQsCols; u++)
            if (cg + u < nc) p = fma(v[u], v[u], p);
        glb(t.M)[(int64_t)((c0 + cg) / kQsCols) * ldm + r0 + r] = p;
    }
}

// ---------------------------------------------------------------------------
// QRCP + interpolative decomposition.  Two launch shapes share every piece of
// arithmetic below, so they give bit-identical skeletons:
//  * k_qrcp: one 512-thread workgroup per node (levels with many nodes);
//  * k_qs_*: several workgroups per node, one launch per pivot step (levels
//    with few nodes, where one workgroup per node would leave the GPU idle).
// ---------------------------------------------------------------------------
constexpr int kQrThreads = 512;
constexpr int kQrWaves = kQrThreads / kWave;
constexpr int kQsWaves = kQsThreads / kWave;
static_assert(kQsCols == 2 * kQsWaves, "two columns per wave in the split form");

__device__ inline double wave_sum(double v) { return wave_sum_d(v); }

// block-wide sum over kQrThreads threads (all get the result); red: kQrWaves
__device__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < kQrWaves; i++) s += red[i];
    return s;
}

// LDS budget: norms and pivots per candidate column, Householder vector
constexpr int kQrMaxCols = 2048;
constexpr int kQrMaxRows = 4096;
constexpr int kQrMaxRank = 256;
// positions per lane in the split step's pivot scan (2 kQrMaxRank candidates)
constexpr int kQsScan = 2 * kQrMaxRank / kWave;

__device__ inline int node_ncand(const SkelTask &t) { return t.leaf ? t.n : *glb(t.srl) + *glb(t.srr); }

// squared norm of row i over the columns [c0, c1) of the block
template <typename PM>
__device__ inline double row_part(PM M, int ldm, int i, int c0, int c1) {
    double v[kQsCols];
#pragma unroll
    for (int u = 0; u < kQsCols; u++) v[u] = c0 + u < c1 ? M[(int64_t)(c0 + u) * ldm + i] : 0.0;
    double p = 0.0;
#pragma unroll
    for (int u = 0; u < kQsCols; u++)
        if (c0 + u < c1) p = fma(v[u], v[u], p);
    return p;
}

// Rows of the sampled block whose squared norm is below 1e-44 of the block's
// squared Frobenius norm are dropped (the rest keep their order).  Taken
// together (at most 4096 rows) they are a perturbation of the block of
// Frobenius norm below 6.4e-21 of the block's, some 17,000 times smaller than
// the backward error FP64 Householder QR commits anyway (at least the unit
// roundoff 1.1e-16 times the block's norm), so the pivots, R and T are those
// of the whole block up to rounding; the trailing updates then stream only
// the rows that carry the interaction.  rn: squared row norms (summed over
// groups of kQsCols columns in order); all kQrThreads threads call this;
// returns the number of kept rows and fills rmap (new index or -1).
template <typename PR, typename PI>
__device__ inline int row_map(PR rn, int rows, PI rmap, int32_t *wcnt, double *red) {
    typedef typename std::remove_cv<typename std::remove_reference<decltype(rmap[0])>::type>::type IT;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    double part = 0.0;
    for (int i = tid; i < rows; i += kQrThreads) part += rn[i];
    const double thr = 1e-44 * block_sum(part, red);
    int kept = 0;
    for (int base = 0; base < rows; base += kQrThreads) {
        const int i = base + tid;
        const bool keep = i < rows && rn[i] > thr;
        const unsigned long long bal = __ballot(keep);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[wave] = __popcll(bal);
        __syncthreads();
        int wofs = 0, tot = 0;
        for (int w = 0; w < kQrWaves; w++) {
            if (w < wave) wofs += wcnt[w];
            tot += wcnt[w];
        }
        if (i < rows) rmap[i] = (IT)(keep ? kept + wofs + below : -1);
        kept += tot;
        __syncthreads();
    }
    return kept;
}

// in-place compaction of one column by one wave: rows only move up, and a
// wave reads a block of 1024 rows (16 per lane) before writing it
template <typename PC, typename PI>
__device__ inline void compact_col(PC col, PI rmap, int rows, int lane) {
    for (int base = 0; base < rows; base += 16 * kWave) {
        double v[16];
#pragma unroll
        for (int t = 0; t < 16; t++) {
            const int i = base + lane + t * kWave;
            v[t] = i < rows ? col[i] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 16; t++) {
            const int i = base + lane + t * kWave;
            const int dst = i < rows ? (int)rmap[i] : -1;
            if (dst >= 0) col[dst] = v[t];
        }
    }
}

// squared norm of rows [0, rows) of a column (one wave)
template <typename PC>
__device__ inline double col_norm(PC col, int rows, int lane) {
    double acc = 0.0;
    for (int base = 0; base < rows; base += 4 * kWave) {
        double v[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int i = base + lane + t * kWave;
            v[t] = i < rows ? col[i] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 4; t++)
            if (base + lane + t * kWave < rows) acc = fma(v[t], v[t], acc);
    }
    return wave_sum(acc);
}

// Householder reflector of pivot step j from the pivot column x (one wave):
// LAPACK convention beta = -sign(alpha) |x|, tau = (beta - alpha) / beta,
// v = x / (alpha - beta) below the diagonal.  Lane l sums the rows i > j with
// i = l mod 64 in increasing order.
struct Refl {
    double alpha, beta, tau, sc;
};
template <typename PX>
__device__ inline Refl reflector(PX x, int j, int rows, int lane) {
    double xn = 0.0;
    for (int i = lane; i < rows; i += kWave)
        if (i > j) xn = fma(x[i], x[i], xn);
    xn = wave_sum(xn);
    Refl r;
    r.alpha = x[j];
    if (xn == 0.0) {
        r.beta = r.alpha;
        r.tau = 0.0;
        r.sc = 0.0;
    } else {
        r.beta = -copysign(sqrt(r.alpha * r.alpha + xn), r.alpha);
        r.tau = (r.beta - r.alpha) / r.beta;
        r.sc = 1.0 / (r.alpha - r.beta);
    }
    return r;
}

// the same for rows - j <= 16 * 64 with the column's rows j + lane + 64 t
// kept in xv (zero past the rows): lane l sums the rows i > j with
// i = j + l mod 64, in increasing order
template <typename PX>
__device__ inline Refl reflector_reg(PX x, int j, int rows, int lane, double (&xv)[16]) {
#pragma unroll
    for (int t = 0; t < 16; t++) {
        const int i = j + lane + t * kWave;
        xv[t] = i < rows ? x[i] : 0.0;
    }
    double xn = 0.0;
#pragma unroll
    for (int t = 0; t < 16; t++) {
        const int i = j + lane + t * kWave;
        if (i > j && i < rows) xn = fma(xv[t], xv[t], xn);
    }
    xn = wave_sum(xn);
    Refl r;
    r.alpha = readlane_d(xv[0], 0);
    if (xn == 0.0) {
        r.beta = r.alpha;
        r.tau = 0.0;
        r.sc = 0.0;
    } else {
        r.beta = -copysign(sqrt(r.alpha * r.alpha + xn), r.alpha);
        r.tau = (r.beta - r.alpha) / r.beta;
        r.sc = 1.0 / (r.alpha - r.beta);
    }
    return r;
}

// reflector of pivot step j, its Householder vector written to vh (v_j = 1
// by the caller) unless the rank rule stops; returns whether it stops
template <typename PX>
__device__ inline Refl reflector_to_lds(PX x, int j, int rows, int lane, double r00, double tol, double *vh,
                                        bool &stop);

// the rank is j when |R_jj| falls to the guard 1e-14 |R_00| or below
// tol |R_00| (adaptive rank); a zero block stops at step 0 with rank 1
__device__ inline bool guard_stop(int j, double beta, double r00, double tol) {
    const double r0 = j == 0 ? fabs(beta) : r00;
    return (j > 0 && (fabs(beta) <= kRankGuard * r0 || fabs(beta) < tol * r0)) || (j == 0 && r0 == 0.0);
}

template <typename PX>
__device__ inline Refl reflector_to_lds(PX x, int j, int rows, int lane, double r00, double tol, double *vh,
                                        bool &stop) {
    if (rows - j <= 16 * kWave) {
        double xv[16];
        const Refl r = reflector_reg(x, j, rows, lane, xv);
        stop = guard_stop(j, r.beta, r00, tol);
        if (!stop) {
#pragma unroll
            for (int t = 0; t < 16; t++) {
                const int i = j + lane + t * kWave;
                if (i > j && i < rows) vh[i] = xv[t] * r.sc;
            }
        }
        return r;
    }
    const Refl r = reflector(x, j, rows, lane);
    stop = guard_stop(j, r.beta, r00, tol);
    if (!stop)
        for (int i = j + 1 + lane; i < rows; i += kWave) vh[i] = x[i] * r.sc;
    return r;
}

// apply H = I - tau v v^T (v in LDS, v_j = 1) to rows [j, rows) of one column
// (one wave) and return the new squared norm of its rows below j
template <typename PC>
__device__ inline double apply_col(PC col, const double *vh, int j, int rows, double tau, int lane) {
    if (rows - j <= 16 * kWave) {
        double a[16], vr[16];
#pragma unroll
        for (int t = 0; t < 16; t++) {
            const int i = j + lane + t * kWave;
            vr[t] = i < rows ? vh[i] : 0.0;
            a[t] = i < rows ? col[i] : 0.0;
        }
        double w = 0.0;
#pragma unroll
        for (int t = 0; t < 16; t++) w = fma(vr[t], a[t], w);
        w = wave_sum(w) * tau;
        double n = 0.0;
#pragma unroll
        for (int t = 0; t < 16; t++) {
            const int i = j + lane + t * kWave;
            a[t] = fma(-vr[t], w, a[t]);
            if (i > j && i < rows) n = fma(a[t], a[t], n);
        }
#pragma unroll
        for (int t = 0; t < 16; t++) {
            const int i = j + lane + t * kWave;
            if (i < rows) col[i] = a[t];
        }
        return wave_sum(n);
    }
    double w = 0.0;
    for (int i = j + lane; i < rows; i += kWave) w = fma(vh[i], col[i], w);
    w = wave_sum(w) * tau;
    double n = 0.0;
    for (int i = j + lane; i < rows; i += kWave) {
        const double v = fma(-vh[i], w, col[i]);
        col[i] = v;
        if (i > j) n = fma(v, v, n);
    }
    return wave_sum(n);
}

// the same update for NC columns at once (positions q0 + u qstride < qend):
// all their loads are issued before the first product; rows - j <= 64 NT.
// The per-column arithmetic is that of apply_col (chunks past the rows add
// exact zeros), so the grouping does not change any result.
template <int NT, int NC, typename PM, typename PP, typename PN>
__device__ inline void apply_group(PM M, int ldm, PP pos, int q0, int qstride, int qend, const double *vh, int j,
                                   int rows, double tau, int lane, PN nrm) {
    double vr[NT], a[NC][NT];
    int c[NC];
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int i = j + lane + t * kWave;
        vr[t] = i < rows ? vh[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NC; u++) {
        const int q = q0 + u * qstride;
        c[u] = q < qend ? pos[q] : -1;
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int i = j + lane + t * kWave;
            a[u][t] = (c[u] >= 0 && i < rows) ? M[(int64_t)c[u] * ldm + i] : 0.0;
        }
    }
#pragma unroll
    for (int u = 0; u < NC; u++) {
        if (c[u] < 0) break;
        double w = 0.0;
#pragma unroll
        for (int t = 0; t < NT; t++) w = fma(vr[t], a[u][t], w);
        w = wave_sum(w) * tau;
        double n = 0.0;
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int i = j + lane + t * kWave;
            a[u][t] = fma(-vr[t], w, a[u][t]);
            if (i > j && i < rows) n = fma(a[u][t], a[u][t], n);
        }
        auto col = M + (int64_t)c[u] * ldm;
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int i = j + lane + t * kWave;
            if (i < rows) col[i] = a[u][t];
        }
        n = wave_sum(n);
        if (lane == 0) nrm[c[u]] = n;
    }
}

template <int NT, int NC, typename PM, typename PP, typename PN>
__device__ inline void apply_all(PM M, int ldm, PP pos, int j, int ncand, const double *vh, int rows, double tau,
                                 int lane, int wave, PN nrm) {
    for (int q0 = j + 1 + wave; q0 < ncand; q0 += kQrWaves * NC)
        apply_group<NT, NC>(M, ldm, pos, q0, kQrWaves, ncand, vh, j, rows, tau, lane, nrm);
}

// T = R11^{-1} R12 and the rows of P_{C alpha~} that it fills, for the
// column groups g0, g0 + gstep, ... of kTq right-hand columns (positions
// rank + g ..); pos[q] = column at pivot position q, Rjj = diagonal of R.
// One wave per group: lane l holds the group's rows l + 64 u in registers;
// from the last row up, t_i = r_i / R_ii is taken from its lane and column i
// of R11 (rows 0 .. i-1 of column pos[i], contiguous, loaded one step ahead)
// updates the rows above.  The solved column is stored straight into its row
// of P (lanes along the row).
constexpr int kTq = 8;
constexpr int kTu = kQrMaxRank / kWave;
static_assert(kQrWaves * kTq == kQsFinishCols, "k_qs_finish column split");
__device__ inline int p_row(const SkelTask &t, int c, int s, int sl) {
    return t.leaf ? c : (c < sl ? c : s + (c - sl));
}
template <typename PM, typename PP, typename PR>
__device__ inline void id_solve_rows(const SkelTask &t, PM M, int ldm, int s, int sl, int ncand, int rank, bool zero,
                                     PP pos, PR Rjj, int g0, int gstep) {
    const int lane = threadIdx.x % kWave;
    const int nr = ncand - rank;
    for (int g = g0; g < nr; g += gstep) {
        double r[kTq][kTu];
        int cq[kTq];
#pragma unroll
        for (int u = 0; u < kTq; u++) {
            const int q = rank + g + u;
            cq[u] = q < ncand ? pos[q] : -1;
#pragma unroll
            for (int v = 0; v < kTu; v++) {
                const int k = lane + v * kWave;
                r[u][v] = (cq[u] >= 0 && k < rank && !zero) ? M[(int64_t)cq[u] * ldm + k] : 0.0;
            }
        }
        if (!zero) {
            double rk[kTu], rn[kTu];
            {
                const auto Ri = M + (int64_t)pos[rank - 1] * ldm;
#pragma unroll
                for (int v = 0; v < kTu; v++) {
                    const int k = lane + v * kWave;
                    rk[v] = k < rank - 1 ? Ri[k] : 0.0;
                }
            }
#pragma unroll
            for (int vi = kTu - 1; vi >= 0; vi--) {
                for (int src = kWave - 1; src >= 0; src--) {
                    const int i = vi * kWave + src;
                    if (i >= rank) continue;
                    if (i > 0) {
                        const auto Rn = M + (int64_t)pos[i - 1] * ldm;
#pragma unroll
                        for (int v = 0; v < kTu; v++) {
                            const int k = lane + v * kWave;
                            rn[v] = k < i - 1 ? Rn[k] : 0.0;
                        }
                    }
                    const double d = Rjj[i];
#pragma unroll
                    for (int u = 0; u < kTq; u++) {
                        const double ti = readlane_d(r[u][vi], src) / d;
                        if (lane == src) r[u][vi] = ti;
#pragma unroll
                        for (int v = 0; v <= vi; v++) r[u][v] = fma(-rk[v], ti, r[u][v]);
                    }
#pragma unroll
                    for (int v = 0; v < kTu; v++) rk[v] = rn[v];
                }
            }
        }
        // P is written in the rows of the candidates and the columns below
        // the rank only: nothing reads the rest of the padded slot
#pragma unroll
        for (int u = 0; u < kTq; u++) {
            if (cq[u] < 0) break;
            GLB double *row = glb(t.Pt) + (int64_t)p_row(t, cq[u], s, sl) * s;
#pragma unroll
            for (int v = 0; v < kTu; v++) {
                const int k = lane + v * kWave;
                if (k < rank) row[k] = r[u][v];
            }
        }
    }
}

// the skeleton positions, rank, truncation flag and the identity rows of P
// (one wave per row).  All kQrThreads threads.
template <typename PP>
__device__ inline void id_outputs(const SkelTask &t, int s, int sl, int ncand, int rank, PP pos) {
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    for (int k = tid; k < s; k += kQrThreads) glb(t.skel)[k] = k < rank ? cand_pos(t, pos[k], sl) : -1;
    if (tid == 0) {
        *glb(t.sr) = rank;
        *glb(t.trunc) = (rank < (s < ncand ? s : ncand)) ? 1 : 0;
    }
    for (int q = wave; q < rank; q += kQrWaves) {
        GLB double *row = glb(t.Pt) + (int64_t)p_row(t, pos[q], s, sl) * s;
        for (int k = lane; k < rank; k += kWave) row[k] = k == q ? 1.0 : 0.0;
    }
}

// pivot choice: largest norm over positions [j, ncand) (value nrm[pos[k]]),
// lowest position on ties; one wave, result in every lane
template <typename PN, typename PP>
__device__ inline int pick_pivot(PN nrm, PP pos, int j, int ncand, int lane) {
    double bv = -1.0;
    int bk = 0x7fffffff;
    for (int k = j + lane; k < ncand; k += kWave) {
        const double v = nrm[pos[k]];
        if (v > bv) {  // positions ascend within a lane: the first of equal norms stays
            bv = v;
            bk = k;
        }
    }
    const int k = wave_argmax(bv, bk);
    return k == 0x7fffffff ? j : k;  // no comparable norm (NaN): keep the order
}

// Rows of the sampled block generated in place, compacted: entry (k, c) =
// K(x of sampled row src[k], x of candidate c) for k < nk, by the arithmetic
// of k_sample_block (so the values are those the block would hold).  The
// candidate points are staged in xs (capacity xcap doubles) by chunks of
// xcap / d columns; each wave takes the chunk's columns wave, wave +
// kQrWaves, ...; lane l the rows l + 64 u.  For d <= kXrDim a lane keeps its
// row point in registers.  All kQrThreads threads call this.
template <typename PM, typename PS>
__device__ inline void gen_rows(const SkelTask &t, PM M, int ldm, int d, int sl, int ncand, PS src, int nk,
                                double *xs, int xcap) {
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const GLB double *X = glb(t.X);
    const GLB int32_t *q = glb(t.q);
    const int cc = xcap / d;
    for (int c0 = 0; c0 < ncand; c0 += cc) {
        const int nc = min(cc, ncand - c0);
        __syncthreads();
        for (int e = tid; e < nc * d; e += kQrThreads) xs[e] = X[(int64_t)cand_pos(t, c0 + e / d, sl) * d + e % d];
        __syncthreads();
        for (int k0 = 0; k0 < nk; k0 += kWave) {
            const int k = k0 + lane;
            const bool live = k < nk;
            const int64_t yrow = live ? (int64_t)q[src[k]] * d : 0;
            if (d <= kXrDim) {
                double y[kXrDim];
#pragma unroll
                for (int e = 0; e < kXrDim; e++) y[e] = e < d ? X[yrow + e] : 0.0;
                for (int c = wave; c < nc; c += kQrWaves) {
                    const double *xc = xs + c * d;
                    double r2 = 0.0;
#pragma unroll
                    for (int e = 0; e < kXrDim; e++)
                        if (e < d) {
                            const double df = xc[e] - y[e];
                            r2 = fma(df, df, r2);
                        }
                    if (live) M[(int64_t)(c0 + c) * ldm + k] = exp(r2 * t.scale);
                }
            } else {
                for (int c = wave; c < nc; c += kQrWaves) {
                    const double *xc = xs + c * d;
                    double r2 = 0.0;
                    for (int e = 0; e < d; e++) {
                        const double df = xc[e] - X[yrow + e];
                        r2 = fma(df, df, r2);
                    }
                    if (live) M[(int64_t)(c0 + c) * ldm + k] = exp(r2 * t.scale);
                }
            }
        }
    }
}

// squared norms of rows [0, rows) of the columns at positions 0 .. ncand-1
// (as col_norm, with the loads of eight columns issued together when
// rows <= 4 * kWave); one wave per column group
template <typename PM, typename PN>
__device__ inline void col_norms(PM M, int ldm, int ncand, int rows, PN nrm, int lane, int wave) {
    if (rows > 4 * kWave) {
        for (int c = wave; c < ncand; c += kQrWaves) {
            const double v = col_norm(M + (int64_t)c * ldm, rows, lane);
            if (lane == 0) nrm[c] = v;
        }
        return;
    }
    constexpr int G = 8;
    for (int c0 = wave; c0 < ncand; c0 += kQrWaves * G) {
        double v[G][4];
#pragma unroll
        for (int u = 0; u < G; u++) {
            const int c = c0 + u * kQrWaves;
#pragma unroll
            for (int t4 = 0; t4 < 4; t4++) {
                const int i = lane + t4 * kWave;
                v[u][t4] = (c < ncand && i < rows) ? M[(int64_t)c * ldm + i] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < G; u++) {
            const int c = c0 + u * kQrWaves;
            double acc = 0.0;
#pragma unroll
            for (int t4 = 0; t4 < 4; t4++)
                if (lane + t4 * kWave < rows) acc = fma(v[u][t4], v[u][t4], acc);
            acc = wave_sum(acc);
            if (lane == 0 && c < ncand) nrm[c] = acc;
        }
    }
}

// Nodes with |C| <= s: skeleton = candidates, P = I (all kQrThreads threads)
__device__ inline void qr_identity(const SkelTask &t, int s, int sl, int ncand) {
    const int tid = threadIdx.x;
    auto prow = [&](int c) { return t.leaf ? c : (c < sl ? c : s + (c - sl)); };
    for (int k = tid; k < s; k += kQrThreads) glb(t.skel)[k] = k < ncand ? cand_pos(t, k, sl) : -1;
    for (int64_t i = tid; i < (int64_t)ncand * ncand; i += kQrThreads) {
        const int c = (int)(i / ncand), k = (int)(i % ncand);
        glb(t.Pt)[(int64_t)prow(c) * s + k] = k == c ? 1.0 : 0.0;
    }
    if (tid == 0) {
        *glb(t.sr) = ncand;
        *glb(t.trunc) = 0;
    }
}

// Rows kept by the QR (R29): row norms from the group sums k_sample_rownorm
// left in the block's first columns, the row map, and src[k] = sampled row
// of kept row k (in vh, reused as int32).  Returns the rows in use: the kept
// ones, all rows when none is dropped, row 0 when every row is zero.  All
// kQrThreads threads; the block itself is not touched.
template <typename PM>
__device__ inline int qr_row_select(const SkelTask &t, PM M, int ldm, int ncand, double *vh, int16_t *rmap,
                                    int32_t *wcnt, double *red) {
    const int tid = threadIdx.x;
    int rows = t.nq;
    const int ngrp = (ncand + kQsCols - 1) / kQsCols;
    for (int i = tid; i < rows; i += kQrThreads) {
        double a = 0.0;
        for (int g0 = 0; g0 < ngrp; g0 += 16) {  // 16 loads in flight, then added in order
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; u++) v[u] = g0 + u < ngrp ? M[(int64_t)(g0 + u) * ldm + i] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; u++)
                if (g0 + u < ngrp) a += v[u];
        }
        vh[i] = a;
    }
    __syncthreads();
    const int kept = row_map(vh, rows, rmap, wcnt, red);
    int32_t *src = reinterpret_cast<int32_t *>(vh);  // the row norms are consumed
    for (int i = tid; i < rows; i += kQrThreads) {
        const int k = kept > 0 ? (int)rmap[i] : (i == 0 ? 0 : -1);
        if (k >= 0) src[k] = i;
    }
    if (kept < rows) rows = kept > 0 ? kept : 1;
    __syncthreads();
    return rows;
}

// ---------------------------------------------------------------------------
// one workgroup per node: block, norms and reflector traffic through L2/HBM,
// the pivot bookkeeping in LDS
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kQrThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_qrcp(const SkelTask *__restrict__ tasks, int s, int ldm, int d) {
    __shared__ double nrm[kQrMaxCols];
    __shared__ int32_t pos[kQrMaxCols];
    __shared__ double Rjj[kQrMaxRank];
    __shared__ double vh[kQrMaxRows];
    __shared__ int16_t rmap[kQrMaxRows];
    __shared__ double red[kQrWaves];
    __shared__ int32_t wcnt[kQrWaves];
    __shared__ int32_t s_stop, s_rank, s_zero;
    __shared__ double s_tau;

    const SkelTask t = tasks[blockIdx.x];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int sl = t.leaf ? 0 : *glb(t.srl);
    const int ncand = node_ncand(t);
    GLB double *M = glb(t.M);
    if (ncand <= s) {  // no compression: skeleton = candidates, P = I
        qr_identity(t, s, sl, ncand);
        return;
    }
    int rows = qr_row_select(t, M, ldm, ncand, vh, rmap, wcnt, red);
    if (tid == 0) *glb(t.qrows) = rows;
    const int32_t *src = reinterpret_cast<const int32_t *>(vh);
    gen_rows(t, M, ldm, d, sl, ncand, src, rows, nrm, kQrMaxCols);  // nrm is free until the norms
    __syncthreads();
    const int steps = s < rows ? s : rows;
    for (int c = tid; c < ncand; c += kQrThreads) pos[c] = c;
    col_norms(M, ldm, ncand, rows, nrm, lane, wave);
    if (tid == 0) {
        s_rank = steps;
        s_zero = 0;
        s_stop = 0;
    }
    __syncthreads();
    // Pivot steps (columns stay in place; pos is the pivot order): wave 0
    // picks the pivot, builds the reflector in LDS and swaps the positions;
    // one barrier; all waves update the trailing columns and their norms;
    // one barrier.
    double r00 = 0.0;
    for (int j = 0; j < steps; j++) {
        if (wave == 0) {
            const int k = pick_pivot(nrm, pos, j, ncand, lane);
            const int p = pos[k];
            bool stop;
            const Refl r = reflector_to_lds(M + (int64_t)p * ldm, j, rows, lane, r00, t.tol, vh, stop);
            if (stop) {
                if (lane == 0) {
                    s_rank = j == 0 ? 1 : j;
                    s_zero = (j == 0);
                    s_stop = 1;
                }
            } else {
                if (lane == 0) {
                    vh[j] = 1.0;
                    s_tau = r.tau;
                    Rjj[j] = r.beta;
                    pos[k] = pos[j];
                    pos[j] = p;
                }
            }
        }
        __syncthreads();
        if (s_stop) break;
        if (j == 0) r00 = fabs(Rjj[0]);
        const double tau = s_tau;
        const int span = rows - j;
        if (span <= kWave) apply_all<1, 16>(M, ldm, pos, j, ncand, vh, rows, tau, lane, wave, nrm);
        else if (span <= 2 * kWave) apply_all<2, 8>(M, ldm, pos, j, ncand, vh, rows, tau, lane, wave, nrm);
        else if (span <= 4 * kWave) apply_all<4, 4>(M, ldm, pos, j, ncand, vh, rows, tau, lane, wave, nrm);
        else if (span <= 8 * kWave) apply_all<8, 2>(M, ldm, pos, j, ncand, vh, rows, tau, lane, wave, nrm);
        else
            for (int q = j + 1 + wave; q < ncand; q += kQrWaves) {
                const int c = pos[q];
                const double v = apply_col(M + (int64_t)c * ldm, vh, j, rows, tau, lane);
                if (lane == 0) nrm[c] = v;
            }
        __syncthreads();
    }
    id_solve_rows(t, M, ldm, s, sl, ncand, s_rank, s_zero != 0, pos, Rjj, wave * kTq, kQrWaves * kTq);
    id_outputs(t, s, sl, ncand, s_rank, pos);
}

// ---------------------------------------------------------------------------
// split form: kQsCols columns per 256-thread workgroup, one launch per step
// ---------------------------------------------------------------------------
// partial squared row norms over the workgroup's column group
__global__ __launch_bounds__(kQsThreads) void k_qs_rows(const SkelTask *__restrict__ tasks, QrWork w, int ldm) {
    const int node = blockIdx.x / w.slices, slice = blockIdx.x % w.slices;
    const SkelTask t = tasks[node];
    const int ncand = node_ncand(t), c0 = slice * kQsCols;
    if (c0 >= ncand) return;
    GLB double *part = glb(w.part) + ((int64_t)node * w.slices + slice) * w.rcap;
    const GLB double *M = glb(t.M);
    for (int i = threadIdx.x; i < t.nq; i += kQsThreads) part[i] = row_part(M, ldm, i, c0, min(ncand, c0 + kQsCols));
}

// row norms (groups summed in order), kept rows and their new indices
__global__ __launch_bounds__(kQrThreads) void k_qs_rowmap(const SkelTask *__restrict__ tasks, QrWork w) {
    __shared__ double rn[kQrMaxRows];
    __shared__ double red[kQrWaves];
    __shared__ int32_t wcnt[kQrWaves];
    const int node = blockIdx.x;
    const SkelTask t = tasks[node];
    const int ncand = node_ncand(t), groups = (ncand + kQsCols - 1) / kQsCols, rows = t.nq;
    const GLB double *part = glb(w.part) + (int64_t)node * w.slices * w.rcap;
    for (int i = threadIdx.x; i < rows; i += kQrThreads) {
        double a = 0.0;
        for (int g = 0; g < groups; g++) a += part[(int64_t)g * w.rcap + i];
        rn[i] = a;
    }
    __syncthreads();
    const int kept = row_map(rn, rows, glb(w.rmap) + (int64_t)node * w.rcap, wcnt, red);
    if (threadIdx.x == 0) glb(w.rows)[node] = kept;
}

// compaction of the group's columns, initial norms, pivot order and state.
// From here on a workgroup owns pivot positions (not columns): norms are kept
// by position and the column at a position is read from the pivot order.
__global__ __launch_bounds__(kQsThreads) void k_qs_init(const SkelTask *__restrict__ tasks, QrWork w, int s,
                                                         int ldm) {
    const int node = blockIdx.x / w.slices, slice = blockIdx.x % w.slices;
    const SkelTask t = tasks[node];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int ncand = node_ncand(t), kept = glb(w.rows)[node];
    const int rows = kept < t.nq ? (kept > 0 ? kept : 1) : t.nq;  // as in k_qrcp
    const GLB int32_t *rmap = glb(w.rmap) + (int64_t)node * w.rcap;
    GLB double *nrm = glb(w.nrm) + (int64_t)node * 2 * w.cmax;
    GLB int32_t *pos = glb(w.pos) + (int64_t)node * 2 * w.cmax;
    for (int q = 0; q < 2; q++) {
        const int c = slice * kQsCols + 2 * wave + q;
        if (c >= ncand) continue;
        GLB double *col = glb(t.M) + (int64_t)c * ldm;
        if (kept < t.nq) compact_col(col, rmap, t.nq, lane);
        const double v = col_norm(col, rows, lane);
        if (lane == 0) {
            nrm[c] = v;
            pos[c] = c;
        }
    }
    if (slice == 0 && tid == 0) {
        GLB int32_t *st = glb(w.st) + kQsState * node;
        st[0] = 0;
        st[1] = 0;
        st[2] = 0;
        st[3] = s < rows ? s : rows;
        st[4] = rows;
        st[5] = ncand;
        *glb(t.qrows) = rows;
    }
}

// Pivot step j of a split node.  qs_pivot: every workgroup of a node picks the same
// pivot (largest norm over positions j .., lowest position on ties) and
// builds the same reflector from the state of step j - 1 (buffers j % 2);
// wave 0 works, the result lands in LDS.  The writer workgroup records R_jj
// or the stop.  qs_update: the workgroup updates the columns at the
// positions > j of its column groups (s0, s0 + sstep, .. of kQsCols
// positions each) into the other buffers; in the next pivot order positions
// j and k are exchanged, and the column now at position q is updated and its
// norm stored at q.
struct QsPivot {
    double tau;
    int32_t k, p, stop;
};

// leading dimension of the split nodes' sampled blocks (the sample capacity)
__device__ inline int ldm_of(const QrWork &w) { return w.rcap; }

__device__ inline void qs_pivot(const SkelTask *tasks, const QrWork &w, int node, int j, bool writer, double *vh,
                                QsPivot *sp) {
    const GLB int32_t *st = glb(w.st) + kQsState * node;
    const int rows = st[4], ncand = st[5];
    GLB double *M = glb(tasks[node].M);
    // |R_00| for the rank rule (meaningless, and unused, at step 0)
    const double r00 = fabs(glb(w.diag)[(int64_t)node * w.cmax]);
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    if (wave != 0) return;
    const GLB double *nin = glb(w.nrm) + (int64_t)node * 2 * w.cmax + (int64_t)(j & 1) * w.cmax;
    const GLB int32_t *pin = glb(w.pos) + (int64_t)node * 2 * w.cmax + (int64_t)(j & 1) * w.cmax;
    GLB double *Rjj = glb(w.diag) + (int64_t)node * w.cmax;
    // each lane reads the norms and the columns of its positions (at most
    // kQsScan: a split node has at most 2 s <= 2 kQrMaxRank candidates), all
    // loads before the first comparison, so the pivot's column comes from
    // the winning lane instead of another load
    double nv[kQsScan];
    int pc[kQsScan];
#pragma unroll
    for (int u = 0; u < kQsScan; u++) {
        const int k = j + lane + u * kWave;
        nv[u] = k < ncand ? nin[k] : -1.0;
        pc[u] = k < ncand ? pin[k] : -1;
    }
    double bv = -1.0;
    int bk = 0x7fffffff, bc = -1;
#pragma unroll
    for (int u = 0; u < kQsScan; u++) {
        if (nv[u] > bv) {  // positions ascend within a lane: the first of equal norms stays
            bv = nv[u];
            bk = j + lane + u * kWave;
            bc = pc[u];
        }
    }
    const int kw = wave_argmax(bv, bk);
    bk = kw == 0x7fffffff ? j : kw;  // no comparable norm (NaN): keep the order
    const int p = kw == 0x7fffffff ? pin[j] : __builtin_amdgcn_readlane(bc, (kw - j) & (kWave - 1));
    bool stop;
    const Refl r = reflector_to_lds(M + (int64_t)p * ldm_of(w), j, rows, lane, j == 0 ? 0.0 : r00, tasks[node].tol, vh,
                                    stop);
    if (lane == 0) {
        sp->stop = stop;
        sp->k = bk;
        sp->p = p;
        sp->tau = r.tau;
        vh[j] = 1.0;
        if (writer) {
            if (stop) {
                GLB int32_t *stw = glb(w.st) + kQsState * node;
                stw[0] = 1;
                stw[1] = j;
                stw[2] = (j == 0);
            } else {
                Rjj[j] = r.beta;
            }
        }
    }
}

// the update of one workgroup's positions; columns of a wave are loaded
// NC at a time before their products when rows - j <= 64 NT (the
// per-column arithmetic is apply_col's, so the grouping changes no result)
template <int NT, int NC>
__device__ inline void qs_update_grouped(const QrWork &w, GLB double *M, int ldm, int node, int j, int rows,
                                         int ncand, int s0, int sstep, const double *vh, const QsPivot &pv) {
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const GLB int32_t *pin = glb(w.pos) + (int64_t)node * 2 * w.cmax + (int64_t)(j & 1) * w.cmax;
    GLB double *nout = glb(w.nrm) + (int64_t)node * 2 * w.cmax + (int64_t)((j + 1) & 1) * w.cmax;
    GLB int32_t *pout = glb(w.pos) + (int64_t)node * 2 * w.cmax + (int64_t)((j + 1) & 1) * w.cmax;
    // this workgroup's positions: group g of s0, s0 + sstep, ..; position
    // i of the workgroup's list is q(i) = (s0 + (i / kQsCols) sstep) kQsCols + i % kQsCols
    const int ngroups = (w.slices - s0 + sstep - 1) / sstep;
    const int npos = ngroups * kQsCols;
    auto qpos = [&](int i) { return (s0 + (i / kQsCols) * sstep) * kQsCols + i % kQsCols; };
    const int pj = pin[j];
    double vr[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int i = j + lane + t * kWave;
        vr[t] = i < rows ? vh[i] : 0.0;
    }
    for (int i0 = wave; i0 < npos; i0 += kQsWaves * NC) {
        int q[NC], c[NC];
        double a[NC][NT];
#pragma unroll
        for (int u = 0; u < NC; u++) {
            const int i = i0 + u * kQsWaves;
            q[u] = i < npos ? qpos(i) : ncand;
            c[u] = -1;
            if (q[u] < ncand) {
                c[u] = q[u] == j ? pv.p : (q[u] == pv.k ? pj : pin[q[u]]);
                if (lane == 0) pout[q[u]] = c[u];
                if (q[u] <= j) c[u] = -1;  // placed, nothing to update
            }
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int r = j + lane + t * kWave;
                a[u][t] = (c[u] >= 0 && r < rows) ? M[(int64_t)c[u] * ldm + r] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < NC; u++) {
            if (c[u] < 0) continue;
            double wsum = 0.0;
#pragma unroll
            for (int t = 0; t < NT; t++) wsum = fma(vr[t], a[u][t], wsum);
            wsum = wave_sum(wsum) * pv.tau;
            double n = 0.0;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int r = j + lane + t * kWave;
                a[u][t] = fma(-vr[t], wsum, a[u][t]);
                if (r > j && r < rows) n = fma(a[u][t], a[u][t], n);
            }
            GLB double *col = M + (int64_t)c[u] * ldm;
#pragma unroll
            for (int t = 0; t < NT; t++) {
                const int r = j + lane + t * kWave;
                if (r < rows) col[r] = a[u][t];
            }
            n = wave_sum(n);
            if (lane == 0) nout[q[u]] = n;
        }
    }
}

// spans above 16 x 64 rows: one column at a time (apply_col)
__device__ inline void qs_update_plain(const QrWork &w, GLB double *M, int ldm, int node, int j, int rows, int ncand,
                                       int s0, int sstep, const double *vh, const QsPivot &pv) {
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const GLB int32_t *pin = glb(w.pos) + (int64_t)node * 2 * w.cmax + (int64_t)(j & 1) * w.cmax;
    GLB double *nout = glb(w.nrm) + (int64_t)node * 2 * w.cmax + (int64_t)((j + 1) & 1) * w.cmax;
    GLB int32_t *pout = glb(w.pos) + (int64_t)node * 2 * w.cmax + (int64_t)((j + 1) & 1) * w.cmax;
    const int npos = ((w.slices - s0 + sstep - 1) / sstep) * kQsCols;
    const int pj = pin[j];
    for (int i = wave; i < npos; i += kQsWaves) {
        const int q = (s0 + (i / kQsCols) * sstep) * kQsCols + i % kQsCols;
        if (q >= ncand) continue;
        const int c = q == j ? pv.p : (q == pv.k ? pj : pin[q]);
        if (lane == 0) pout[q] = c;
        if (q <= j) continue;
        const double v = apply_col(M + (int64_t)c * ldm, vh, j, rows, pv.tau, lane);
        if (lane == 0) nout[q] = v;
    }
}

__device__ inline void qs_update(const SkelTask *tasks, const QrWork &w, int node, int j, int s0, int sstep,
                                 const double *vh, const QsPivot &pv) {
    const GLB int32_t *st = glb(w.st) + kQsState * node;
    const int rows = st[4], ncand = st[5];
    GLB double *M = glb(tasks[node].M);
    const int ldm = ldm_of(w), span = rows - j;
    if (span <= kWave) qs_update_grouped<1, 8>(w, M, ldm, node, j, rows, ncand, s0, sstep, vh, pv);
    else if (span <= 2 * kWave) qs_update_grouped<2, 4>(w, M, ldm, node, j, rows, ncand, s0, sstep, vh, pv);
    else if (span <= 4 * kWave) qs_update_grouped<4, 2>(w, M, ldm, node, j, rows, ncand, s0, sstep, vh, pv);
    else if (span <= 8 * kWave) qs_update_grouped<8, 2>(w, M, ldm, node, j, rows, ncand, s0, sstep, vh, pv);
    else if (span <= 16 * kWave) qs_update_grouped<16, 1>(w, M, ldm, node, j, rows, ncand, s0, sstep, vh, pv);
    else qs_update_plain(w, M, ldm, node, j, rows, ncand, s0, sstep, vh, pv);
}

// one launch per pivot step: workgroup = (node, column group)
// The launch covers the slices s0 .. w.slices - 1 of every node, s0 =
// (j - 1) / kQsCols: a position placed at step p is copied into the other
// buffer of the pivot order at step p + 1 and changes in neither after, so
// the slices below s0, whose positions are all <= j - 2, have nothing left
// to do.  The first launched slice records R_jj and the stop (a split node
// has more than s candidates, so its positions reach past j).
__global__ __launch_bounds__(kQsThreads) void k_qs_step(const SkelTask *__restrict__ tasks, QrWork w, int j,
                                                         int s0) {
    __shared__ double vh[kQrMaxRows];
    __shared__ QsPivot sp;
    const int nsl = w.slices - s0;
    const int node = blockIdx.x / nsl, slice = s0 + blockIdx.x % nsl;
    const GLB int32_t *st = glb(w.st) + kQsState * node;
    const int stopped = st[0], steps = st[3], ncand = st[5];
    if (stopped || j >= steps) return;
    if (slice * kQsCols >= ncand) return;
    qs_pivot(tasks, w, node, j, slice == s0, vh, &sp);
    __syncthreads();
    const QsPivot pv = sp;
    if (pv.stop) return;
    qs_update(tasks, w, node, j, slice, w.slices, vh, pv);
}

// T = R11^{-1} R12 and the outputs; blockIdx.y takes the column groups
// y, y + gridDim.y, ... of kQsFinishCols columns each, workgroup 0 of a node
// also writes the per-node outputs
__global__ __launch_bounds__(kQrThreads) void k_qs_finish(const SkelTask *__restrict__ tasks, QrWork w, int s,
                                                           int ldm) {
    const int node = blockIdx.x, wave = threadIdx.x / kWave;
    const SkelTask t = tasks[node];
    const GLB int32_t *st = glb(w.st) + kQsState * node;
    const int sl = t.leaf ? 0 : *glb(t.srl), ncand = node_ncand(t);
    const bool stopped = st[0] != 0, zero = st[2] != 0;
    const int jstop = st[1], steps = st[3];
    const int done = stopped ? jstop : steps;
    const int rank = stopped ? (jstop == 0 ? 1 : jstop) : steps;
    const GLB int32_t *pos = glb(w.pos) + (int64_t)node * 2 * w.cmax + (int64_t)(done & 1) * w.cmax;
    id_solve_rows(t, glb(t.M), ldm, s, sl, ncand, rank, zero, pos, glb(w.diag) + (int64_t)node * w.cmax,
                  (int)(blockIdx.y * kQrWaves + wave) * kTq, (int)gridDim.y * kQsFinishCols);
    if (blockIdx.y == 0) id_outputs(t, s, sl, ncand, rank, pos);
}

}  // namespace askit
