// k_skel.hip -- skeletonization kernels (Sec. 2.1, "Computing low rank
// approximations"; Alg. 1; the ID of eq. (4)).
//
//  * k_sample: the sampled rows S' of a node: min(nsamp, N - n) distinct
//    positions outside the node, drawn uniformly with SplitMix64 (Steele, Lea
//    & Flood 2014) from the node's own stream, duplicates rejected; when the
//    complement has at most nsamp positions it is taken whole, in order.
//  * k_sample_block: the kernel block K(X_S', X_C) in FP64, column-major.
//  * k_qrcp: column-pivoted Householder QR of that block, truncated at the
//    rank s (trailing column norms recomputed at every step, largest norm
//    first, lowest column on ties), the rank guard |R_jj| <= 1e-14 |R_00|,
//    T = R11^{-1} R12 and the projection P = [I T] Pi^T, written transposed.
#include "askit_dev.h"

namespace askit {

// ---------------------------------------------------------------------------
// sampling: one wave per node; lane 0 runs the sequential rejection loop with
// an open-addressing set in LDS
// ---------------------------------------------------------------------------
constexpr int kSampHashBits = 13;  // 8192 slots: nsamp <= 4096

__device__ inline uint64_t splitmix_next(uint64_t &st) {
    uint64_t z = (st += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(64) void k_sample(const SampTask *__restrict__ tasks, int nsamp, int32_t *__restrict__ err) {
    __shared__ int32_t table[1 << kSampHashBits];
    const SampTask t = tasks[blockIdx.x];
    const int64_t n = t.e - t.b, c = t.N - n;
    if (c <= nsamp) {
        for (int64_t i = threadIdx.x; i < c; i += kWave) t.out[i] = (int32_t)(i < t.b ? i : i + n);
        return;
    }
    for (int i = threadIdx.x; i < (1 << kSampHashBits); i += kWave) table[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t st = t.state;
        const uint64_t cap = 64ULL * (uint64_t)(c + nsamp);
        int k = 0;
        uint64_t draws = 0;
        while (k < nsamp) {
            if (++draws > cap) {
                atomicOr(err, 1);
                break;
            }
            uint64_t r = __umul64hi(splitmix_next(st), (uint64_t)c);
            int64_t pos = (int64_t)r < t.b ? (int64_t)r : (int64_t)r + n;
            uint32_t key = (uint32_t)pos + 1u;
            uint32_t slot = (uint32_t)(((uint64_t)pos * 0x9E3779B97F4A7C15ULL) >> (64 - kSampHashBits));
            bool dup = false;
            while (true) {
                int32_t v = table[slot];
                if (v == 0) {
                    table[slot] = (int32_t)key;
                    break;
                }
                if ((uint32_t)v == key) {
                    dup = true;
                    break;
                }
                slot = (slot + 1) & ((1u << kSampHashBits) - 1);
            }
            if (!dup) t.out[k++] = (int32_t)pos;
        }
    }
}

// ---------------------------------------------------------------------------
// sampled kernel block M = K(X_S', X_C), column-major (ldm rows)
// ---------------------------------------------------------------------------
__device__ inline int32_t cand_pos(const SkelTask &t, int c, int sl) {
    if (t.leaf) return (int32_t)(t.b + c);
    return c < sl ? t.skl[c] : t.skr[c - sl];
}

__device__ inline double sqdist(const double *x, const double *y, int d) {
    double r2 = 0.0;
    for (int k = 0; k < d; k++) {
        double df = x[k] - y[k];
        r2 = fma(df, df, r2);
    }
    return r2;
}

// block: 256 threads on a 64 x 64 tile (sampled rows x candidate columns);
// both point sets are staged in LDS, each thread writes 16 entries of one
// column (consecutive rows across lanes: coalesced column-major stores)
__global__ __launch_bounds__(256) void k_sample_block(const SkelTask *__restrict__ tasks, int rowtiles, int ldm, int d,
                                                      int coltiles) {
    extern __shared__ double dyn_lds[];  // 2 x 64 x d doubles
    double *ys = dyn_lds, *xs = dyn_lds + 64 * d;
    const int per = rowtiles * coltiles;
    const int task = blockIdx.x / per, rt = (blockIdx.x % per) % rowtiles, ct = (blockIdx.x % per) / rowtiles;
    const SkelTask t = tasks[task];
    const int r0 = rt * 64, c0 = ct * 64;
    const int sl = t.leaf ? 0 : *t.srl;
    const int ncand = t.leaf ? t.n : sl + *t.srr;
    if (r0 >= t.nq || c0 >= ncand) return;
    const int nr = min(64, t.nq - r0), nc = min(64, ncand - c0);
    for (int i = threadIdx.x; i < 64 * d; i += blockDim.x) {
        const int a = i / d, k = i % d;
        ys[i] = a < nr ? t.X[(int64_t)t.q[r0 + a] * d + k] : 0.0;
        xs[i] = a < nc ? t.X[(int64_t)cand_pos(t, c0 + a, sl) * d + k] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x % 64;
    if (r >= nr) return;
    const double *y = ys + r * d;
    for (int c = threadIdx.x / 64; c < nc; c += 4)
        t.M[(int64_t)(c0 + c) * ldm + r0 + r] = exp(sqdist(xs + c * d, y, d) * t.scale);
}

// ---------------------------------------------------------------------------
// QRCP + interpolative decomposition, one workgroup per node
// ---------------------------------------------------------------------------
constexpr int kQrThreads = 512;
constexpr int kQrWaves = kQrThreads / kWave;

__device__ inline double wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// block-wide sum (all threads get the result); red: kQrWaves doubles of LDS
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

__global__ __launch_bounds__(kQrThreads) void k_qrcp(const SkelTask *__restrict__ tasks, int s, int ldm) {
    __shared__ double nrm[kQrMaxCols];
    __shared__ int32_t piv[kQrMaxCols];
    __shared__ double vh[kQrMaxRows];
    __shared__ double red[kQrWaves];
    __shared__ int32_t rmap[kQrMaxRows];
    __shared__ int32_t wcnt[kQrWaves];
    __shared__ int32_t s_rank, s_zero;

    const SkelTask t = tasks[blockIdx.x];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int sl = t.leaf ? 0 : *t.srl;
    const int ncand = t.leaf ? t.n : sl + *t.srr;
    int rows = t.nq;
    double *M = t.M;
    // padded row of candidate c in P_{C alpha~}: internal nodes keep the two
    // children's skeletons in the halves [0, s) and [s, 2s)
    auto prow = [&](int c) { return t.leaf ? c : (c < sl ? c : s + (c - sl)); };

    // P is written in the rows of the candidates and the columns below the
    // rank only: nothing reads the rest of the padded slot
    if (ncand <= s) {  // no compression: skeleton = candidates, P = I
        for (int k = tid; k < s; k += kQrThreads) t.skel[k] = k < ncand ? cand_pos(t, k, sl) : -1;
        for (int64_t i = tid; i < (int64_t)ncand * ncand; i += kQrThreads) {
            const int c = (int)(i / ncand), k = (int)(i % ncand);
            t.Pt[(int64_t)prow(c) * s + k] = k == c ? 1.0 : 0.0;
        }
        if (tid == 0) {
            *t.sr = ncand;
            *t.trunc = 0;
        }
        return;
    }
    // Rows of the sampled block whose squared norm is below 1e-60 of the
    // block's squared Frobenius norm are dropped (the rest keep their order).
    // Their total weight, under 1e-57 of the block's, is far below FP64
    // rounding of every column norm and of the rank guard's threshold, so the
    // pivots, R and T are those of the whole block up to rounding; the trailing
    // updates then stream only the rows that carry the interaction.
    {
        for (int i = tid; i < rows; i += kQrThreads) {
            double a = 0.0;
            for (int c = 0; c < ncand; c++) {
                const double v = M[(int64_t)c * ldm + i];
                a = fma(v, v, a);
            }
            vh[i] = a;
        }
        __syncthreads();
        double part = 0.0;
        for (int i = tid; i < rows; i += kQrThreads) part += vh[i];
        const double thr = 1e-60 * block_sum(part, red);
        int kept = 0;
        for (int base = 0; base < rows; base += kQrThreads) {
            const int i = base + tid;
            const bool keep = i < rows && vh[i] > thr;
            const unsigned long long bal = __ballot(keep);
            const int below = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) wcnt[wave] = __popcll(bal);
            __syncthreads();
            int wofs = 0, tot = 0;
            for (int w = 0; w < kQrWaves; w++) {
                if (w < wave) wofs += wcnt[w];
                tot += wcnt[w];
            }
            if (i < rows) rmap[i] = keep ? kept + wofs + below : -1;
            kept += tot;
            __syncthreads();
        }
        if (kept < rows) {
            // compaction in place, one wave per column: every row moves up or
            // stays, and a wave reads a 64-row chunk before writing it
            for (int c = wave; c < ncand; c += kQrWaves) {
                double *col = M + (int64_t)c * ldm;
                for (int base = 0; base < rows; base += kWave) {
                    const int i = base + lane;
                    const double v = i < rows ? col[i] : 0.0;
                    const int dst = i < rows ? rmap[i] : -1;
                    if (dst >= 0) col[dst] = v;
                }
            }
            rows = kept > 0 ? kept : 1;
            __syncthreads();
        }
    }
    int steps = s < rows ? s : rows;
    for (int c = tid; c < ncand; c += kQrThreads) piv[c] = c;
    // initial squared column norms (one wave per column)
    for (int c = wave; c < ncand; c += kQrWaves) {
        double acc = 0.0;
        for (int i = lane; i < rows; i += kWave) {
            double v = M[(int64_t)c * ldm + i];
            acc = fma(v, v, acc);
        }
        acc = wave_sum(acc);
        if (lane == 0) nrm[c] = acc;
    }
    if (tid == 0) {
        s_rank = steps;
        s_zero = 0;
    }
    __syncthreads();
    // Pivot steps.  Every wave finds the pivot itself from the norms in LDS
    // (no barrier); wave 0 swaps the columns in memory, builds the reflector
    // and publishes it in LDS; one barrier; all waves apply it to the
    // trailing columns (two at a time, held in registers when the sampled
    // block has at most 1024 rows) and recompute their norms; one barrier.
    __shared__ double s_tau;
    __shared__ int32_t s_stop;
    if (tid == 0) s_stop = 0;
    __syncthreads();
    double r00 = 0.0;
    for (int j = 0; j < steps; j++) {
        double bv = -1.0;
        int bi = 0x7fffffff;
        for (int c = j + lane; c < ncand; c += kWave) {
            const double v = nrm[c];
            if (v > bv || (v == bv && c < bi)) {
                bv = v;
                bi = c;
            }
        }
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        const int p = bi;
        if (wave == 0) {
            double *col = M + (int64_t)j * ldm;
            double xn = 0.0, aj = 0.0;  // aj: entry (j, j) after the swap, held by lane j % 64
            if (p != j) {
                double *cp = M + (int64_t)p * ldm;
                for (int i = lane; i < rows; i += kWave) {
                    const double a = col[i], b = cp[i];
                    col[i] = b;
                    cp[i] = a;
                    if (i > j) xn = fma(b, b, xn);
                    if (i == j) aj = b;
                }
                if (lane == 0) {
                    const int ti = piv[j];
                    piv[j] = piv[p];
                    piv[p] = ti;
                }
            } else {
                for (int i = j + 1 + lane; i < rows; i += kWave) xn = fma(col[i], col[i], xn);
                if (lane == j % kWave) aj = col[j];
            }
            xn = wave_sum(xn);
            const double alpha = __shfl(aj, j % kWave);
            double beta, tau, sc;
            if (xn == 0.0) {
                beta = alpha; tau = 0.0; sc = 0.0;
            } else {
                beta = -copysign(sqrt(alpha * alpha + xn), alpha);
                tau = (beta - alpha) / beta;
                sc = 1.0 / (alpha - beta);
            }
            const double r0 = j == 0 ? fabs(beta) : r00;
            const bool stop = (j > 0 && fabs(beta) <= kRankGuard * r0) || (j == 0 && r0 == 0.0);
            if (stop) {
                if (lane == 0) {
                    s_rank = j == 0 ? 1 : j;
                    s_zero = (j == 0);
                    s_stop = 1;
                }
            } else {
                for (int i = j + 1 + lane; i < rows; i += kWave) {
                    const double v = col[i] * sc;
                    vh[i] = v;
                    col[i] = v;
                }
                if (lane == 0) {
                    vh[j] = 1.0;
                    col[j] = beta;
                    s_tau = tau;
                }
            }
        }
        __syncthreads();
        if (s_stop) break;
        if (j == 0) r00 = fabs(M[0]);
        const double tau = s_tau;
        // apply H to the columns right of j; new squared norms over rows j+1..
        if (rows - j <= 16 * kWave) {
            double vr[16];
#pragma unroll
            for (int t = 0; t < 16; t++) {
                const int i = j + lane + t * kWave;
                vr[t] = i < rows ? vh[i] : 0.0;
            }
            for (int c = j + 1 + 2 * wave; c < ncand; c += 2 * kQrWaves) {
                const bool two = c + 1 < ncand;
                double *c0 = M + (int64_t)c * ldm, *c1 = M + (int64_t)(two ? c + 1 : c) * ldm;
                double a0[16], a1[16];
                double w0 = 0.0, w1 = 0.0;
#pragma unroll
                for (int t = 0; t < 16; t++) {
                    const int i = j + lane + t * kWave;
                    a0[t] = i < rows ? c0[i] : 0.0;
                    a1[t] = i < rows ? c1[i] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < 16; t++) {
                    w0 = fma(vr[t], a0[t], w0);
                    w1 = fma(vr[t], a1[t], w1);
                }
                for (int o = kWave / 2; o > 0; o >>= 1) {
                    w0 += __shfl_xor(w0, o);
                    w1 += __shfl_xor(w1, o);
                }
                w0 *= tau;
                w1 *= tau;
                double n0 = 0.0, n1 = 0.0;
#pragma unroll
                for (int t = 0; t < 16; t++) {
                    const int i = j + lane + t * kWave;
                    a0[t] = fma(-vr[t], w0, a0[t]);
                    a1[t] = fma(-vr[t], w1, a1[t]);
                    if (i > j && i < rows) {
                        n0 = fma(a0[t], a0[t], n0);
                        n1 = fma(a1[t], a1[t], n1);
                    }
                }
#pragma unroll
                for (int t = 0; t < 16; t++) {
                    const int i = j + lane + t * kWave;
                    if (i < rows) {
                        c0[i] = a0[t];
                        if (two) c1[i] = a1[t];
                    }
                }
                for (int o = kWave / 2; o > 0; o >>= 1) {
                    n0 += __shfl_xor(n0, o);
                    n1 += __shfl_xor(n1, o);
                }
                if (lane == 0) {
                    nrm[c] = n0;
                    if (two) nrm[c + 1] = n1;
                }
            }
        } else {
            for (int c = j + 1 + wave; c < ncand; c += kQrWaves) {
                double *ck = M + (int64_t)c * ldm;
                double w = 0.0;
                for (int i = j + lane; i < rows; i += kWave) w = fma(vh[i], ck[i], w);
                w = wave_sum(w) * tau;
                double acc = 0.0;
                for (int i = j + lane; i < rows; i += kWave) {
                    const double v = fma(-vh[i], w, ck[i]);
                    ck[i] = v;
                    if (i > j) acc = fma(v, v, acc);
                }
                acc = wave_sum(acc);
                if (lane == 0) nrm[c] = acc;
            }
        }
        __syncthreads();
    }
    const int rank = s_rank;
    const bool zero = s_zero != 0;
    // T = R11^{-1} R12 in place of R12 (one thread per column)
    const int nr = ncand - rank;
    for (int c = tid; c < nr; c += kQrThreads) {
        double *tc = M + (int64_t)(rank + c) * ldm;
        for (int i = rank - 1; i >= 0; i--) {
            if (zero) {
                tc[i] = 0.0;
                continue;
            }
            double acc = tc[i];
            for (int k = i + 1; k < rank; k++) acc = fma(-M[(int64_t)k * ldm + i], tc[k], acc);
            tc[i] = acc / M[(int64_t)i * ldm + i];
        }
    }
    __syncthreads();
    // outputs: skeleton positions, rank, P_{C alpha~} rows
    for (int k = tid; k < s; k += kQrThreads) t.skel[k] = k < rank ? cand_pos(t, piv[k], sl) : -1;
    if (tid == 0) {
        *t.sr = rank;
        *t.trunc = (rank < (s < ncand ? s : ncand)) ? 1 : 0;
    }
    for (int jc = tid; jc < ncand; jc += kQrThreads) {
        double *row = t.Pt + (int64_t)prow(piv[jc]) * s;
        if (jc < rank) {
            for (int k = 0; k < rank; k++) row[k] = k == jc ? 1.0 : 0.0;
        } else {
            const double *tc = M + (int64_t)jc * ldm;
            for (int k = 0; k < rank; k++) row[k] = tc[k];
        }
    }
}

}  // namespace askit
