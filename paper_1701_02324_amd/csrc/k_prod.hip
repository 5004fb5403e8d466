// k_prod.hip -- tiled MFMA products of the factorization and the solves.
//
// k_kmm: the fused kernel-block product C op= K(R, S) B of Sec. 2.4 (kernel
// summation without storing the block): a 64 x 16 tile of Gaussian kernel
// entries (eq. (1)) is generated from LDS-staged coordinates and fed straight
// to the matrix cores together with a 16 x TC tile of B.  It forms the
// reduced-system blocks K_{l~ r} Phat_r and K_{r~ l} Phat_l of eq. (8), the
// products V v of Alg. 3 and their transposes, and the matvec of eq. (6).
//
// k_gmm: the plain products with the hat factors (telescoping of eq. (10),
// W y of Alg. 3, W^T g of the transpose solve) with arbitrary strides.
//
// Both use v_mfma_f64_16x16x4f64 (FP64 path) or v_mfma_f32_16x16x4f32
// (mixed path): a 256-thread workgroup owns a 64 x TC output tile, wave w
// owns rows 16w..16w+15 and TC/16 accumulator blocks.  MFMA operand layout
// (16x16x4, both types): lane l holds A[l%16][l/16] and B[l/16][l%16].
// Accumulator register r of lane l holds C[i][l%16] with i = 4(l/16) + r for
// FP32 and i = 4r + l/16 for FP64 (measured on gfx950).
#include "askit_dev.h"

namespace askit {

template <typename T> struct Acc;
template <> struct Acc<double> {
    typedef dbl4 type;
    static __device__ inline dbl4 mma(double a, double b, dbl4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int r) { return 4 * r + lane / 16; }
};
template <> struct Acc<float> {
    typedef flt4 type;
    static __device__ inline flt4 mma(float a, float b, flt4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

__device__ inline double kexp(double x) { return exp(x); }
__device__ inline float kexp(float x) { return expf(x); }

constexpr int kTR = 64;   // tile rows
constexpr int kKS = 16;   // contraction per stage

template <typename P, typename T>
__device__ inline void store_out(P C, int64_t off, T v, int op) {
    if (op == OP_STORE) C[off] = v;
    else if (op == OP_ADD) C[off] += v;
    else C[off] -= v;
}

__device__ inline int src_count(const PtSrc &s) { return s.cnt ? *glb(s.cnt) : s.n; }
__device__ inline int64_t src_pos(const PtSrc &s, int i) { return s.idx ? (int64_t)glb(s.idx)[i] : s.base + i; }

// XR (d <= kXrDim): lane l generates the kernel entries of tile row l only,
// so its row point stays in registers for the whole contraction and the
// contraction points are staged at stride kXrDim, zero-padded (the padded
// coordinates add exact zeros to the squared distance).  Otherwise the row
// points are staged in LDS at an odd stride (lanes read different rows: no
// bank conflicts) and the contraction points at stride d (broadcast within a
// wave).
//
// CG column groups of four waves each (256 CG threads) share one generated
// kernel tile: the output tile is 64 x (CG TC), wave w owns rows
// 16 (w % 4) .. + 15 of columns TC (w / 4) .. + TC - 1, so the exponentials
// of a tile are computed once for CG TC columns.
template <typename T, typename TB, typename TO, int TC, bool XR, int CG>
__global__ __launch_bounds__(256 * CG) void k_kmm(const KmmTask *__restrict__ tasks,
                                                  const TileItem *__restrict__ items, int ncol, int d) {
    constexpr int NB = TC / 16, NT = 256 * CG;
    __shared__ T sA[kTR][kKS + 1];
    __shared__ T sB[kKS][TC * CG + 1];
    // XR: 16 kXrDim elements of T; else 64 (d | 1) + 16 d
    extern __shared__ double dyn_lds[];
    const int dp = d | 1;
    T *sR = (T *)dyn_lds, *sS = XR ? (T *)dyn_lds : (T *)dyn_lds + kTR * dp;
    const TileItem it = items[blockIdx.x];
    if (it.task < 0) return;
    const KmmTask t = tasks[it.task];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave, wr = wave % 4, wc = wave / 4;
    const int nrow = src_count(t.R);
    if (t.ncol > 0) ncol = min(ncol, t.ncol);
    const int r0 = it.rt * kTR, c0 = it.ct * TC * CG;
    GLB TO *C = glb((TO *)t.C);
    const GLB double *X = glb(t.X);
    if (r0 >= nrow) {  // tile of padded rows: zero-fill on store
        if (t.op == OP_STORE)
            for (int i = tid; i < kTR * TC * CG; i += NT) {
                int r = r0 + i / (TC * CG), c = c0 + i % (TC * CG);
                if (r < t.rcap && c < ncol) C[(int64_t)r * t.crs + (int64_t)c * t.ccs] = (TO)0;
            }
        return;
    }
    int k1 = t.k1;
    if (t.S.cnt) k1 = min(k1, *glb(t.S.cnt));
    const T scale = (T)t.scale, hinv = (T)t.hinv;
    // the row points (fixed for the whole contraction)
    T xr[XR ? kXrDim : 1];
    if constexpr (XR) {
        const bool live = r0 + lane < nrow;
        const int64_t pr = live ? src_pos(t.R, r0 + lane) * d : 0;
#pragma unroll
        for (int q = 0; q < kXrDim; q++) xr[q] = (live && q < d) ? (T)X[pr + q] : (T)0;
    } else {
        for (int i = tid; i < kTR * d; i += NT) {
            int r = i / d, k = i % d;
            sR[r * dp + k] = r0 + r < nrow ? (T)X[src_pos(t.R, r0 + r) * d + k] : (T)0;
        }
    }
    typename Acc<T>::type acc[NB];
    for (int b = 0; b < NB; b++) acc[b] = typename Acc<T>::type{0, 0, 0, 0};
    const GLB TB *B = glb((const TB *)t.B);
    // the next stage's contraction points and B rows are fetched into
    // registers while the current stage is generated and multiplied.  Thread
    // tid stages the same tile positions at every stage: the B addresses
    // are set once and advance by one stage per fetch
    constexpr int SS = XR ? kKS * kXrDim : kKS * kMaxDim;  // staged contraction values (max)
    constexpr int PS = (SS + NT - 1) / NT, PB = kKS * TC * CG / NT;
    T pS[PS], pB[PB];
    const GLB TB *qb[PB];
    int kbb[PB];
    bool okb[PB];
#pragma unroll
    for (int u = 0; u < PB; u++) {
        const int i = tid + u * NT, k = i / (TC * CG), c = i % (TC * CG);
        kbb[u] = k;
        okb[u] = c0 + c < ncol;
        qb[u] = B + (okb[u] ? (int64_t)k * t.ldb + c0 + c : 0);
    }
    const int64_t stepb = (int64_t)kKS * t.ldb;
    auto fetch = [&](int ks) {
        const int kn = min(kKS, k1 - ks);
#pragma unroll
        for (int u = 0; u < PS; u++) {
            const int i = tid + u * NT;
            if constexpr (XR) {
                const int r = i / kXrDim, k = i % kXrDim;
                pS[u] = (i < SS && k < d && r < kn) ? (T)X[src_pos(t.S, ks + r) * d + k] : (T)0;
            } else {
                const int r = i / d, k = i % d;
                pS[u] = (i < kKS * d && r < kn) ? (T)X[src_pos(t.S, ks + r) * d + k] : (T)0;
            }
        }
#pragma unroll
        for (int u = 0; u < PB; u++) {
            pB[u] = (okb[u] && kbb[u] < kn) ? (T)*qb[u] : (T)0;
            qb[u] += stepb;
        }
    };
    if (t.k0 < k1) fetch(t.k0);
    for (int ks = t.k0; ks < k1; ks += kKS) {
        const int kn = min(kKS, k1 - ks);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PS; u++) {
            const int i = tid + u * NT;
            if (XR ? i < SS : i < kKS * d) sS[i] = pS[u];
        }
#pragma unroll
        for (int u = 0; u < PB; u++) {
            const int i = tid + u * NT;
            sB[i / (TC * CG)][i % (TC * CG)] = pB[u];
        }
        __syncthreads();
        if (ks + kKS < k1) fetch(ks + kKS);
        // generate the kernel tile: 64 x 16 entries, 4 / CG per thread
        // (thread tid: row tid % 64 = its lane, columns tid / 64 + 4 CG m)
        if constexpr (XR) {
#pragma unroll
            for (int m = 0; m < kKS / (4 * CG); m++) {
                const int k = wave + 4 * CG * m;
                T v = (T)0;
                if (k < kn && r0 + lane < nrow) {
                    const T *y = sS + k * kXrDim;
                    T r2 = 0;
#pragma unroll
                    for (int q = 0; q < kXrDim; q++) {
                        T df = xr[q] - y[q];
                        r2 = fma(df, df, r2);
                    }
                    v = kexp(r2 * scale);
                    if (t.which) v = v * r2 * hinv * hinv * hinv;
                }
                sA[lane][k] = v;
            }
        } else {
            for (int i = tid; i < kTR * kKS; i += NT) {
                int r = i % kTR, k = i / kTR;
                T v = (T)0;
                if (k < kn && r0 + r < nrow) {
                    const T *x = sR + r * dp, *y = sS + k * d;
                    T r2 = 0;
                    for (int q = 0; q < d; q++) {
                        T df = x[q] - y[q];
                        r2 = fma(df, df, r2);
                    }
                    v = kexp(r2 * scale);
                    if (t.which) v = v * r2 * hinv * hinv * hinv;
                }
                sA[r][k] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < kKS; k4 += 4) {
            T a = sA[wr * 16 + lane % 16][k4 + lane / 16];
#pragma unroll
            for (int b = 0; b < NB; b++) {
                T bb = sB[k4 + lane / 16][wc * TC + b * 16 + lane % 16];
                acc[b] = Acc<T>::mma(a, bb, acc[b]);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int c = c0 + wc * TC + b * 16 + lane % 16;
        if (c >= ncol) continue;
        for (int q = 0; q < 4; q++) {
            const int r = r0 + wr * 16 + Acc<T>::row(lane, q);
            if (r < nrow) store_out(C, (int64_t)r * t.crs + (int64_t)c * t.ccs, (TO)acc[b][q], t.op);
            else if (r < t.rcap && t.op == OP_STORE) C[(int64_t)r * t.crs + (int64_t)c * t.ccs] = (TO)0;
        }
    }
}

template <typename T, int TC>
__global__ __launch_bounds__(256) void k_gmm(const GmmTask *__restrict__ tasks, const TileItem *__restrict__ items,
                                             int ncol, int kchunk) {
    constexpr int NB = TC / 16;
    __shared__ T sA[kTR][kKS + 1];
    __shared__ T sB[kKS][TC + 1];
    const TileItem it = items[blockIdx.x];
    if (it.task < 0) return;
    const GmmTask t = tasks[it.task];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int r0 = it.rt * kTR, c0 = it.ct * TC;
    if (r0 >= t.rows) return;
    if (t.ncol > 0) ncol = min(ncol, t.ncol);
    // optional split of the contraction: item.pad = chunk index
    const int kb = it.pad * kchunk, ke = min(t.kdim, kb + kchunk);
    const GLB T *A = glb((const T *)t.A), *B = glb((const T *)t.B);
    const bool a_kfast = (t.acs == 1), b_cfast = (t.bcs == 1);
    typename Acc<T>::type acc[NB];
    for (int b = 0; b < NB; b++) acc[b] = typename Acc<T>::type{0, 0, 0, 0};
    // the next stage's A and B tiles are fetched into registers while the
    // current stage is multiplied.  Thread tid stages the same tile
    // positions at every stage: their coordinates, bounds and addresses are
    // set once and the addresses advance by one stage per fetch (no
    // per-element index arithmetic in the loop)
    constexpr int PA = kTR * kKS / 256, PB = kKS * TC / 256;
    T pA[PA], pB[PB];
    const GLB T *qa[PA], *qb[PB];
    int ia[PA], ib[PB];  // LDS offsets of the staged elements
    int kaa[PA], kbb[PB];  // contraction index within the stage
    bool oka[PA], okb[PB];
#pragma unroll
    for (int u = 0; u < PA; u++) {
        const int i = tid + u * 256;
        const int r = a_kfast ? i / kKS : i % kTR, k = a_kfast ? i % kKS : i / kTR;
        kaa[u] = k;
        oka[u] = r0 + r < t.rows;
        ia[u] = r * (kKS + 1) + k;
        qa[u] = A + (oka[u] ? (int64_t)(r0 + r) * t.ars + (int64_t)(kb + k) * t.acs : 0);
    }
#pragma unroll
    for (int u = 0; u < PB; u++) {
        const int i = tid + u * 256;
        const int k = b_cfast ? i / TC : i % kKS, c = b_cfast ? i % TC : i / kKS;
        kbb[u] = k;
        okb[u] = c0 + c < ncol;
        ib[u] = k * (TC + 1) + c;
        qb[u] = B + (okb[u] ? (int64_t)(kb + k) * t.brs + (int64_t)(c0 + c) * t.bcs : 0);
    }
    const int64_t stepa = (int64_t)kKS * t.acs, stepb = (int64_t)kKS * t.brs;
    auto fetch = [&](int ks) {
        const int kn = min(kKS, ke - ks);
#pragma unroll
        for (int u = 0; u < PA; u++) {
            pA[u] = (oka[u] && kaa[u] < kn) ? *qa[u] : (T)0;
            qa[u] += stepa;
        }
#pragma unroll
        for (int u = 0; u < PB; u++) {
            pB[u] = (okb[u] && kbb[u] < kn) ? *qb[u] : (T)0;
            qb[u] += stepb;
        }
    };
    if (kb < ke) fetch(kb);
    for (int ks = kb; ks < ke; ks += kKS) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PA; u++) (&sA[0][0])[ia[u]] = pA[u];
#pragma unroll
        for (int u = 0; u < PB; u++) (&sB[0][0])[ib[u]] = pB[u];
        __syncthreads();
        if (ks + kKS < ke) fetch(ks + kKS);
#pragma unroll
        for (int k4 = 0; k4 < kKS; k4 += 4) {
            T a = sA[wave * 16 + lane % 16][k4 + lane / 16];
#pragma unroll
            for (int b = 0; b < NB; b++) {
                T bb = sB[k4 + lane / 16][b * 16 + lane % 16];
                acc[b] = Acc<T>::mma(a, bb, acc[b]);
            }
        }
    }
    GLB T *C = glb((T *)t.C);
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int c = c0 + b * 16 + lane % 16;
        if (c >= ncol) continue;
        for (int q = 0; q < 4; q++) {
            const int r = r0 + wave * 16 + Acc<T>::row(lane, q);
            if (r < t.rows) store_out(C, (int64_t)r * t.crs + (int64_t)c * t.ccs, (T)acc[b][q], t.op);
        }
    }
}

// dst(r, c) op= sum_p src_p(r, c), partials summed in index order
template <typename T, typename TO>
__global__ void k_reduce(const RedTask *__restrict__ tasks, int ncol, int blocks_per_task) {
    const RedTask t = tasks[blockIdx.x / blocks_per_task];
    const int64_t e = (int64_t)(blockIdx.x % blocks_per_task) * blockDim.x + threadIdx.x;
    if (t.ncol > 0) ncol = min(ncol, t.ncol);
    if (e >= (int64_t)t.rows * ncol) return;
    const int r = (int)(e / ncol), c = (int)(e % ncol);
    const GLB T *src = glb((const T *)t.src);
    double acc = 0.0;
    for (int p = 0; p < t.np; p++) acc += (double)src[p * t.pstride + (int64_t)r * t.prs + c];
    store_out(glb((TO *)t.dst), (int64_t)r * t.drs + (int64_t)c * t.dcs, (TO)acc, t.op);
}

#define KMM_INST(T, TB, TO, TC, CG)                                                                    \
    template __global__ void k_kmm<T, TB, TO, TC, false, CG>(const KmmTask *, const TileItem *, int, int); \
    template __global__ void k_kmm<T, TB, TO, TC, true, CG>(const KmmTask *, const TileItem *, int, int);
#define KMM_ALL(T, TB, TO) KMM_INST(T, TB, TO, 16, 1) KMM_INST(T, TB, TO, 64, 1) KMM_INST(T, TB, TO, 128, 1)
KMM_ALL(double, double, double)
KMM_INST(double, double, double, 128, 2)
KMM_ALL(float, float, float)
KMM_ALL(float, float, double)
KMM_ALL(double, float, double)
#define GMM_INST(T, TC) template __global__ void k_gmm<T, TC>(const GmmTask *, const TileItem *, int, int);
GMM_INST(double, 16) GMM_INST(double, 64) GMM_INST(double, 128) GMM_INST(double, 256)
GMM_INST(float, 16) GMM_INST(float, 64) GMM_INST(float, 128)
template __global__ void k_reduce<double, double>(const RedTask *, int, int);
template __global__ void k_reduce<float, float>(const RedTask *, int, int);
template __global__ void k_reduce<float, double>(const RedTask *, int, int);

}  // namespace askit
