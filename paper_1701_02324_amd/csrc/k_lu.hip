// k_lu.hip -- batched FP64 LU with partial pivoting (the GETRF of Sec. 2.2:
// leaf blocks lambda I + K_aa and reduced systems Z of eq. (8)) and the
// matching batched solves (GETRS), plain and transposed.
//
// One workgroup per matrix.  Column-major matrices; pivot = row of largest
// |a| in the column, lowest row on ties; piv[k] = row exchanged with row k.
// The factor works blocked: a panel of kPanel columns is factored with
// rank-1 updates restricted to the panel (rows held in registers, one thread
// per row), the row exchanges are kept as a permutation of row positions,
// the block row of U is solved with the unit lower panel triangle, and the
// trailing matrix receives one rank-kPanel update computed with FP64 MFMA
// (v_mfma_f64_16x16x4f64) from the LDS-staged U block row.
#include "askit_dev.h"

namespace askit {

constexpr int kPanel = kLuPanel;
static_assert(kLuFThreads % kWave == 0, "whole waves");
static_assert(kLuFThreads >= kLuMaxN, "one thread per row of the largest matrix");

// ---------------------------------------------------------------------------
// Trailing update A22 -= L21 U12 of a blocked LU of depth KP (kPanel): the
// rows r0 + ci (ci < nr) and columns c0 + cj (cj < nc) of A receive the
// product of L21 = A(rows, kb .. kb+KP-1) and U12, computed as its transpose
// U12^T L21^T so that an accumulator register holds 16 consecutive rows of a
// column (coalesced column-major access).  Logical row i of A is physical
// row rowof(i).  U12 is staged in LDS, row-major: W[k * ldw + cj] for cj in
// whole 64-column blocks covering nc (values past nc are never written
// back).  With LOWER, column blocks entirely above the diagonal (global
// column > global row) are skipped.  Wave w takes the 16-row stripes w, w + NW, ...: it loads the
// stripe's L21 rows once, then goes over 64-column blocks, fetching the next
// block's A22 values before the current block's products; a block's U12
// operands are read from LDS (4 rows of k at a time) before their products.
// ---------------------------------------------------------------------------
template <int NW, int KP, bool LOWER = false, class RowOf>
__device__ inline void trailing_update(GLB double *A, int lda, int kb, int r0, int nr, int c0, int nc,
                                       const double *W, int ldw, RowOf rowof, int wave, int lane) {
    static_assert(KP % 16 == 0, "depth in multiples of 16");
    const int bt = (nr + 15) / 16, ncb_all = (nc + 63) / 64;
    const int row = lane % 16, kq = lane / 16;
    for (int st = wave; st < bt; st += NW) {
        // LOWER: only the column blocks that reach the diagonal or below
        const int ncb = LOWER ? min(ncb_all, (r0 - c0 + st * 16 + 15) / 64 + 1) : ncb_all;
        const int ci = st * 16 + row;
        const int64_t rb = ci < nr ? rowof(r0 + ci) : 0;
        // this stripe's L21 rows, kept for all its column blocks
        double l[KP / 4];
#pragma unroll
        for (int kk = 0; kk < KP / 4; kk++) l[kk] = ci < nr ? A[rb + (int64_t)(kb + 4 * kk + kq) * lda] : 0.0;
        // element (q, r) of column block cbk is column c0 + 64 cbk + 16 q +
        // 4 r + kq of this lane's row: one base pointer per stripe and
        // strides instead of a 64-bit product per element, and no bounds
        // tests in the blocks that lie inside the matrix
        const bool live = ci < nr;
        GLB double *rp = A + rb + (int64_t)(c0 + kq) * lda;
        const int64_t l4 = 4 * (int64_t)lda, l16 = 16 * (int64_t)lda, l64 = 64 * (int64_t)lda;
        auto fetch = [&](int cbk, double (&c)[4][4]) {
            GLB double *bp = rp + (int64_t)cbk * l64;
            if (live && 64 * (cbk + 1) <= nc) {
#pragma unroll
                for (int q = 0; q < 4; q++)
#pragma unroll
                    for (int r = 0; r < 4; r++) c[q][r] = bp[q * l16 + r * l4];
            } else {
#pragma unroll
                for (int q = 0; q < 4; q++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int cj = (4 * cbk + q) * 16 + 4 * r + kq;
                        c[q][r] = (live && cj < nc) ? bp[q * l16 + r * l4] : 0.0;
                    }
            }
        };
        auto update = [&](int cbk, const double (&c)[4][4]) {
            const int cb0 = 4 * cbk;
            dbl4 acc[4];
#pragma unroll
            for (int q = 0; q < 4; q++) acc[q] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int h = 0; h < KP / 16; h++) {
                double ua[4][4];
#pragma unroll
                for (int kk = 0; kk < 4; kk++)
#pragma unroll
                    for (int q = 0; q < 4; q++)
                        ua[kk][q] = W[(4 * (4 * h + kk) + kq) * ldw + (cb0 + q) * 16 + row];
#pragma unroll
                for (int kk = 0; kk < 4; kk++)
#pragma unroll
                    for (int q = 0; q < 4; q++)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[kk][q], l[4 * h + kk], acc[q], 0, 0, 0);
            }
            // acc[q][r] = entry (row st*16 + lane%16, column (cb0+q)*16 + 4r + lane/16)
            GLB double *bp = rp + (int64_t)cbk * l64;
            if (live && 64 * (cbk + 1) <= nc) {
#pragma unroll
                for (int q = 0; q < 4; q++)
#pragma unroll
                    for (int r = 0; r < 4; r++) bp[q * l16 + r * l4] = c[q][r] - acc[q][r];
            } else if (live) {
#pragma unroll
                for (int q = 0; q < 4; q++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int cj = (cb0 + q) * 16 + 4 * r + kq;
                        if (cj < nc) bp[q * l16 + r * l4] = c[q][r] - acc[q][r];
                    }
            }
        };
        double cA[4][4], cB[4][4];
        fetch(0, cA);
        for (int cbk = 0; cbk < ncb; cbk += 2) {
            if (cbk + 1 < ncb) fetch(cbk + 1, cB);
            update(cbk, cA);
            if (cbk + 1 < ncb) {
                if (cbk + 2 < ncb) fetch(cbk + 2, cA);
                update(cbk + 1, cB);
            }
        }
    }
}

// Shared memory of one panel of the blocked LU: L11 the unit lower panel
// triangle; redv / redk the per-wave pivot candidates; prb the pivot row;
// sp the panel's pivot rows.
struct LuPanelLds {
    double L11[kPanel * kPanel];
    double redv[kLuFThreads / kWave];
    int redk[kLuFThreads / kWave];
    double prb[kPanel];
    int32_t sp[kPanel];
};

// Panel kb of the blocked LU (columns kb .. kb+nb-1, rows kb .. n-1) and the
// U block row right of it, by one workgroup of kLuFThreads threads.
// Logical row i of the matrix is stored in physical row prow[i] (LDS): row
// exchanges only swap entries there.  With STAGE the U block row is also
// left in W (row-major, ld = trailing columns rounded up to 64) for the
// trailing update.  Ends with a barrier.  Returns the
// number of trailing columns n - kb - nb.
template <bool STAGE>
__device__ inline int lu_panel(GLB double *A, GLB int32_t *piv, int n, int lda, int kb, int32_t *prow,
                               LuPanelLds &S, double *W, double &s_min, double &s_max, int tid, int lane, int wave) {
    constexpr int NW = kLuFThreads / kWave;
    const int nb = n - kb < kPanel ? n - kb : kPanel, m = n - kb;
    // ---- panel: thread r < m holds panel row r in registers.  Rows do not
    // move: each keeps its logical position lp and an exchange only swaps two
    // positions, so a column step is one pivot search over the rows not
    // chosen yet, one broadcast of the pivot row through LDS and a local
    // rank-1 update.
    {
        const bool own = tid < m;
        const int32_t arow = own ? prow[kb + tid] : 0;
        double rw[kPanel];
#pragma unroll
        for (int j = 0; j < kPanel; j++) rw[j] = (own && j < nb) ? A[arow + (int64_t)(kb + j) * lda] : 0.0;
        int lp = tid;
        bool done = !own;
#pragma unroll
        for (int k = 0; k < kPanel; k++) {
            if (k < nb) {
                // largest |a| of column k over the remaining rows (a NaN
                // counts as infinite), ties to the lowest position: the
                // maximum first, then the smallest key = position * 1024
                // + row among the rows holding it
                const double a = rw[k];
                const double v = done ? -1.0 : (a != a ? INFINITY : fabs(a));
                const double wm = wave_max_d(v);
                const int wk = wave_min_i(v == wm ? ((lp << 10) | tid) : 0x7fffffff);
                if (lane == 0) {
                    S.redv[wave] = wm;
                    S.redk[wave] = wk;
                }
                __syncthreads();
                double bv = S.redv[0];
#pragma unroll
                for (int w = 1; w < NW; w++) bv = fmax(bv, S.redv[w]);
                int bk = 0x7fffffff;
#pragma unroll
                for (int w = 0; w < NW; w++) bk = S.redv[w] == bv ? min(bk, S.redk[w]) : bk;
                const int P = bk & 1023, p = bk >> 10;
                if (tid == P) {
#pragma unroll
                    for (int j = 0; j < kPanel; j++) S.prb[j] = rw[j];
                    done = true;
                }
                if (tid == 0) S.sp[k] = kb + p;
                if (lp == k) lp = p;  // the row at position k moves to p
                if (tid == P) lp = k;
                __syncthreads();
                const double ukk = S.prb[k];
                const double au = fabs(ukk);
                s_min = au == au ? fmin(s_min, au) : 0.0;
                s_max = fmax(s_max, au);
                if (!done && ukk != 0.0) {
                    const double l = rw[k] / ukk;
                    rw[k] = l;
#pragma unroll
                    for (int j = k + 1; j < kPanel; j++) rw[j] = fma(-l, S.prb[j], rw[j]);
                }
            }
        }
        // rows stay where they are in A; their positions go into prow
        if (own) {
#pragma unroll
            for (int j = 0; j < kPanel; j++)
                if (j < nb) A[arow + (int64_t)(kb + j) * lda] = rw[j];
            if (lp < nb) {
#pragma unroll
                for (int c = 0; c < kPanel; c++)
                    if (c < nb) S.L11[lp + c * kPanel] = rw[c];
            }
            prow[kb + lp] = arow;
        }
        if (tid < nb) piv[kb + tid] = S.sp[tid];
        __syncthreads();
    }
    const int j0 = kb + nb, nt = n - j0;
    if (nt <= 0) return nt;  // only the last panel can be narrower than kPanel
    // ---- U block row: A[kb:kb+32, j0:n] = L11^{-1} A[kb:kb+32, j0:n],
    // thread j solves column j0 + j in registers (the same operations, in
    // the same order, as row-by-row substitution); with STAGE the rows are
    // also staged in W, zero-padded to ldw columns
    const int ldw = (nt + 63) & ~63;
    if (STAGE && tid >= nt && tid < ldw) {
#pragma unroll
        for (int r = 0; r < kPanel; r++) W[r * ldw + tid] = 0.0;
    }
    if (tid < nt) {
        const int64_t col = (int64_t)(j0 + tid) * lda;
        double u[kPanel];
#pragma unroll
        for (int r = 0; r < kPanel; r++) u[r] = A[prow[kb + r] + col];
#pragma unroll
        for (int c = 0; c < kPanel; c++)
#pragma unroll
            for (int r = c + 1; r < kPanel; r++) u[r] = fma(-S.L11[r + c * kPanel], u[c], u[r]);
#pragma unroll
        for (int r = 0; r < kPanel; r++) {
            A[prow[kb + r] + col] = u[r];
            if (STAGE) W[r * ldw + tid] = u[r];
        }
    }
    __syncthreads();
    return nt;
}

// Rows in place (physical row prow[i] becomes row i): column batches of
// kPanel staged in W.
__device__ inline void lu_rows_in_place(GLB double *A, int n, int lda, const int32_t *prow, double *W, int tid) {
    constexpr int NT = kLuFThreads;
    for (int cb = 0; cb < n; cb += kPanel) {
        const int nc = n - cb < kPanel ? n - cb : kPanel;
        for (int e = tid; e < n * nc; e += NT) {
            const int r = e % n, c = e / n;
            W[e] = A[prow[r] + (int64_t)(cb + c) * lda];
        }
        __syncthreads();
        for (int e = tid; e < n * nc; e += NT) {
            const int r = e % n, c = e / n;
            A[r + (int64_t)(cb + c) * lda] = W[e];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kLuFThreads) void k_lu(const LuTask *__restrict__ tasks) {
    constexpr int NT = kLuFThreads, NW = NT / kWave;
    // W: the U block row, then staging of the final row pass
    __shared__ double W[kPanel * kLuMaxN];
    __shared__ LuPanelLds S;
    __shared__ int32_t prow[kLuMaxN];
    const LuTask t = tasks[blockIdx.x];
    const int n = t.n, lda = t.lda, tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    GLB double *A = glb(t.A);
    // smallest and largest |pivot| (every thread sees every pivot)
    double s_min = INFINITY, s_max = 0.0;
    for (int i = tid; i < n; i += NT) prow[i] = i;
    __syncthreads();
    for (int kb = 0; kb < n; kb += kPanel) {
        const int nt = lu_panel<true>(A, glb(t.piv), n, lda, kb, prow, S, W, s_min, s_max, tid, lane, wave);
        if (nt <= 0) continue;
        const int j0 = n - nt, ldw = (nt + 63) & ~63;
        trailing_update<NW, kPanel>(A, lda, kb, j0, nt, j0, nt, W, ldw, [&](int i) -> int64_t { return prow[i]; },
                                    wave, lane);
        __syncthreads();
    }
    lu_rows_in_place(A, n, lda, prow, W, tid);
    if (tid == 0 && t.ratio) *glb(t.ratio) = n ? (s_max > 0.0 ? s_min / s_max : 0.0) : 1.0;
}

// ---------------------------------------------------------------------------
// The same factorization split over launches, for batches whose largest
// matrices leave most compute units idle under one workgroup per matrix:
// per panel, k_lup_panel factors the panel and solves the U block row (one
// workgroup per matrix, the code of k_lu), then k_lup_update applies the
// trailing update in 64 x 64 tiles, one workgroup each (the trailing update
// of k_lu restricted to the tile: the same products in the same order, so
// the factors are bit for bit those of k_lu); k_lup_finish puts the rows in
// place, a few columns per workgroup.  Between launches each matrix's row positions and pivot extremes
// live in LuSplit.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kLuFThreads) void k_lup_panel(const LuTask *__restrict__ tasks, LuSplit w, int kb) {
    constexpr int NT = kLuFThreads;
    __shared__ LuPanelLds S;
    __shared__ int32_t prow[kLuMaxN];
    const LuTask t = tasks[blockIdx.x];
    const int n = t.n, lda = t.lda, tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    if (kb >= n) return;
    GLB int32_t *gp = glb(w.prow) + (int64_t)blockIdx.x * kLuMaxN;
    GLB double *gs = glb(w.smm) + 2 * (int64_t)blockIdx.x;
    double s_min = INFINITY, s_max = 0.0;
    if (kb == 0) {
        for (int i = tid; i < n; i += NT) prow[i] = i;
    } else {
        for (int i = tid; i < n; i += NT) prow[i] = gp[i];
        s_min = gs[0];
        s_max = gs[1];
    }
    __syncthreads();
    lu_panel<false>(glb(t.A), glb(t.piv), n, lda, kb, prow, S, nullptr, s_min, s_max, tid, lane, wave);
    // the panel moved positions kb .. n-1 only
    for (int i = kb + tid; i < n; i += NT) gp[i] = prow[i];
    if (tid == 0) {
        gs[0] = s_min;
        gs[1] = s_max;
    }
}

__global__ __launch_bounds__(kLupThreads) void k_lup_update(const LuTask *__restrict__ tasks, LuSplit w,
                                                             const TileItem *__restrict__ items, int kb) {
    __shared__ double W[kPanel * 64];
    const TileItem it = items[blockIdx.x];
    if (it.task < 0) return;  // padding of the compute-die order
    const LuTask t = tasks[it.task];
    const int n = t.n, lda = t.lda, tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int j0 = kb + kPanel, r0 = j0 + 64 * it.rt, c0 = j0 + 64 * it.ct;
    const int nr = min(64, n - r0), nc = min(64, n - c0);
    GLB double *A = glb(t.A);
    const GLB int32_t *gp = glb(w.prow) + (int64_t)it.task * kLuMaxN;
    // the tile's columns of the U block row, zero past nc
    for (int e = tid; e < kPanel * 64; e += kLupThreads) {
        const int k = e / 64, cj = e % 64;
        W[e] = cj < nc ? A[gp[kb + k] + (int64_t)(c0 + cj) * lda] : 0.0;
    }
    __syncthreads();
    trailing_update<kLupThreads / kWave, kPanel>(A, lda, kb, r0, nr, c0, nc, W, 64,
                                                 [&](int i) -> int64_t { return gp[i]; }, wave, lane);
}

// Rows in place, kLupFinCols columns per workgroup (the columns are
// independent): lanes 32 c .. 32 c + 31 move column c0 + c, each lane every
// 32nd row, through registers; the barrier separates the reads of the
// workgroup's columns from its writes.
__global__ __launch_bounds__(kLupThreads) void k_lup_finish(const LuTask *__restrict__ tasks, LuSplit w,
                                                             const TileItem *__restrict__ items) {
    static_assert(kLupThreads == 32 * kLupFinCols, "32 lanes per column");
    constexpr int RPL = kLuMaxN / 32;  // rows per lane
    const TileItem it = items[blockIdx.x];
    const LuTask t = tasks[it.task];
    const int n = t.n, lda = t.lda, tid = threadIdx.x;
    const int c = it.rt * kLupFinCols + tid / 32, r0 = tid % 32;
    const bool live = c < n;
    GLB double *col = glb(t.A) + (int64_t)c * lda;
    const GLB int32_t *gp = glb(w.prow) + (int64_t)it.task * kLuMaxN;
    double v[RPL];
#pragma unroll
    for (int i = 0; i < RPL; i++) {
        const int r = r0 + 32 * i;
        v[i] = live && r < n ? col[gp[r]] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPL; i++) {
        const int r = r0 + 32 * i;
        if (live && r < n) col[r] = v[i];
    }
    if (it.rt == 0 && tid == 0 && t.ratio) {
        const GLB double *gs = glb(w.smm) + 2 * (int64_t)it.task;
        *glb(t.ratio) = n ? (gs[1] > 0.0 ? gs[0] / gs[1] : 0.0) : 1.0;
    }
}

// ---------------------------------------------------------------------------
// LU without row exchanges for symmetric positive definite matrices (the leaf
// blocks lambda I + K_aa, lambda > 0): elimination without pivoting is
// backward stable there and gives the factors GETRF gives whenever it
// exchanges no rows.  Blocked by 32 columns: the diagonal block is factored
// by one wave with its rows in registers (pivot rows shared by lane
// shuffles); U11 is inverted in registers; L21 = A21 U11^{-1} is a product on
// FP64 MFMA and U12 = D L21^T (D = diag(U11)), as the factors of a symmetric
// matrix without row exchanges satisfy U = D L^T.  The trailing matrix stays
// symmetric, so only its blocks on or below the diagonal are updated (the
// trailing update of k_lu restricted to them); each upper entry is written
// once, as part of U12.  piv[k] = k.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kLuFThreads) void k_lu_nopiv(const LuTask *__restrict__ tasks) {
    constexpr int NT = kLuFThreads, NW = NT / kWave, DL = kPanel + 1;
    __shared__ double Up[kPanel * kLuMaxN];  // U block row (row-major, ld = nt rounded up to 64)
    __shared__ double Dg[kPanel * DL];       // factored diagonal block (row-major)
    __shared__ double UI[kPanel * DL];       // U11^{-1} (row-major)
    __shared__ double s_min, s_max;
    const LuTask t = tasks[blockIdx.x];
    const int n = t.n, lda = t.lda, tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    GLB double *A = glb(t.A);
    if (tid == 0) {
        s_min = INFINITY;
        s_max = 0.0;
    }
    for (int i = tid; i < n; i += NT) glb(t.piv)[i] = i;
    for (int kb = 0; kb < n; kb += kPanel) {
        const int nb = n - kb < kPanel ? n - kb : kPanel;
        // ---- diagonal block, factored by wave 0: lane i < nb holds row i in
        // registers, the pivot row is broadcast by lane shuffles (fully
        // unrolled: every register index is static)
        if (wave == 0) {
            double rw[kPanel];
#pragma unroll
            for (int j = 0; j < kPanel; j++)
                rw[j] = (lane < nb && j < nb) ? A[kb + lane + (int64_t)(kb + j) * lda] : (lane == j ? 1.0 : 0.0);
#pragma unroll
            for (int k = 0; k < kPanel; k++) {
                const double ukk = readlane_d(rw[k], k);
                const bool act = k < nb && lane > k && lane < nb;
                const double l = (act && ukk != 0.0) ? rw[k] / ukk : 0.0;
                if (act) rw[k] = l;
#pragma unroll
                for (int j = k + 1; j < kPanel; j++) {
                    const double pj = readlane_d(rw[j], k);
                    if (act) rw[j] = fma(-l, pj, rw[j]);
                }
            }
            if (lane < kPanel) {
#pragma unroll
                for (int j = 0; j < kPanel; j++) Dg[lane * DL + j] = rw[j];
            }
            if (lane < nb) {
#pragma unroll
                for (int j = 0; j < kPanel; j++)
                    if (j < nb) A[kb + lane + (int64_t)(kb + j) * lda] = rw[j];
            }
        }
        __syncthreads();
        // ---- inverse of U11, one column per lane in registers: column j
        // of U^{-1} by lane j of wave 1 (terms with a zero factor included:
        // they leave the sums unchanged); pivot magnitudes by wave 3
        if (wave == 1 && lane < kPanel) {
            const int j = lane;
            double x[kPanel];
#pragma unroll
            for (int i = kPanel - 1; i >= 0; i--) {
                double acc = i == j ? 1.0 : 0.0;
#pragma unroll
                for (int k = i + 1; k < kPanel; k++) acc = fma(-Dg[i * DL + k], x[k], acc);
                const double u = Dg[i * DL + i];
                x[i] = i > j ? 0.0 : (u != 0.0 ? acc / u : 0.0);
            }
#pragma unroll
            for (int i = 0; i < kPanel; i++) UI[i * DL + j] = x[i];
        } else if (wave == 3 && lane == 0) {
            for (int i = 0; i < nb; i++) {
                const double au = fabs(Dg[i * DL + i]);
                s_min = fmin(s_min, au);
                s_max = fmax(s_max, au);
            }
        }
        __syncthreads();
        const int j0 = kb + nb, nt = n - j0;
        if (nt <= 0) continue;  // only the last panel can be narrower than kPanel
        const int rr = lane % 16, kq = lane / 16;
        // ---- L21 = A21 U11^{-1}, 16-row stripes, and with it U12 = D L21^T
        // (D = diag(U11)): without row exchanges the factors of a symmetric
        // matrix satisfy U = D L^T, so the block row of U comes from L21 (the
        // trailing matrix's upper part is not kept up to date).  U12 is also
        // staged in Up (zero-padded to ldw columns).
        const int ldw = (nt + 63) & ~63;
        for (int e = tid; e < kPanel * (ldw - nt); e += NT) Up[(e / (ldw - nt)) * ldw + nt + e % (ldw - nt)] = 0.0;
#pragma unroll 1
        for (int st = wave; st < (nt + 15) / 16; st += NW) {
            const int i0 = st * 16;
            dbl4 acc[2] = {dbl4{0, 0, 0, 0}, dbl4{0, 0, 0, 0}};
            double a[kPanel / 4];
#pragma unroll
            for (int kk = 0; kk < kPanel / 4; kk++)
                a[kk] = i0 + rr < nt ? A[j0 + i0 + rr + (int64_t)(kb + 4 * kk + kq) * lda] : 0.0;
#pragma unroll
            for (int kk = 0; kk < kPanel / 4; kk++)
#pragma unroll
                for (int cb = 0; cb < 2; cb++)
                    acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], UI[(4 * kk + kq) * DL + cb * 16 + rr],
                                                                   acc[cb], 0, 0, 0);
#pragma unroll
            for (int cb = 0; cb < 2; cb++) {
                const int k = cb * 16 + rr;
                const double dk = Dg[k * DL + k];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int r = i0 + 4 * q + kq;
                    if (r < nt) {
                        A[j0 + r + (int64_t)(kb + k) * lda] = acc[cb][q];
                        const double u = dk * acc[cb][q];
                        A[kb + k + (int64_t)(j0 + r) * lda] = u;
                        Up[k * ldw + r] = u;
                    }
                }
            }
        }
        __syncthreads();
        // ---- trailing update A22 -= L21 U12
        trailing_update<NW, kPanel, true>(A, lda, kb, j0, nt, j0, nt, Up, ldw, [](int i) -> int64_t { return i; }, wave,
                                          lane);
        __syncthreads();
    }
    if (tid == 0 && t.ratio) *glb(t.ratio) = n ? (s_max > 0.0 ? s_min / s_max : 0.0) : 1.0;
}

// ---------------------------------------------------------------------------
// Inverses of the 16 x 16 diagonal blocks of L (unit lower) and U, used by the
// blocked triangular solves: Dinv[2b] = L_bb^{-1}, Dinv[2b+1] = U_bb^{-1}
// (column-major 16 x 16; a partial last block is completed by the identity).
// One workgroup per matrix, one lane per block column.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lu_diaginv(const LuTask *__restrict__ tasks) {
    // the 16 x 16 diagonal blocks of a pass (eight: 32 jobs each) are staged
    // in LDS once, completed by the identity beyond n, then read by the jobs
    __shared__ double sT[8][256];
    const LuTask t = tasks[blockIdx.x];
    const int n = t.n, lda = t.lda, nb = (n + 15) / 16;
    const int tid = threadIdx.x, tile = tid / 32;
    for (int base = 0; base < nb * 32; base += 256) {
        const int bs = base / 32 + tile;  // the block this thread stages and solves
        if (bs < nb) {
            const int b0 = bs * 16;
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int e = tid % 32 + 32 * u, r = e % 16, c = e / 16, gr = b0 + r, gc = b0 + c;
                sT[tile][e] = (gr >= n || gc >= n) ? (r == c ? 1.0 : 0.0) : glb((const double *)t.A)[gr + (int64_t)gc * lda];
            }
        }
        __syncthreads();
        const int job = base + tid;
        if (job < nb * 32) {
            const int b = job / 32, j = job % 16, upper = (job % 32) / 16;
            const double *T = sT[tile];
            auto a = [&](int r, int c) -> double { return T[r + 16 * c]; };
            double x[16];
            GLB double *out = glb(t.dinv) + ((int64_t)(2 * b + upper)) * 256;
            if (!upper) {  // x = L^{-1} e_j, unit diagonal
                for (int i = 0; i < 16; i++) {
                    double acc = (i == j) ? 1.0 : 0.0;
                    for (int k = 0; k < i; k++) acc = fma(-a(i, k), x[k], acc);
                    x[i] = acc;
                }
            } else {  // x = U^{-1} e_j
                for (int i = 15; i >= 0; i--) {
                    double acc = (i == j) ? 1.0 : 0.0;
                    for (int k = i + 1; k < 16; k++) acc = fma(-a(i, k), x[k], acc);
                    x[i] = acc / a(i, i);
                }
            }
            for (int i = 0; i < 16; i++) out[i + 16 * j] = x[i];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Batched LU solves (GETRS) A X = B or A^T X = B for right-hand sides stored
// row-major (n x nrhs, row stride ldb), FP32 or FP64 storage, FP64
// arithmetic.  One workgroup per (matrix, panel of NR columns); the panel is
// held in LDS.  Each triangular sweep goes over 16-row blocks: the block is
// finished with its precomputed diagonal inverse, then the remaining blocks
// receive a rank-16 update, both on the FP64 matrix cores.
// ---------------------------------------------------------------------------
// The sweeps below load the operands of block step ib + 1 (its diagonal
// inverse and its coupling blocks, which do not depend on the right-hand
// sides) while step ib is applied, so that each step waits on LDS and the
// matrix cores only.  A step's coupling jobs (J, column block) fit one
// batch of kLsU jobs per wave: (nb - 1) CB <= 31 * 2 < 16 * 4.
constexpr int kLsU = 4;
static_assert((kLuMaxN / 16 - 1) * 2 <= (kLsThreads / kWave) * kLsU, "one batch of coupling jobs per step");

// this lane's operand of the diagonal product: D'(row, k) for its k4 steps
__device__ inline void load_diag(double (&dv)[4], const GLB double *D, bool transD, int lane, bool use) {
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const int row = lane % 16, kk = 4 * s + lane / 16;
        dv[s] = use ? (transD ? D[kk + 16 * row] : D[row + 16 * kk]) : 0.0;
    }
}

// S[r0:r0+16, :] = D' S[r0:r0+16, :]: wave cb < CB reads and rewrites the
// 16 x 16 block of its own columns only, so no barrier separates its reads
// from its writes; the barrier after them publishes the block to the update
template <int NR>
__device__ inline void diag_apply_reg(double (*S)[NR + 1], int r0, const double (&dv)[4], int lane, int wave) {
    constexpr int CB = NR / 16;
    const int cb = wave;
    if (cb < CB) {
        dbl4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const double b = S[r0 + 4 * s + lane / 16][cb * 16 + lane % 16];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(dv[s], b, acc, 0, 0, 0);
        }
        for (int q = 0; q < 4; q++) S[r0 + 4 * q + lane / 16][cb * 16 + lane % 16] = acc[q];
    }
    __syncthreads();
}

// this wave's coupling values of the jobs of one block step (blocks J in
// [jb0, jb1) against rows i0 .. i0 + 15)
template <int NR, typename G>
__device__ inline void load_coupling(double (&a)[kLsU][4], int i0, int jb0, int jb1, G get, int lane, int wave) {
    constexpr int CB = NR / 16, NW = kLsThreads / kWave;
    const int njobs = (jb1 - jb0) * CB;
#pragma unroll
    for (int u = 0; u < kLsU; u++) {
        const int job = wave + u * NW;
        const int J = jb0 + job / CB;
#pragma unroll
        for (int k4 = 0; k4 < 4; k4++) a[u][k4] = job < njobs ? get(J * 16 + lane % 16, i0 + 4 * k4 + lane / 16) : 0.0;
    }
}

template <int NR>
__device__ inline void block_update_reg(double (*S)[NR + 1], int i0, int jb0, int jb1, const double (&a)[kLsU][4],
                                        int lane, int wave) {
    constexpr int CB = NR / 16, NW = kLsThreads / kWave;
    const int njobs = (jb1 - jb0) * CB;
#pragma unroll
    for (int u = 0; u < kLsU; u++) {
        const int job = wave + u * NW;
        if (job >= njobs) break;
        const int J = jb0 + job / CB, cb = job % CB;
        dbl4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int k4 = 0; k4 < 4; k4++) {
            double b = S[i0 + 4 * k4 + lane / 16][cb * 16 + lane % 16];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][k4], b, acc, 0, 0, 0);
        }
        for (int q = 0; q < 4; q++) S[J * 16 + 4 * q + lane / 16][cb * 16 + lane % 16] -= acc[q];
    }
    __syncthreads();
}

// one triangular sweep: forward (ib = 0 .. nb - 1, coupling blocks below)
// or backward (ib = nb - 1 .. 0, coupling blocks above); D(ib) is the
// diagonal inverse of step ib
template <int NR, typename G, typename DP>
__device__ inline void sweep(double (*S)[NR + 1], int nb, bool forward, DP dptr, bool transD, G get, int lane,
                             int wave) {
    constexpr int CB = NR / 16;
    double dv[4], a[kLsU][4];
    const int ib0 = forward ? 0 : nb - 1;
    auto range = [&](int ib, int &j0, int &j1) {
        j0 = forward ? ib + 1 : 0;
        j1 = forward ? nb : ib;
    };
    int j0, j1;
    range(ib0, j0, j1);
    load_diag(dv, dptr(ib0), transD, lane, wave < CB);
    load_coupling<NR>(a, ib0 * 16, j0, j1, get, lane, wave);
    for (int t = 0; t < nb; t++) {
        const int ib = forward ? t : nb - 1 - t;
        double dc[4], ac[kLsU][4];
#pragma unroll
        for (int s2 = 0; s2 < 4; s2++) dc[s2] = dv[s2];
#pragma unroll
        for (int u = 0; u < kLsU; u++)
#pragma unroll
            for (int k4 = 0; k4 < 4; k4++) ac[u][k4] = a[u][k4];
        if (t + 1 < nb) {  // the next step's operands, loaded while this one is applied
            const int in = forward ? ib + 1 : ib - 1;
            range(in, j0, j1);
            load_diag(dv, dptr(in), transD, lane, wave < CB);
            load_coupling<NR>(a, in * 16, j0, j1, get, lane, wave);
        }
        range(ib, j0, j1);
        diag_apply_reg<NR>(S, ib * 16, dc, lane, wave);
        block_update_reg<NR>(S, ib * 16, j0, j1, ac, lane, wave);
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8); the (matrix, panel) pairs are numbered so that the panels of one
// matrix land on the same XCD and share its factors in that XCD's L2.
template <typename T, int NR, bool TRANS>
__global__ __launch_bounds__(kLsThreads) void k_lusolve(const LuTask *__restrict__ tasks, int ntask, int nrhs,
                                                        int panels) {
    __shared__ double S[kLuMaxN][NR + 1];
    __shared__ int32_t P[kLuMaxN];  // row interchanges, applied in order from LDS
    const int total = ntask * panels, chunk = (total + 7) / 8;
    const int L = (blockIdx.x % 8) * chunk + blockIdx.x / 8;
    if (L >= total) return;
    const LuTask t = tasks[L / panels];
    const int c0 = (L % panels) * NR;
    if (t.nrhs > 0) nrhs = min(nrhs, t.nrhs);
    if (c0 >= nrhs) return;
    const int ncols = min(NR, nrhs - c0);
    const int n = t.n, lda = t.lda, nb = (n + 15) / 16, tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const GLB double *A = glb((const double *)t.A);
    GLB T *B = glb((T *)t.B);
    const GLB double *dinv = glb((const double *)t.dinv);
    const GLB int32_t *piv = glb((const int32_t *)t.piv);
    for (int i = tid; i < nb * 16 * NR; i += kLsThreads) {
        const int r = i / NR, c = i % NR;
        S[r][c] = (r < n && c < ncols) ? (double)B[(int64_t)r * t.ldb + c0 + c] : 0.0;
    }
    for (int k = tid; k < n; k += kLsThreads) P[k] = piv[k];
    __syncthreads();
    auto Lget = [&](int r, int c) -> double { return (r < n && c < n && r > c) ? A[r + (int64_t)c * lda] : 0.0; };
    auto Uget = [&](int r, int c) -> double { return (r < n && c < n && r <= c) ? A[r + (int64_t)c * lda] : 0.0; };
    if (!TRANS) {
        if (tid < NR)
            for (int k = 0; k < n; k++) {
                const int p = P[k];
                if (p != k) {
                    double a = S[k][tid];
                    S[k][tid] = S[p][tid];
                    S[p][tid] = a;
                }
            }
        __syncthreads();
        // L y = P b, then U x = y
        sweep<NR>(S, nb, true, [&](int ib) { return dinv + (int64_t)(2 * ib) * 256; }, false, Lget, lane, wave);
        sweep<NR>(S, nb, false, [&](int ib) { return dinv + (int64_t)(2 * ib + 1) * 256; }, false, Uget, lane, wave);
    } else {
        auto UTget = [&](int r, int c) -> double { return Uget(c, r); };
        auto LTget = [&](int r, int c) -> double { return Lget(c, r); };
        // U^T z = b, then L^T w = z
        sweep<NR>(S, nb, true, [&](int ib) { return dinv + (int64_t)(2 * ib + 1) * 256; }, true, UTget, lane, wave);
        sweep<NR>(S, nb, false, [&](int ib) { return dinv + (int64_t)(2 * ib) * 256; }, true, LTget, lane, wave);
        if (tid < NR)
            for (int k = n - 1; k >= 0; k--) {
                const int p = P[k];
                if (p != k) {
                    double a = S[k][tid];
                    S[k][tid] = S[p][tid];
                    S[p][tid] = a;
                }
            }
        __syncthreads();
    }
    for (int i = tid; i < n * NR; i += kLsThreads) {
        const int r = i / NR, c = i % NR;
        if (c < ncols) B[(int64_t)r * t.ldb + c0 + c] = (T)S[r][c];
    }
}

#define LUS_INST(T, NR)                                                              \
    template __global__ void k_lusolve<T, NR, false>(const LuTask *, int, int, int); \
    template __global__ void k_lusolve<T, NR, true>(const LuTask *, int, int, int);
LUS_INST(double, 16) LUS_INST(double, 32) LUS_INST(float, 16) LUS_INST(float, 32)

}  // namespace askit
