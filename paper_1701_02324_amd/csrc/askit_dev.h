// askit_dev.h -- device-side types shared by the HIP translation units of
// libaskit (gfx950).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace askit {

constexpr int kWave = 64;
constexpr int kMaxDim = 64;      // largest point dimension d accepted
constexpr int kTreeChunk = 256;  // positions per chunk of the tree reductions
constexpr int kPowerIters = 50;  // power iterations for the principal axis
constexpr double kRankGuard = 1e-14;
constexpr int kQsThreads = 256;  // threads per workgroup of the split QRCP
constexpr int kQsCols = 8;       // columns per workgroup of the split QRCP (two per wave)
constexpr int kQsFinishCols = 64;  // columns of T = R11^-1 R12 per workgroup of the split QRCP's last kernel
constexpr int kQsState = 8;      // ints of per-node state of the split QRCP
constexpr int kOneWgLevel = 10;  // pipelined call, by default: tree levels from here (>= 1024 nodes) use one workgroup per node
constexpr int kLsThreads = 1024; // batched LU solves: 16 waves keep many block loads in flight
constexpr int kLuFThreads = 512; // batched LU factorization
constexpr int kLuMaxN = 512;     // largest matrix of the batched LU
constexpr int kLuPanel = 32;     // panel width of the blocked LU
constexpr int kLupThreads = 256; // LU split over launches: threads of a trailing-update tile
constexpr int kLupFinCols = 8;   // LU split over launches: columns per workgroup of the final row pass
constexpr int kLuSplitN = 256;   // LU batches whose largest matrix is larger are split over launches
constexpr int kXrDim = 16;       // kernel-block products keep row points in registers up to this dimension
constexpr int kNbrThreads = 1024; // neighbour-list ranking: threads per node
constexpr int kNbrLds = 4096;     // neighbour-list ranking: keys sorted in LDS (more go to a scratch slot)
constexpr int kKnnMax = 64;       // largest kappa of the neighbour search (32 for d > 32)

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Pointers taken from task structs are generic (flat) to the compiler, and
// flat loads count against the LDS wait counter too: a kernel that waits for
// an LDS read then also waits for every global load in flight.  Kernels hold
// such pointers as global-address-space pointers (GLB) instead.
#define GLB __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ GLB T *glb(T *p) { return (GLB T *)p; }
typedef float flt4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Cross-lane reductions: rows of 16 lanes by DPP (quad xor 1, quad xor 2,
// half-row mirror, row mirror), then the four row results by readlane.
// Every lane receives the wave's result, and the same value (the pairings
// are symmetric).  The whole wave must be active.
// ---------------------------------------------------------------------------
template <int CTRL> __device__ inline int dpp_i(int x) { return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false); }
template <int CTRL> __device__ inline double dpp_d(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// value of x in lane l (l uniform across the wave)
__device__ inline double readlane_d(double x, int l) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double wave_max_d(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    v = fmax(v, dpp_d<0x140>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ inline int wave_min_i(int k) {
    k = min(k, dpp_i<0xB1>(k));
    k = min(k, dpp_i<0x4E>(k));
    k = min(k, dpp_i<0x141>(k));
    k = min(k, dpp_i<0x140>(k));
    return min(min(__builtin_amdgcn_readlane(k, 0), __builtin_amdgcn_readlane(k, 16)),
               min(__builtin_amdgcn_readlane(k, 32), __builtin_amdgcn_readlane(k, 48)));
}
// sum over the wave: pairs within quads, quads, half rows, rows, then
// (row 0 + row 1) + (row 2 + row 3)
__device__ inline double wave_sum_d(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
// index of the largest v over the wave, the smallest index k on ties (v >= 0
// for candidates; -1 or NaN never wins); 0x7fffffff if no lane has v >= 0
__device__ inline int wave_argmax(double v, int k) {
    const double m = wave_max_d(v);
    return wave_min_i(v == m && m >= 0.0 ? k : 0x7fffffff);
}

// ---------------------------------------------------------------------------
// Point sources: a contiguous range of tree positions, or a list of positions
// (skeletons) whose length lives in device memory (ranks are decided on the
// device).  Positions index the permuted point array.
// ---------------------------------------------------------------------------
struct PtSrc {
    const int32_t *idx;    // list of positions, or nullptr for a range
    const int32_t *cnt;    // device count for a list (nullptr -> n)
    int64_t base;          // first position of a range
    int32_t n;             // range length / list capacity
    int32_t pad;
};

// One product task of the fused kernel-matrix kernel:
//   C(r, c) op= sum_k K(R_r, S_k) B(k, c)   (r < rows, c < ncol, k in chunk)
// R and S are point sources of the same problem (points X, bandwidth).
struct KmmTask {
    const double *X;       // permuted points of the problem, d per point
    PtSrc R, S;
    int32_t k0, k1;        // contraction sub-range [k0, k1) of S
    const void *B;         // B(k, c) = B[(k - k0) * ldb + c]
    int64_t ldb;
    void *C;               // C(r, c) = C[r * crs + c * ccs]
    int64_t crs, ccs;
    double scale;          // -1 / (2 h^2)
    double hinv;           // 1 / h (for dK/dh = K r^2 / h^3)
    int32_t which;         // 0: K, 1: dK/dh
    int32_t op;            // OutOp
    int32_t rcap;          // rows written: r < count gets the product, count <= r < rcap
                           // gets 0 when op == OP_STORE (padded skeleton slots)
    int32_t ncol;          // columns of this task (0: the launch's column count)
};

// One plain product task:  C(r, c) op= sum_k A(r, k) B(k, c)
struct GmmTask {
    const void *A;  int64_t ars, acs;
    const void *B;  int64_t brs, bcs;
    void *C;        int64_t crs, ccs;
    int32_t rows, kdim;
    int32_t op, ncol;      // ncol: columns of this task (0: the launch's column count)
};

// Work item of a tiled launch: task index, row tile, column tile.
struct TileItem {
    int32_t task, rt, ct, pad;
};

// Partial-sum reduction: dst(r, c) op= sum_{p < np} src[p](r, c), partials
// contiguous with stride pstride, each partial rows x ncol row-major.
struct RedTask {
    const void *src;
    int64_t pstride;       // elements between partials
    int64_t prs;           // row stride inside a partial
    int32_t np, rows;
    void *dst;
    int64_t drs, dcs;
    int32_t op, ncol;      // ncol: columns of this task (0: the launch's column count)
};

// Strided block copy / cast: dst(r, c) = src(r, c), r < rows, c < cols.
struct CopyTask {
    const void *src;
    void *dst;
    int64_t sld, dld;
    int32_t rows, cols;
};

// Leaf block lambda I + K_aa (column-major, lda) of the points [b, b+n).
struct LeafTask {
    const double *X;
    int64_t b;
    int32_t n, lda;
    double *A;
    double scale, lambda;
};

// Permutation of one problem's right-hand sides into tree order (batched
// solves): W(pos, c) = B_i[perm[pos] + c N] and back.
struct GatherTask {
    const int64_t *perm;
    int64_t N;
    void *W;
    int64_t ldw;
};

// n x n identity block (column-major, ld = n) for a reduced system.
struct IdTask {
    double *Z;
    int32_t n, pad;
};

// Batched LU / LU-solve task (column-major matrix).
struct LuTask {
    double *A;
    int32_t *piv;
    int32_t n, lda;
    void *B;              // right-hand sides, row-major n x nrhs, row stride ldb
    int64_t ldb;
    double *ratio;        // pivot ratio output (factor)
    double *dinv;         // inverses of the 16 x 16 diagonal blocks of L and U
    int32_t nrhs, pad;    // right-hand sides of this task (0: the launch's count)
};

// State of the LU split over launches (one slot per task of the launch):
// the physical row of each logical row, and the smallest and largest
// |pivot| so far.
struct LuSplit {
    int32_t *prow;        // tasks x kLuMaxN
    double *smm;          // tasks x 2
};

// Sampling task (rows outside a node): the npre positions of pre first (the
// node's neighbour list), then uniform draws from its SplitMix64 stream.
struct SampTask {
    int64_t b, e, N;
    uint64_t state;
    int32_t *out;
    const int32_t *pre;
    int32_t npre, pad;
};

// Ranked neighbour lists of the nodes of one level (kappa-NN sampling):
// list of node id = pos/w[id * cap .. + len[id]).
struct NbrTask {
    const int64_t *nb, *ne;  // device node ranges
    const int32_t *knn;      // N x kappa neighbour positions (-1: none)
    int32_t *pos, *w, *len;
    int32_t kappa, cap, leaf, pad;
};

// Sampled kernel block + QRCP task for one non-root node.
struct SkelTask {
    const double *X;
    const int32_t *q;      // sampled positions (nsamp capacity)
    int32_t nq;            // number of sampled rows
    int32_t leaf;          // 1: candidates = [b, b+n); 0: [skl[:sl], skr[:sr]]
    int64_t b;
    int32_t n;
    int32_t cmax;          // rows of this tree's P slots (max(leaf size, 2s))
    const int32_t *skl, *skr, *srl, *srr;
    double *M;             // nsamp_cap x cmax column-major
    int32_t *skel;         // out: s positions (-1 padded)
    int32_t *sr;           // out: rank
    int32_t *trunc;        // out: rank-guard flag
    int32_t *qrows;        // out: rows of the sampled block the QR factors (numerically zero rows dropped)
    double *Pt;            // out: cmax x s row-major P_{C alpha~} (rows padded)
    double scale;          // -1 / (2 h^2)
    double tol;            // adaptive rank: stop at |R_jj| < tol |R_00| (0: fixed rank)
};

// Work arrays of the split QRCP (several workgroups per node, one launch per
// pivot step); node i of a launch owns the i-th slot of every array.
struct QrWork {
    double *part;      // slices x rcap partial squared row norms per node
    int32_t *rmap;     // rcap: new row index or -1
    int32_t *rows;     // 1: kept rows, then rows in use
    double *nrm;       // 2 x cmax squared trailing norms by pivot position (buffers by step parity)
    int32_t *pos;      // 2 x cmax pivot order: column at each position (buffers by step parity)
    double *diag;      // cmax: R_jj
    int32_t *st;       // kQsState: stopped, stop step, zero block, steps, rows, candidates
    int32_t cmax, rcap, slices, pad;
};

// Output operations of the product kernels.
enum OutOp : int { OP_STORE = 0, OP_ADD = 1, OP_SUB = 2 };

}  // namespace askit
