// api.hip -- host orchestration and C ABI of libaskit (see include/askit.h).
//
// The host only sequences launches: every arithmetic step of the tree build,
// the skeletonization, the factorization and the solves runs in the kernels
// of the k_*.hip files.  Each phase is expressed as a "plan": a list of
// launches whose task descriptors (one per tree node and product chunk) are
// built once on the host, uploaded once, and replayed level by level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "askit.h"
#include "askit_kernels.h"

using namespace askit;

namespace {

thread_local std::string g_err;

askit_status fail(askit_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIP_TRY(x)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) return fail(ASKIT_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define ST_TRY(x)                          \
    do {                                   \
        askit_status s_ = (x);             \
        if (s_ != ASKIT_OK) return s_;     \
    } while (0)

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
// Cache of large device blocks.  A factorization's arenas (leaf LUs, the
// per-level bases, the refinement's Krylov basis) are several GB each; a
// fresh hipMalloc of that size can stall for hundreds of ms in the runtime,
// and repeated factorizations of one problem (new lambda, another precision,
// a serving loop) ask for the same sizes again.  Blocks of kCacheMin bytes or
// more are therefore kept on a per-device free list when released and handed
// out again to a request of at most 1/8 less; the device is synchronized
// before a block enters the list (as hipFree would), so no queued kernel
// still uses it when it is reused.  A failed hipMalloc empties the list of
// that device and tries once more; askit_release_cached_memory empties it on
// request.
constexpr size_t kCacheMin = (size_t)64 << 20;
constexpr size_t kCacheGrain = (size_t)2 << 20;
struct CachedBlock {
    void *p;
    size_t bytes;
    int dev;
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;

void cache_flush(int dev) {  // dev < 0: every device
    std::vector<CachedBlock> out;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        std::vector<CachedBlock> keep;
        for (auto &b : g_cache) (dev < 0 || b.dev == dev ? out : keep).push_back(b);
        g_cache.swap(keep);
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &b : out) {
        if (b.dev != cur) (void)hipSetDevice(b.dev);
        (void)hipFree(b.p);
        if (b.dev != cur) (void)hipSetDevice(cur);
    }
}

hipError_t dev_malloc(void **p, size_t *n, int *dev) {
    (void)hipGetDevice(dev);
    if (*n < kCacheMin) return hipMalloc(p, *n);
    *n = (*n + kCacheGrain - 1) / kCacheGrain * kCacheGrain;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        int best = -1;
        for (int i = 0; i < (int)g_cache.size(); i++) {
            const CachedBlock &b = g_cache[i];
            if (b.dev == *dev && b.bytes >= *n && b.bytes - *n <= *n / 8 &&
                (best < 0 || b.bytes < g_cache[best].bytes))
                best = i;
        }
        if (best >= 0) {
            *p = g_cache[best].p;
            *n = g_cache[best].bytes;
            g_cache.erase(g_cache.begin() + best);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, *n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        cache_flush(*dev);
        e = hipMalloc(p, *n);
    }
    return e;
}

void dev_free(void *p, size_t n, int dev) {
    if (n < kCacheMin) {
        (void)hipFree(p);
        return;
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (dev != cur) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    if (dev != cur) (void)hipSetDevice(cur);
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_cache.push_back({p, n, dev});
}

struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int dev = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) dev_free(p, bytes, dev);
        p = nullptr;
        bytes = 0;
    }
    askit_status alloc(size_t n) {
        release();
        if (n == 0) n = 8;
        if (dev_malloc(&p, &n, &dev) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(ASKIT_ERR_ALLOC, "device allocation of " + std::to_string(n) + " bytes failed");
        }
        bytes = n;
        return ASKIT_OK;
    }
    template <class T> T *as() const { return (T *)p; }
    void swap(DBuf &o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(dev, o.dev);
    }
};

// Host-to-device uploads of task lists are synchronous copies, except while
// an upload stream is set (UploadOnStream): then they are queued on that
// stream from host copies kept until the guard ends, so they neither wait
// for nor delay the kernels queued on other streams.
thread_local bool g_upload_async = false;  // per calling thread: calls on other handles may overlap
thread_local hipStream_t g_upload_stream = nullptr;  // may be the null stream
thread_local std::vector<std::vector<char>> g_upload_keep;

static askit_status copy_up(void *dst, const void *src, size_t bytes) {
    if (g_upload_async) {
        g_upload_keep.emplace_back((const char *)src, (const char *)src + bytes);
        HIP_TRY(hipMemcpyAsync(dst, g_upload_keep.back().data(), bytes, hipMemcpyHostToDevice, g_upload_stream));
    } else {
        HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    }
    return ASKIT_OK;
}

// uploads queued on `s` while the guard lives; the kept host copies are
// released at the end of the call that owns the guard (after it has
// synchronized with `s`)
struct UploadOnStream {
    explicit UploadOnStream(hipStream_t s) {
        g_upload_async = true;
        g_upload_stream = s;
    }
    ~UploadOnStream() {
        g_upload_async = false;
        g_upload_stream = nullptr;
    }
};

template <class T> askit_status upload(DBuf &b, const std::vector<T> &v) {
    ST_TRY(b.alloc(sizeof(T) * std::max<size_t>(v.size(), 1)));
    if (!v.empty()) ST_TRY(copy_up(b.p, v.data(), sizeof(T) * v.size()));
    return ASKIT_OK;
}

// device buffer that only grows: a height reuses the previous height's
// allocation when it fits (no hipFree, which would wait for every stream)
template <class T> askit_status upload_grow(DBuf &b, const std::vector<T> &v) {
    if (b.bytes < sizeof(T) * std::max<size_t>(v.size(), 1)) ST_TRY(b.alloc(sizeof(T) * std::max<size_t>(v.size(), 1)));
    if (!v.empty()) ST_TRY(copy_up(b.p, v.data(), sizeof(T) * v.size()));
    return ASKIT_OK;
}
static askit_status grow(DBuf &b, size_t n) {
    if (b.bytes < n) ST_TRY(b.alloc(n));
    return ASKIT_OK;
}

// the same, with an outgrown buffer moved to `retired` instead of released
// (a release synchronizes the device)
static askit_status grow_keep(std::vector<std::unique_ptr<DBuf>> &retired, DBuf &b, size_t n) {
    if (b.bytes >= n) return ASKIT_OK;
    if (b.p) {
        retired.emplace_back(new DBuf());
        retired.back()->swap(b);
    }
    return b.alloc(n);
}
template <class T>
askit_status upload_grow_keep(std::vector<std::unique_ptr<DBuf>> &retired, DBuf &b, const std::vector<T> &v) {
    ST_TRY(grow_keep(retired, b, sizeof(T) * std::max<size_t>(v.size(), 1)));
    if (!v.empty()) ST_TRY(copy_up(b.p, v.data(), sizeof(T) * v.size()));
    return ASKIT_OK;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline unsigned grid1(int64_t n, int bs = 256) { return (unsigned)std::max<int64_t>(1, cdiv(n, bs)); }

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), used to seed the per-node
// sampling streams: node state = output number k = id + 1 + problem 2^32 of
// the generator started at `seed`.
uint64_t splitmix_out(uint64_t st) {
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
uint64_t node_state(uint64_t seed, int64_t problem, int64_t id) {
    uint64_t k = (uint64_t)id + 1ULL + ((uint64_t)problem << 32);
    return splitmix_out(seed + k * 0x9E3779B97F4A7C15ULL);
}

// ---------------------------------------------------------------------------
// plans: a list of enqueue closures plus the device buffers they reference
// ---------------------------------------------------------------------------
typedef std::function<hipError_t(hipStream_t, int)> Launch;

// Optional per-kernel timing with HIP events recorded on the launch stream
// (askit_profile_enable); totals per kernel name are read back by
// askit_profile_report.
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
    int64_t launches;  // launches between the two events
};
struct Prof {
    bool on = false;
    bool heights = false;   // label each launch with the tree height it serves
    bool timeline = false;  // keep every launch's start and end
    std::vector<ProfRec> pend;
    std::map<std::string, std::pair<double, int64_t>> acc;
    hipEvent_t origin = nullptr;  // times of the timeline are relative to this event
    std::vector<std::pair<std::string, std::pair<double, double>>> tl;
};
Prof g_prof;

// f issues `launches` launches (a chain of dependent launches is timed as
// one interval, without events between its launches)
template <class F> hipError_t timed(const std::string &name, hipStream_t st, F &&f, int64_t launches = 1) {
    if (!g_prof.on) return f();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, st);
    if (e != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        return e;
    }
    e = f();
    const hipError_t e2 = hipEventRecord(b, st);
    g_prof.pend.push_back({name, a, b, launches});
    return e != hipSuccess ? e : e2;
}

// "@h<height>" when launches are profiled per tree height, else ""
std::string prof_height(int hgt) { return g_prof.heights ? "@h" + std::to_string(hgt) : std::string(); }

hipError_t prof_flush() {
    for (auto &r : g_prof.pend) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return e;
        auto &v = g_prof.acc[r.name];
        v.first += ms;
        v.second += r.launches;
        if (g_prof.timeline) {
            if (!g_prof.origin) {
                g_prof.origin = r.a;  // kept until profiling is reset
                r.a = nullptr;
            }
            float t0 = 0.f, t1 = 0.f;
            if (r.a) e = hipEventElapsedTime(&t0, g_prof.origin, r.a);
            if (e == hipSuccess) e = hipEventElapsedTime(&t1, g_prof.origin, r.b);
            if (e != hipSuccess) return e;
            g_prof.tl.push_back({r.name, {t0, t1}});
        }
        if (r.a) (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.pend.clear();
    return hipSuccess;
}

struct Plan {
    std::string tag, sub;  // step names are tag:name<sub>
    std::vector<std::pair<std::string, Launch>> steps;
    std::vector<std::unique_ptr<DBuf>> bufs;
    DBuf *own() {
        bufs.emplace_back(new DBuf());
        return bufs.back().get();
    }
    void add(const char *name, Launch f) { steps.emplace_back(tag + ":" + name + sub, std::move(f)); }
    hipError_t run(hipStream_t st, int ncol) const { return run_from(st, ncol, 0); }
    // enqueue steps i0 .. end
    hipError_t run_from(hipStream_t st, int ncol, size_t i0) const {
        for (size_t i = i0; i < steps.size(); i++) {
            hipError_t e = timed(steps[i].first, st, [&] { return steps[i].second(st, ncol); });
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
};

enum Prec { P64 = 0, P32 = 1 };

// a launch of the fused kernel-matrix product with optional split of the
// contraction into chunks (partials in a workspace, reduced in index order)
struct KmmBuild {
    std::vector<KmmTask> tasks;
    std::vector<TileItem> items;
    std::vector<RedTask> reds;
    int tc = 64;
    int64_t ws_elems = 0;  // partial elements needed (output type)
    int out_size = 8;
};

// `off` counts the partial elements already handed out in the workspace `ws`
// (one counter per workspace; the total is recorded in kb.ws_elems)
void kmm_add(KmmBuild &kb, KmmTask t, int kcap, int ncap, int64_t KC, int b_elem, char *ws, int64_t &off) {
    const int nrt = (int)cdiv(t.rcap, 64), nct = (int)cdiv(ncap, kb.tc);
    const int64_t nch = std::max<int64_t>(1, cdiv(kcap, KC));
    if (nch == 1) {
        t.k0 = 0;
        t.k1 = kcap;
        int ti = (int)kb.tasks.size();
        kb.tasks.push_back(t);
        for (int r = 0; r < nrt; r++)
            for (int c = 0; c < nct; c++) kb.items.push_back({ti, r, c, 0});
        return;
    }
    const int64_t per = (int64_t)t.rcap * ncap;
    RedTask rd{};
    rd.src = ws + off * kb.out_size;
    rd.pstride = per;
    rd.prs = ncap;
    rd.np = (int32_t)nch;
    rd.rows = t.rcap;
    rd.dst = t.C;
    rd.drs = t.crs;
    rd.dcs = t.ccs;
    rd.op = t.op;
    rd.ncol = t.ncol;
    for (int64_t c = 0; c < nch; c++) {
        KmmTask u = t;
        u.k0 = (int32_t)(c * KC);
        u.k1 = (int32_t)std::min<int64_t>(kcap, (c + 1) * KC);
        u.B = (const char *)t.B + (int64_t)u.k0 * t.ldb * b_elem;
        u.C = ws + (off + c * per) * kb.out_size;
        u.crs = ncap;
        u.ccs = 1;
        u.op = OP_STORE;
        int ti = (int)kb.tasks.size();
        kb.tasks.push_back(u);
        for (int r = 0; r < nrt; r++)
            for (int cc = 0; cc < nct; cc++) kb.items.push_back({ti, r, cc, 0});
    }
    kb.reds.push_back(rd);
    off += nch * per;
    kb.ws_elems = std::max(kb.ws_elems, off);
}

struct GmmBuild {
    std::vector<GmmTask> tasks;
    std::vector<TileItem> items;
    std::vector<RedTask> reds;
    int tc = 64;
    int64_t ws_elems = 0;
    int elem = 8;
};

// C(r, c) op= sum_k A(r, k) B(k, c); split of k into chunks of KC if kdim > KC
void gmm_add(GmmBuild &gb, GmmTask t, int ncap, int64_t KC, char *ws, int64_t &off) {
    const int nrt = (int)cdiv(t.rows, 64), nct = (int)cdiv(ncap, gb.tc);
    const int64_t nch = std::max<int64_t>(1, cdiv(t.kdim, KC));
    if (nch == 1) {
        int ti = (int)gb.tasks.size();
        gb.tasks.push_back(t);
        for (int r = 0; r < nrt; r++)
            for (int c = 0; c < nct; c++) gb.items.push_back({ti, r, c, 0});
        return;
    }
    const int64_t per = (int64_t)t.rows * ncap;
    RedTask rd{};
    rd.src = ws + off * gb.elem;
    rd.pstride = per;
    rd.prs = ncap;
    rd.np = (int32_t)nch;
    rd.rows = t.rows;
    rd.dst = t.C;
    rd.drs = t.crs;
    rd.dcs = t.ccs;
    rd.op = t.op;
    rd.ncol = t.ncol;
    for (int64_t c = 0; c < nch; c++) {
        GmmTask u = t;
        int64_t k0 = c * KC;
        u.kdim = (int32_t)std::min<int64_t>(t.kdim - k0, KC);
        u.A = (const char *)t.A + k0 * t.acs * gb.elem;
        u.B = (const char *)t.B + k0 * t.brs * gb.elem;
        u.C = ws + (off + c * per) * gb.elem;
        u.crs = ncap;
        u.ccs = 1;
        u.op = OP_STORE;
        int ti = (int)gb.tasks.size();
        gb.tasks.push_back(u);
        for (int r = 0; r < nrt; r++)
            for (int cc = 0; cc < nct; cc++) gb.items.push_back({ti, r, cc, 0});
    }
    gb.reds.push_back(rd);
    off += nch * per;
    gb.ws_elems = std::max(gb.ws_elems, off);
}

// Renumber tile items so that consecutive items (which share operands) run
// on one XCD: block b executes item xcd * chunk + slot with xcd = b % 8,
// slot = b / 8; positions past the end hold a no-op item (task -1).
void xcd_order(std::vector<TileItem> &items) {
    const int64_t n = (int64_t)items.size(), chunk = cdiv(n, 8);
    std::vector<TileItem> out((size_t)(8 * chunk), TileItem{-1, 0, 0, 0});
    for (int64_t b = 0; b < 8 * chunk; b++) {
        const int64_t L = (b % 8) * chunk + b / 8;
        if (L < n) out[(size_t)b] = items[(size_t)L];
    }
    items.swap(out);
}

template <typename T, typename TB, typename TO>
hipError_t launch_kmm(const KmmTask *tasks, const TileItem *items, int nitems, int ncol, int d, int tc,
                      hipStream_t st) {
    const size_t lds = d <= kXrDim ? sizeof(T) * 16 * kXrDim : sizeof(T) * (64 * (d | 1) + 16 * d);
    constexpr bool f64 = std::is_same<T, double>::value && std::is_same<TB, double>::value &&
                         std::is_same<TO, double>::value;
    if constexpr (f64) {
        if (tc == 256) {  // two 128-column halves sharing the generated kernel tile
            if (d <= kXrDim)
                hipLaunchKernelGGL((k_kmm<T, TB, TO, 128, true, 2>), dim3(nitems), dim3(512), lds, st, tasks, items,
                                   ncol, d);
            else
                hipLaunchKernelGGL((k_kmm<T, TB, TO, 128, false, 2>), dim3(nitems), dim3(512), lds, st, tasks, items,
                                   ncol, d);
            return hipGetLastError();
        }
    }
    if (tc == 256) return hipErrorInvalidValue;  // 256-column tiles exist in FP64 only
    if (d <= kXrDim) {  // row points in registers
        if (tc == 128)
            hipLaunchKernelGGL((k_kmm<T, TB, TO, 128, true, 1>), dim3(nitems), dim3(256), lds, st, tasks, items, ncol,
                               d);
        else if (tc == 64)
            hipLaunchKernelGGL((k_kmm<T, TB, TO, 64, true, 1>), dim3(nitems), dim3(256), lds, st, tasks, items, ncol,
                               d);
        else
            hipLaunchKernelGGL((k_kmm<T, TB, TO, 16, true, 1>), dim3(nitems), dim3(256), lds, st, tasks, items, ncol,
                               d);
        return hipGetLastError();
    }
    if (tc == 128)
        hipLaunchKernelGGL((k_kmm<T, TB, TO, 128, false, 1>), dim3(nitems), dim3(256), lds, st, tasks, items, ncol, d);
    else if (tc == 64)
        hipLaunchKernelGGL((k_kmm<T, TB, TO, 64, false, 1>), dim3(nitems), dim3(256), lds, st, tasks, items, ncol, d);
    else
        hipLaunchKernelGGL((k_kmm<T, TB, TO, 16, false, 1>), dim3(nitems), dim3(256), lds, st, tasks, items, ncol, d);
    return hipGetLastError();
}

template <typename T, int TC>
hipError_t launch_gmm(const GmmTask *tasks, const TileItem *items, int nitems, int ncol, hipStream_t st) {
    hipLaunchKernelGGL((k_gmm<T, TC>), dim3(nitems), dim3(256), 0, st, tasks, items, ncol, 1 << 30);
    return hipGetLastError();
}

// finalize a kmm build into plan steps: tc = compute precision, tb = storage
// of B, tout = output precision
askit_status kmm_commit(Plan &P, KmmBuild &kb, Prec tin, Prec tout, int d, int rows_red_max, int tbin = -1) {
    if (kb.tasks.empty()) return ASKIT_OK;
    const Prec tb = tbin < 0 ? tin : (Prec)tbin;
    DBuf *bt = P.own(), *bi = P.own();
    xcd_order(kb.items);
    ST_TRY(upload(*bt, kb.tasks));
    ST_TRY(upload(*bi, kb.items));
    const KmmTask *tp = bt->as<KmmTask>();
    const TileItem *ip = bi->as<TileItem>();
    const int nitems = (int)kb.items.size(), tc = kb.tc;
    P.add("k_kmm", [=](hipStream_t st, int ncol) -> hipError_t {
        if (tin == P64 && tb == P64) return launch_kmm<double, double, double>(tp, ip, nitems, ncol, d, tc, st);
        if (tin == P64) return launch_kmm<double, float, double>(tp, ip, nitems, ncol, d, tc, st);
        if (tout == P64) return launch_kmm<float, float, double>(tp, ip, nitems, ncol, d, tc, st);
        return launch_kmm<float, float, float>(tp, ip, nitems, ncol, d, tc, st);
    });
    if (!kb.reds.empty()) {
        DBuf *br = P.own();
        ST_TRY(upload(*br, kb.reds));
        const RedTask *rp = br->as<RedTask>();
        const int nred = (int)kb.reds.size();
        P.add("k_reduce", [=](hipStream_t st, int ncol) -> hipError_t {
            int bpt = (int)cdiv((int64_t)rows_red_max * ncol, 256);
            if (tout == P64) hipLaunchKernelGGL((k_reduce<double, double>), dim3(nred * bpt), dim3(256), 0, st, rp, ncol, bpt);
            else hipLaunchKernelGGL((k_reduce<float, float>), dim3(nred * bpt), dim3(256), 0, st, rp, ncol, bpt);
            return hipGetLastError();
        });
    }
    return ASKIT_OK;
}

askit_status gmm_commit(Plan &P, GmmBuild &gb, Prec t, int rows_red_max) {
    if (gb.tasks.empty()) return ASKIT_OK;
    DBuf *bt = P.own(), *bi = P.own();
    xcd_order(gb.items);
    ST_TRY(upload(*bt, gb.tasks));
    ST_TRY(upload(*bi, gb.items));
    const GmmTask *tp = bt->as<GmmTask>();
    const TileItem *ip = bi->as<TileItem>();
    const int nitems = (int)gb.items.size(), tc = gb.tc;
    P.add("k_gmm", [=](hipStream_t st, int ncol) -> hipError_t {
        if (t == P64) {
            if (tc == 256) return launch_gmm<double, 256>(tp, ip, nitems, ncol, st);
            if (tc == 128) return launch_gmm<double, 128>(tp, ip, nitems, ncol, st);
            if (tc == 64) return launch_gmm<double, 64>(tp, ip, nitems, ncol, st);
            return launch_gmm<double, 16>(tp, ip, nitems, ncol, st);
        }
        if (tc == 128) return launch_gmm<float, 128>(tp, ip, nitems, ncol, st);
        if (tc == 64) return launch_gmm<float, 64>(tp, ip, nitems, ncol, st);
        return launch_gmm<float, 16>(tp, ip, nitems, ncol, st);
    });
    if (!gb.reds.empty()) {
        DBuf *br = P.own();
        ST_TRY(upload(*br, gb.reds));
        const RedTask *rp = br->as<RedTask>();
        const int nred = (int)gb.reds.size();
        P.add("k_reduce", [=](hipStream_t st, int ncol) -> hipError_t {
            int bpt = (int)cdiv((int64_t)rows_red_max * ncol, 256);
            if (t == P64) hipLaunchKernelGGL((k_reduce<double, double>), dim3(nred * bpt), dim3(256), 0, st, rp, ncol, bpt);
            else hipLaunchKernelGGL((k_reduce<float, float>), dim3(nred * bpt), dim3(256), 0, st, rp, ncol, bpt);
            return hipGetLastError();
        });
    }
    return ASKIT_OK;
}

// spd: every matrix is symmetric positive definite (factored without row
// exchanges)
// The matrices of one LU launch differ in order, and a launch lasts as long
// as its slowest workgroups: the largest matrices go first (workgroups are
// dispatched in index order), so that the small ones fill in beside them
// instead of delaying a large one to the end.  Each task writes only its
// own outputs, so the order changes no result.  (The solves keep the plan's
// order: sorted, they measured slower.)
static std::vector<LuTask> largest_first(const std::vector<LuTask> &v) {
    std::vector<LuTask> o(v);
    std::stable_sort(o.begin(), o.end(), [](const LuTask &a, const LuTask &b) { return a.n > b.n; });
    return o;
}

askit_status lu_commit(Plan &P, const std::vector<LuTask> &v0, bool spd, int32_t split_n) {
    if (v0.empty()) return ASKIT_OK;
    const std::vector<LuTask> v = largest_first(v0);
    DBuf *b = P.own();
    ST_TRY(upload(*b, v));
    const LuTask *tp = b->as<LuTask>();
    const int n = (int)v.size(), nmax = v[0].n;
    if (!spd && nmax > split_n) {
        // split over launches (k_lup_*): per panel, the tasks still
        // factoring (a prefix, largest first) and the 64 x 64 tiles of their
        // trailing matrices
        DBuf *bw = P.own(), *bi = P.own();
        const size_t prow_bytes = (size_t)n * kLuMaxN * sizeof(int32_t);
        ST_TRY(bw->alloc(prow_bytes + (size_t)n * 2 * sizeof(double)));
        const LuSplit w{bw->as<int32_t>(), (double *)((char *)bw->p + prow_bytes)};
        std::vector<TileItem> items;
        std::vector<int> active, off;
        for (int kb = 0; kb < nmax; kb += kLuPanel) {
            int act = 0;
            std::vector<TileItem> pi;
            for (int i = 0; i < n; i++) {
                if (v[(size_t)i].n <= kb) break;
                act++;
                const int rest = v[(size_t)i].n - kb - kLuPanel;  // trailing order after this panel
                const int tt = rest > 0 ? (int)cdiv(rest, 64) : 0;
                for (int rt = 0; rt < tt; rt++)
                    for (int ct = 0; ct < tt; ct++) pi.push_back(TileItem{i, rt, ct, 0});
            }
            xcd_order(pi);
            active.push_back(act);
            off.push_back((int)items.size());
            items.insert(items.end(), pi.begin(), pi.end());
        }
        off.push_back((int)items.size());
        // the final row pass: kLupFinCols columns per workgroup; a task of
        // order 0 still gets one (its pivot ratio)
        for (int i = 0; i < n; i++)
            for (int cg = 0; cg < std::max<int64_t>(1, cdiv(v[(size_t)i].n, kLupFinCols)); cg++)
                items.push_back(TileItem{i, cg, 0, 0});
        const int nfin = (int)items.size() - off.back();
        ST_TRY(upload(*bi, items));
        const TileItem *ip = bi->as<TileItem>();
        P.add("k_lu", [=](hipStream_t st, int) -> hipError_t {
            for (size_t p = 0; p < active.size(); p++) {
                const int kb = (int)p * kLuPanel;
                hipLaunchKernelGGL(k_lup_panel, dim3(active[p]), dim3(kLuFThreads), 0, st, tp, w, kb);
                if (off[p + 1] > off[p])
                    hipLaunchKernelGGL(k_lup_update, dim3(off[p + 1] - off[p]), dim3(kLupThreads), 0, st, tp, w,
                                       ip + off[p], kb);
            }
            hipLaunchKernelGGL(k_lup_finish, dim3(nfin), dim3(kLupThreads), 0, st, tp, w, ip + off.back());
            return hipGetLastError();
        });
    } else {
        P.add(spd ? "k_lu_nopiv" : "k_lu", [=](hipStream_t st, int) -> hipError_t {
            if (spd) hipLaunchKernelGGL(k_lu_nopiv, dim3(n), dim3(kLuFThreads), 0, st, tp);
            else hipLaunchKernelGGL(k_lu, dim3(n), dim3(kLuFThreads), 0, st, tp);
            return hipGetLastError();
        });
    }
    P.add("k_lu_diaginv", [=](hipStream_t st, int) -> hipError_t {
        hipLaunchKernelGGL(k_lu_diaginv, dim3(n), dim3(256), 0, st, tp);
        return hipGetLastError();
    });
    return ASKIT_OK;
}

// LU solves with nrhs = fixed (>0) or the run-time column count (fixed = 0)
template <typename T, bool TR>
hipError_t launch_lusolve(const LuTask *tp, int n, int nrhs, hipStream_t st) {
    const int panels = nrhs > 16 ? (int)cdiv(nrhs, 32) : 1;
    const int grid = 8 * (int)cdiv((int64_t)n * panels, 8);
    if (nrhs > 16)
        hipLaunchKernelGGL((k_lusolve<T, 32, TR>), dim3(grid), dim3(kLsThreads), 0, st, tp, n, nrhs, panels);
    else hipLaunchKernelGGL((k_lusolve<T, 16, TR>), dim3(grid), dim3(kLsThreads), 0, st, tp, n, nrhs, 1);
    return hipGetLastError();
}


askit_status getrs_commit(Plan &P, const std::vector<LuTask> &v, Prec t, bool trans, int fixed) {
    if (v.empty()) return ASKIT_OK;
    DBuf *b = P.own();
    ST_TRY(upload(*b, v));
    const LuTask *tp = b->as<LuTask>();
    const int n = (int)v.size();
    P.add(trans ? "k_lusolve_t" : "k_lusolve", [=](hipStream_t st, int ncol) -> hipError_t {
        const int nrhs = fixed ? fixed : ncol;
        if (t == P64) return trans ? launch_lusolve<double, true>(tp, n, nrhs, st) : launch_lusolve<double, false>(tp, n, nrhs, st);
        return trans ? launch_lusolve<float, true>(tp, n, nrhs, st) : launch_lusolve<float, false>(tp, n, nrhs, st);
    });
    return ASKIT_OK;
}

askit_status copy_commit(Plan &P, const std::vector<CopyTask> &v, Prec from, Prec to, int rows_max, int cols_max) {
    if (v.empty()) return ASKIT_OK;
    DBuf *b = P.own();
    ST_TRY(upload(*b, v));
    const CopyTask *tp = b->as<CopyTask>();
    const int n = (int)v.size();
    const int rb = (int)cdiv((int64_t)rows_max, 4);  // four rows per 256-thread block
    (void)cols_max;
    P.add("k_copy", [=](hipStream_t st, int) -> hipError_t {
        if (from == P64 && to == P64) hipLaunchKernelGGL((k_copy<double, double>), dim3(n * rb), dim3(256), 0, st, tp, rb);
        else if (from == P64) hipLaunchKernelGGL((k_copy<double, float>), dim3(n * rb), dim3(256), 0, st, tp, rb);
        else hipLaunchKernelGGL((k_copy<float, double>), dim3(n * rb), dim3(256), 0, st, tp, rb);
        return hipGetLastError();
    });
    return ASKIT_OK;
}

askit_status ident_commit(Plan &P, const std::vector<IdTask> &v, int n) {
    if (v.empty()) return ASKIT_OK;
    DBuf *b = P.own();
    ST_TRY(upload(*b, v));
    const IdTask *tp = b->as<IdTask>();
    const int cnt = (int)v.size();
    const int bpm = (int)cdiv((int64_t)n, 4);  // four columns per 256-thread block
    P.add("k_identity", [=](hipStream_t st, int) -> hipError_t {
        hipLaunchKernelGGL(k_identity, dim3(cnt * bpm), dim3(256), 0, st, tp, bpm);
        return hipGetLastError();
    });
    return ASKIT_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// Temporaries of the tree build of N points in d dimensions at depth D, as
// byte offsets into one arena (each array 256-byte aligned).
struct TreeScratch {
    size_t nb, ne, pa, pc, part, mu, S, axis, key, kid, key2, kid2, total;
};
static TreeScratch tree_scratch_layout(int64_t N, int d, int D) {
    const int npair = d * (d + 1) / 2;
    const int64_t nnodes = ((int64_t)2 << D) - 1;
    int64_t part_max = 1;
    for (int l = 0; l < D; l++) {
        const int64_t cnt = (int64_t)1 << l, nmax = cdiv(N, cnt), maxch = cdiv(nmax, kTreeChunk);
        part_max = std::max(part_max, cnt * maxch * std::max(d, npair));
    }
    const int64_t cnt_max = D > 0 ? ((int64_t)1 << (D - 1)) : 1;
    TreeScratch L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    L.nb = take(sizeof(int64_t) * nnodes);
    L.ne = take(sizeof(int64_t) * nnodes);
    L.pa = take(sizeof(int16_t) * npair);
    L.pc = take(sizeof(int16_t) * npair);
    L.part = take(sizeof(double) * part_max);
    L.mu = take(sizeof(double) * cnt_max * d);
    L.S = take(sizeof(double) * cnt_max * d * d);
    L.axis = take(sizeof(double) * cnt_max * d);
    L.key = take(sizeof(double) * N);
    L.kid = take(sizeof(int64_t) * N);
    L.key2 = take(sizeof(double) * N);
    L.kid2 = take(sizeof(int64_t) * N);
    L.total = off;
    return L;
}

// The levels of the tree build (Sec. 2.1, "Partitioning the matrix"): for
// each level, chunk sums -> means -> scatter matrices -> principal axes ->
// keys -> tile sort + merges -> the permutation reordered within every node.
// perm holds the identity on entry and the tree order on exit; nb/ne are the
// node ranges (heap order), pa/pc the index pairs of the scatter matrix; the
// other pointers are temporaries sized as in tree_scratch_layout.
static askit_status tree_levels(const double *X, int64_t N, int d, int D, int64_t *perm, const int64_t *nb,
                                const int64_t *ne, const int16_t *pa, const int16_t *pc, double *part, double *mu,
                                double *S, double *axis, double *key, int64_t *kid, double *key2, int64_t *kid2,
                                hipStream_t st) {
    const int npair = d * (d + 1) / 2;
    for (int l = 0; l < D; l++) {
        const int cnt = 1 << l;
        const int64_t first = (((int64_t)1 << l) - 1), nmax = cdiv(N, cnt);
        const int maxch = (int)cdiv(nmax, kTreeChunk);
        hipLaunchKernelGGL(k_tree_chunk_mean, dim3(grid1((int64_t)cnt * maxch * d)), dim3(256), 0, st,
                           X, perm, d, nb, ne, first, cnt, maxch, part);
        hipLaunchKernelGGL(k_tree_mean, dim3(grid1((int64_t)cnt * d)), dim3(256), 0, st, nb, ne, first, cnt, maxch, d,
                           part, mu);
        hipLaunchKernelGGL(k_tree_chunk_scatter, dim3(grid1((int64_t)cnt * maxch * npair)), dim3(256), 0, st,
                           X, perm, d, nb, ne, first, cnt, maxch, mu,
                           pa, pc, npair, part);
        hipLaunchKernelGGL(k_tree_scatter, dim3(grid1((int64_t)cnt * npair)), dim3(256), 0, st, nb, ne, first, cnt,
                           maxch, d, pa, pc, npair, part, S);
        hipLaunchKernelGGL(k_tree_axis, dim3(grid1(cnt, 64)), dim3(64), 0, st, cnt, d, S,
                           axis);
        const int bpn = (int)cdiv(nmax, 256);
        hipLaunchKernelGGL(k_tree_keys, dim3(cnt * bpn), dim3(256), 0, st, X, perm, d,
                           nb, ne, first, bpn, mu, axis, key, kid);
        const int tpn = (int)cdiv(nmax, 1024);
        hipLaunchKernelGGL(k_tree_sort_tiles, dim3(cnt * tpn), dim3(512), 0, st, nb, ne, first, tpn, key,
                           kid);
        double *ka = key, *kb2 = key2;
        int64_t *ia = kid, *ib = kid2;
        for (int64_t w = 1024; w < nmax; w *= 2) {
            hipLaunchKernelGGL(k_tree_merge, dim3(cnt * bpn), dim3(256), 0, st, nb, ne, first, bpn, w, ka, ia, kb2, ib);
            std::swap(ka, kb2);
            std::swap(ia, ib);
        }
        hipLaunchKernelGGL(k_copy_ids, dim3(grid1(N)), dim3(256), 0, st, ia, perm, N);
        HIP_TRY(hipGetLastError());
    }
    return ASKIT_OK;
}

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
// By default the internal levels run the split QRCP (several workgroups per
// node, one launch per pivot step) and the leaves, the widest level, one
// workgroup per node.  Both give identical skeletons.

// Tile configuration of the factorization's level products at one tree
// height (0 fields: the built-in choice from the column count)
struct Tune {
    int kmm_tc = 0, gmm_tc = 0;  // output columns per tile of k_kmm / k_gmm
    int64_t kmm_kc = 0;          // contraction points per split chunk of k_kmm
};

struct askit_tree_s {
    int64_t N = 0;
    int d = 0, m = 0, s = 0, nsamp = 0, D = 0, cmax = 0, mmax = 0;
    int64_t nnodes = 0, problem = 0;
    uint64_t seed = 0;
    double h = 1.0;      // bandwidth of the skeletonization
    double hfac = 1.0;   // bandwidth of the next factorization (skeletons frozen)
    double tol = 0.0;    // adaptive rank tolerance tau (0: fixed rank s)
    int knn = 0;         // kappa of the neighbour sampling (0: uniform rows)
    DBuf knnidx, nbpos, nbw, nblen;  // N x kappa neighbours; per node: ranked list (nsamp slots), length
    std::vector<int32_t> hnn;        // host copy of the list lengths
    double t_knn = 0;
    unsigned long long knn_points = 0;  // points the neighbour search compared, summed over its waves
    std::vector<Tune> tune;  // per tree height, from askit_tune_factorization (empty: built-in choices)
    int32_t lu_split = kLuSplitN;  // LU batches with a larger matrix are split over launches (askit_tree_set_lu_split)
    int32_t *hsr_pinned = nullptr;  // pinned landing buffer of the rank reads (nnodes)
    ~askit_tree_s() {
        if (hsr_pinned) (void)hipHostFree(hsr_pinned);
    }
    std::vector<int64_t> nb, ne;  // host node ranges
    DBuf X, Xp, perm, iperm, dnb, dne;  // iperm[original index] = tree position
    DBuf srank, trunc, skel, Pt, samp, qrows;
    std::vector<int32_t> hsr;  // host copy of the ranks s_alpha (root: 0)
    int split_levels = 0;      // tree levels 1 .. split_levels use the split QRCP
    bool split_default = true; // split_levels was left to the library
    bool skel_ok = false;
    int refs = 0;
    double t_tree = 0, t_skel = 0;
    int64_t first(int l) const { return ((int64_t)1 << l) - 1; }
};

struct askit_factor_s {
    askit_tree t = nullptr;
    double lambda = 0;
    double h = 1.0;
    Prec prec = P64;
    DBuf LU, piv, ratio, Xc, Xcf, ws, dinv;
    std::vector<std::unique_ptr<DBuf>> PH;  // levels 1..D
    int64_t leafLU = 0, zLU = 0;            // element offsets of the arenas
    // solve state
    int cap = 0;
    DBuf W, TB, WX, WY, CB, wsS, R, Dx, nrm, Vk, kpart, ksmall;
    std::unique_ptr<Plan> solve_plan, solvet_plan, mv_plan[3];
    int max_refine = 10;
    double refine_tol = 1e-11;
    askit_solve_info info{};
    double min_ratio = 1.0;
    int min_node = -1;
    double t_factor = 0, t_solve = 0;
    // level restriction (hybrid solver): frontier level L >= 1, or 0 for the
    // full direct factorization.  The reduced system I + V W has order hM;
    // frontier node j (heap id first(L) + j) owns its rows hoff[j] ..
    int hyb = 0;
    int64_t hM = 0;
    std::vector<int64_t> hoff;
    DBuf HZ, HT, HK, HR, HU, hws;  // N x cap scratch, reduced-system vectors, Krylov basis, V partials
    std::unique_ptr<Plan> hv_w, hv_z, hw_store, hw_sub;
    void *ph(int level) const { return PH[level - 1]->p; }
    size_t elem() const { return prec == P64 ? 8 : 4; }
    double *lu_of(int64_t id) const {
        int64_t leaf0 = t->first(t->D);
        if (id >= leaf0) return LU.as<double>() + leafLU + (id - leaf0) * (int64_t)t->mmax * t->mmax;
        return LU.as<double>() + zLU + id * (int64_t)(2 * t->s) * (2 * t->s);
    }
    double *dinv_of(int64_t id) const {
        int64_t leaf0 = t->first(t->D), lb = (t->mmax + 15) / 16, zb = (2 * t->s + 15) / 16;
        if (id >= leaf0) return dinv.as<double>() + (id - leaf0) * lb * 512;
        return dinv.as<double>() + (leaf0 + 1) * lb * 512 + id * zb * 512;
    }
    int32_t *piv_of(int64_t id) const {
        int64_t leaf0 = t->first(t->D);
        if (id >= leaf0) return piv.as<int32_t>() + (id - leaf0) * (int64_t)t->mmax;
        return piv.as<int32_t>() + (leaf0 + 1) * t->mmax + id * (int64_t)(2 * t->s);
    }
};

extern "C" {

const char *askit_last_error(void) { return g_err.c_str(); }

askit_status askit_release_cached_memory(uint64_t *bytes_released) {
    uint64_t tot = 0;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        for (auto &b : g_cache) tot += b.bytes;
    }
    cache_flush(-1);
    if (bytes_released) *bytes_released = tot;
    return ASKIT_OK;
}

askit_status askit_profile_enable(int32_t on) {
    HIP_TRY(prof_flush());
    g_prof.acc.clear();
    g_prof.tl.clear();
    if (g_prof.origin) (void)hipEventDestroy(g_prof.origin);
    g_prof.origin = nullptr;
    g_prof.on = on != 0;
    g_prof.heights = on == 2 || on == 3;
    g_prof.timeline = on == 3;
    return ASKIT_OK;
}

askit_status askit_profile_report(char *json, size_t cap) {
    if (!json || cap == 0) return fail(ASKIT_ERR_ARG, "NULL buffer");
    HIP_TRY(prof_flush());
    std::string o = "{";
    bool first = true;
    for (auto &kv : g_prof.acc) {
        char b[256];
        snprintf(b, sizeof b, "%s\"%s\": [%.6f, %lld]", first ? "" : ", ", kv.first.c_str(), kv.second.first,
                 (long long)kv.second.second);
        o += b;
        first = false;
    }
    if (g_prof.timeline) {
        o += first ? "\"@timeline\": [" : ", \"@timeline\": [";
        for (size_t i = 0; i < g_prof.tl.size(); i++) {
            char b[256];
            snprintf(b, sizeof b, "%s[\"%s\", %.4f, %.4f]", i ? ", " : "", g_prof.tl[i].first.c_str(),
                     g_prof.tl[i].second.first, g_prof.tl[i].second.second);
            o += b;
        }
        o += "]";
    }
    o += "}";
    if (o.size() + 1 > cap) return fail(ASKIT_ERR_ARG, "buffer too small");
    memcpy(json, o.c_str(), o.size() + 1);
    return ASKIT_OK;
}

// ---------------------------------------------------------------------------
// tree
// ---------------------------------------------------------------------------
}  // extern "C"

// Neighbours of every point (exact, k_knn) and the ranked neighbour list of
// every non-root node, bottom-up (k_nbr_rank); list lengths copied to the host.
template <int K>
static void launch_knn(int dpad, const double *Xp, int64_t N, int d, const float *lo, const float *hi,
                       const int64_t *levoff, int top, int kappa, int32_t *out, unsigned long long *visits,
                       hipStream_t st) {
    const dim3 g((unsigned)cdiv(N, kWave)), b(kWave);
    if (dpad == 16)
        hipLaunchKernelGGL((k_knn<K, 16>), g, b, 0, st, Xp, N, d, lo, hi, levoff, top, kappa, out, visits);
    else if (dpad == 32)
        hipLaunchKernelGGL((k_knn<K, 32>), g, b, 0, st, Xp, N, d, lo, hi, levoff, top, kappa, out, visits);
    else if constexpr (K <= 32)
        hipLaunchKernelGGL((k_knn<K, 64>), g, b, 0, st, Xp, N, d, lo, hi, levoff, top, kappa, out, visits);
}

static askit_status build_neighbor_lists(askit_tree t, hipStream_t st) {
    const int64_t N = t->N;
    const int d = t->d, kappa = t->knn;
    const int dpad = d <= 16 ? 16 : (d <= 32 ? 32 : 64);
    const int64_t nrun = cdiv(N, 64);
    // box tree over the runs: level 0 = the runs, each level half the one below
    std::vector<int64_t> levoff{0};
    for (int64_t n = nrun;; n = (n + 1) / 2) {
        levoff.push_back(levoff.back() + n);
        if (n == 1) break;
    }
    const int top = (int)levoff.size() - 2;
    const int64_t nbox = levoff.back();
    DBuf lo, hi, scratch, visits, dlev;
    ST_TRY(visits.alloc(sizeof(unsigned long long)));
    HIP_TRY(hipMemsetAsync(visits.p, 0, sizeof(unsigned long long), st));
    ST_TRY(lo.alloc(sizeof(float) * nbox * dpad));
    ST_TRY(hi.alloc(sizeof(float) * nbox * dpad));
    ST_TRY(upload(dlev, levoff));
    ST_TRY(t->knnidx.alloc(sizeof(int32_t) * N * kappa));
    ST_TRY(t->nbpos.alloc(sizeof(int32_t) * t->nnodes * t->nsamp));
    ST_TRY(t->nbw.alloc(sizeof(int32_t) * t->nnodes * t->nsamp));
    ST_TRY(t->nblen.alloc(sizeof(int32_t) * t->nnodes));
    HIP_TRY(hipMemsetAsync(t->nblen.p, 0, sizeof(int32_t) * t->nnodes, st));
    HIP_TRY(timed("tree:k_knn_boxes", st, [&] {
        hipLaunchKernelGGL(k_knn_boxes, dim3(grid1(nrun * dpad)), dim3(256), 0, st, t->Xp.as<double>(), N, d, dpad,
                           lo.as<float>(), hi.as<float>());
        for (int l = 1; l <= top; l++) {
            const int64_t nat = levoff[l + 1] - levoff[l];
            hipLaunchKernelGGL(k_knn_box_up, dim3(grid1(nat * dpad)), dim3(256), 0, st, lo.as<float>(),
                               hi.as<float>(), levoff[l - 1], levoff[l] - levoff[l - 1], levoff[l], nat, dpad);
        }
        return hipGetLastError();
    }));
    HIP_TRY(timed("tree:k_knn", st, [&] {
        const double *Xp = t->Xp.as<double>();
        const float *L = lo.as<float>(), *H = hi.as<float>();
        const int64_t *lv = dlev.as<int64_t>();
        int32_t *o = t->knnidx.as<int32_t>();
        unsigned long long *v = visits.as<unsigned long long>();
        if (kappa <= 8) launch_knn<8>(dpad, Xp, N, d, L, H, lv, top, kappa, o, v, st);
        else if (kappa <= 16) launch_knn<16>(dpad, Xp, N, d, L, H, lv, top, kappa, o, v, st);
        else if (kappa <= 32) launch_knn<32>(dpad, Xp, N, d, L, H, lv, top, kappa, o, v, st);
        else launch_knn<64>(dpad, Xp, N, d, L, H, lv, top, kappa, o, v, st);
        return hipGetLastError();
    }));
    for (int l = t->D; l >= 1; l--) {
        NbrTask nt{};
        nt.nb = t->dnb.as<int64_t>();
        nt.ne = t->dne.as<int64_t>();
        nt.knn = t->knnidx.as<int32_t>();
        nt.pos = t->nbpos.as<int32_t>();
        nt.w = t->nbw.as<int32_t>();
        nt.len = t->nblen.as<int32_t>();
        nt.kappa = kappa;
        nt.cap = t->nsamp;
        nt.leaf = l == t->D;
        const int64_t cnt = (int64_t)1 << l, nent = nt.leaf ? (int64_t)t->mmax * kappa : 2 * (int64_t)t->nsamp;
        int64_t pmax = 2;
        while (pmax < nent) pmax <<= 1;
        if (pmax > kNbrLds) ST_TRY(scratch.alloc(sizeof(uint64_t) * cnt * 2 * pmax));
        HIP_TRY(timed("tree:k_nbr_rank", st, [&] {
            hipLaunchKernelGGL(k_nbr_rank, dim3((unsigned)cnt), dim3(kNbrThreads), 0, st, nt, t->first(l), pmax,
                               pmax > kNbrLds ? scratch.as<uint64_t>() : nullptr);
            return hipGetLastError();
        }));
        if (pmax > kNbrLds) {
            HIP_TRY(hipStreamSynchronize(st));  // the scratch of this level is released next
            scratch.release();
        }
    }
    t->hnn.assign(t->nnodes, 0);
    HIP_TRY(hipMemcpyAsync(t->hnn.data(), t->nblen.p, sizeof(int32_t) * t->nnodes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&t->knn_points, visits.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return ASKIT_OK;
}

extern "C" {

askit_status askit_build_tree(const double *X, int64_t N, int32_t d, const askit_options *opt, void *stream,
                              askit_tree *out) {
    if (!out) return fail(ASKIT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!X || !opt) return fail(ASKIT_ERR_ARG, "X or options is NULL");
    if (N < 1 || N >= (int64_t)1 << 31) return fail(ASKIT_ERR_ARG, "N must be in [1, 2^31)");
    if (d < 1 || d > kMaxDim) return fail(ASKIT_ERR_ARG, "d must be in [1, 64]");
    if (opt->leaf_size < 2) return fail(ASKIT_ERR_ARG, "leaf_size must be >= 2");
    if (opt->rank < 1) return fail(ASKIT_ERR_ARG, "rank must be >= 1");
    if (!(opt->h > 0.0) || !std::isfinite(opt->h)) return fail(ASKIT_ERR_ARG, "h must be positive and finite");
    if (opt->n_samples < 0) return fail(ASKIT_ERR_ARG, "n_samples must be >= 0");
    if (opt->qr_split_levels < -1) return fail(ASKIT_ERR_ARG, "qr_split_levels must be >= -1");
    if (!(opt->tol >= 0.0 && opt->tol < 1.0)) return fail(ASKIT_ERR_ARG, "tol must be in [0, 1)");
    if (opt->knn < 0 || opt->knn > kKnnMax || (d > 32 && opt->knn > 32))
        return fail(ASKIT_ERR_ARG, "knn must be in [0, 64] (in [0, 32] for d > 32)");
    if ((int64_t)opt->knn * N >= ((int64_t)1 << 31)) return fail(ASKIT_ERR_ARG, "knn * N must be below 2^31");
    hipStream_t st = (hipStream_t)stream;
    std::unique_ptr<askit_tree_s> t(new askit_tree_s());
    t->N = N;
    t->d = d;
    t->m = opt->leaf_size;
    t->s = opt->rank;
    t->nsamp = opt->n_samples ? opt->n_samples : 4 * opt->rank;

    t->seed = opt->seed;
    t->problem = opt->problem;
    t->h = opt->h;
    t->hfac = opt->h;
    t->tol = opt->tol;
    t->knn = opt->knn;
    while ((int64_t)t->m * ((int64_t)1 << t->D) < N) t->D++;
    t->nnodes = ((int64_t)2 << t->D) - 1;
    // default: the split QR on every internal level (the pipelined call
    // narrows it, see SkelRun::split_of)
    t->split_levels = opt->qr_split_levels == 0 ? t->D - 1 : std::max(0, opt->qr_split_levels);
    t->split_default = opt->qr_split_levels == 0;
    t->mmax = (int)cdiv(N, (int64_t)1 << t->D);
    t->cmax = std::max(t->mmax, 2 * t->s);
    if (t->mmax > 512 || 2 * t->s > 512)
        return fail(ASKIT_ERR_ARG, "leaf size and 2 * rank must not exceed 512");
    if (t->nsamp > 4096) return fail(ASKIT_ERR_ARG, "n_samples must be <= 4096");
    t->nb.assign(t->nnodes, 0);
    t->ne.assign(t->nnodes, 0);
    t->ne[0] = N;
    for (int64_t id = 0; id < t->first(t->D); id++) {
        int64_t b = t->nb[id], n = t->ne[id] - b;
        t->nb[2 * id + 1] = b;
        t->ne[2 * id + 1] = b + n / 2;
        t->nb[2 * id + 2] = b + n / 2;
        t->ne[2 * id + 2] = t->ne[id];
    }
    auto t0 = std::chrono::steady_clock::now();
    ST_TRY(t->X.alloc(sizeof(double) * N * d));
    ST_TRY(t->Xp.alloc(sizeof(double) * N * d));
    ST_TRY(t->perm.alloc(sizeof(int64_t) * N));
    ST_TRY(upload(t->dnb, t->nb));
    ST_TRY(upload(t->dne, t->ne));
    // X may be in host or device memory (unified addressing)
    HIP_TRY(hipMemcpyAsync(t->X.p, X, sizeof(double) * N * d, hipMemcpyDefault, st));
    // scratch for the level reductions and the sort
    const int npair = d * (d + 1) / 2;
    std::vector<int16_t> pa, pc;
    for (int a = 0; a < d; a++)
        for (int c = a; c < d; c++) {
            pa.push_back((int16_t)a);
            pc.push_back((int16_t)c);
        }
    DBuf dpa, dpc, part, mu, S, axis, key, kid, key2, kid2, bad;
    ST_TRY(upload(dpa, pa));
    ST_TRY(upload(dpc, pc));
    int64_t part_max = 0;
    for (int l = 0; l < t->D; l++) {
        int64_t cnt = (int64_t)1 << l, nmax = cdiv(N, cnt), maxch = cdiv(nmax, kTreeChunk);
        part_max = std::max(part_max, cnt * maxch * std::max(d, npair));
    }
    int64_t cnt_max = t->D > 0 ? ((int64_t)1 << (t->D - 1)) : 1;
    ST_TRY(part.alloc(sizeof(double) * std::max<int64_t>(part_max, 1)));
    ST_TRY(mu.alloc(sizeof(double) * cnt_max * d));
    ST_TRY(S.alloc(sizeof(double) * cnt_max * d * d));
    ST_TRY(axis.alloc(sizeof(double) * cnt_max * d));
    ST_TRY(key.alloc(sizeof(double) * N));
    ST_TRY(kid.alloc(sizeof(int64_t) * N));
    ST_TRY(key2.alloc(sizeof(double) * N));
    ST_TRY(kid2.alloc(sizeof(int64_t) * N));
    ST_TRY(bad.alloc(sizeof(int32_t)));
    HIP_TRY(hipMemsetAsync(bad.p, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_check_finite, dim3(grid1(N * d)), dim3(256), 0, st, t->X.as<double>(), N * d, bad.as<int32_t>());
    hipLaunchKernelGGL(k_iota, dim3(grid1(N)), dim3(256), 0, st, t->perm.as<int64_t>(), N);
    ST_TRY(tree_levels(t->X.as<double>(), N, d, t->D, t->perm.as<int64_t>(), t->dnb.as<int64_t>(),
                       t->dne.as<int64_t>(), dpa.as<int16_t>(), dpc.as<int16_t>(), part.as<double>(),
                       mu.as<double>(), S.as<double>(), axis.as<double>(), key.as<double>(), kid.as<int64_t>(),
                       key2.as<double>(), kid2.as<int64_t>(), st));
    hipLaunchKernelGGL(k_gather_points, dim3(grid1(N * d)), dim3(256), 0, st, t->X.as<double>(),
                       t->perm.as<int64_t>(), d, N, t->Xp.as<double>());
    ST_TRY(t->iperm.alloc(sizeof(int64_t) * N));
    hipLaunchKernelGGL(k_invert_perm, dim3(grid1(N)), dim3(256), 0, st, t->perm.as<int64_t>(), N,
                       t->iperm.as<int64_t>());
    HIP_TRY(hipGetLastError());
    int32_t hbad = 0;
    HIP_TRY(hipMemcpyAsync(&hbad, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hbad) return fail(ASKIT_ERR_ARG, "X has non-finite coordinates");
    // skeleton arrays
    ST_TRY(t->srank.alloc(sizeof(int32_t) * t->nnodes));
    ST_TRY(t->trunc.alloc(sizeof(int32_t) * t->nnodes));
    ST_TRY(t->qrows.alloc(sizeof(int32_t) * t->nnodes));
    ST_TRY(t->skel.alloc(sizeof(int32_t) * t->nnodes * t->s));
    ST_TRY(t->Pt.alloc(sizeof(double) * t->nnodes * t->cmax * t->s));
    HIP_TRY(hipMemsetAsync(t->srank.p, 0, sizeof(int32_t) * t->nnodes, st));
    HIP_TRY(hipMemsetAsync(t->skel.p, 0xff, sizeof(int32_t) * t->nnodes * t->s, st));  // -1: no skeleton yet
    HIP_TRY(hipMemsetAsync(t->trunc.p, 0, sizeof(int32_t) * t->nnodes, st));
    HIP_TRY(hipMemsetAsync(t->qrows.p, 0, sizeof(int32_t) * t->nnodes, st));
    HIP_TRY(hipStreamSynchronize(st));
    t->t_tree = ms_since(t0);
    if (t->knn > 0) {
        auto t1 = std::chrono::steady_clock::now();
        ST_TRY(build_neighbor_lists(t.get(), st));
        t->t_knn = ms_since(t1);
    }
    *out = t.release();
    return ASKIT_OK;
}

askit_status askit_tree_knn(askit_tree t, int32_t *idx) {
    if (!t || !idx) return fail(ASKIT_ERR_ARG, "NULL argument");
    if (t->knn <= 0) return fail(ASKIT_ERR_STATE, "the tree was built without neighbour sampling (knn = 0)");
    HIP_TRY(hipMemcpy(idx, t->knnidx.p, sizeof(int32_t) * t->N * t->knn, hipMemcpyDefault));
    return ASKIT_OK;
}

askit_status askit_tree_neighbor_lists(askit_tree t, int32_t *pos, int32_t *weight, int32_t *len) {
    if (!t || !pos || !weight || !len) return fail(ASKIT_ERR_ARG, "NULL argument");
    if (t->knn <= 0) return fail(ASKIT_ERR_STATE, "the tree was built without neighbour sampling (knn = 0)");
    const size_t n = sizeof(int32_t) * t->nnodes * t->nsamp;
    HIP_TRY(hipMemcpy(pos, t->nbpos.p, n, hipMemcpyDefault));
    HIP_TRY(hipMemcpy(weight, t->nbw.p, n, hipMemcpyDefault));
    HIP_TRY(hipMemcpy(len, t->nblen.p, sizeof(int32_t) * t->nnodes, hipMemcpyDefault));
    return ASKIT_OK;
}

askit_status askit_tree_depth(askit_tree t, int32_t *D) {
    if (!t || !D) return fail(ASKIT_ERR_ARG, "NULL argument");
    *D = t->D;
    return ASKIT_OK;
}

askit_status askit_tree_qr_rows(askit_tree t, int32_t *rows) {
    if (!t || !rows) return fail(ASKIT_ERR_ARG, "NULL argument");
    if (!t->skel_ok) return fail(ASKIT_ERR_STATE, "the tree is not skeletonized");
    HIP_TRY(hipMemcpy(rows, t->qrows.p, sizeof(int32_t) * t->nnodes, hipMemcpyDefault));
    return ASKIT_OK;
}

askit_status askit_tree_samples(askit_tree t, int32_t *samples) {
    if (!t || !samples) return fail(ASKIT_ERR_ARG, "NULL argument");
    if (!t->skel_ok || !t->samp.p) return fail(ASKIT_ERR_STATE, "the tree is not skeletonized");
    HIP_TRY(hipMemcpy(samples, t->samp.p, sizeof(int32_t) * t->nnodes * t->nsamp, hipMemcpyDefault));
    return ASKIT_OK;
}

askit_status askit_tree_perm(askit_tree t, int64_t *perm) {
    if (!t || !perm) return fail(ASKIT_ERR_ARG, "NULL argument");
    HIP_TRY(hipMemcpy(perm, t->perm.p, sizeof(int64_t) * t->N, hipMemcpyDefault));
    return ASKIT_OK;
}

void askit_tree_destroy(askit_tree t) { delete t; }

// ---------------------------------------------------------------------------
// skeletonization (Alg. 1), level by level from the leaves up
// ---------------------------------------------------------------------------
// One skeletonization pass over a set of trees, height by height.  prepare()
// waits for the previous height, reads the ranks it decided (they fix the
// candidate counts and so every launch shape of this height) and uploads the
// task lists; launch() only enqueues kernels, so that a caller can enqueue
// other work in between without waiting on this stream.
struct SkelRun {
    askit_tree *trees = nullptr;
    int count = 0, Hmax = 0, nsamp_max = 0, cmax = 0, s = 0, d = 0;
    hipStream_t st = nullptr;
    DBuf M, err, dsamp, dsk, dqr, dsplit;
    DBuf wpart, wrmap, wrows, wnrm, wpos, wdiag, wst;
    // Buffers outgrown by a later height are released when the run ends, not
    // when they are replaced: a release synchronizes the device, which in the
    // pipelined call would wait for the factorization queued on the other
    // stream and stall the skeleton chain.
    std::vector<std::unique_ptr<DBuf>> retired;
    // launch parameters of the prepared height
    int nqr = 0, n1 = 0, nsp = 0, split_steps = 0;
    QrWork w{};


    // In the pipelined call the skeletonization of a level overlaps the
    // factorization below it; there a level with 2^kOneWgLevel nodes or more
    // does better with one workgroup per node than with one launch per pivot
    // step (measured at the 1M workload), so the library's default narrows to
    // the levels with fewer nodes.  Both shapes give the same skeletons.
    bool pipelined = false;
    int split_of(askit_tree t) const {
        return pipelined && t->split_default ? std::min(t->split_levels, kOneWgLevel - 1) : t->split_levels;
    }

    askit_status begin(askit_tree *tr, int cnt, hipStream_t stream) {
        trees = tr;
        count = cnt;
        st = stream;
        for (int i = 0; i < count; i++) Hmax = std::max(Hmax, trees[i]->D);
        s = trees[0]->s;
        d = trees[0]->d;
        for (int i = 0; i < count; i++) {
            nsamp_max = std::max(nsamp_max, trees[i]->nsamp);
            cmax = std::max(cmax, trees[i]->cmax);
            if (trees[i]->s != s || trees[i]->d != d)
                return fail(ASKIT_ERR_ARG, "batched trees must share rank and dimension");
            if (!trees[i]->samp.p) ST_TRY(trees[i]->samp.alloc(sizeof(int32_t) * trees[i]->nnodes * trees[i]->nsamp));
            HIP_TRY(hipMemsetAsync(trees[i]->qrows.p, 0, sizeof(int32_t) * trees[i]->nnodes, stream));
            trees[i]->hsr.assign(trees[i]->nnodes, 0);
            trees[i]->skel_ok = false;
        }
        ST_TRY(err.alloc(sizeof(int32_t)));
        HIP_TRY(hipMemsetAsync(err.p, 0, sizeof(int32_t), st));
        return ASKIT_OK;
    }

    // the ranks decided so far, on the host (through pinned memory: a copy
    // to pageable memory goes through the runtime's staging path, which
    // does not stay ordered on `st` alone)
    askit_status read_ranks() {
        for (int i = 0; i < count; i++) {
            askit_tree t = trees[i];
            if (!t->hsr_pinned) HIP_TRY(hipHostMalloc((void **)&t->hsr_pinned, sizeof(int32_t) * t->nnodes));
            HIP_TRY(hipMemcpyAsync(t->hsr_pinned, t->srank.p, sizeof(int32_t) * t->nnodes, hipMemcpyDeviceToHost,
                                   st));
        }
        HIP_TRY(hipStreamSynchronize(st));
        for (int i = 0; i < count; i++) {
            std::copy(trees[i]->hsr_pinned, trees[i]->hsr_pinned + trees[i]->nnodes, trees[i]->hsr.begin());
            trees[i]->hsr[0] = 0;
        }
        return ASKIT_OK;
    }

    askit_status prepare(int hgt) {
        // the children's ranks (decided at the previous height) fix the
        // candidate counts: nodes with |C| <= s keep all candidates (P = I)
        // and need neither samples nor a QR
        if (hgt > 0) ST_TRY(read_ranks());
        else HIP_TRY(hipStreamSynchronize(st));
        // in the pipelined call the task lists are queued on the skeleton
        // stream itself (host copies kept until the call ends): a synchronous
        // copy would also wait for the factorization queued on the other
        // stream, and stall the skeleton chain for as long
        std::unique_ptr<UploadOnStream> on_stream;
        if (pipelined) on_stream.reset(new UploadOnStream(st));
        std::vector<SampTask> samp_one, samp_split;
        std::vector<SkelTask> qr_one, qr_split, ident;
        int split_cols = 0;
        split_steps = 0;
        for (int i = 0; i < count; i++) {
            askit_tree t = trees[i];
            const int l = t->D - hgt;
            if (l < 1) continue;
            for (int64_t id = t->first(l); id < t->first(l + 1); id++) {
                SkelTask k{};
                k.X = t->Xp.as<double>();
                k.leaf = (l == t->D);
                k.b = t->nb[id];
                k.n = (int32_t)(t->ne[id] - t->nb[id]);
                k.cmax = t->cmax;
                if (!k.leaf) {
                    k.skl = t->skel.as<int32_t>() + (2 * id + 1) * t->s;
                    k.skr = t->skel.as<int32_t>() + (2 * id + 2) * t->s;
                    k.srl = t->srank.as<int32_t>() + 2 * id + 1;
                    k.srr = t->srank.as<int32_t>() + 2 * id + 2;
                }
                k.skel = t->skel.as<int32_t>() + id * t->s;
                k.sr = t->srank.as<int32_t>() + id;
                k.trunc = t->trunc.as<int32_t>() + id;
                k.qrows = t->qrows.as<int32_t>() + id;
                k.Pt = t->Pt.as<double>() + id * (int64_t)t->cmax * t->s;
                k.scale = -1.0 / (2.0 * t->h * t->h);
                k.tol = t->tol;
                const int ncand = k.leaf ? k.n : t->hsr[2 * id + 1] + t->hsr[2 * id + 2];
                if (ncand <= s) {
                    ident.push_back(k);
                    continue;
                }
                SampTask a{};
                a.b = t->nb[id];
                a.e = t->ne[id];
                a.N = t->N;
                a.state = node_state(t->seed, t->problem, id);
                a.out = t->samp.as<int32_t>() + id * t->nsamp;
                if (t->knn > 0) {  // the node's neighbour list opens its sample
                    a.pre = t->nbpos.as<int32_t>() + id * t->nsamp;
                    a.npre = t->hnn[id];
                }
                k.q = a.out;
                k.nq = (int32_t)std::min<int64_t>(t->nsamp, t->N - (a.e - a.b));
                if (l <= split_of(t)) {
                    samp_split.push_back(a);
                    qr_split.push_back(k);
                    split_cols = std::max(split_cols, ncand);
                    split_steps = std::max(split_steps, std::min(s, k.nq));
                } else {
                    samp_one.push_back(a);
                    qr_one.push_back(k);
                }
            }
        }
        // sampled nodes: one-workgroup ones first, then the split ones
        std::vector<SampTask> samp(samp_one);
        samp.insert(samp.end(), samp_split.begin(), samp_split.end());
        std::vector<SkelTask> qr(qr_one);
        qr.insert(qr.end(), qr_split.begin(), qr_split.end());
        nqr = (int)qr.size();
        nsp = (int)qr_split.size();
        const int none_ = (int)qr_one.size();
        const int64_t slot = (int64_t)nsamp_max * cmax;  // sampled block per node, column-major, ld nsamp_max
        ST_TRY(grow_keep(retired, M, sizeof(double) * std::max(nqr, 1) * slot));
        for (int j = 0; j < nqr; j++) qr[j].M = M.as<double>() + (int64_t)j * slot;
        for (int j = 0; j < nsp; j++) qr_split[j].M = qr[none_ + j].M;
        std::vector<SkelTask> one(qr.begin(), qr.begin() + none_);
        one.insert(one.end(), ident.begin(), ident.end());
        n1 = (int)one.size();
        if (nqr > 0) {
            ST_TRY(upload_grow_keep(retired, dsamp, samp));
            ST_TRY(upload_grow_keep(retired, dsk, qr));
        }
        if (n1 > 0) ST_TRY(upload_grow_keep(retired, dqr, one));
        if (nsp > 0) {
            w = QrWork{};
            w.cmax = cmax;
            w.rcap = nsamp_max;
            w.slices = (int)cdiv(split_cols, kQsCols);
            ST_TRY(upload_grow_keep(retired, dsplit, qr_split));
            ST_TRY(grow_keep(retired, wpart, sizeof(double) * (size_t)nsp * w.slices * w.rcap));
            ST_TRY(grow_keep(retired, wrmap, sizeof(int32_t) * (size_t)nsp * w.rcap));
            ST_TRY(grow_keep(retired, wrows, sizeof(int32_t) * (size_t)nsp));
            ST_TRY(grow_keep(retired, wnrm, sizeof(double) * (size_t)nsp * 2 * cmax));
            ST_TRY(grow_keep(retired, wpos, sizeof(int32_t) * (size_t)nsp * 2 * cmax));
            ST_TRY(grow_keep(retired, wdiag, sizeof(double) * (size_t)nsp * cmax));
            ST_TRY(grow_keep(retired, wst, sizeof(int32_t) * (size_t)nsp * kQsState));
            w.part = wpart.as<double>();
            w.rmap = wrmap.as<int32_t>();
            w.rows = wrows.as<int32_t>();
            w.nrm = wnrm.as<double>();
            w.pos = wpos.as<int32_t>();
            w.diag = wdiag.as<double>();
            w.st = wst.as<int32_t>();
        }
        return ASKIT_OK;
    }

    askit_status launch(int hgt) {
        if (nqr > 0) {
            // all trees of a batch share nsamp (checked by the batched entry point)
            HIP_TRY(timed("skel:k_sample" + prof_height(hgt), st, [&] {
                hipLaunchKernelGGL(k_sample, dim3(nqr), dim3(64), 0, st, dsamp.as<SampTask>(), nsamp_max,
                                   err.as<int32_t>());
                return hipGetLastError();
            }));
            // the QR tasks hold the one-workgroup nodes first, then the split ones
            const int rt = (int)cdiv(nsamp_max, 64), ct = (int)cdiv(cmax, 64), none_ = nqr - nsp;
            const size_t lds = sizeof(double) * (64 * (d | 1) + 64 * std::max(d, kXrDim));
            if (none_ > 0)
                HIP_TRY(timed("skel:k_sample_rownorm" + prof_height(hgt), st, [&] {
                    hipLaunchKernelGGL(k_sample_rownorm, dim3(none_ * rt * ct), dim3(256), lds, st,
                                       dsk.as<SkelTask>(), rt, nsamp_max, d, ct);
                    return hipGetLastError();
                }));
            if (nsp > 0)
                HIP_TRY(timed("skel:k_sample_block" + prof_height(hgt), st, [&] {
                    hipLaunchKernelGGL(k_sample_block, dim3(nsp * rt * ct), dim3(256), lds, st,
                                       dsk.as<SkelTask>() + none_, rt, nsamp_max, d, ct);
                    return hipGetLastError();
                }));
        }
        if (n1 > 0) {
            HIP_TRY(timed("skel:k_qrcp" + prof_height(hgt), st, [&] {
                hipLaunchKernelGGL(k_qrcp, dim3(n1), dim3(512), 0, st, dqr.as<SkelTask>(), s, nsamp_max, d);
                return hipGetLastError();
            }));
        }
        if (nsp > 0) ST_TRY(split_qr(hgt));
        return ASKIT_OK;
    }

    // The pivoted QR of the split nodes: row norms, row map, compaction and
    // initial norms, one launch per pivot step, then T and the outputs.
    askit_status split_qr(int hgt) {
        const SkelTask *tp = dsplit.as<SkelTask>();
        const QrWork wk = w;
        const unsigned g = (unsigned)(nsp * wk.slices);
        const std::string hs = prof_height(hgt);
        HIP_TRY(timed("skel:k_qs_rows" + hs, st, [&] {
            hipLaunchKernelGGL(k_qs_rows, dim3(g), dim3(kQsThreads), 0, st, tp, wk, nsamp_max);
            return hipGetLastError();
        }));
        HIP_TRY(timed("skel:k_qs_rowmap" + hs, st, [&] {
            hipLaunchKernelGGL(k_qs_rowmap, dim3(nsp), dim3(512), 0, st, tp, wk);
            return hipGetLastError();
        }));
        HIP_TRY(timed("skel:k_qs_init" + hs, st, [&] {
            hipLaunchKernelGGL(k_qs_init, dim3(g), dim3(kQsThreads), 0, st, tp, wk, s, nsamp_max);
            return hipGetLastError();
        }));
        // the pivot steps: one launch each, timed as one chain; step j
        // launches the slices from (j - 1) / kQsCols on (k_qs_step)
        HIP_TRY(timed(
            "skel:k_qs_step" + hs, st,
            [&] {
                for (int j = 0; j < split_steps; j++) {
                    const int s0 = j > 0 ? (j - 1) / kQsCols : 0;
                    hipLaunchKernelGGL(k_qs_step, dim3((unsigned)(nsp * (wk.slices - s0))), dim3(kQsThreads), 0, st,
                                       tp, wk, j, s0);
                }
                return hipGetLastError();
            },
            split_steps));
        HIP_TRY(timed("skel:k_qs_finish" + hs, st, [&] {
            hipLaunchKernelGGL(k_qs_finish, dim3(nsp, (unsigned)cdiv(wk.slices * kQsCols, kQsFinishCols)), dim3(512), 0,
                               st, tp, wk, s, nsamp_max);
            return hipGetLastError();
        }));
        return ASKIT_OK;
    }

    // the ranks decide the shapes of every later launch: keep them on the host
    askit_status end() {
        int32_t herr = 0;
        HIP_TRY(hipMemcpyAsync(&herr, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        ST_TRY(read_ranks());
        if (herr) return fail(ASKIT_ERR_HIP, "row sampling did not terminate");
        for (int i = 0; i < count; i++) trees[i]->skel_ok = true;
        return ASKIT_OK;
    }
};

// skeletonization (Alg. 1), level by level from the leaves up
static askit_status skeletonize_impl(askit_tree *trees, int count, hipStream_t st) {
    SkelRun R;
    ST_TRY(R.begin(trees, count, st));
    for (int hgt = 0; hgt < R.Hmax; hgt++) {
        ST_TRY(R.prepare(hgt));
        ST_TRY(R.launch(hgt));
    }
    return R.end();
}

askit_status askit_skeletonize(askit_tree t, void *stream) {
    if (!t) return fail(ASKIT_ERR_ARG, "NULL tree");
    if (t->refs) return fail(ASKIT_ERR_STATE, "destroy the factors of this tree before re-skeletonizing");
    auto t0 = std::chrono::steady_clock::now();
    ST_TRY(skeletonize_impl(&t, 1, (hipStream_t)stream));
    t->t_skel = ms_since(t0);
    return ASKIT_OK;
}

askit_status askit_skeletons_export(askit_tree t, int32_t *ids, double *P, int32_t *sizes) {
    if (!t || !sizes || (!ids) != (!P)) return fail(ASKIT_ERR_ARG, "NULL argument");
    if (!t->skel_ok) return fail(ASKIT_ERR_STATE, "tree not skeletonized");
    if (!ids) {  // sizes only
        for (int64_t id = 0; id < t->nnodes; id++) {
            int lvl = 0;
            while (((int64_t)2 << lvl) - 1 <= id) lvl++;
            const bool leaf = (lvl == t->D);
            sizes[2 * id] = id ? t->hsr[id] : 0;
            sizes[2 * id + 1] = !id ? 0 : leaf ? (int)(t->ne[id] - t->nb[id]) : t->hsr[2 * id + 1] + t->hsr[2 * id + 2];
        }
        return ASKIT_OK;
    }
    std::vector<int32_t> sr(t->nnodes);
    HIP_TRY(hipMemcpy(ids, t->skel.p, sizeof(int32_t) * t->nnodes * t->s, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(sr.data(), t->srank.p, sizeof(int32_t) * t->nnodes, hipMemcpyDeviceToHost));
    std::vector<double> Pt((size_t)t->nnodes * t->cmax * t->s);
    HIP_TRY(hipMemcpy(Pt.data(), t->Pt.p, sizeof(double) * Pt.size(), hipMemcpyDeviceToHost));
    // P_{alpha~ C} (s_alpha x |C|, compact columns) from the padded transposed rows
    for (int64_t id = 0; id < t->nnodes; id++) {
        sizes[2 * id] = id ? sr[id] : 0;
        int nc = 0;
        int lvl = 0;
        while (((int64_t)2 << lvl) - 1 <= id) lvl++;
        if (id == 0) {
            sizes[1] = 0;
            continue;
        }
        bool leaf = (lvl == t->D);
        int sl = leaf ? 0 : sr[2 * id + 1];
        nc = leaf ? (int)(t->ne[id] - t->nb[id]) : sl + sr[2 * id + 2];
        sizes[2 * id + 1] = nc;
        double *dst = P + id * (int64_t)t->s * t->cmax;
        for (int k = 0; k < sr[id]; k++)
            for (int c = 0; c < nc; c++) {
                int row = leaf ? c : (c < sl ? c : t->s + (c - sl));
                dst[(int64_t)k * nc + c] = Pt[(size_t)id * t->cmax * t->s + (size_t)row * t->s + k];
            }
    }
    return ASKIT_OK;
}

askit_status askit_skeletons_import(askit_tree t, const int32_t *ids, const double *P, const int32_t *sizes) {
    if (!t || !ids || !P || !sizes) return fail(ASKIT_ERR_ARG, "NULL argument");
    if (t->refs) return fail(ASKIT_ERR_STATE, "destroy the factors of this tree first");
    std::vector<int32_t> sr(t->nnodes, 0), sk((size_t)t->nnodes * t->s, -1), tr(t->nnodes, 0);
    std::vector<double> Pt((size_t)t->nnodes * t->cmax * t->s, 0.0);
    for (int64_t id = 1; id < t->nnodes; id++) {
        int lvl = 0;
        while (((int64_t)2 << lvl) - 1 <= id) lvl++;
        bool leaf = (lvl == t->D);
        int r = sizes[2 * id], nc = sizes[2 * id + 1];
        int want_nc = leaf ? (int)(t->ne[id] - t->nb[id]) : sizes[2 * (2 * id + 1)] + sizes[2 * (2 * id + 2)];
        if (r < 1 || r > t->s || nc != want_nc) return fail(ASKIT_ERR_ARG, "inconsistent skeleton sizes");
        sr[id] = r;
        int sl = leaf ? 0 : sizes[2 * (2 * id + 1)];
        for (int k = 0; k < r; k++) {
            int32_t p = ids[id * t->s + k];
            if (p < t->nb[id] || p >= t->ne[id]) return fail(ASKIT_ERR_ARG, "skeleton point outside its node");
            sk[(size_t)id * t->s + k] = p;
        }
        const double *src = P + id * (int64_t)t->s * t->cmax;
        for (int k = 0; k < r; k++)
            for (int c = 0; c < nc; c++) {
                int row = leaf ? c : (c < sl ? c : t->s + (c - sl));
                Pt[(size_t)id * t->cmax * t->s + (size_t)row * t->s + k] = src[(int64_t)k * nc + c];
            }
    }
    HIP_TRY(hipMemcpy(t->srank.p, sr.data(), sizeof(int32_t) * t->nnodes, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t->trunc.p, tr.data(), sizeof(int32_t) * t->nnodes, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t->skel.p, sk.data(), sizeof(int32_t) * sk.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t->Pt.p, Pt.data(), sizeof(double) * Pt.size(), hipMemcpyHostToDevice));
    t->hsr = sr;
    t->skel_ok = true;
    return ASKIT_OK;
}

// ---------------------------------------------------------------------------
// factorization (Alg. 2)
// ---------------------------------------------------------------------------
static const int64_t kChunk = 4096;  // contraction chunk of the split products

// Factorization plan for one or several factors of equal rank, dimension and
// precision: one launch per kernel and tree height (distance from the
// leaves), covering the nodes of every tree at that height.
// One part of the factorization plan: part -1 = the leaf LUs of
// lambda I + K_aa (they need no skeletons), part 0 = the leaves' Phat, part
// h >= 1 = the internal nodes at height h.  Part h >= 0 reads the ranks and
// skeletons of heights <= h only, and of a part h >= 1 the half `PartZ` (Z
// and its LU) only those of heights <= h - 1; the half `PartPhat` (Xc =
// Z^{-1} P_c and the telescoped Phat) needs the node's own skeleton.
static int builtin_tc(int cols) { return cols >= 128 ? 128 : (cols >= 64 ? 64 : 16); }

// smallest split chunk the factorization of t may use (sizes its workspace)
static int64_t tree_kc_min(askit_tree t) {
    int64_t kc = kChunk;
    for (const Tune &u : t->tune)
        if (u.kmm_kc > 0) kc = std::min(kc, u.kmm_kc);
    return kc;
}

// force: the tile configuration of every height of this part (tuning runs);
// else a single tree's tuned configuration, else the built-in choice
enum PartHalf { PartAll = 3, PartZ = 1, PartPhat = 2 };

// the smallest split size of the trees factored together
static int32_t lu_split_of(const std::vector<askit_factor> &fs) {
    int32_t n = kLuSplitN;
    for (size_t i = 0; i < fs.size(); i++) n = i ? std::min(n, fs[i]->t->lu_split) : fs[i]->t->lu_split;
    return n;
}

static askit_status factor_plan_part(const std::vector<askit_factor> &fs, Plan &P, int part,
                                     const Tune *force = nullptr, int half = PartAll) {
    askit_tree t0 = fs[0]->t;
    const int s = t0->s, d = t0->d, s2 = 2 * s;
    const Prec pr = fs[0]->prec;
    const int el = (int)fs[0]->elem();
    int Hmax = 0, mmax = 0;
    for (auto f : fs) {
        Hmax = std::max(Hmax, f->t->D);
        mmax = std::max(mmax, f->t->mmax);
    }
    P.sub = prof_height(std::max(part, 0));
    // height 0: leaves -- lambda I + K_aa, LU, Phat = A^{-1} P_{alpha alpha~}
    if (part <= 0) {
        std::vector<LeafTask> lt;
        std::vector<LuTask> lu, rs;
        std::vector<CopyTask> cp;
        for (auto f : fs) {
            askit_tree t = f->t;
            const int D = t->D;
            for (int64_t id = t->first(D); id < t->nnodes; id++) {
                LeafTask a{};
                a.X = t->Xp.as<double>();
                a.b = t->nb[id];
                a.n = (int32_t)(t->ne[id] - t->nb[id]);
                a.lda = t->mmax;
                a.A = f->lu_of(id);
                a.scale = -1.0 / (2.0 * f->h * f->h);
                a.lambda = f->lambda;
                lt.push_back(a);
                LuTask u{};
                u.A = a.A;
                u.piv = f->piv_of(id);
                u.dinv = f->dinv_of(id);
                u.n = a.n;
                u.lda = t->mmax;
                u.ratio = f->ratio.as<double>() + id;
                lu.push_back(u);
                if (D > 0) {
                    CopyTask c{};
                    c.src = t->Pt.as<double>() + id * (int64_t)t->cmax * s;
                    c.dst = (char *)f->ph(D) + t->nb[id] * s * el;
                    c.sld = s;
                    c.dld = s;
                    c.rows = a.n;
                    c.cols = t->hsr[id];
                    cp.push_back(c);
                    u.B = c.dst;
                    u.ldb = s;
                    u.nrhs = t->hsr[id];
                    rs.push_back(u);
                }
            }
        }
        if (part < 0) {
            DBuf *b = P.own();
            ST_TRY(upload(*b, lt));
            const LeafTask *lp = b->as<LeafTask>();
            const int nl = (int)lt.size(), tl = (int)cdiv(mmax, 64);
            P.add("k_leaf_block", [=](hipStream_t st, int) -> hipError_t {
                hipLaunchKernelGGL(k_leaf_block, dim3(nl * tl * tl), dim3(256),
                                   sizeof(double) * (64 * (d | 1) + 64 * std::max(d, kXrDim)), st, lp, tl, d);
                return hipGetLastError();
            });
            // lambda I + K_aa is symmetric positive definite for lambda > 0
            bool spd = true;
            for (auto f : fs) spd = spd && f->lambda > 0.0;
            ST_TRY(lu_commit(P, lu, spd, lu_split_of(fs)));
        } else {
            ST_TRY(copy_commit(P, cp, P64, pr, mmax, s));
            ST_TRY(getrs_commit(P, rs, pr, false, s));
        }
    }
    // heights 1 .. Hmax: internal nodes, bottom-up
    for (int hgt = std::max(part, 1); hgt <= std::min(part, Hmax); hgt++) {
        std::vector<IdTask> ident;
        const Tune *tn = force;
        if (!tn && fs.size() == 1 && (size_t)hgt < fs[0]->t->tune.size()) tn = &fs[0]->t->tune[hgt];
        KmmBuild kb;
        kb.tc = tn && tn->kmm_tc ? tn->kmm_tc : builtin_tc(s);
        const int64_t kc = tn && tn->kmm_kc ? tn->kmm_kc : kChunk;
        kb.out_size = 8;
        std::vector<LuTask> lu, rs;
        std::vector<CopyTask> cp, cp32;
        GmmBuild gb;
        gb.tc = tn && tn->gmm_tc ? tn->gmm_tc : builtin_tc(s);
        if (pr != P64) {  // 256-column tiles exist in FP64 only
            kb.tc = std::min(kb.tc, 128);
            gb.tc = std::min(gb.tc, 128);
        }
        gb.elem = el;
        for (auto f : fs) {
            askit_tree t = f->t;
            const int l = t->D - hgt;
            if (l < 0) continue;
            const int64_t f0 = t->first(l), cnt = (int64_t)1 << l;
            int64_t wsoff = 0;
            for (int64_t id = f0; id < f0 + cnt; id++) {
                const int64_t lc = 2 * id + 1, rc = 2 * id + 2;
                // Z = [I, K1 Phat_r; K2 Phat_l, I] of order n = s_l + s_r,
                // column-major with leading dimension n (eq. (8))
                const int sl = t->hsr[lc], sr = t->hsr[rc], n = sl + sr, sa = t->hsr[id];
                double *Z = f->lu_of(id);
                if (half & PartZ) ident.push_back({Z, n, 0});
                for (int side = 0; side < 2 && (half & PartZ); side++) {
                    const int64_t a = side ? rc : lc, o = side ? lc : rc;  // skeleton of a vs points of o
                    KmmTask k{};
                    k.X = t->Xp.as<double>();
                    k.R.idx = t->skel.as<int32_t>() + a * s;
                    k.R.n = t->hsr[a];
                    k.S.base = t->nb[o];
                    k.S.n = (int32_t)(t->ne[o] - t->nb[o]);
                    k.B = (const char *)f->ph(l + 1) + t->nb[o] * s * el;
                    k.ldb = s;
                    k.C = side ? Z + sl : Z + (int64_t)sl * n;
                    k.crs = 1;
                    k.ccs = n;
                    k.scale = -1.0 / (2.0 * f->h * f->h);
                    k.op = OP_STORE;
                    k.rcap = t->hsr[a];
                    k.ncol = t->hsr[o];
                    kmm_add(kb, k, k.S.n, k.ncol, kc, el, f->ws.as<char>(), wsoff);
                }
                LuTask u{};
                u.A = Z;
                u.piv = f->piv_of(id);
                u.dinv = f->dinv_of(id);
                u.n = n;
                u.lda = n;
                u.ratio = f->ratio.as<double>() + id;
                if (half & PartZ) lu.push_back(u);
                if (l >= 1 && (half & PartPhat)) {
                    // Xc = Z^{-1} P_c with P_c = P_{alpha~ [l~ r~]}^T (n x s_alpha,
                    // row stride s), then Phat_alpha = blockdiag(Phat_l, Phat_r) Xc
                    double *xc = f->Xc.as<double>() + (id - f0) * (int64_t)s2 * s;
                    const double *pt = t->Pt.as<double>() + id * (int64_t)t->cmax * s;
                    cp.push_back(CopyTask{pt, xc, s, s, sl, sa});
                    cp.push_back(CopyTask{pt + (int64_t)s * s, xc + (int64_t)sl * s, s, s, sr, sa});
                    u.B = xc;
                    u.ldb = s;
                    u.nrhs = sa;
                    rs.push_back(u);
                    const void *xb = xc;
                    if (pr == P32) {
                        float *xf = f->Xcf.as<float>() + (id - f0) * (int64_t)s2 * s;
                        cp32.push_back(CopyTask{xc, xf, s, s, n, sa});
                        xb = xf;
                    }
                    for (int side = 0; side < 2; side++) {
                        const int64_t ch = side ? rc : lc;
                        GmmTask g{};
                        g.A = (const char *)f->ph(l + 1) + t->nb[ch] * s * el;
                        g.ars = s;
                        g.acs = 1;
                        g.B = (const char *)xb + (int64_t)(side ? sl : 0) * s * el;
                        g.brs = s;
                        g.bcs = 1;
                        g.C = (char *)f->ph(l) + t->nb[ch] * s * el;
                        g.crs = s;
                        g.ccs = 1;
                        g.rows = (int32_t)(t->ne[ch] - t->nb[ch]);
                        g.kdim = t->hsr[ch];
                        g.op = OP_STORE;
                        g.ncol = sa;
                        int64_t none = 0;
                        gmm_add(gb, g, sa, 1 << 30, nullptr, none);
                    }
                }
            }
            if (wsoff * 8 > (int64_t)f->ws.bytes) return fail(ASKIT_ERR_STATE, "internal: workspace too small");
        }
        ST_TRY(ident_commit(P, ident, s2));
        ST_TRY(kmm_commit(P, kb, pr, P64, d, s));
        ST_TRY(lu_commit(P, lu, false, lu_split_of(fs)));
        ST_TRY(copy_commit(P, cp, P64, P64, s2, s));
        ST_TRY(getrs_commit(P, rs, P64, false, s));
        if (pr == P32) ST_TRY(copy_commit(P, cp32, P64, P32, s2, s));
        ST_TRY(gmm_commit(P, gb, pr, 0));
    }
    P.sub.clear();
    return ASKIT_OK;
}

static int factor_height_max(const std::vector<askit_factor> &fs) {
    int H = 0;
    for (auto f : fs) H = std::max(H, f->t->D);
    return H;
}

static askit_status factor_plan(const std::vector<askit_factor> &fs, Plan &P) {
    // with a level restriction only the frontier's subtrees are factored
    const int top = (fs.size() == 1 && fs[0]->hyb) ? fs[0]->t->D - fs[0]->hyb : factor_height_max(fs);
    for (int part = -1; part <= top; part++) ST_TRY(factor_plan_part(fs, P, part));
    return ASKIT_OK;
}

// partial-sum workspace needed by the split products of one level
static int64_t split_ws_elems(askit_tree t, int ncol, int64_t KC) {
    int64_t worst = 0;
    for (int l = 0; l < t->D; l++) {
        int64_t tot = 0;
        for (int64_t id = t->first(l); id < t->first(l + 1); id++)
            for (int side = 0; side < 2; side++) {
                int64_t o = 2 * id + 1 + (side ? 0 : 1);
                int64_t n = t->ne[o] - t->nb[o];
                int64_t nch = cdiv(n, KC);
                if (nch > 1) tot += nch * (int64_t)t->s * ncol;
            }
        worst = std::max(worst, tot);
    }
    return worst;
}

// allocation of a factor's arenas (no work enqueued)
static askit_status factor_alloc(askit_tree t, double lambda, int precision, std::unique_ptr<askit_factor_s> &f) {
    f.reset(new askit_factor_s());
    f->t = t;
    f->lambda = lambda;
    f->h = t->hfac;
    f->prec = precision == ASKIT_MIXED ? P32 : P64;
    f->max_refine = f->prec == P32 ? 100 : 0;
    const int s = t->s, D = t->D, s2 = 2 * s;
    const int64_t leaf0 = t->first(D), nleaf = (int64_t)1 << D;
    f->leafLU = 0;
    f->zLU = nleaf * (int64_t)t->mmax * t->mmax;
    ST_TRY(f->LU.alloc(sizeof(double) * (f->zLU + leaf0 * (int64_t)s2 * s2)));
    ST_TRY(f->piv.alloc(sizeof(int32_t) * (nleaf * t->mmax + leaf0 * s2)));
    ST_TRY(f->ratio.alloc(sizeof(double) * t->nnodes));
    ST_TRY(f->dinv.alloc(sizeof(double) * 512 * (nleaf * ((t->mmax + 15) / 16) + leaf0 * ((s2 + 15) / 16))));
    for (int l = 1; l <= D; l++) {
        f->PH.emplace_back(new DBuf());
        ST_TRY(f->PH.back()->alloc(f->elem() * t->N * s));
    }
    const int64_t lvl_max = D >= 2 ? ((int64_t)1 << (D - 1)) : 1;  // nodes of the widest level with a telescoping step
    ST_TRY(f->Xc.alloc(sizeof(double) * lvl_max * s2 * s));
    if (f->prec == P32) ST_TRY(f->Xcf.alloc(sizeof(float) * lvl_max * s2 * s));
    ST_TRY(f->ws.alloc(sizeof(double) * std::max<int64_t>(1, split_ws_elems(t, s, tree_kc_min(t)))));
    return ASKIT_OK;
}

// smallest pivot ratio of a finished factorization (synchronizes `st`)
static askit_status factor_ratio(askit_factor f, hipStream_t st) {
    askit_tree t = f->t;
    std::vector<double> ratio(t->nnodes);
    HIP_TRY(hipMemcpyAsync(ratio.data(), f->ratio.p, sizeof(double) * t->nnodes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    f->min_ratio = 1.0;
    f->min_node = -1;
    for (int64_t id = f->hyb ? t->first(f->hyb) : 0; id < t->nnodes; id++) {
        if (ratio[id] < f->min_ratio) {
            f->min_ratio = ratio[id];
            f->min_node = (int)id;
        }
    }
    return ASKIT_OK;
}

static askit_status ratio_status(askit_factor f) {
    if (f->min_ratio == 0.0) return fail(ASKIT_ERR_SINGULAR, "exactly singular pivot in a leaf or reduced system");
    if (f->min_ratio < 1e-12) return fail(ASKIT_WARN_ILLCOND, "pivot ratio below 1e-12: factorization unstable");
    return ASKIT_OK;
}

static askit_status factorize_impl(askit_tree t, double lambda, int precision, hipStream_t st, askit_factor *out) {
    std::unique_ptr<askit_factor_s> f;
    ST_TRY(factor_alloc(t, lambda, precision, f));
    Plan P;
    P.tag = "factor";
    ST_TRY(factor_plan({f.get()}, P));
    HIP_TRY(P.run(st, t->s));
    ST_TRY(factor_ratio(f.get(), st));
    t->refs++;
    *out = f.release();
    return ratio_status(*out);
}

// Skeletonization and factorization as one pipeline over two streams: the
// caller's stream skeletonizes height h while an internal stream factorizes
// height h - 1 (which reads only the ranks, skeletons and projections of
// heights <= h - 1); the leaf LUs, which need no skeletons, start at once.
// Each kernel sees the inputs it sees in the two separate calls, so the
// results are the same bit for bit.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    ~SideStream() {
        if (e) (void)hipEventDestroy(e);
        if (s) (void)hipStreamDestroy(s);
    }
};

// releases the host copies of queued uploads once every stream that read
// them has been synchronized (end of the owning call, also on errors: the
// error paths synchronize the device first)
struct UploadKeep {
    ~UploadKeep() {
        if (!g_upload_keep.empty()) {
            (void)hipDeviceSynchronize();
            g_upload_keep.clear();
        }
    }
};

static askit_status skel_factor_impl(askit_tree t, double lambda, int precision, hipStream_t st, askit_factor *out,
                                     double &t_skel) {
    auto t0 = std::chrono::steady_clock::now();
    SkelRun R;
    R.pipelined = true;
    ST_TRY(R.begin(&t, 1, st));
    std::unique_ptr<askit_factor_s> f;
    ST_TRY(factor_alloc(t, lambda, precision, f));
    SideStream B;
    // non-blocking: no implicit ordering against the legacy default stream
    HIP_TRY(hipStreamCreateWithFlags(&B.s, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&B.e, hipEventDisableTiming));
    // uploads of the factorization's task lists go through their own
    // stream, so building the plan of height h - 1 neither waits for the
    // skeletonization of height h queued before it nor holds it back
    SideStream U;
    HIP_TRY(hipStreamCreateWithFlags(&U.s, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&U.e, hipEventDisableTiming));
    UploadKeep keep;
    const std::vector<askit_factor> fs{f.get()};
    Plan P;
    P.tag = "factor";
    ST_TRY(factor_plan_part(fs, P, -1));
    // the side stream starts after the work already queued on the caller's
    HIP_TRY(hipEventRecord(B.e, st));
    HIP_TRY(hipStreamWaitEvent(B.s, B.e, 0));
    HIP_TRY(P.run_from(B.s, t->s, 0));
    size_t done = P.steps.size();
    auto factor_part = [&](int part, int half) -> askit_status {
        {
            UploadOnStream g(U.s);
            ST_TRY(factor_plan_part(fs, P, part, nullptr, half));
        }
        HIP_TRY(hipEventRecord(U.e, U.s));
        HIP_TRY(hipStreamWaitEvent(B.s, U.e, 0));
        HIP_TRY(P.run_from(B.s, t->s, done));
        done = P.steps.size();
        return ASKIT_OK;
    };
    for (int hgt = 0; hgt <= R.Hmax; hgt++) {
        // wait for height hgt - 1 and read its ranks (the skeletonization
        // uploads are made while the skeleton stream is idle), launch height
        // hgt, then queue the rest of the factorization of height hgt - 1
        // (Xc and Phat, which need its skeletons) and the Z blocks and LUs of
        // height hgt (which need only those of its children), so that they
        // run while height hgt is skeletonized
        if (hgt < R.Hmax) {
            ST_TRY(R.prepare(hgt));
            ST_TRY(R.launch(hgt));
        } else {
            ST_TRY(R.end());
            t_skel = ms_since(t0);
        }
        if (hgt > 0) {
            ST_TRY(factor_part(hgt - 1, hgt - 1 == 0 ? PartAll : PartPhat));
            ST_TRY(factor_part(hgt, PartZ));
        }
    }
    ST_TRY(factor_part(R.Hmax, PartPhat));  // empty at the root
    // the caller's stream continues after the factorization
    HIP_TRY(hipEventRecord(B.e, B.s));
    HIP_TRY(hipStreamWaitEvent(st, B.e, 0));
    ST_TRY(factor_ratio(f.get(), st));
    t->refs++;
    *out = f.release();
    return ratio_status(*out);
}

askit_status askit_skeletonize_factorize(askit_tree t, double lambda, int32_t precision, void *stream,
                                         askit_factor *out) {
    if (!t || !out) return fail(ASKIT_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (t->refs) return fail(ASKIT_ERR_STATE, "destroy the factors of this tree before re-skeletonizing");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ASKIT_ERR_ARG, "lambda must be >= 0 and finite");
    if (precision != ASKIT_FP64 && precision != ASKIT_MIXED) return fail(ASKIT_ERR_ARG, "unknown precision");
    auto t0 = std::chrono::steady_clock::now();
    double ts = 0.0;
    askit_status st = skel_factor_impl(t, lambda, precision, (hipStream_t)stream, out, ts);
    t->t_skel = ts;
    if (*out) (*out)->t_factor = ms_since(t0) - ts;
    return st;
}

askit_status askit_factorize(askit_tree t, double lambda, int32_t precision, void *stream, askit_factor *out) {
    if (!t || !out) return fail(ASKIT_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (!t->skel_ok) return fail(ASKIT_ERR_STATE, "skeletonize the tree first");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ASKIT_ERR_ARG, "lambda must be >= 0 and finite");
    if (precision != ASKIT_FP64 && precision != ASKIT_MIXED) return fail(ASKIT_ERR_ARG, "unknown precision");
    auto t0 = std::chrono::steady_clock::now();
    askit_status st = factorize_impl(t, lambda, precision, (hipStream_t)stream, out);
    if (*out) (*out)->t_factor = ms_since(t0);
    return st;
}

askit_status askit_tune_factorization(askit_tree t, double lambda, void *stream) {
    if (!t) return fail(ASKIT_ERR_ARG, "NULL tree");
    if (!t->skel_ok) return fail(ASKIT_ERR_STATE, "skeletonize the tree first");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ASKIT_ERR_ARG, "lambda must be >= 0 and finite");
    hipStream_t st = (hipStream_t)stream;
    const int D = t->D, s = t->s;
    std::vector<int> tcs;
    for (int tc : {64, 128, 256})
        if (tc <= 2 * std::max(64, builtin_tc(s))) tcs.push_back(tc);
    const int64_t kcs[] = {2048, 4096, 8192};
    // workspace for the smallest chunk, then one factorization with the
    // built-in choices: every height's inputs (the children's Phat) are valid
    t->tune.assign(D + 1, Tune{0, 0, kcs[0]});
    std::unique_ptr<askit_factor_s> f;
    askit_status rc = factor_alloc(t, lambda, ASKIT_FP64, f);
    t->tune.clear();
    ST_TRY(rc);
    {
        Plan P;
        P.tag = "tune";
        ST_TRY(factor_plan({f.get()}, P));
        HIP_TRY(P.run(st, s));
    }
    hipEvent_t ev[2];
    HIP_TRY(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return fail(ASKIT_ERR_HIP, "hipEventCreate failed");
    }
    // kernel time of the steps of one height whose names contain `what`
    auto time_steps = [&](const Plan &P, float &kmm_ms, float &gmm_ms) -> hipError_t {
        kmm_ms = gmm_ms = 0.f;
        for (const auto &step : P.steps) {
            const bool k = step.first.find("k_kmm") != std::string::npos ||
                           step.first.find("k_reduce") != std::string::npos;
            const bool g = step.first.find("k_gmm") != std::string::npos;
            if (k || g) {
                hipError_t e = hipEventRecord(ev[0], st);
                if (e == hipSuccess) e = step.second(st, s);
                if (e == hipSuccess) e = hipEventRecord(ev[1], st);
                if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
                if (e != hipSuccess) return e;
                (k ? kmm_ms : gmm_ms) += ms;
            } else {
                hipError_t e = step.second(st, s);
                if (e != hipSuccess) return e;
            }
        }
        return hipSuccess;
    };
    std::vector<Tune> best(D + 1);
    hipError_t err = hipSuccess;
    askit_status ast = ASKIT_OK;
    for (int hgt = 1; hgt <= D && err == hipSuccess && ast == ASKIT_OK; hgt++) {
        float bk = INFINITY, bg = INFINITY;
        for (int tc : tcs)
            for (int64_t kc : kcs) {
                Tune cand{tc, tc, kc};
                Plan P;
                P.tag = "tune";
                ast = factor_plan_part({f.get()}, P, hgt, &cand);
                if (ast != ASKIT_OK) break;
                float km = 0.f, gm = 0.f, k2 = 0.f, g2 = 0.f;
                err = time_steps(P, km, gm);  // first run warms the tile configuration
                if (err == hipSuccess) err = time_steps(P, k2, g2);
                if (err != hipSuccess) break;
                if (k2 < bk) {
                    bk = k2;
                    best[hgt].kmm_tc = tc;
                    best[hgt].kmm_kc = kc;
                }
                if (g2 < bg) {
                    bg = g2;
                    best[hgt].gmm_tc = tc;
                }
            }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    ST_TRY(ast);
    HIP_TRY(err);
    HIP_TRY(hipStreamSynchronize(st));
    t->tune = best;
    return ASKIT_OK;
}

askit_status askit_tree_set_tiling(askit_tree t, const int32_t *table, int32_t heights) {
    if (!t) return fail(ASKIT_ERR_ARG, "NULL tree");
    if (heights == 0) {
        t->tune.clear();
        return ASKIT_OK;
    }
    if (!table) return fail(ASKIT_ERR_ARG, "table is NULL");
    if (heights != t->D) return fail(ASKIT_ERR_ARG, "heights must equal the tree depth " + std::to_string(t->D));
    std::vector<Tune> tn(t->D + 1);
    auto width = [](int32_t v) { return v == 64 || v == 128 || v == 256; };
    for (int h = 1; h <= t->D; h++) {
        const int32_t *e = table + 3 * (h - 1);
        if (!width(e[0]) || !width(e[2]) || !(e[1] == 2048 || e[1] == 4096 || e[1] == 8192))
            return fail(ASKIT_ERR_ARG, "height " + std::to_string(h) + ": tile widths 64, 128 or 256 and chunks of "
                                       "2048, 4096 or 8192 points");
        tn[h] = Tune{e[0], e[2], e[1]};
    }
    t->tune = tn;
    return ASKIT_OK;
}

askit_status askit_tree_set_lu_split(askit_tree t, int32_t n) {
    if (!t) return fail(ASKIT_ERR_ARG, "NULL tree");
    if (n < 0) return fail(ASKIT_ERR_ARG, "n must be >= 0");
    t->lu_split = n;
    return ASKIT_OK;
}

askit_status askit_factorize_hybrid(askit_tree t, double lambda, int32_t level, void *stream, askit_factor *out) {
    if (!out) return fail(ASKIT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!t) return fail(ASKIT_ERR_ARG, "NULL tree");
    if (!t->skel_ok) return fail(ASKIT_ERR_STATE, "skeletonize first");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ASKIT_ERR_ARG, "lambda must be finite and >= 0");
    if (level < 1 || level > t->D) return fail(ASKIT_ERR_ARG, "level must be in [1, D]");
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<askit_factor_s> f;
    ST_TRY(factor_alloc(t, lambda, ASKIT_FP64, f));
    f->hyb = level;
    f->hoff.assign((size_t)1 << level, 0);
    int64_t M = 0;
    for (int64_t id = t->first(level); id < t->first(level + 1); id++) {
        f->hoff[id - t->first(level)] = M;
        M += t->hsr[id];
    }
    f->hM = M;
    f->max_refine = 2000;
    f->refine_tol = 1e-12;
    Plan P;
    P.tag = "factor";
    ST_TRY(factor_plan({f.get()}, P));
    HIP_TRY(P.run(st, t->s));
    ST_TRY(factor_ratio(f.get(), st));
    f->t_factor = ms_since(t0);
    t->refs++;
    *out = f.release();
    return ratio_status(*out);
}

void askit_factor_destroy(askit_factor f) {
    if (!f) return;
    f->t->refs--;
    delete f;
}

askit_status askit_factor_pivot_ratio(askit_factor f, double *ratio, int32_t *node) {
    if (!f || !ratio || !node) return fail(ASKIT_ERR_ARG, "NULL argument");
    *ratio = f->min_ratio;
    *node = f->min_node;
    return ASKIT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// solves and matvec: plans per right-hand-side capacity
// ---------------------------------------------------------------------------
static askit_status ensure_cap(askit_factor f, int nrhs) {
    if (nrhs <= f->cap) return ASKIT_OK;
    askit_tree t = f->t;
    int cap = std::max(nrhs, 1);
    cap = ((cap + 15) / 16) * 16;
    const int s = t->s;
    const size_t el = f->elem();
    ST_TRY(f->W.alloc(el * t->N * cap));
    ST_TRY(f->TB.alloc(el * std::max<int64_t>(1, t->first(t->D)) * 2 * s * cap));
    ST_TRY(f->WX.alloc(sizeof(double) * t->N * cap));
    ST_TRY(f->WY.alloc(sizeof(double) * t->N * cap));
    ST_TRY(f->CB.alloc(sizeof(double) * t->nnodes * s * cap));
    // split-product partials: the larger of the solve (rows s) and transpose
    // solve (rows s) needs, in doubles
    ST_TRY(f->wsS.alloc(sizeof(double) * std::max<int64_t>(1, split_ws_elems(t, cap, kChunk))));
    f->cap = cap;
    f->solve_plan.reset();
    f->solvet_plan.reset();
    f->mv_plan[0].reset();
    f->mv_plan[1].reset();
    f->mv_plan[2].reset();
    f->hv_w.reset();
    f->hv_z.reset();
    f->hw_store.reset();
    f->hw_sub.reset();
    f->hws.release();
    return ASKIT_OK;
}

// ---------------------------------------------------------------------------
// Hybrid solver (Sec. 2.3, "Fast hybrid solver"; Alg. HybridSolve, MatVecW,
// MatVecV).  The frontier A is the level L: its nodes and their subtrees are
// skeletonized and factored as usual; above it nothing is compressed, so for
// frontier nodes a != b, Ktilde_ab = P_{a a~} K_{a~ b}.  Then lambda I +
// Ktilde = D (I + W V) with D = blockdiag(lambda I + Ktilde_aa), W =
// blockdiag(Phat_a) and V_ab = K_{a~ b} (a != b), and
//   x = v - W y,  v = D^{-1} u,  (I + V W) y = V v,
// the reduced system of order sum_a s_a solved by GMRES with V and W applied
// matrix-free (V: kernel summations from all other frontier nodes' points to
// a's skeleton, W: the stored Phat of the frontier).
// ---------------------------------------------------------------------------

// partial-sum elements of the V contractions (each frontier node's two
// ranges, split in chunks of kChunk points) for `cap` columns
static int64_t hybrid_ws_elems(askit_factor f, int cap) {
    askit_tree t = f->t;
    int64_t worst = 0;
    for (int half = 0; half < 2; half++) {
        int64_t tot = 0;
        for (int64_t id = t->first(f->hyb); id < t->first(f->hyb + 1); id++) {
            const int64_t r0 = half ? t->ne[id] : 0, r1 = half ? t->N : t->nb[id];
            const int64_t nch = cdiv(r1 - r0, kChunk);
            if (nch > 1) tot += nch * (int64_t)t->hsr[id] * cap;
        }
        worst = std::max(worst, tot);
    }
    return worst;
}

// out rows of frontier node j (= first(L) + j) += or = sum_{b != j}
// K(X_{j~}, X_b) src_b: src is N x cap row-major (tree order); out(j, r, c)
// = cptr(j)[r * crs + c * ccs].  The range [0, b_j) is stored first, then
// [e_j, N) added, in two launches (they write the same rows).
template <class CP>
static askit_status hybrid_v_commit(askit_factor f, Plan &P, const double *src, CP cptr, int64_t crs, int64_t ccs,
                                    int which, bool add_first) {
    askit_tree t = f->t;
    const int s = t->s, cap = f->cap;
    for (int half = 0; half < 2; half++) {
        KmmBuild kb;
        kb.tc = cap >= 128 ? 128 : (cap >= 64 ? 64 : 16);
        int64_t wsoff = 0;
        for (int64_t id = t->first(f->hyb); id < t->first(f->hyb + 1); id++) {
            // the first non-empty range of a node stores (unless add_first), the second adds
            const int64_t r0 = half ? t->ne[id] : 0, r1 = half ? t->N : t->nb[id];
            if (r1 <= r0) continue;
            const bool first_range = half == 0 || t->nb[id] == 0;
            KmmTask k{};
            k.X = t->Xp.as<double>();
            k.R.idx = t->skel.as<int32_t>() + id * s;
            k.R.n = t->hsr[id];
            k.S.base = r0;
            k.S.n = (int32_t)(r1 - r0);
            k.B = src + r0 * cap;
            k.ldb = cap;
            k.C = cptr(id - t->first(f->hyb));
            k.crs = crs;
            k.ccs = ccs;
            k.scale = -1.0 / (2.0 * f->h * f->h);
            k.hinv = 1.0 / f->h;
            k.which = which;
            k.op = (first_range && !add_first) ? OP_STORE : OP_ADD;
            k.rcap = t->hsr[id];
            kmm_add(kb, k, k.S.n, cap, kChunk, 8, f->hws.as<char>(), wsoff);
        }
        if (wsoff * 8 > (int64_t)f->hws.bytes) return fail(ASKIT_ERR_STATE, "internal: hybrid workspace too small");
        ST_TRY(kmm_commit(P, kb, P64, P64, t->d, s));
    }
    return ASKIT_OK;
}

// dst (N x cap row-major, tree order) op= W y: rows of frontier node b get
// Phat_b y_b, y the reduced-system vector (hM x ncol column-major)
static askit_status hybrid_w_commit(askit_factor f, Plan &P, const double *y, double *dst, int op) {
    askit_tree t = f->t;
    const int s = t->s, cap = f->cap, L = f->hyb;
    GmmBuild gb;
    gb.tc = cap >= 128 ? 128 : (cap >= 64 ? 64 : 16);
    gb.elem = 8;
    for (int64_t id = t->first(L); id < t->first(L + 1); id++) {
        GmmTask g{};
        g.A = (const double *)f->ph(L) + t->nb[id] * s;
        g.ars = s;
        g.acs = 1;
        g.B = y + f->hoff[id - t->first(L)];
        g.brs = 1;
        g.bcs = f->hM;
        g.C = dst + t->nb[id] * cap;
        g.crs = cap;
        g.ccs = 1;
        g.rows = (int32_t)(t->ne[id] - t->nb[id]);
        g.kdim = t->hsr[id];
        g.op = op;
        int64_t none = 0;
        gmm_add(gb, g, cap, 1 << 30, nullptr, none);
    }
    return gmm_commit(P, gb, P64, 0);
}

static askit_status hybrid_plans(askit_factor f) {
    const int64_t M = f->hM, cap = f->cap, N = f->t->N;
    if (f->hv_w) return ASKIT_OK;
    ST_TRY(f->hws.alloc(sizeof(double) * std::max<int64_t>(1, hybrid_ws_elems(f, (int)cap))));
    ST_TRY(f->HZ.alloc(sizeof(double) * N * cap));
    ST_TRY(f->HT.alloc(sizeof(double) * M * cap));
    double *HT = f->HT.as<double>(), *HZ = f->HZ.as<double>(), *W = f->W.as<double>();
    auto rows_of = [&](double *base) { return [=](int64_t j) { return (void *)(base + f->hoff[j]); }; };
    f->hv_w.reset(new Plan());
    f->hv_w->tag = "hybrid";
    ST_TRY(hybrid_v_commit(f, *f->hv_w, W, rows_of(HT), 1, M, 0, false));
    f->hw_sub.reset(new Plan());
    f->hw_sub->tag = "hybrid";
    ST_TRY(hybrid_w_commit(f, *f->hw_sub, HT, W, OP_SUB));
    // operator: HZ = W y (y in HT), then out = V HZ; the caller adds y
    f->hw_store.reset(new Plan());
    f->hw_store->tag = "hybrid";
    ST_TRY(hybrid_w_commit(f, *f->hw_store, HT, HZ, OP_STORE));
    f->hv_z.reset(new Plan());
    f->hv_z->tag = "hybrid";
    ST_TRY(f->HU.alloc(sizeof(double) * M * cap));
    ST_TRY(hybrid_v_commit(f, *f->hv_z, HZ, rows_of(f->HU.as<double>()), 1, M, 0, false));
    return ASKIT_OK;
}

// Solve plan (Alg. 3) for one or several factors sharing rank, dimension,
// precision and right-hand-side capacity: leaf LU solves of every tree in one
// launch, then per height the node steps of every tree.
static askit_status solve_plan(const std::vector<askit_factor> &fs, Plan &P) {
    askit_tree t0 = fs[0]->t;
    const int s = t0->s, d = t0->d, cap = fs[0]->cap, s2 = 2 * s;
    const Prec pr = fs[0]->prec;
    const int el = (int)fs[0]->elem();
    int Hmax = 0;
    for (auto f : fs) Hmax = std::max(Hmax, f->t->D);
    std::vector<LuTask> leaves;
    for (auto f : fs) {
        askit_tree t = f->t;
        char *W = f->W.as<char>();
        for (int64_t id = t->first(t->D); id < t->nnodes; id++) {
            LuTask u{};
            u.A = f->lu_of(id);
            u.piv = f->piv_of(id);
            u.dinv = f->dinv_of(id);
            u.n = (int32_t)(t->ne[id] - t->nb[id]);
            u.lda = t->mmax;
            u.B = W + t->nb[id] * cap * el;
            u.ldb = cap;
            leaves.push_back(u);
        }
    }
    ST_TRY(getrs_commit(P, leaves, pr, false, 0));
    // with a level restriction the node steps stop at the frontier (v = D^{-1} u)
    if (fs.size() == 1 && fs[0]->hyb) Hmax = fs[0]->t->D - fs[0]->hyb;
    for (int hgt = 1; hgt <= Hmax; hgt++) {
        KmmBuild kb;
        kb.tc = cap >= 128 ? 128 : (cap >= 64 ? 64 : 16);
        kb.out_size = el;
        GmmBuild gb;
        gb.tc = kb.tc;
        gb.elem = el;
        std::vector<LuTask> zs;
        for (auto f : fs) {
            askit_tree t = f->t;
            const int l = t->D - hgt;
            if (l < 0) continue;
            char *W = f->W.as<char>();
            int64_t wsoff = 0;
            for (int64_t id = t->first(l); id < t->first(l + 1); id++) {
                const int64_t lc = 2 * id + 1, rc = 2 * id + 2;
                // t = [K1 w_r; K2 w_l] (s_l + s_r rows), y = Z^{-1} t,
                // w_l -= Phat_l y_top, w_r -= Phat_r y_bot
                char *tb = f->TB.as<char>() + id * (int64_t)s2 * cap * el;
                const int sl = t->hsr[lc], n = sl + t->hsr[rc];
                for (int side = 0; side < 2; side++) {
                    const int64_t a = side ? rc : lc, o = side ? lc : rc;
                    KmmTask k{};
                    k.X = t->Xp.as<double>();
                    k.R.idx = t->skel.as<int32_t>() + a * s;
                    k.R.n = t->hsr[a];
                    k.S.base = t->nb[o];
                    k.S.n = (int32_t)(t->ne[o] - t->nb[o]);
                    k.B = W + t->nb[o] * cap * el;
                    k.ldb = cap;
                    k.C = tb + (int64_t)(side ? sl : 0) * cap * el;
                    k.crs = cap;
                    k.ccs = 1;
                    k.scale = -1.0 / (2.0 * f->h * f->h);
                    k.op = OP_STORE;
                    k.rcap = t->hsr[a];
                    kmm_add(kb, k, k.S.n, cap, kChunk, el, f->wsS.as<char>(), wsoff);
                }
                LuTask u{};
                u.A = f->lu_of(id);
                u.piv = f->piv_of(id);
                u.dinv = f->dinv_of(id);
                u.n = n;
                u.lda = n;
                u.B = tb;
                u.ldb = cap;
                zs.push_back(u);
                for (int side = 0; side < 2; side++) {
                    const int64_t ch = side ? rc : lc;
                    GmmTask g{};
                    g.A = (const char *)f->ph(l + 1) + t->nb[ch] * s * el;
                    g.ars = s;
                    g.acs = 1;
                    g.B = tb + (int64_t)(side ? sl : 0) * cap * el;
                    g.brs = cap;
                    g.bcs = 1;
                    g.C = W + t->nb[ch] * cap * el;
                    g.crs = cap;
                    g.ccs = 1;
                    g.rows = (int32_t)(t->ne[ch] - t->nb[ch]);
                    g.kdim = t->hsr[ch];
                    g.op = OP_SUB;
                    int64_t none = 0;
                    gmm_add(gb, g, cap, 1 << 30, nullptr, none);
                }
            }
        }
        ST_TRY(kmm_commit(P, kb, pr, pr, d, s));
        ST_TRY(getrs_commit(P, zs, pr, false, 0));
        ST_TRY(gmm_commit(P, gb, pr, 0));
    }
    return ASKIT_OK;
}

static askit_status solvet_plan(askit_factor f, Plan &P) {
    askit_tree t = f->t;
    const int s = t->s, D = t->D, d = t->d, cap = f->cap, s2 = 2 * s;
    const Prec pr = f->prec;
    const int el = (int)f->elem();
    char *W = f->W.as<char>();
    for (int l = 0; l < D; l++) {
        GmmBuild gb;
        gb.tc = cap >= 128 ? 128 : (cap >= 64 ? 64 : 16);
        gb.elem = el;
        KmmBuild kb;
        kb.tc = gb.tc;
        kb.out_size = el;
        std::vector<LuTask> zs;
        int64_t wsoff = 0, none = 0;
        for (int64_t id = t->first(l); id < t->first(l + 1); id++) {
            const int64_t lc = 2 * id + 1, rc = 2 * id + 2;
            char *tb = f->TB.as<char>() + id * (int64_t)s2 * cap * el;
            const int sl = t->hsr[lc], n = sl + t->hsr[rc];
            for (int side = 0; side < 2; side++) {  // gt = [Phat_l^T w_l ; Phat_r^T w_r]
                const int64_t ch = side ? rc : lc;
                GmmTask g{};
                g.A = (const char *)f->ph(l + 1) + t->nb[ch] * s * el;
                g.ars = 1;
                g.acs = s;
                g.B = W + t->nb[ch] * cap * el;
                g.brs = cap;
                g.bcs = 1;
                g.C = tb + (int64_t)(side ? sl : 0) * cap * el;
                g.crs = cap;
                g.ccs = 1;
                g.rows = t->hsr[ch];
                g.kdim = (int32_t)(t->ne[ch] - t->nb[ch]);
                g.op = OP_STORE;
                gmm_add(gb, g, cap, kChunk, f->wsS.as<char>(), wsoff);
            }
            LuTask u{};
            u.A = f->lu_of(id);
            u.piv = f->piv_of(id);
            u.dinv = f->dinv_of(id);
            u.n = n;
            u.lda = n;
            u.B = tb;
            u.ldb = cap;
            zs.push_back(u);
            for (int side = 0; side < 2; side++) {  // w_l -= K_{r~ l}^T y_bot, w_r -= K_{l~ r}^T y_top
                const int64_t ch = side ? rc : lc, a = side ? lc : rc;
                KmmTask k{};
                k.X = t->Xp.as<double>();
                k.R.base = t->nb[ch];
                k.R.n = (int32_t)(t->ne[ch] - t->nb[ch]);
                k.S.idx = t->skel.as<int32_t>() + a * s;
                k.S.n = t->hsr[a];
                k.B = tb + (int64_t)(side ? 0 : sl) * cap * el;
                k.ldb = cap;
                k.C = W + t->nb[ch] * cap * el;
                k.crs = cap;
                k.ccs = 1;
                k.scale = -1.0 / (2.0 * f->h * f->h);
                k.op = OP_SUB;
                k.rcap = k.R.n;
                kmm_add(kb, k, k.S.n, cap, 1 << 30, el, nullptr, none);
            }
        }
        ST_TRY(gmm_commit(P, gb, pr, s));
        ST_TRY(getrs_commit(P, zs, pr, true, 0));
        ST_TRY(kmm_commit(P, kb, pr, pr, d, 0));
    }
    std::vector<LuTask> leaves;
    for (int64_t id = t->first(D); id < t->nnodes; id++) {
        LuTask u{};
        u.A = f->lu_of(id);
        u.piv = f->piv_of(id);
        u.dinv = f->dinv_of(id);
        u.n = (int32_t)(t->ne[id] - t->nb[id]);
        u.lda = t->mmax;
        u.B = W + t->nb[id] * cap * el;
        u.ldb = cap;
        leaves.push_back(u);
    }
    ST_TRY(getrs_commit(P, leaves, pr, true, 0));
    return ASKIT_OK;
}

// (lambda I + Ktilde) x or dKtilde/dh x in FP64 (WX -> WY)
static askit_status matvec_t_plan(askit_factor f, Plan &P);

static askit_status matvec_plan(askit_factor f, int which, Plan &P) {
    if (which == 2) return matvec_t_plan(f, P);
    askit_tree t = f->t;
    const int s = t->s, D = t->D, d = t->d, cap = f->cap;
    double *WX = f->WX.as<double>(), *WY = f->WY.as<double>(), *CB = f->CB.as<double>();
    const double scale = -1.0 / (2.0 * f->h * f->h);
    {  // leaves: exact diagonal blocks
        KmmBuild kb;
        kb.tc = cap >= 128 ? 128 : (cap >= 64 ? 64 : 16);
        int64_t wsoff = 0;
        for (int64_t id = t->first(D); id < t->nnodes; id++) {
            KmmTask k{};
            k.X = t->Xp.as<double>();
            k.R.base = t->nb[id];
            k.R.n = (int32_t)(t->ne[id] - t->nb[id]);
            k.S = k.R;
            k.B = WX + t->nb[id] * cap;
            k.ldb = cap;
            k.C = WY + t->nb[id] * cap;
            k.crs = cap;
            k.ccs = 1;
            k.scale = scale;
            k.hinv = 1.0 / f->h;
            k.which = which;
            k.op = OP_STORE;
            k.rcap = k.R.n;
            kmm_add(kb, k, k.S.n, cap, 1 << 30, 8, nullptr, wsoff);
        }
        ST_TRY(kmm_commit(P, kb, P64, P64, d, 0));
        if (!which) {
            const double lam = f->lambda;
            const int64_t N = t->N;
            P.add("k_axpy", [=](hipStream_t st, int ncol) -> hipError_t {
                hipLaunchKernelGGL(k_axpy<double>, dim3(grid1(N * ncol)), dim3(256), 0, st, WY, WX, (int64_t)cap, N,
                                   ncol, lam);
                return hipGetLastError();
            });
        }
    }
    if (D == 0) return ASKIT_OK;
    // with a level restriction (Sec. 2.3) each frontier node a gets
    // c_a = sum_{b != a} K_{a~ b} x_b, and the nodes above add nothing
    if (f->hyb) {
        if (!f->hws.p) ST_TRY(f->hws.alloc(sizeof(double) * std::max<int64_t>(1, hybrid_ws_elems(f, cap))));
        ST_TRY(hybrid_v_commit(
            f, P, WX, [=](int64_t j) { return (void *)(CB + (t->first(f->hyb) + j) * (int64_t)s * cap); }, cap, 1,
            which, false));
    }
    // skeleton potentials c_l = K_{l~ r} x_r, c_r = K_{r~ l} x_l, one launch per level
    for (int l = f->hyb; l < D; l++) {
        KmmBuild kl;
        kl.tc = cap >= 128 ? 128 : (cap >= 64 ? 64 : 16);
        int64_t wsoff = 0;
        for (int64_t id = t->first(l); id < t->first(l + 1); id++) {
            const int64_t lc = 2 * id + 1, rc = 2 * id + 2;
            for (int side = 0; side < 2; side++) {
                const int64_t a = side ? rc : lc, o = side ? lc : rc;
                KmmTask k{};
                k.X = t->Xp.as<double>();
                k.R.idx = t->skel.as<int32_t>() + a * s;
                k.R.n = t->hsr[a];
                k.S.base = t->nb[o];
                k.S.n = (int32_t)(t->ne[o] - t->nb[o]);
                k.B = WX + t->nb[o] * cap;
                k.ldb = cap;
                k.C = CB + a * (int64_t)s * cap;
                k.crs = cap;
                k.ccs = 1;
                k.scale = scale;
                k.hinv = 1.0 / f->h;
                k.which = which;
                k.op = OP_STORE;
                k.rcap = t->hsr[a];
                kmm_add(kl, k, k.S.n, cap, kChunk, 8, f->wsS.as<char>(), wsoff);
            }
        }
        ST_TRY(kmm_commit(P, kl, P64, P64, d, s));
    }
    // push down: [c_l; c_r] += P_c c_beta, levels 1 .. D-1 in order (from
    // the frontier down with a level restriction)
    for (int l = std::max(1, f->hyb); l < D; l++) {
        GmmBuild gb;
        gb.tc = cap >= 128 ? 128 : (cap >= 64 ? 64 : 16);
        int64_t wsoff = 0;
        for (int64_t id = t->first(l); id < t->first(l + 1); id++) {
            for (int side = 0; side < 2; side++) {
                GmmTask g{};
                g.A = t->Pt.as<double>() + id * (int64_t)t->cmax * s + (int64_t)side * s * s;
                g.ars = s;
                g.acs = 1;
                g.B = CB + id * (int64_t)s * cap;
                g.brs = cap;
                g.bcs = 1;
                g.C = CB + (2 * id + 1 + side) * (int64_t)s * cap;
                g.crs = cap;
                g.ccs = 1;
                g.rows = t->hsr[2 * id + 1 + side];
                g.kdim = t->hsr[id];
                g.op = OP_ADD;
                gmm_add(gb, g, cap, 1 << 30, nullptr, wsoff);
            }
        }
        ST_TRY(gmm_commit(P, gb, P64, 0));
    }
    {  // leaves: y_a += P_{alpha alpha~} c_a
        GmmBuild gb;
        gb.tc = cap >= 128 ? 128 : (cap >= 64 ? 64 : 16);
        int64_t wsoff = 0;
        for (int64_t id = t->first(D); id < t->nnodes; id++) {
            GmmTask g{};
            g.A = t->Pt.as<double>() + id * (int64_t)t->cmax * s;
            g.ars = s;
            g.acs = 1;
            g.B = CB + id * (int64_t)s * cap;
            g.brs = cap;
            g.bcs = 1;
            g.C = WY + t->nb[id] * cap;
            g.crs = cap;
            g.ccs = 1;
            g.rows = (int32_t)(t->ne[id] - t->nb[id]);
            g.kdim = t->hsr[id];
            g.op = OP_ADD;
            gmm_add(gb, g, cap, 1 << 30, nullptr, wsoff);
        }
        ST_TRY(gmm_commit(P, gb, P64, 0));
    }
    return ASKIT_OK;
}

// (lambda I + Ktilde)^T x in FP64 (WX -> WY).  The off-diagonal block (l, r)
// of Ktilde is P_{l l~} K_{l~ r}, so its transpose K_{r l~} P_{l l~}^T acts
// through skeleton charges q_a = P_{a a~}^T x_a, gathered upward with the
// telescoped projections (q_a = P_c^T [q_l; q_r]), then evaluated at the
// sibling's points: y_r += K_{r l~} q_l, y_l += K_{l r~} q_r.
static askit_status matvec_t_plan(askit_factor f, Plan &P) {
    askit_tree t = f->t;
    const int s = t->s, D = t->D, d = t->d, cap = f->cap;
    double *WX = f->WX.as<double>(), *WY = f->WY.as<double>(), *CB = f->CB.as<double>();
    const double scale = -1.0 / (2.0 * f->h * f->h);
    const int tc = cap >= 128 ? 128 : (cap >= 64 ? 64 : 16);
    {  // leaves: symmetric diagonal blocks, plus lambda x
        KmmBuild kb;
        kb.tc = tc;
        int64_t none = 0;
        for (int64_t id = t->first(D); id < t->nnodes; id++) {
            KmmTask k{};
            k.X = t->Xp.as<double>();
            k.R.base = t->nb[id];
            k.R.n = (int32_t)(t->ne[id] - t->nb[id]);
            k.S = k.R;
            k.B = WX + t->nb[id] * cap;
            k.ldb = cap;
            k.C = WY + t->nb[id] * cap;
            k.crs = cap;
            k.ccs = 1;
            k.scale = scale;
            k.op = OP_STORE;
            k.rcap = k.R.n;
            kmm_add(kb, k, k.S.n, cap, 1 << 30, 8, nullptr, none);
        }
        ST_TRY(kmm_commit(P, kb, P64, P64, d, 0));
        const double lam = f->lambda;
        const int64_t N = t->N;
        P.add("k_axpy", [=](hipStream_t st, int ncol) -> hipError_t {
            hipLaunchKernelGGL(k_axpy<double>, dim3(grid1(N * ncol)), dim3(256), 0, st, WY, WX, (int64_t)cap, N,
                               ncol, lam);
            return hipGetLastError();
        });
    }
    if (D == 0) return ASKIT_OK;
    {  // leaf charges q_a = P_{a~ a} x_a
        GmmBuild gb;
        gb.tc = tc;
        int64_t none = 0;
        for (int64_t id = t->first(D); id < t->nnodes; id++) {
            GmmTask g{};
            g.A = t->Pt.as<double>() + id * (int64_t)t->cmax * s;
            g.ars = 1;
            g.acs = s;
            g.B = WX + t->nb[id] * cap;
            g.brs = cap;
            g.bcs = 1;
            g.C = CB + id * (int64_t)s * cap;
            g.crs = cap;
            g.ccs = 1;
            g.rows = t->hsr[id];
            g.kdim = (int32_t)(t->ne[id] - t->nb[id]);
            g.op = OP_STORE;
            gmm_add(gb, g, cap, 1 << 30, nullptr, none);
        }
        ST_TRY(gmm_commit(P, gb, P64, 0));
    }
    for (int l = D - 1; l >= 1; l--) {  // q_a = P_c^T [q_l; q_r], bottom-up
        for (int side = 0; side < 2; side++) {
            GmmBuild gb;
            gb.tc = tc;
            int64_t none = 0;
            for (int64_t id = t->first(l); id < t->first(l + 1); id++) {
                const int64_t ch = 2 * id + 1 + side;
                GmmTask g{};
                g.A = t->Pt.as<double>() + id * (int64_t)t->cmax * s + (int64_t)side * s * s;
                g.ars = 1;
                g.acs = s;
                g.B = CB + ch * (int64_t)s * cap;
                g.brs = cap;
                g.bcs = 1;
                g.C = CB + id * (int64_t)s * cap;
                g.crs = cap;
                g.ccs = 1;
                g.rows = t->hsr[id];
                g.kdim = t->hsr[ch];
                g.op = side ? OP_ADD : OP_STORE;
                gmm_add(gb, g, cap, 1 << 30, nullptr, none);
            }
            ST_TRY(gmm_commit(P, gb, P64, 0));
        }
    }
    for (int l = 0; l < D; l++) {  // y_r += K_{r l~} q_l, y_l += K_{l r~} q_r
        KmmBuild kb;
        kb.tc = tc;
        int64_t none = 0;
        for (int64_t id = t->first(l); id < t->first(l + 1); id++) {
            for (int side = 0; side < 2; side++) {
                const int64_t src = 2 * id + 1 + side, dst = 2 * id + 2 - side;
                KmmTask k{};
                k.X = t->Xp.as<double>();
                k.R.base = t->nb[dst];
                k.R.n = (int32_t)(t->ne[dst] - t->nb[dst]);
                k.S.idx = t->skel.as<int32_t>() + src * s;
                k.S.n = t->hsr[src];
                k.B = CB + src * (int64_t)s * cap;
                k.ldb = cap;
                k.C = WY + t->nb[dst] * cap;
                k.crs = cap;
                k.ccs = 1;
                k.scale = scale;
                k.op = OP_ADD;
                k.rcap = k.R.n;
                kmm_add(kb, k, k.S.n, cap, 1 << 30, 8, nullptr, none);
            }
        }
        ST_TRY(kmm_commit(P, kb, P64, P64, d, 0));
    }
    return ASKIT_OK;
}

// Arrays of right-hand sides, solutions and adjoints may live in host or
// device memory.  Host arrays (pageable or pinned) are staged through device
// buffers of the call; the call then synchronizes its stream before it
// returns.
static bool is_host_ptr(const void *p) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // unknown to the runtime: plain host memory
        return true;
    }
    return a.type == hipMemoryTypeHost || a.type == hipMemoryTypeUnregistered;
}

// runs body(B', ldb', X', ldx') with device views of two N x nrhs arrays
// (the first read, the second written unless `out2` is false)
template <class F>
static askit_status with_device_arrays(int64_t N, int nrhs, const double *B, int64_t ldb, double *X, int64_t ldx,
                                       bool out2, hipStream_t st, F &&body) {
    const bool hb = is_host_ptr(B), hx = is_host_ptr(X);
    if (!hb && !hx) return body(B, ldb, X, ldx);
    const size_t col = sizeof(double) * (size_t)N;
    DBuf db, dx;
    const double *Bd = B;
    double *Xd = X;
    int64_t lb = ldb, lx = ldx;
    if (hb) {
        ST_TRY(db.alloc(col * nrhs));
        HIP_TRY(hipMemcpy2DAsync(db.p, col, B, sizeof(double) * ldb, col, nrhs, hipMemcpyHostToDevice, st));
        Bd = db.as<double>();
        lb = N;
    }
    if (hx) {
        ST_TRY(dx.alloc(col * nrhs));
        if (!out2)
            HIP_TRY(hipMemcpy2DAsync(dx.p, col, X, sizeof(double) * ldx, col, nrhs, hipMemcpyHostToDevice, st));
        Xd = dx.as<double>();
        lx = N;
    }
    const askit_status rc = body(Bd, lb, Xd, lx);
    if (rc == ASKIT_OK && hx && out2)
        HIP_TRY(hipMemcpy2DAsync(X, sizeof(double) * ldx, Xd, col, col, nrhs, hipMemcpyDeviceToHost, st));
    // the staging buffers are released only after the queued work is done
    const hipError_t e = hipStreamSynchronize(st);
    if (rc != ASKIT_OK) return rc;
    HIP_TRY(e);
    return ASKIT_OK;
}

static askit_status check_solve_args(askit_factor f, const double *B, int64_t ldb, int32_t nrhs, double *X,
                                     int64_t ldx) {
    if (!f) return fail(ASKIT_ERR_ARG, "NULL factor");
    if (!B || !X) return fail(ASKIT_ERR_ARG, "NULL array");
    if (nrhs < 1) return fail(ASKIT_ERR_ARG, "nrhs must be >= 1");
    if (ldb < f->t->N || ldx < f->t->N) return fail(ASKIT_ERR_ARG, "leading dimension smaller than N");
    return ASKIT_OK;
}

// one application of the stored factors: X = A^{-1} B (or A^{-T} B)
static askit_status apply_inverse(askit_factor f, const double *B, int64_t ldb, int nrhs, double *X, int64_t ldx,
                                  bool trans, hipStream_t st) {
    askit_tree t = f->t;
    ST_TRY(ensure_cap(f, nrhs));
    std::unique_ptr<Plan> &pl = trans ? f->solvet_plan : f->solve_plan;
    if (!pl) {
        pl.reset(new Plan());
        pl->tag = trans ? "solve_t" : "solve";
        ST_TRY(trans ? solvet_plan(f, *pl) : solve_plan({f}, *pl));
    }
    const int64_t N = t->N;
    const dim3 tg((unsigned)cdiv(N, 64), (unsigned)cdiv(nrhs, 64));
    if (f->prec == P64)
        hipLaunchKernelGGL(k_gather_rhs_t<double>, tg, dim3(256), 0, st, B, ldb, t->iperm.as<int64_t>(), N, nrhs,
                           f->W.as<double>(), (int64_t)f->cap);
    else
        hipLaunchKernelGGL(k_gather_rhs_t<float>, tg, dim3(256), 0, st, B, ldb, t->iperm.as<int64_t>(), N, nrhs,
                           f->W.as<float>(), (int64_t)f->cap);
    HIP_TRY(hipGetLastError());
    HIP_TRY(pl->run(st, nrhs));
    if (f->prec == P64)
        hipLaunchKernelGGL(k_scatter_rhs_t<double>, tg, dim3(256), 0, st, f->W.as<double>(), (int64_t)f->cap,
                           t->iperm.as<int64_t>(), N, nrhs, X, ldx, 0);
    else
        hipLaunchKernelGGL(k_scatter_rhs_t<float>, tg, dim3(256), 0, st, f->W.as<float>(), (int64_t)f->cap,
                           t->iperm.as<int64_t>(), N, nrhs, X, ldx, 0);
    HIP_TRY(hipGetLastError());
    return ASKIT_OK;
}

static askit_status matvec_impl(askit_factor f, int which, const double *Xin, int64_t ldx, int nrhs, double *Y,
                                int64_t ldy, hipStream_t st) {
    askit_tree t = f->t;
    ST_TRY(ensure_cap(f, nrhs));
    if (!f->mv_plan[which]) {
        f->mv_plan[which].reset(new Plan());
        f->mv_plan[which]->tag = which == 1 ? "matvec_dh" : which == 2 ? "matvec_t" : "matvec";
        ST_TRY(matvec_plan(f, which, *f->mv_plan[which]));
    }
    const int64_t N = t->N;
    const dim3 tg((unsigned)cdiv(N, 64), (unsigned)cdiv(nrhs, 64));
    hipLaunchKernelGGL(k_gather_rhs_t<double>, tg, dim3(256), 0, st, Xin, ldx, t->iperm.as<int64_t>(), N, nrhs,
                       f->WX.as<double>(), (int64_t)f->cap);
    HIP_TRY(hipGetLastError());
    HIP_TRY(f->mv_plan[which]->run(st, nrhs));
    hipLaunchKernelGGL(k_scatter_rhs_t<double>, tg, dim3(256), 0, st, f->WY.as<double>(), (int64_t)f->cap,
                       t->iperm.as<int64_t>(), N, nrhs, Y, ldy, 0);
    HIP_TRY(hipGetLastError());
    return ASKIT_OK;
}

// ---------------------------------------------------------------------------
// Refinement against the FP64 operator: restarted GMRES on (lambda I +
// Ktilde) x = b, right-preconditioned with the stored factorization (GMRES-IR,
// Carson & Higham 2018).  Plain refinement x += Ahat^{-1}(b - A x) diverges
// once the factorization error times the growth of the recursion exceeds one;
// the Krylov form keeps converging as long as the preconditioned spectrum is
// clustered.  All columns iterate in lockstep; the small Hessenberg systems
// are solved on the host.
// ---------------------------------------------------------------------------
static const int kRestart = 30;

// out[j * nrhs + c] = <V_j(:, c), W(:, c)>, j < nv (device -> host)
static askit_status mdot(askit_factor f, const double *V, const double *W, int nv, int nrhs, hipStream_t st,
                         std::vector<double> &out, int64_t len = -1) {
    const int64_t N = len >= 0 ? len : f->t->N;
    const int64_t chunk = std::max<int64_t>(4096, cdiv(N, 256));
    const int nchunk = (int)cdiv(N, chunk);
    const int njc = nv * nrhs;
    if (f->kpart.bytes < sizeof(double) * ((size_t)njc * nchunk + njc)) {
        HIP_TRY(hipStreamSynchronize(st));
        ST_TRY(f->kpart.alloc(sizeof(double) * ((size_t)njc * nchunk + njc) * 2));
    }
    double *part = f->kpart.as<double>(), *res = part + (size_t)njc * nchunk;
    hipLaunchKernelGGL(k_mdot_part, dim3(njc, nchunk), dim3(256), 0, st, V, W, N, nrhs, chunk, part);
    hipLaunchKernelGGL(k_mdot_finish, dim3(grid1(njc)), dim3(256), 0, st, part, nchunk, njc, res);
    HIP_TRY(hipGetLastError());
    out.resize(njc);
    HIP_TRY(hipMemcpyAsync(out.data(), res, sizeof(double) * njc, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return ASKIT_OK;
}

static askit_status put_small(askit_factor f, const std::vector<double> &v, hipStream_t st) {
    if (f->ksmall.bytes < sizeof(double) * v.size()) {
        HIP_TRY(hipStreamSynchronize(st));
        ST_TRY(f->ksmall.alloc(sizeof(double) * v.size() * 2));
    }
    HIP_TRY(hipMemcpyAsync(f->ksmall.p, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice, st));
    return ASKIT_OK;
}

static askit_status gmres_refine(askit_factor f, const double *B, int64_t ldb, int nrhs, double *X, int64_t ldx,
                                 bool trans, hipStream_t st) {
    const int op = trans ? 2 : 0;  // operator: A or A^T
    const int64_t N = f->t->N, NR = N * (int64_t)nrhs;
    const int m = kRestart;
    const size_t need = sizeof(double) * (size_t)NR;
    if (f->Vk.bytes < need * (m + 1) || f->R.bytes < need || f->Dx.bytes < need) {
        HIP_TRY(hipStreamSynchronize(st));
        ST_TRY(f->Vk.alloc(need * (m + 1)));
        ST_TRY(f->R.alloc(need));
        ST_TRY(f->Dx.alloc(need));
    }
    double *V = f->Vk.as<double>(), *R = f->R.as<double>(), *Z = f->Dx.as<double>();
    // |b| per column
    HIP_TRY(hipMemcpy2DAsync(R, sizeof(double) * N, B, sizeof(double) * ldb, sizeof(double) * N, nrhs,
                             hipMemcpyDeviceToDevice, st));
    std::vector<double> bn, h1, h2, hn;
    ST_TRY(mdot(f, R, R, 1, nrhs, st, bn));
    for (auto &v : bn) v = v > 0 ? std::sqrt(v) : 1.0;
    // x0 = Ahat^{-1} b  (B may alias X: it is not read again after the copy in R
    // ... except for the residuals, so keep b in the last Krylov slot)
    double *Bc = V + (size_t)m * NR;
    HIP_TRY(hipMemcpyAsync(Bc, R, need, hipMemcpyDeviceToDevice, st));
    ST_TRY(apply_inverse(f, B, ldb, nrhs, X, ldx, trans, st));
    int it = 0;
    double res = INFINITY, res0 = -1.0, prev = INFINITY;
    std::vector<double> H((size_t)nrhs * (m + 1) * m), g((size_t)nrhs * (m + 1)), cs((size_t)nrhs * m),
        sn((size_t)nrhs * m), sc(nrhs), y;
    while (true) {
        // r = b - A x
        ST_TRY(matvec_impl(f, op, X, ldx, nrhs, R, N, st));
        hipLaunchKernelGGL(k_sub_from, dim3(grid1(NR)), dim3(256), 0, st, Bc, N, R, N, nrhs);
        HIP_TRY(hipGetLastError());
        std::vector<double> rn;
        ST_TRY(mdot(f, R, R, 1, nrhs, st, rn));
        res = 0.0;
        for (int c = 0; c < nrhs; c++) {
            rn[c] = std::sqrt(std::max(rn[c], 0.0));
            const double rc = rn[c] / bn[c];
            if (!(rc <= res)) res = rc;  // a NaN residual propagates (and never converges)
        }
        if (std::isnan(res)) break;
        if (res0 < 0) res0 = res;
        if (res <= f->refine_tol || it >= f->max_refine) break;
        // stagnation: a restart cycle that did not halve the true residual
        // ends the refinement (rounding floor reached, or a preconditioner
        // too far from the operator)
        if (res > 0.5 * prev) break;
        prev = res;
        // Arnoldi with the last Krylov slot kept for b: at most m - 1 steps
        const int mm = m - 1;
        for (int c = 0; c < nrhs; c++) sc[c] = rn[c] > 0 ? 1.0 / rn[c] : 0.0;
        ST_TRY(put_small(f, sc, st));
        hipLaunchKernelGGL(k_scale_cols, dim3(grid1(NR)), dim3(256), 0, st, V, R, f->ksmall.as<double>(), N, nrhs);
        std::fill(g.begin(), g.end(), 0.0);
        for (int c = 0; c < nrhs; c++) g[(size_t)c * (m + 1)] = rn[c];
        int used = 0;
        std::vector<double> est;  // estimated residual after each Arnoldi step
        for (int j = 0; j < mm && it < f->max_refine; j++) {
            double *Vj = V + (size_t)j * NR, *W = R;
            ST_TRY(apply_inverse(f, Vj, N, nrhs, Z, N, trans, st));
            ST_TRY(matvec_impl(f, op, Z, N, nrhs, W, N, st));
            // classical Gram-Schmidt, twice
            ST_TRY(mdot(f, V, W, j + 1, nrhs, st, h1));
            ST_TRY(put_small(f, h1, st));
            hipLaunchKernelGGL(k_maxpy, dim3(grid1(NR)), dim3(256), 0, st, W, V, f->ksmall.as<double>(), j + 1, N, nrhs);
            ST_TRY(mdot(f, V, W, j + 1, nrhs, st, h2));
            ST_TRY(put_small(f, h2, st));
            hipLaunchKernelGGL(k_maxpy, dim3(grid1(NR)), dim3(256), 0, st, W, V, f->ksmall.as<double>(), j + 1, N, nrhs);
            ST_TRY(mdot(f, W, W, 1, nrhs, st, hn));
            for (int c = 0; c < nrhs; c++) {
                hn[c] = std::sqrt(std::max(hn[c], 0.0));
                sc[c] = hn[c] > 0 ? 1.0 / hn[c] : 0.0;
            }
            ST_TRY(put_small(f, sc, st));
            hipLaunchKernelGGL(k_scale_cols, dim3(grid1(NR)), dim3(256), 0, st, V + (size_t)(j + 1) * NR, W,
                               f->ksmall.as<double>(), N, nrhs);
            HIP_TRY(hipGetLastError());
            it++;
            used = j + 1;
            double worst = 0.0;
            for (int c = 0; c < nrhs; c++) {
                double *Hc = H.data() + (size_t)c * (m + 1) * m, *gc = g.data() + (size_t)c * (m + 1);
                double *csc = cs.data() + (size_t)c * m, *snc = sn.data() + (size_t)c * m;
                auto Hat = [&](int r, int k) -> double & { return Hc[(size_t)r * m + k]; };
                for (int r = 0; r <= j; r++) Hat(r, j) = h1[(size_t)r * nrhs + c] + h2[(size_t)r * nrhs + c];
                Hat(j + 1, j) = hn[c];
                for (int r = 0; r < j; r++) {
                    double a = Hat(r, j), b = Hat(r + 1, j);
                    Hat(r, j) = csc[r] * a + snc[r] * b;
                    Hat(r + 1, j) = -snc[r] * a + csc[r] * b;
                }
                double a = Hat(j, j), b = Hat(j + 1, j), rr = std::hypot(a, b);
                csc[j] = rr > 0 ? a / rr : 1.0;
                snc[j] = rr > 0 ? b / rr : 0.0;
                Hat(j, j) = rr;
                Hat(j + 1, j) = 0.0;
                gc[j + 1] = -snc[j] * gc[j];
                gc[j] = csc[j] * gc[j];
                worst = std::max(worst, std::fabs(gc[j + 1]) / bn[c]);
            }
            if (worst <= 0.5 * f->refine_tol) break;
            // the cycle stalls when four steps gain less than 5%
            est.push_back(worst);
            if (est.size() >= 5 && worst > 0.95 * est[est.size() - 5]) break;
        }
        if (used == 0) break;
        // x += Ahat^{-1} V y
        y.assign((size_t)used * nrhs, 0.0);
        for (int c = 0; c < nrhs; c++) {
            double *Hc = H.data() + (size_t)c * (m + 1) * m, *gc = g.data() + (size_t)c * (m + 1);
            for (int r = used - 1; r >= 0; r--) {
                double acc = gc[r];
                for (int k = r + 1; k < used; k++) acc -= Hc[(size_t)r * m + k] * y[(size_t)k * nrhs + c];
                double d = Hc[(size_t)r * m + r];
                y[(size_t)r * nrhs + c] = d != 0.0 ? acc / d : 0.0;
            }
        }
        ST_TRY(put_small(f, y, st));
        hipLaunchKernelGGL(k_lincomb, dim3(grid1(NR)), dim3(256), 0, st, R, V, f->ksmall.as<double>(), used, N, nrhs);
        HIP_TRY(hipGetLastError());
        ST_TRY(apply_inverse(f, R, N, nrhs, Z, N, trans, st));
        hipLaunchKernelGGL(k_update, dim3(grid1(NR)), dim3(256), 0, st, X, ldx, Z, N, N, nrhs);
        HIP_TRY(hipGetLastError());
    }
    f->info.iterations = it;
    f->info.converged = res <= f->refine_tol;
    f->info.initial_residual = res0;
    f->info.residual = res;
    HIP_TRY(hipStreamSynchronize(st));
    return ASKIT_OK;
}


// HybridSolve (Alg. HybridSolve): v = D^{-1} u by the node steps up to the
// frontier; t = V v (MatVecV); (I + V W) y = t by GMRES (classical
// Gram-Schmidt, twice; x0 = 0; the small Hessenberg systems on the host);
// x = v - W y (MatVecW).  Reduced-system vectors are hM x nrhs column-major.
static askit_status hybrid_solve(askit_factor f, const double *B, int64_t ldb, int nrhs, double *X, int64_t ldx,
                                 hipStream_t st) {
    askit_tree t = f->t;
    ST_TRY(ensure_cap(f, nrhs));
    if (!f->solve_plan) {
        f->solve_plan.reset(new Plan());
        f->solve_plan->tag = "solve";
        ST_TRY(solve_plan({f}, *f->solve_plan));
    }
    ST_TRY(hybrid_plans(f));
    const int64_t N = t->N, M = f->hM, MR = M * (int64_t)nrhs;
    // restart length: the whole reduced system when its order is at most
    // 1024 (GMRES then needs no restart), else 1024 basis vectors
    const int m = (int)std::max<int64_t>(1, std::min<int64_t>(M, 1024));
    const dim3 tg((unsigned)cdiv(N, 64), (unsigned)cdiv(nrhs, 64));
    hipLaunchKernelGGL(k_gather_rhs_t<double>, tg, dim3(256), 0, st, B, ldb, t->iperm.as<int64_t>(), N, nrhs,
                       f->W.as<double>(), (int64_t)f->cap);
    HIP_TRY(hipGetLastError());
    HIP_TRY(f->solve_plan->run(st, nrhs));  // W = v = D^{-1} u
    HIP_TRY(f->hv_w->run(st, nrhs));        // HT = t = V v
    // Krylov basis V_0 .. V_m, then t, y and a work vector: m + 4 slots
    if (f->HK.bytes < sizeof(double) * (size_t)MR * (m + 4)) {
        HIP_TRY(hipStreamSynchronize(st));
        ST_TRY(f->HK.alloc(sizeof(double) * (size_t)MR * (m + 4)));
    }
    double *V = f->HK.as<double>(), *Bt = V + (size_t)(m + 1) * MR, *Y = Bt + MR, *R = Y + MR;
    double *HT = f->HT.as<double>(), *HU = f->HU.as<double>();
    HIP_TRY(hipMemcpyAsync(Bt, HT, sizeof(double) * MR, hipMemcpyDeviceToDevice, st));

    hipLaunchKernelGGL(k_zero, dim3(grid1(MR)), dim3(256), 0, st, Y, MR);
    HIP_TRY(hipGetLastError());
    // out = (I + V W) in, in and out M x nrhs (out may be HU itself)
    auto apply = [&](const double *in, double *outp) -> askit_status {
        HIP_TRY(hipMemcpyAsync(HT, in, sizeof(double) * MR, hipMemcpyDeviceToDevice, st));
        HIP_TRY(f->hw_store->run(st, nrhs));
        HIP_TRY(f->hv_z->run(st, nrhs));
        hipLaunchKernelGGL(k_update, dim3(grid1(MR)), dim3(256), 0, st, HU, M, HT, M, M, nrhs);
        HIP_TRY(hipGetLastError());
        if (outp != HU) HIP_TRY(hipMemcpyAsync(outp, HU, sizeof(double) * MR, hipMemcpyDeviceToDevice, st));
        return ASKIT_OK;
    };
    std::vector<double> bn, rn, h1, h2, hn, y;
    ST_TRY(mdot(f, Bt, Bt, 1, nrhs, st, bn, M));
    for (auto &v : bn) v = v > 0 ? std::sqrt(v) : 1.0;
    std::vector<double> H((size_t)nrhs * (m + 1) * m), g((size_t)nrhs * (m + 1)), cs((size_t)nrhs * m),
        sn((size_t)nrhs * m), sc(nrhs);
    int it = 0;
    double res = INFINITY, res0 = -1.0, prev = INFINITY;
    bool first = true;
    while (true) {
        // r = t - (I + V W) y
        if (first) {
            HIP_TRY(hipMemcpyAsync(R, Bt, sizeof(double) * MR, hipMemcpyDeviceToDevice, st));
        } else {
            ST_TRY(apply(Y, R));
            hipLaunchKernelGGL(k_sub_from, dim3(grid1(MR)), dim3(256), 0, st, Bt, M, R, M, nrhs);
            HIP_TRY(hipGetLastError());
        }
        first = false;
        ST_TRY(mdot(f, R, R, 1, nrhs, st, rn, M));
        res = 0.0;
        for (int c = 0; c < nrhs; c++) {
            rn[c] = std::sqrt(std::max(rn[c], 0.0));
            const double rc = rn[c] / bn[c];
            if (!(rc <= res)) res = rc;  // a NaN residual propagates (and never converges)
        }
        if (std::isnan(res)) break;
        if (res0 < 0) res0 = res;
        if (res <= f->refine_tol || it >= f->max_refine) break;
        if (res > 0.99 * prev) break;  // a whole restart cycle gained less than 1%
        prev = res;
        for (int c = 0; c < nrhs; c++) sc[c] = rn[c] > 0 ? 1.0 / rn[c] : 0.0;
        ST_TRY(put_small(f, sc, st));
        hipLaunchKernelGGL(k_scale_cols, dim3(grid1(MR)), dim3(256), 0, st, V, R, f->ksmall.as<double>(), M, nrhs);
        std::fill(g.begin(), g.end(), 0.0);
        for (int c = 0; c < nrhs; c++) g[(size_t)c * (m + 1)] = rn[c];
        int used = 0;
        for (int j = 0; j < m && it < f->max_refine; j++) {
            double *Vj = V + (size_t)j * MR, *Wv = R;
            ST_TRY(apply(Vj, Wv));
            ST_TRY(mdot(f, V, Wv, j + 1, nrhs, st, h1, M));
            ST_TRY(put_small(f, h1, st));
            hipLaunchKernelGGL(k_maxpy, dim3(grid1(MR)), dim3(256), 0, st, Wv, V, f->ksmall.as<double>(), j + 1, M,
                               nrhs);
            ST_TRY(mdot(f, V, Wv, j + 1, nrhs, st, h2, M));
            ST_TRY(put_small(f, h2, st));
            hipLaunchKernelGGL(k_maxpy, dim3(grid1(MR)), dim3(256), 0, st, Wv, V, f->ksmall.as<double>(), j + 1, M,
                               nrhs);
            ST_TRY(mdot(f, Wv, Wv, 1, nrhs, st, hn, M));
            for (int c = 0; c < nrhs; c++) {
                hn[c] = std::sqrt(std::max(hn[c], 0.0));
                sc[c] = hn[c] > 0 ? 1.0 / hn[c] : 0.0;
            }
            ST_TRY(put_small(f, sc, st));
            hipLaunchKernelGGL(k_scale_cols, dim3(grid1(MR)), dim3(256), 0, st, V + (size_t)(j + 1) * MR, Wv,
                               f->ksmall.as<double>(), M, nrhs);
            HIP_TRY(hipGetLastError());
            it++;
            used = j + 1;
            double worst = 0.0;
            for (int c = 0; c < nrhs; c++) {
                double *Hc = H.data() + (size_t)c * (m + 1) * m, *gc = g.data() + (size_t)c * (m + 1);
                double *csc = cs.data() + (size_t)c * m, *snc = sn.data() + (size_t)c * m;
                auto Hat = [&](int r, int k) -> double & { return Hc[(size_t)r * m + k]; };
                for (int r = 0; r <= j; r++) Hat(r, j) = h1[(size_t)r * nrhs + c] + h2[(size_t)r * nrhs + c];
                Hat(j + 1, j) = hn[c];
                for (int r = 0; r < j; r++) {
                    double a = Hat(r, j), b = Hat(r + 1, j);
                    Hat(r, j) = csc[r] * a + snc[r] * b;
                    Hat(r + 1, j) = -snc[r] * a + csc[r] * b;
                }
                double a = Hat(j, j), b = Hat(j + 1, j), rr = std::hypot(a, b);
                csc[j] = rr > 0 ? a / rr : 1.0;
                snc[j] = rr > 0 ? b / rr : 0.0;
                Hat(j, j) = rr;
                Hat(j + 1, j) = 0.0;
                gc[j + 1] = -snc[j] * gc[j];
                gc[j] = csc[j] * gc[j];
                worst = std::max(worst, std::fabs(gc[j + 1]) / bn[c]);
            }
            if (worst <= 0.5 * f->refine_tol) break;
        }
        if (used == 0) break;
        // y += V z, z from the triangular Hessenberg system
        y.assign((size_t)used * nrhs, 0.0);
        for (int c = 0; c < nrhs; c++) {
            double *Hc = H.data() + (size_t)c * (m + 1) * m, *gc = g.data() + (size_t)c * (m + 1);
            for (int r = used - 1; r >= 0; r--) {
                double acc = gc[r];
                for (int k = r + 1; k < used; k++) acc -= Hc[(size_t)r * m + k] * y[(size_t)k * nrhs + c];
                double d = Hc[(size_t)r * m + r];
                y[(size_t)r * nrhs + c] = d != 0.0 ? acc / d : 0.0;
            }
        }
        ST_TRY(put_small(f, y, st));
        hipLaunchKernelGGL(k_lincomb, dim3(grid1(MR)), dim3(256), 0, st, R, V, f->ksmall.as<double>(), used, M, nrhs);
        hipLaunchKernelGGL(k_update, dim3(grid1(MR)), dim3(256), 0, st, Y, M, R, M, M, nrhs);
        HIP_TRY(hipGetLastError());
    }
    // x = v - W y
    HIP_TRY(hipMemcpyAsync(HT, Y, sizeof(double) * MR, hipMemcpyDeviceToDevice, st));
    HIP_TRY(f->hw_sub->run(st, nrhs));
    hipLaunchKernelGGL(k_scatter_rhs_t<double>, tg, dim3(256), 0, st, f->W.as<double>(), (int64_t)f->cap,
                       t->iperm.as<int64_t>(), N, nrhs, X, ldx, 0);
    HIP_TRY(hipGetLastError());
    f->info.iterations = it;
    f->info.converged = res <= f->refine_tol;
    f->info.initial_residual = res0;
    f->info.residual = res;
    HIP_TRY(hipStreamSynchronize(st));
    return ASKIT_OK;
}

extern "C" {

askit_status askit_solve(askit_factor f, const double *B, int64_t ldb, int32_t nrhs, double *X, int64_t ldx,
                         void *stream) {
    ST_TRY(check_solve_args(f, B, ldb, nrhs, X, ldx));
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    f->info = askit_solve_info{};
    ST_TRY(with_device_arrays(f->t->N, nrhs, B, ldb, X, ldx, true, st,
                              [&](const double *Bd, int64_t lb, double *Xd, int64_t lx) {
                                  if (f->hyb) return hybrid_solve(f, Bd, lb, nrhs, Xd, lx, st);
                                  if (f->max_refine == 0) return apply_inverse(f, Bd, lb, nrhs, Xd, lx, false, st);
                                  return gmres_refine(f, Bd, lb, nrhs, Xd, lx, false, st);
                              }));
    f->t_solve = ms_since(t0);
    return ASKIT_OK;
}

askit_status askit_solve_transpose(askit_factor f, const double *B, int64_t ldb, int32_t nrhs, double *X,
                                   int64_t ldx, void *stream) {
    ST_TRY(check_solve_args(f, B, ldb, nrhs, X, ldx));
    if (f->hyb) return fail(ASKIT_ERR_STATE, "no transpose solve for a level-restricted (hybrid) factor");
    hipStream_t st = (hipStream_t)stream;
    f->info = askit_solve_info{};
    return with_device_arrays(f->t->N, nrhs, B, ldb, X, ldx, true, st,
                              [&](const double *Bd, int64_t lb, double *Xd, int64_t lx) {
                                  if (f->max_refine == 0) return apply_inverse(f, Bd, lb, nrhs, Xd, lx, true, st);
                                  return gmres_refine(f, Bd, lb, nrhs, Xd, lx, true, st);
                              });
}

askit_status askit_matvec(askit_factor f, int32_t which, const double *Xin, int64_t ldx, int32_t nrhs, double *Y,
                          int64_t ldy, void *stream) {
    ST_TRY(check_solve_args(f, Xin, ldx, nrhs, Y, ldy));
    if (which < 0 || which > 2) return fail(ASKIT_ERR_ARG, "which must be 0, 1 or 2");
    if (which == 2 && f->hyb) return fail(ASKIT_ERR_STATE, "no transposed matvec for a level-restricted (hybrid) factor");
    hipStream_t st = (hipStream_t)stream;
    return with_device_arrays(f->t->N, nrhs, Xin, ldx, Y, ldy, true, st,
                              [&](const double *Xd, int64_t lxd, double *Yd, int64_t lyd) {
                                  return matvec_impl(f, which, Xd, lxd, nrhs, Yd, lyd, st);
                              });
}

askit_status askit_set_refinement(askit_factor f, int32_t max_refine, double refine_tol) {
    if (!f || max_refine < 0 || !(refine_tol > 0.0)) return fail(ASKIT_ERR_ARG, "bad refinement controls");
    f->max_refine = max_refine;
    f->refine_tol = refine_tol;
    return ASKIT_OK;
}

askit_status askit_last_solve_info(askit_factor f, askit_solve_info *info) {
    if (!f || !info) return fail(ASKIT_ERR_ARG, "NULL argument");
    *info = f->info;
    return ASKIT_OK;
}

askit_status askit_tree_set_bandwidth(askit_tree t, double h) {
    if (!t) return fail(ASKIT_ERR_ARG, "NULL tree");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(ASKIT_ERR_ARG, "h must be positive and finite");
    t->hfac = h;
    return ASKIT_OK;
}

static askit_status adjoint_impl(askit_factor f, const double *Xs, int64_t ldx, const double *Zs, int64_t ldz,
                                 int32_t nrhs, double *dlambda, double *dh, hipStream_t st);

askit_status askit_adjoint_scalars(askit_factor f, const double *Xs, const double *Zs, int64_t ld, int32_t nrhs,
                                   double *dlambda, double *dh, void *stream) {
    ST_TRY(check_solve_args(f, Xs, ld, nrhs, (double *)Zs, ld));
    if (!dlambda || !dh) return fail(ASKIT_ERR_ARG, "NULL output");
    hipStream_t st = (hipStream_t)stream;
    // X and Z are both inputs here
    return with_device_arrays(f->t->N, nrhs, Xs, ld, (double *)Zs, ld, false, st,
                              [&](const double *Xd, int64_t lxd, double *Zd, int64_t lzd) {
                                  return adjoint_impl(f, Xd, lxd, Zd, lzd, nrhs, dlambda, dh, st);
                              });
}

static askit_status adjoint_impl(askit_factor f, const double *Xs, int64_t ldx, const double *Zs, int64_t ldz,
                                 int32_t nrhs, double *dlambda, double *dh, hipStream_t st) {
    const int64_t N = f->t->N, NR = N * (int64_t)nrhs;
    if (f->R.bytes < sizeof(double) * NR || f->Dx.bytes < sizeof(double) * NR) {
        HIP_TRY(hipStreamSynchronize(st));
        ST_TRY(f->R.alloc(sizeof(double) * NR));
        ST_TRY(f->Dx.alloc(sizeof(double) * NR));
    }
    double *Xc = f->Dx.as<double>(), *Y = f->R.as<double>();
    HIP_TRY(hipMemcpy2DAsync(Xc, sizeof(double) * N, Xs, sizeof(double) * ldx, sizeof(double) * N, nrhs,
                             hipMemcpyDeviceToDevice, st));
    ST_TRY(matvec_impl(f, 1, Xc, N, nrhs, Y, N, st));
    // Zs may have a leading dimension above N: the dots read it through a
    // compact copy in the first Krylov slot
    if (f->Vk.bytes < sizeof(double) * NR) {
        HIP_TRY(hipStreamSynchronize(st));
        ST_TRY(f->Vk.alloc(sizeof(double) * NR));
    }
    double *Zc = f->Vk.as<double>();
    HIP_TRY(hipMemcpy2DAsync(Zc, sizeof(double) * N, Zs, sizeof(double) * ldz, sizeof(double) * N, nrhs,
                             hipMemcpyDeviceToDevice, st));
    std::vector<double> zx, zy;
    ST_TRY(mdot(f, Zc, Xc, 1, nrhs, st, zx));
    ST_TRY(mdot(f, Zc, Y, 1, nrhs, st, zy));
    double a = 0.0, b = 0.0;
    for (int c = 0; c < nrhs; c++) {
        a += zx[c];
        b += zy[c];
    }
    *dlambda = -a;
    *dh = -b;
    return ASKIT_OK;
}

// ---------------------------------------------------------------------------
// batches of independent problems: one launch per kernel and tree height for
// all problems, the factorization and the solve each captured in a hipGraph
// ---------------------------------------------------------------------------
}  // extern "C"

struct askit_batch_s {
    std::vector<askit_factor> fs;
    int nrhs = 0;
    Plan fplan, splan;
    hipGraphExec_t fexec = nullptr, sexec = nullptr;
    hipGraph_t fgraph = nullptr, sgraph = nullptr;
    DBuf ptrs, gtasks;
    ~askit_batch_s() {
        if (fexec) (void)hipGraphExecDestroy(fexec);
        if (sexec) (void)hipGraphExecDestroy(sexec);
        if (fgraph) (void)hipGraphDestroy(fgraph);
        if (sgraph) (void)hipGraphDestroy(sgraph);
        for (auto f : fs) askit_factor_destroy(f);
    }
};

// record a plan into a graph on a private capture stream
static askit_status capture(const Plan &P, int ncol, hipGraph_t *g, hipGraphExec_t *ex,
                            const std::function<hipError_t(hipStream_t)> &pre = nullptr,
                            const std::function<hipError_t(hipStream_t)> &post = nullptr) {
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const bool prof = g_prof.on;
    g_prof.on = false;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess && pre) e = pre(cs);
    if (e == hipSuccess) e = P.run(cs, ncol);
    if (e == hipSuccess && post) e = post(cs);
    hipError_t e2 = hipStreamEndCapture(cs, g);
    g_prof.on = prof;
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(ex, *g, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    HIP_TRY(e);
    return ASKIT_OK;
}

extern "C" {

askit_status askit_skeletonize_batched(askit_tree *trees, int32_t count, void *stream) {
    if (!trees || count < 1) return fail(ASKIT_ERR_ARG, "no trees");
    for (int i = 0; i < count; i++) {
        if (!trees[i]) return fail(ASKIT_ERR_ARG, "NULL tree");
        if (trees[i]->refs) return fail(ASKIT_ERR_STATE, "destroy the factors of the trees first");
        if (trees[i]->nsamp != trees[0]->nsamp || trees[i]->s != trees[0]->s || trees[i]->d != trees[0]->d)
            return fail(ASKIT_ERR_ARG, "batched trees must share rank, sample count and dimension");
    }
    auto t0 = std::chrono::steady_clock::now();
    ST_TRY(skeletonize_impl(trees, count, (hipStream_t)stream));
    double ms = ms_since(t0);
    for (int i = 0; i < count; i++) trees[i]->t_skel = ms;
    return ASKIT_OK;
}

askit_status askit_batch_create(askit_tree *trees, int32_t count, const double *lambdas, int32_t precision,
                                int32_t nrhs, askit_batch *out) {
    if (!out) return fail(ASKIT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!trees || !lambdas || count < 1 || nrhs < 1) return fail(ASKIT_ERR_ARG, "bad batch arguments");
    if (precision != ASKIT_FP64 && precision != ASKIT_MIXED) return fail(ASKIT_ERR_ARG, "unknown precision");
    for (int i = 0; i < count; i++) {
        if (!trees[i] || !trees[i]->skel_ok) return fail(ASKIT_ERR_STATE, "every tree must be skeletonized");
        if (trees[i]->s != trees[0]->s || trees[i]->d != trees[0]->d)
            return fail(ASKIT_ERR_ARG, "batched trees must share rank and dimension");
        if (!(lambdas[i] >= 0.0) || !std::isfinite(lambdas[i])) return fail(ASKIT_ERR_ARG, "bad lambda");
    }
    std::unique_ptr<askit_batch_s> b(new askit_batch_s());
    b->nrhs = nrhs;
    for (int i = 0; i < count; i++) {
        std::unique_ptr<askit_factor_s> f;
        ST_TRY(factor_alloc(trees[i], lambdas[i], precision, f));
        trees[i]->refs++;
        b->fs.push_back(f.release());
        ST_TRY(ensure_cap(b->fs.back(), nrhs));
    }
    b->fplan.tag = "batch_factor";
    ST_TRY(factor_plan(b->fs, b->fplan));
    b->splan.tag = "batch_solve";
    ST_TRY(solve_plan(b->fs, b->splan));
    // gather / scatter descriptors: one per problem; user pointers come from a
    // device table (B[0..count), X[0..count)) refreshed by every solve call
    std::vector<GatherTask> gt;
    int64_t nmax = 0;
    for (auto f : b->fs) {
        GatherTask g{};
        g.perm = f->t->perm.as<int64_t>();
        g.N = f->t->N;
        g.W = f->W.p;
        g.ldw = f->cap;
        gt.push_back(g);
        nmax = std::max(nmax, f->t->N);
    }
    ST_TRY(upload(b->gtasks, gt));
    ST_TRY(b->ptrs.alloc(sizeof(double *) * 2 * count));
    const GatherTask *gp = b->gtasks.as<GatherTask>();
    const double *const *pB = b->ptrs.as<const double *>();
    double *const *pX = b->ptrs.as<double *>() + count;
    const Prec pr = b->fs[0]->prec;
    const int bpt = (int)cdiv(nmax * nrhs, 256);
    auto gather = [=](hipStream_t st) -> hipError_t {
        if (pr == P64) hipLaunchKernelGGL(k_gather_multi<double>, dim3(count * bpt), dim3(256), 0, st, gp, pB, nrhs, bpt);
        else hipLaunchKernelGGL(k_gather_multi<float>, dim3(count * bpt), dim3(256), 0, st, gp, pB, nrhs, bpt);
        return hipGetLastError();
    };
    auto scatter = [=](hipStream_t st) -> hipError_t {
        if (pr == P64) hipLaunchKernelGGL(k_scatter_multi<double>, dim3(count * bpt), dim3(256), 0, st, gp, pX, nrhs, bpt);
        else hipLaunchKernelGGL(k_scatter_multi<float>, dim3(count * bpt), dim3(256), 0, st, gp, pX, nrhs, bpt);
        return hipGetLastError();
    };
    ST_TRY(capture(b->fplan, trees[0]->s, &b->fgraph, &b->fexec));
    ST_TRY(capture(b->splan, nrhs, &b->sgraph, &b->sexec, gather, scatter));
    *out = b.release();
    return ASKIT_OK;
}

askit_status askit_batch_factorize(askit_batch b, void *stream) {
    if (!b) return fail(ASKIT_ERR_ARG, "NULL batch");
    HIP_TRY(hipGraphLaunch(b->fexec, (hipStream_t)stream));
    return ASKIT_OK;
}

askit_status askit_factorize_batched(askit_tree *trees, int32_t count, const double *lambdas, int32_t precision,
                                     int32_t nrhs, void *stream, askit_batch *out) {
    ST_TRY(askit_batch_create(trees, count, lambdas, precision, nrhs, out));
    const askit_status rc = askit_batch_factorize(*out, stream);
    if (rc != ASKIT_OK) {
        askit_batch_destroy(*out);
        *out = nullptr;
    }
    return rc;
}

askit_status askit_batch_check(askit_batch b, double *min_ratio, int32_t *problem, void *stream) {
    if (!b || !min_ratio || !problem) return fail(ASKIT_ERR_ARG, "NULL argument");
    *min_ratio = 1.0;
    *problem = -1;
    for (size_t i = 0; i < b->fs.size(); i++) {
        ST_TRY(factor_ratio(b->fs[i], (hipStream_t)stream));
        if (b->fs[i]->min_ratio < *min_ratio) {
            *min_ratio = b->fs[i]->min_ratio;
            *problem = (int32_t)i;
        }
    }
    return ASKIT_OK;
}

askit_status askit_batch_solve(askit_batch b, const double *const *B, double *const *X, void *stream) {
    if (!b || !B || !X) return fail(ASKIT_ERR_ARG, "NULL argument");
    const int count = (int)b->fs.size();
    std::vector<const void *> tab(2 * count);
    for (int i = 0; i < count; i++) {
        if (!B[i] || !X[i]) return fail(ASKIT_ERR_ARG, "NULL right-hand side");
        tab[i] = B[i];
        tab[count + i] = X[i];
    }
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(b->ptrs.p, tab.data(), sizeof(void *) * 2 * count, hipMemcpyHostToDevice, st));
    HIP_TRY(hipGraphLaunch(b->sexec, st));
    HIP_TRY(hipStreamSynchronize(st));  // the pointer table is host memory of this call
    return ASKIT_OK;
}

askit_status askit_batch_factor(askit_batch b, int32_t i, askit_factor *f) {
    if (!b || !f || i < 0 || i >= (int32_t)b->fs.size()) return fail(ASKIT_ERR_ARG, "bad batch index");
    *f = b->fs[i];
    return ASKIT_OK;
}

void askit_batch_destroy(askit_batch b) { delete b; }

askit_status askit_get_stats(askit_tree t, askit_factor f, char *json, size_t cap) {
    if (!json || cap == 0) return fail(ASKIT_ERR_ARG, "NULL buffer");
    char buf[1024];
    int n = snprintf(buf, sizeof buf,
                     "{\"N\": %lld, \"d\": %d, \"depth\": %d, \"leaf_size\": %d, \"rank\": %d, "
                     "\"tree_ms\": %.3f, \"knn\": %d, \"knn_ms\": %.3f, \"knn_wave_points\": %llu, "
                     "\"skeletonize_ms\": %.3f, \"factorize_ms\": %.3f, \"solve_ms\": %.3f, "
                     "\"precision\": \"%s\", \"min_pivot_ratio\": %.3e, \"refine_iterations\": %d}",
                     t ? (long long)t->N : 0LL, t ? t->d : 0, t ? t->D : 0, t ? t->m : 0, t ? t->s : 0,
                     t ? t->t_tree : 0.0, t ? t->knn : 0, t ? t->t_knn : 0.0, t ? t->knn_points : 0ULL,
                     t ? t->t_skel : 0.0,
                     f ? f->t_factor : 0.0, f ? f->t_solve : 0.0,
                     f ? (f->prec == P64 ? "fp64" : "mixed") : "none", f ? f->min_ratio : 0.0,
                     f ? f->info.iterations : 0);
    if (n < 0 || (size_t)n >= sizeof buf) return fail(ASKIT_ERR_ARG, "buffer too small");
    std::string js(buf, (size_t)n);
    if (t && !t->tune.empty()) {  // tuned tiles per height: [kmm columns, kmm chunk, gmm columns]
        js.pop_back();
        js += ", \"tune\": {";
        for (size_t h = 1; h < t->tune.size(); h++) {
            const Tune &u = t->tune[h];
            js += (h > 1 ? ", \"" : "\"") + std::to_string(h) + "\": [" + std::to_string(u.kmm_tc) + ", " +
                  std::to_string(u.kmm_kc) + ", " + std::to_string(u.gmm_tc) + "]";
        }
        js += "}}";
    }
    if (js.size() >= cap) return fail(ASKIT_ERR_ARG, "buffer too small");
    memcpy(json, js.c_str(), js.size() + 1);
    return ASKIT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free tree permutation.  Every temporary of the tree build lives
// in this array: one copy per device, held until the process ends.  Host code
// uses the device address hipGetSymbolAddress gives for the current device,
// never the array's name.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<unsigned char *> g_scratch_ptr;  // per device ordinal

askit_status scratch_of_current_device(unsigned char **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[dev];
    return ASKIT_OK;
}
}  // namespace

extern "C" askit_status askit_tree_permutation_noalloc(const double *X, int64_t N, int32_t d, int32_t leaf_size,
                                                       int64_t *perm, void *stream) {
    if (!X || !perm) return fail(ASKIT_ERR_ARG, "X or perm is NULL");
    if (N < 1 || N >= (int64_t)1 << 31) return fail(ASKIT_ERR_ARG, "N must be in [1, 2^31)");
    if (d < 1 || d > kMaxDim) return fail(ASKIT_ERR_ARG, "d must be in [1, 64]");
    if (leaf_size < 2) return fail(ASKIT_ERR_ARG, "leaf_size must be >= 2");
    int D = 0;
    while ((int64_t)leaf_size * ((int64_t)1 << D) < N) D++;
    const TreeScratch L = tree_scratch_layout(N, d, D);
    if (L.total > kNoAllocScratchBytes)
        return fail(ASKIT_ERR_ARG, "the tree build of " + std::to_string(N) + " points in " + std::to_string(d) +
                                       "-D needs " + std::to_string(L.total) + " bytes of scratch; the allocation-free "
                                       "entry point has " + std::to_string(kNoAllocScratchBytes));
    unsigned char *w = nullptr;
    ST_TRY(scratch_of_current_device(&w));
    hipStream_t st = (hipStream_t)stream;
    int64_t *nb = (int64_t *)(w + L.nb), *ne = (int64_t *)(w + L.ne);
    int16_t *pa = (int16_t *)(w + L.pa), *pc = (int16_t *)(w + L.pc);
    const int64_t nnodes = ((int64_t)2 << D) - 1;
    const int npair = d * (d + 1) / 2;
    hipLaunchKernelGGL(k_node_ranges, dim3(grid1(nnodes)), dim3(256), 0, st, nb, ne, N, D);
    hipLaunchKernelGGL(k_pair_index, dim3(grid1(npair)), dim3(256), 0, st, pa, pc, d);
    hipLaunchKernelGGL(k_iota, dim3(grid1(N)), dim3(256), 0, st, perm, N);
    HIP_TRY(hipGetLastError());
    return tree_levels(X, N, d, D, perm, nb, ne, pa, pc, (double *)(w + L.part), (double *)(w + L.mu),
                       (double *)(w + L.S), (double *)(w + L.axis), (double *)(w + L.key), (int64_t *)(w + L.kid),
                       (double *)(w + L.key2), (int64_t *)(w + L.kid2), st);
}
