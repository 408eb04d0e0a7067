// C ABI of libuoi: argument validation, scratch pool, and the orchestration of
// UoI_LASSO (Alg. 1) and UoI_VAR (Alg. 2) over the device kernels.  Every step
// of the fit runs in this library's kernels; the host only validates, sizes
// scratch memory, launches, and reads back small control values (convergence
// counts, support sizes).
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace uoi {

static thread_local std::string g_last_error;
void set_last_error(const std::string &m) { g_last_error = m; }

// ---------------------------------------------------------------------------
// grow-only scratch pool, one per device
// ---------------------------------------------------------------------------
namespace {
struct PoolEntry {
    void *ptr = nullptr;
    size_t cap = 0;
};
std::mutex g_pool_mu;
std::map<int, PoolEntry> g_pool;
std::map<std::pair<int, int>, PoolEntry> g_pinned;  // (device, slot)
}  // namespace

AuxStream &aux_stream() {
    static std::mutex mu;
    static std::map<int, AuxStream> m;
    int dev = 0;
    UOI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    AuxStream &a = m[dev];
    if (!a.s) {
        UOI_HIP(hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking));
        UOI_HIP(hipEventCreateWithFlags(&a.e0, hipEventDisableTiming));
        UOI_HIP(hipEventCreateWithFlags(&a.e1, hipEventDisableTiming));
        UOI_HIP(hipEventCreateWithFlags(&a.e2, hipEventDisableTiming));
    }
    return a;
}

void *pinned_slot(int slot, size_t bytes) {
    int dev = 0;
    UOI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_pool_mu);
    PoolEntry &e = g_pinned[std::make_pair(dev, slot)];
    bytes = std::max<size_t>(bytes, 256);
    if (e.cap < bytes) {
        if (e.ptr) {
            UOI_HIP(hipDeviceSynchronize());
            UOI_HIP(hipHostFree(e.ptr));
            e.ptr = nullptr;
            e.cap = 0;
        }
        if (hipHostMalloc(&e.ptr, bytes) != hipSuccess) {
            e.ptr = nullptr;
            (void)hipGetLastError();
            throw Error(UOI_ENOMEM, "pinned host allocation failed");
        }
        e.cap = bytes;
    }
    return e.ptr;
}

int *pinned_ints(size_t n) { return (int *)pinned_slot(kPinnedCounts, sizeof(int) * n); }

namespace {
struct GraphCache {
    hipStream_t cs = nullptr;  // capture stream (default priority)
    std::map<std::string, hipGraphExec_t> exec;
};
std::mutex g_graph_mu;
std::map<int, GraphCache> g_graphs;
constexpr size_t kGraphCacheMax = 64;
}  // namespace

void graph_launch(hipStream_t s, const GraphKey &key, const std::function<void(hipStream_t)> &record) {
    int dev = 0;
    UOI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_graph_mu);
    GraphCache &gc = g_graphs[dev];
    if (!gc.cs) UOI_HIP(hipStreamCreateWithFlags(&gc.cs, hipStreamNonBlocking));
    auto it = gc.exec.find(key.bytes);
    if (it == gc.exec.end()) {
        if (gc.exec.size() >= kGraphCacheMax) {
            UOI_HIP(hipDeviceSynchronize());  // no cached graph is still running
            for (auto &kv : gc.exec) (void)hipGraphExecDestroy(kv.second);
            gc.exec.clear();
        }
        hipGraph_t g = nullptr;
        UOI_HIP(hipStreamBeginCapture(gc.cs, hipStreamCaptureModeRelaxed));
        try {
            record(gc.cs);
        } catch (...) {
            (void)hipStreamEndCapture(gc.cs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        UOI_HIP(hipStreamEndCapture(gc.cs, &g));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        UOI_HIP(e);
        it = gc.exec.emplace(key.bytes, ex).first;
    }
    UOI_HIP(hipGraphLaunch(it->second, s));
}

namespace {
std::mutex g_event_mu;
std::map<int, std::vector<hipEvent_t>> g_events;  // free timing events per device
}  // namespace

hipEvent_t event_take() {
    int dev = 0;
    UOI_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_event_mu);
        std::vector<hipEvent_t> &v = g_events[dev];
        if (!v.empty()) {
            hipEvent_t e = v.back();
            v.pop_back();
            return e;
        }
    }
    hipEvent_t e;
    UOI_HIP(hipEventCreate(&e));
    return e;
}

void event_give(hipEvent_t e) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipEventDestroy(e);
        return;
    }
    std::lock_guard<std::mutex> lk(g_event_mu);
    g_events[dev].push_back(e);
}

void *pool_get(size_t bytes) {
    int dev = 0;
    UOI_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_pool_mu);
    PoolEntry &e = g_pool[dev];
    if (e.cap < bytes) {
        if (e.ptr) {
            UOI_HIP(hipDeviceSynchronize());
            UOI_HIP(hipFree(e.ptr));
            e.ptr = nullptr;
            e.cap = 0;
        }
        size_t want = bytes + bytes / 8 + (1 << 20);
        hipError_t err = hipMalloc(&e.ptr, want);
        if (err != hipSuccess) {
            e.ptr = nullptr;
            (void)hipGetLastError();
            throw Error(UOI_ENOMEM, "scratch allocation of " + std::to_string(want) + " bytes failed");
        }
        e.cap = want;
    }
    return e.ptr;
}

void pool_release() {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    auto it = g_pool.find(dev);
    if (it != g_pool.end() && it->second.ptr) {
        (void)hipDeviceSynchronize();
        (void)hipFree(it->second.ptr);
        it->second = PoolEntry{};
    }
}

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------
static void check_opts(const uoi_opts *o, bool need_boot) {
    UOI_REQUIRE(o != nullptr, "opts is NULL");
    if (need_boot) {
        UOI_REQUIRE(o->B1 >= 1, "B1 must be >= 1");
        UOI_REQUIRE(o->B2 >= 1, "B2 must be >= 1");
        UOI_REQUIRE(o->train_den > 0 && o->train_num > 0 && o->train_num < o->train_den,
                    "train_num/train_den must be a fraction in (0, 1)");
    }
    UOI_REQUIRE(o->q >= 1, "q must be >= 1");
    UOI_REQUIRE(o->lambdas != nullptr, "lambdas is NULL");
    for (int j = 0; j < o->q; ++j) {
        UOI_REQUIRE(std::isfinite(o->lambdas[j]) && o->lambdas[j] >= 0.0,
                    "lambdas must be finite and >= 0");
        if (j) UOI_REQUIRE(o->lambdas[j] < o->lambdas[j - 1], "lambdas must be strictly decreasing");
    }
    UOI_REQUIRE(std::isfinite(o->rho) && o->rho >= 0.0, "rho must be >= 0 (0: scaled to the data)");
    UOI_REQUIRE(std::isfinite(o->kkt_tol) && o->kkt_tol > 0.0, "kkt_tol must be > 0");
    UOI_REQUIRE(o->max_iter >= 1, "max_iter must be >= 1");
    UOI_REQUIRE(o->check_every >= 1, "check_every must be >= 1");
    UOI_REQUIRE(o->cg_max_iter >= 1, "cg_max_iter must be >= 1");
    UOI_REQUIRE(std::isfinite(o->relax) && o->relax >= 1.0 && o->relax <= 1.95,
                "relax must be in [1, 1.95]");
    UOI_REQUIRE(o->precision == UOI_FP64 || o->precision == UOI_MIXED, "unknown precision");
    UOI_REQUIRE(o->warm_start == UOI_COLD || o->warm_start == UOI_MLP, "unknown warm start");
    UOI_REQUIRE(o->warm_start != UOI_MLP || o->mlp != nullptr, "warm start by network: no network given");
    UOI_REQUIRE(o->warm_start != UOI_MLP || o->solver == UOI_SOLVER_BATCHED,
                "warm start by network needs the batched solver");
    UOI_REQUIRE(o->solver == UOI_SOLVER_BATCHED || o->solver == UOI_SOLVER_PLAIN, "unknown solver");
}

// NaN / Inf in the inputs: one flag per array in the workspace, one readback.
struct FiniteArg {
    const double *x;
    size_t n;
    const char *what;
};
static void check_finite(hipStream_t s, int *flags, std::initializer_list<FiniteArg> args) {
    const int na = (int)args.size();
    UOI_HIP(hipMemsetAsync(flags, 0, sizeof(int) * na, s));
    int i = 0;
    for (const FiniteArg &a : args) launch_finite_check(s, a.x, a.n, flags + i++);
    int *h = pinned_ints(na);
    UOI_HIP(hipMemcpyAsync(h, flags, sizeof(int) * na, hipMemcpyDeviceToHost, s));
    UOI_HIP(hipStreamSynchronize(s));
    i = 0;
    for (const FiniteArg &a : args)
        if (h[i++]) throw Error(UOI_EINVAL, std::string(a.what) + " contains NaN or Inf");
}

// z in [nb][p][R] (feature-major) <-> [nb][R][p] (solve-major)
__global__ void k_transpose(int nb, int p, int R, const double *__restrict__ a, double *__restrict__ b,
                            int to_solve_major) {
    __shared__ double t[32][33];
    int bb = blockIdx.z;
    int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    int rows = to_solve_major ? p : R, cols = to_solve_major ? R : p;
    const double *A = a + (size_t)bb * p * R;
    double *B = b + (size_t)bb * p * R;
    for (int dy = threadIdx.y; dy < 32; dy += 8) {
        int y = y0 + dy, x = x0 + threadIdx.x;
        if (y < rows && x < cols) t[dy][threadIdx.x] = A[(size_t)y * cols + x];
    }
    __syncthreads();
    for (int dy = threadIdx.y; dy < 32; dy += 8) {
        int x = x0 + dy, y = y0 + threadIdx.x;  // out[x][y] = in[y][x]
        if (x < cols && y < rows) B[(size_t)x * rows + y] = t[threadIdx.x][dy];
    }
}

static void transpose(hipStream_t s, int nb, int p, int R, const double *a, double *b, bool to_solve_major) {
    int rows = to_solve_major ? p : R, cols = to_solve_major ? R : p;
    hipLaunchKernelGGL(k_transpose, dim3(cdiv(cols, 32), cdiv(rows, 32), nb), dim3(32, 8), 0, s, nb, p,
                       R, a, b, to_solve_major ? 1 : 0);
    UOI_LAUNCH_CHECK();
}

// Host sum of n device int32 values (after the stream has synchronised).
static long long sum_device_ints(hipStream_t s, const int32_t *d, int n) {
    std::vector<int32_t> h(n);
    UOI_HIP(hipMemcpyAsync(h.data(), d, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    UOI_HIP(hipStreamSynchronize(s));
    long long t = 0;
    for (int v : h) t += v;
    return t;
}

// Times one launch sequence on the stream for a kernel-stat slot; the events are
// read only after the fit's final synchronisation (no wait in between).
struct KernelTimer {
    hipStream_t s;
    uoi_kstat *k;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    KernelTimer(hipStream_t s_, uoi_kstat *k_) : s(s_), k(k_) {}
    void start() {
        if (!k) return;
        e0 = event_take();
        e1 = event_take();
        UOI_HIP(hipEventRecord(e0, s));
    }
    void stop() {
        if (k) UOI_HIP(hipEventRecord(e1, s));
    }
    void resolve(double bytes, double flops) {  // after the stream has synchronised
        if (!k) return;
        float ms = 0.f;
        UOI_HIP(hipEventElapsedTime(&ms, e0, e1));
        k->ms += ms;
        k->bytes += bytes;
        k->flops += flops;
        k->launches += 1;
    }
    ~KernelTimer() {
        if (e0) event_give(e0);
        if (e1) event_give(e1);
    }
};

struct Timer {
    hipStream_t s;
    bool on;
    std::vector<hipEvent_t> ev;
    Timer(hipStream_t s_, bool on_) : s(s_), on(on_) {}
    void mark() {
        if (!on) return;
        hipEvent_t e = event_take();
        UOI_HIP(hipEventRecord(e, s));
        ev.push_back(e);
    }
    float between(size_t a, size_t b) {
        float ms = 0.f;
        if (on && b < ev.size()) UOI_HIP(hipEventElapsedTime(&ms, ev[a], ev[b]));
        return ms;
    }
    ~Timer() {
        for (auto e : ev) event_give(e);
    }
};

// ---------------------------------------------------------------------------
// UoI_LASSO
// ---------------------------------------------------------------------------
static int lasso_fit(int n, int p, const double *X, const double *y, const uoi_opts *o,
                     double *beta_out, uint64_t *supp_out, int32_t *jstar_out, uoi_diag *diag) {
    check_opts(o, true);
    UOI_REQUIRE((o->flags & (UOI_FLAG_INTERCEPT | UOI_FLAG_PER_EQUATION)) == 0,
                "the intercept and per-equation options apply to UoI_VAR");
    UOI_REQUIRE(n >= 2 && p >= 1, "need n >= 2 and p >= 1");
    UOI_REQUIRE(X && y && beta_out && supp_out && jstar_out, "NULL data or output pointer");
    const int ntr = split_count(n, o->train_num, o->train_den), nev = n - ntr;
    UOI_REQUIRE(ntr >= 1 && nev >= 1, "estimation split leaves an empty training or evaluation set");
    UOI_REQUIRE((int64_t)o->B1 * o->q <= (int64_t)1 << 30, "too many solves");
    hipStream_t s = (hipStream_t)o->stream;
    const bool timing = (o->flags & UOI_FLAG_TIMING) != 0;
    float sm[8] = {0};
    if (diag) std::memset(diag->kstat, 0, sizeof(diag->kstat));

    const int B1 = o->B1, B2 = o->B2, q = o->q, R = q;
    AdmmProblem P{B1, p, q, 1, R, nullptr, nullptr, nullptr, o->rho, o->kkt_tol, o->max_iter,
                  o->check_every, o->warm_start == UOI_MLP ? o->mlp : nullptr, o->relax};
    P.graphs = (o->flags & UOI_FLAG_EAGER) == 0;
    P.tune = (o->flags & UOI_FLAG_NO_TUNE) == 0;
    EstimProblem E{B2, p, 1, q, R, nullptr, nullptr, nullptr, nullptr, nullptr, supp_out, o->cg_max_iter};
    size_t nst = (size_t)B1 * p * R;
    // partial tiles of the selection product and of the evaluation product (over
    // any column count up to p: the union of the supports is not known yet)
    size_t gp_bytes = gram_part_bytes(B1, n, p, 1, true, 0, true);
    for (int pp = 1; pp <= p; ++pp) gp_bytes = std::max(gp_bytes, gram_part_bytes(B2, nev, pp, 1, true, 1, false));
    // size the scratch arena
    Arena ar;
    auto layout = [&](Arena &a, int32_t *&rows, double *&G, double *&c, double *&lam, double *&z,
                      double *&u, int32_t *&its, double *&kkt, uint8_t *&flag, int32_t *&tr,
                      int32_t *&ev, double *&GT, double *&CT, double *&GE, double *&CE, double *&sE,
                      void *&admm_w, void *&est_w, void *&cw, int32_t *&gidx, uint64_t *&cs, double *&XU,
                      double *&bc, void *&gp) {
        // draws, counts, distinct rows, weights, sizes, input check flags, union size
        rows = a.take<int32_t>((size_t)4 * B1 * n + B1 + 8 + q);  // + union count and support sizes
        G = a.take<double>((size_t)B1 * p * p);
        c = a.take<double>((size_t)B1 * p);
        lam = a.take<double>(q);
        z = a.take<double>(nst);
        u = a.take<double>(nst);
        its = a.take<int32_t>((size_t)B1 * R);
        kkt = a.take<double>((size_t)B1 * R);
        flag = a.take<uint8_t>((size_t)B2 * n);
        tr = a.take<int32_t>((size_t)B2 * ntr);
        ev = a.take<int32_t>((size_t)B2 * nev);
        GT = a.take<double>((size_t)B2 * p * p);
        CT = a.take<double>((size_t)B2 * p);
        GE = a.take<double>((size_t)B2 * p * p);
        CE = a.take<double>((size_t)B2 * p);
        sE = a.take<double>(B2);
        admm_w = a.take<char>(admm_work_bytes(P, o->precision, o->solver));
        est_w = a.take<char>(estim_work_bytes(E));
        cw = a.take<char>(complement_work_bytes(n, p, 1));
        gidx = a.take<int32_t>(p);
        cs = a.take<uint64_t>((size_t)q * ((p + 63) / 64));
        XU = a.take<double>((size_t)n * p);
        bc = a.take<double>(p);
        gp = a.take<char>(gp_bytes);
    };
    int32_t *rows, *its, *tr, *ev, *gidx;
    double *G, *c, *lam, *z, *u, *kkt, *GT, *CT, *GE, *CE, *sE, *XU, *bc;
    uint8_t *flag;
    uint64_t *cs;
    void *admm_w, *est_w, *cw, *gp;
    layout(ar, rows, G, c, lam, z, u, its, kkt, flag, tr, ev, GT, CT, GE, CE, sE, admm_w, est_w, cw, gidx, cs,
           XU, bc, gp);
    Arena A;
    A.cap = ar.off;
    A.base = (char *)pool_get(ar.off);
    layout(A, rows, G, c, lam, z, u, its, kkt, flag, tr, ev, GT, CT, GE, CE, sE, admm_w, est_w, cw, gidx, cs,
           XU, bc, gp);
    check_finite(s, rows + (size_t)4 * B1 * n + B1, {{X, (size_t)n * p, "X"}, {y, (size_t)n, "y"}});

    Timer tm(s, timing);
    KernelTimer gram_timer(s, timing && diag ? &diag->kstat[UOI_KSTAT_GRAM] : nullptr);
    tm.mark();
    UOI_HIP(hipMemcpyAsync(lam, o->lambdas, sizeof(double) * q, hipMemcpyHostToDevice, s));
    // model selection: bootstrap rows, Gram, ADMM sweep, supports
    launch_boot_rows(s, o->seed, TAG_LASSO_BOOT, B1, n, rows);
    // the estimation splits depend on the seed only: drawn on the second stream
    // beside the selection stage
    AuxStream &ax = aux_stream();
    UOI_HIP(hipEventRecord(ax.e0, s));
    UOI_HIP(hipStreamWaitEvent(ax.s, ax.e0, 0));
    launch_split(ax.s, o->seed, TAG_LASSO_SPLIT, B2, n, ntr, flag);
    launch_compact_rows(ax.s, B2, n, flag, ntr, tr, ev);
    UOI_HIP(hipEventRecord(ax.e2, ax.s));
    {
        // the Gram of a bootstrap sample runs over its distinct rows weighted by
        // their multiplicities (about 63% of n rows) and divides by n
        int32_t *cntb = rows + (size_t)B1 * n, *drow = cntb + (size_t)B1 * n, *dw = drow + (size_t)B1 * n;
        int32_t *nd = dw + (size_t)B1 * n;
        launch_distinct_rows(s, B1, n, n, rows, cntb, drow, dw, nd);
        gram_timer.start();
        launch_gram_f64_weighted(s, B1, n, drow, dw, nd, n, p, X, p, 1, y, 1, G, c, nullptr, gp, gp_bytes);
        gram_timer.stop();
    }
    tm.mark();
    P.G = G;
    P.C = c;
    P.lam = lam;
    AdmmOut out{z, u, diag && diag->iters ? diag->iters : its, diag && diag->kkt ? diag->kkt : kkt, 0, 0,
                timing && diag ? diag->kstat : nullptr, 0};
    DeferredTiming dtm;  // stage and kernel times, read after the final synchronisation
    out.dt = &dtm;
    admm_solve(s, P, o->precision, o->solver, admm_w, false, out, timing ? sm + 1 : nullptr);
    tm.mark();
    launch_support_and(s, B1, p, R, z, supp_out);
    tm.mark();
    // model estimation: splits, training / evaluation statistics, refits, union.
    // The refits read statistics of support columns only: when the union U of the
    // q supports is at most 3/4 of the columns, the products are formed over
    // X[:, U] and the supports renumbered; beta* is scattered back at the end.
    std::vector<int32_t> sizes;
    const int nu = launch_support_union(s, q, p, supp_out, rows + (size_t)4 * B1 * n + B1 + 4, gidx, &sizes);
    const bool compact = nu > 0 && 4 * (int64_t)nu <= 3 * (int64_t)p;
    const int pE = compact ? nu : p;
    const double *XE = X;
    if (compact) {
        launch_compact_design(s, q, p, nu, supp_out, gidx, cs, n, X, p, XU);
        XE = XU;
        E.p = pE;
        E.supp = cs;
    }
    UOI_HIP(hipStreamWaitEvent(s, ax.e2, 0));  // the splits
    // evaluation products directly; training products as their complement in the
    // full-data product (the split partitions the rows), so the larger training
    // side is never gathered
    launch_gram_f64(s, B2, nev, ev, nullptr, pE, XE, pE, 1, y, 1, GE, CE, sE, 1, gp, gp_bytes);
    launch_train_from_eval(s, B2, n, pE, XE, pE, 1, y, 1, GE, CE, ntr, nev, nullptr, nullptr, GT, CT, cw);
    tm.mark();
    E.GT = GT; E.CT = CT; E.GE = GE; E.CE = CE; E.sE = sE;
    // [0] singular refit, [1] refits left unconverged: read after the final synchronisation
    int *eflags = (int *)pinned_slot(kPinnedFlag, 2 * sizeof(int));
    estimate(s, E, est_w, compact ? bc : beta_out, jstar_out, diag ? diag->losses : nullptr,
             timing ? sm + 6 : nullptr, &sizes, eflags, &dtm);
    if (compact) launch_scatter_cols(s, p, nu, gidx, bc, beta_out);
    tm.mark();
    if (diag && diag->sel_beta) transpose(s, B1, p, R, z, diag->sel_beta, true);
    UOI_HIP(hipStreamSynchronize(s));
    dtm.resolve();
    if (eflags[0]) throw Error(UOI_EINVAL, "estimation: a training Gram restricted to a support is singular");
    const int refit_noconv = eflags[1];
    if (timing) {
        sm[0] = tm.between(0, 1);
        sm[4] = tm.between(2, 3);
        sm[5] = tm.between(3, 4);
    }
    admm_finish_stats(out);
    if (timing && diag) {  // the selection Gram's rows actually processed
        const double md = (double)sum_device_ints(s, rows + (size_t)4 * B1 * n, B1);
        gram_timer.resolve(md * (p + 1) * 8 + (double)B1 * p * (p + 1) * 8, md * p * (p + 1) + 2.0 * md * p);
    }
    if (diag) {
        diag->n_solves = (int64_t)B1 * R;
        diag->n_unconverged = out.unconverged;
        diag->max_iters = out.max_iters;
        diag->warm_used = out.warm_used;
        diag->n_refit_unconverged = refit_noconv;
        std::memcpy(diag->stage_ms, sm, sizeof(sm));
    }
    return out.unconverged || refit_noconv ? UOI_ENOCONV : UOI_OK;
}

// ---------------------------------------------------------------------------
// UoI_VAR, order d, optional intercept
// ---------------------------------------------------------------------------
// Regression row r = 0 .. N-1 (N = T - d): response x_{r+d}, design the slice
// series[r .. r+d-1] read in place (row stride p, width P = d p, columns from
// lag d to lag 1); k_var_reorder maps the result to Eq. (7)'s lag order.
static int var_fit(int T, int p, int d, const double *series, int block_len, const uoi_opts *o,
                   double *A_out, double *mu_out, uint64_t *supp_out, int32_t *jstar_out, uoi_diag *diag) {
    check_opts(o, true);
    UOI_REQUIRE(d >= 1, "the autoregressive order d must be >= 1");
    UOI_REQUIRE(p >= 1 && (int64_t)T >= (int64_t)d + 2, "need p >= 1 and T >= d + 2");
    UOI_REQUIRE(series && A_out && mu_out && supp_out && jstar_out, "NULL data or output pointer");
    UOI_REQUIRE((int64_t)d * p <= 65536, "d * p must be <= 65536");
    const int N = T - d, P = d * p;
    const int L = block_len > 0 ? block_len : var_block_len_default(N);
    UOI_REQUIRE(L <= N, "block_len must be <= T-d");
    const int nblk = (N + L - 1) / L;
    const int nbt = split_count(nblk, o->train_num, o->train_den);
    UOI_REQUIRE(nbt >= 1 && nbt < nblk, "estimation split leaves no training or evaluation block");
    UOI_REQUIRE((int64_t)o->B1 * o->q * p <= (int64_t)1 << 30, "too many solves");
    hipStream_t s = (hipStream_t)o->stream;
    const bool timing = (o->flags & UOI_FLAG_TIMING) != 0;
    const bool icpt = (o->flags & UOI_FLAG_INTERCEPT) != 0;
    float sm[8] = {0};
    if (diag) std::memset(diag->kstat, 0, sizeof(diag->kstat));

    const int B1 = o->B1, B2 = o->B2, q = o->q, pe = p, R = q * p;
    const int W = (P + 63) / 64;
    UOI_REQUIRE(o->warm_start == UOI_COLD, "warm start by network is for UoI_LASSO only");
    AdmmProblem Pb{B1, P, q, pe, R, nullptr, nullptr, nullptr, o->rho, o->kkt_tol, o->max_iter,
                   o->check_every, nullptr, o->relax};
    Pb.graphs = (o->flags & UOI_FLAG_EAGER) == 0;
    Pb.tune = (o->flags & UOI_FLAG_NO_TUNE) == 0;
    EstimProblem E{B2, P, pe, q, R, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, o->cg_max_iter};
    E.per_eq = (o->flags & UOI_FLAG_PER_EQUATION) != 0;
    const size_t nst = (size_t)B1 * P * R;
    struct Buf {
        int32_t *rows, *its, *tr, *ev, *ntr, *nev;
        double *G, *C, *lam, *z, *u, *kkt, *GT, *CT, *GE, *CE, *sE;
        double *xS, *yS, *xE, *yE, *xT, *yT, *xA, *yA, *beta;  // means (intercept), beta* (d > 1)
        uint64_t *supp;                                       // internal-order supports (d > 1)
        uint8_t *flag;
        void *admm_w, *est_w, *cw, *gp;
    } bf{};
    // partial tiles of the selection and evaluation products
    const size_t gp_bytes = std::max(gram_part_bytes(B1, N, P, pe, true, 0, true),
                                     gram_part_bytes(B2, N, P, pe, true, 1, false));
    auto layout = [&](Arena &a, Buf &x) {
        // draws, counts, distinct rows, weights, sizes, input check flag
        x.rows = a.take<int32_t>((size_t)4 * B1 * N + B1 + 4);
        x.G = a.take<double>((size_t)B1 * P * P);
        x.C = a.take<double>((size_t)B1 * P * pe);
        x.lam = a.take<double>(q);
        x.z = a.take<double>(nst);
        x.u = a.take<double>(nst);
        x.its = a.take<int32_t>((size_t)B1 * R);
        x.kkt = a.take<double>((size_t)B1 * R);
        x.flag = a.take<uint8_t>((size_t)B2 * nblk);
        x.tr = a.take<int32_t>((size_t)B2 * N);
        x.ev = a.take<int32_t>((size_t)B2 * N);
        x.ntr = a.take<int32_t>(B2);
        x.nev = a.take<int32_t>(B2);
        x.GT = a.take<double>((size_t)B2 * P * P);
        x.CT = a.take<double>((size_t)B2 * P * pe);
        x.GE = a.take<double>((size_t)B2 * P * P);
        x.CE = a.take<double>((size_t)B2 * P * pe);
        x.sE = a.take<double>((size_t)B2 * pe);
        if (icpt) {
            x.xS = a.take<double>((size_t)B1 * P);
            x.yS = a.take<double>((size_t)B1 * pe);
            x.xE = a.take<double>((size_t)B2 * P);
            x.yE = a.take<double>((size_t)B2 * pe);
            x.xT = a.take<double>((size_t)B2 * P);
            x.yT = a.take<double>((size_t)B2 * pe);
            x.xA = a.take<double>(P);
            x.yA = a.take<double>(pe);
        }
        if (d > 1) {
            x.beta = a.take<double>((size_t)pe * P);
            x.supp = a.take<uint64_t>((size_t)q * pe * W);
        }
        x.admm_w = a.take<char>(admm_work_bytes(Pb, o->precision, o->solver));
        x.est_w = a.take<char>(estim_work_bytes(E));
        x.cw = a.take<char>(complement_work_bytes(N, P, pe));
        x.gp = a.take<char>(gp_bytes);
    };
    Arena ar;
    layout(ar, bf);
    Arena A;
    A.cap = ar.off;
    A.base = (char *)pool_get(ar.off);
    layout(A, bf);
    uint64_t *supp = d > 1 ? bf.supp : supp_out;    // supports in the internal column order
    double *beta = d > 1 ? bf.beta : A_out;          // beta* [equation][internal column]
    E.supp = supp;
    check_finite(s, bf.rows + (size_t)4 * B1 * N + B1, {{series, (size_t)T * p, "series"}});

    const double *Xd = series, *Yd = series + (size_t)d * p;  // design rows series[r..], responses series[r+d]
    Timer tm(s, timing);
    KernelTimer gram_timer(s, timing && diag ? &diag->kstat[UOI_KSTAT_GRAM] : nullptr);
    tm.mark();
    UOI_HIP(hipMemcpyAsync(bf.lam, o->lambdas, sizeof(double) * q, hipMemcpyHostToDevice, s));
    launch_var_boot_rows(s, o->seed, B1, N, L, bf.rows);
    // the estimation splits depend on the seed only: drawn on the second stream
    // beside the selection stage
    AuxStream &ax = aux_stream();
    UOI_HIP(hipEventRecord(ax.e0, s));
    UOI_HIP(hipStreamWaitEvent(ax.s, ax.e0, 0));
    launch_split(ax.s, o->seed, TAG_VAR_SPLIT, B2, nblk, nbt, bf.flag);
    launch_expand_blocks(ax.s, B2, nblk, N, L, bf.flag, bf.tr, bf.ev, bf.ntr, bf.nev);
    UOI_HIP(hipEventRecord(ax.e2, ax.s));
    {
        // distinct regression rows of each block-bootstrap sample, weighted by
        // their multiplicities
        int32_t *cntb = bf.rows + (size_t)B1 * N, *drow = cntb + (size_t)B1 * N, *dw = drow + (size_t)B1 * N;
        int32_t *nd = dw + (size_t)B1 * N;
        launch_distinct_rows(s, B1, N, N, bf.rows, cntb, drow, dw, nd);
        gram_timer.start();
        launch_gram_f64_weighted(s, B1, N, drow, dw, nd, N, P, Xd, p, pe, Yd, p, bf.G, bf.C, nullptr, bf.gp,
                                 gp_bytes);
        gram_timer.stop();
        if (icpt) {  // every bootstrap sample centred by its own means
            launch_colmeans(s, B1, N, drow, dw, nd, N, P, Xd, p, pe, Yd, p, bf.xS, bf.yS);
            launch_shift_stats(s, B1, P, pe, bf.G, bf.C, nullptr, bf.xS, bf.yS, bf.xS, bf.yS);
        }
    }
    tm.mark();
    Pb.G = bf.G;
    Pb.C = bf.C;
    Pb.lam = bf.lam;
    AdmmOut out{bf.z, bf.u, diag && diag->iters ? diag->iters : bf.its, diag && diag->kkt ? diag->kkt : bf.kkt, 0,
                0, timing && diag ? diag->kstat : nullptr, 0};
    DeferredTiming dtm;  // stage and kernel times, read after the final synchronisation
    out.dt = &dtm;
    admm_solve(s, Pb, o->precision, o->solver, bf.admm_w, false, out, timing ? sm + 1 : nullptr);
    tm.mark();
    launch_support_and(s, B1, P, R, bf.z, supp);
    tm.mark();
    UOI_HIP(hipStreamWaitEvent(s, ax.e2, 0));  // the splits
    launch_gram_f64(s, B2, N, bf.ev, bf.nev, P, Xd, p, pe, Yd, p, bf.GE, bf.CE, nullptr, 1, bf.gp, gp_bytes);
    launch_colsq(s, B2, N, bf.ev, bf.nev, pe, Yd, p, bf.sE);
    launch_train_from_eval(s, B2, N, P, Xd, p, pe, Yd, p, bf.GE, bf.CE, 0, 0, bf.ntr, bf.nev, bf.GT, bf.CT,
                           bf.cw);
    if (icpt) {
        // training means from the full-data and evaluation means; evaluation
        // statistics about the training means, training statistics centred
        launch_colmeans(s, B2, N, bf.ev, nullptr, bf.nev, 0, P, Xd, p, pe, Yd, p, bf.xE, bf.yE);
        launch_colmeans(s, 1, N, nullptr, nullptr, nullptr, 0, P, Xd, p, pe, Yd, p, bf.xA, bf.yA);
        launch_train_means(s, B2, P, pe, N, bf.xA, bf.yA, bf.nev, bf.xE, bf.yE, bf.xT, bf.yT);
        launch_shift_stats(s, B2, P, pe, bf.GE, bf.CE, bf.sE, bf.xE, bf.yE, bf.xT, bf.yT);
        launch_shift_stats(s, B2, P, pe, bf.GT, bf.CT, nullptr, bf.xT, bf.yT, bf.xT, bf.yT);
        E.xT = bf.xT;
        E.yT = bf.yT;
        E.mu = mu_out;
    }
    tm.mark();
    E.GT = bf.GT; E.CT = bf.CT; E.GE = bf.GE; E.CE = bf.CE; E.sE = bf.sE;
    int *eflags = (int *)pinned_slot(kPinnedFlag, 2 * sizeof(int));
    estimate(s, E, bf.est_w, beta, jstar_out, diag ? diag->losses : nullptr, timing ? sm + 6 : nullptr, nullptr,
             eflags, &dtm);
    if (d > 1) launch_var_reorder(s, q, p, d, supp, supp_out, beta, A_out);
    tm.mark();
    if (!icpt) UOI_HIP(hipMemsetAsync(mu_out, 0, sizeof(double) * p, s));
    if (diag && diag->sel_beta) transpose(s, B1, P, R, bf.z, diag->sel_beta, true);
    UOI_HIP(hipStreamSynchronize(s));
    dtm.resolve();
    if (eflags[0]) throw Error(UOI_EINVAL, "estimation: a training Gram restricted to a support is singular");
    const int refit_noconv = eflags[1];
    if (timing) {
        sm[0] = tm.between(0, 1);
        sm[4] = tm.between(2, 3);
        sm[5] = tm.between(3, 4);
    }
    admm_finish_stats(out);
    if (timing && diag) {
        const double md = (double)sum_device_ints(s, bf.rows + (size_t)4 * B1 * N, B1);
        gram_timer.resolve(md * (P + pe) * 8 + (double)B1 * P * (P + pe) * 8,
                           md * P * (P + 1) + 2.0 * md * P * pe);
    }
    if (diag) {
        diag->n_solves = (int64_t)B1 * R;
        diag->n_unconverged = out.unconverged;
        diag->max_iters = out.max_iters;
        diag->warm_used = out.warm_used;
        diag->n_refit_unconverged = refit_noconv;
        std::memcpy(diag->stage_ms, sm, sizeof(sm));
    }
    return out.unconverged || refit_noconv ? UOI_ENOCONV : UOI_OK;
}

// ---------------------------------------------------------------------------
// With scratch_cap > 0 the scratch memory is the caller-provided buffer
// scratch (device, at least scratch_cap bytes): nothing is allocated, and
// sizes beyond the buffer are rejected before any device work.
int solve_batch(int nb, int p, const double *G, const double *c, const uoi_opts *o, const double *z0,
                const double *u0, double *z_out, double *u_out, int32_t *iters, double *kkt,
                void *(*scratch)(), size_t scratch_cap) {
    check_opts(o, false);
    UOI_REQUIRE(nb >= 1 && p >= 1, "need nb >= 1 and p >= 1");
    UOI_REQUIRE(G && c && z_out, "NULL input or output pointer");
    const bool no_alloc = scratch_cap > 0;
    UOI_REQUIRE(!no_alloc || o->warm_start == UOI_COLD,
                "the allocation-free entry point starts cold (no warm start by network)");
    UOI_REQUIRE(!no_alloc || o->rho > 0.0, "the allocation-free entry point needs rho > 0");
    hipStream_t s = (hipStream_t)o->stream;
    const int q = o->q, R = q;
    AdmmProblem P{nb, p, q, 1, R, G, c, nullptr, o->rho, o->kkt_tol, o->max_iter, o->check_every,
                  o->warm_start == UOI_MLP ? o->mlp : nullptr, o->relax};
    P.no_alloc = no_alloc;
    P.graphs = !no_alloc && (o->flags & UOI_FLAG_EAGER) == 0;  // instantiating a graph allocates
    P.tune = !no_alloc && (o->flags & UOI_FLAG_NO_TUNE) == 0;   // timing candidates creates events
    size_t nst = (size_t)nb * p * R;
    auto layout = [&](Arena &a, double *&lam, double *&z, double *&u, int32_t *&its, double *&kk,
                      void *&w) {
        lam = a.take<double>(q);
        z = a.take<double>(nst);
        u = a.take<double>(nst);
        its = a.take<int32_t>((size_t)nb * R);
        kk = a.take<double>((size_t)nb * R);
        w = a.take<char>(admm_work_bytes(P, o->precision, o->solver));
    };
    double *lam, *z, *u, *kk;
    int32_t *its;
    void *w;
    Arena ar;
    layout(ar, lam, z, u, its, kk, w);
    if (no_alloc)
        UOI_REQUIRE(ar.off <= scratch_cap,
                    "problem needs " + std::to_string(ar.off) + " bytes of scratch; the static buffer of the "
                    "allocation-free entry point holds " + std::to_string(scratch_cap));
    Arena A;
    A.cap = ar.off;
    A.base = (char *)(no_alloc ? scratch() : pool_get(ar.off));
    layout(A, lam, z, u, its, kk, w);
    UOI_HIP(hipMemcpyAsync(lam, o->lambdas, sizeof(double) * q, hipMemcpyHostToDevice, s));
    P.lam = lam;
    bool warm = z0 != nullptr || u0 != nullptr;
    if (warm) {
        if (z0) transpose(s, nb, p, R, z0, z, false);
        else UOI_HIP(hipMemsetAsync(z, 0, sizeof(double) * nst, s));
        if (u0) transpose(s, nb, p, R, u0, u, false);
        else UOI_HIP(hipMemsetAsync(u, 0, sizeof(double) * nst, s));
    }
    AdmmOut out{z, u, iters ? iters : its, kkt ? kkt : kk, 0, 0, nullptr, 0, nullptr};
    admm_solve(s, P, o->precision, o->solver, w, warm, out, nullptr);
    transpose(s, nb, p, R, z, z_out, true);
    if (u_out) transpose(s, nb, p, R, u, u_out, true);
    UOI_HIP(hipStreamSynchronize(s));
    admm_finish_stats(out);
    return out.unconverged ? UOI_ENOCONV : UOI_OK;
}

}  // namespace uoi

using namespace uoi;

extern "C" {

void uoi_default_opts(uoi_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rho = 1.0;
    o->kkt_tol = 1e-6;
    o->max_iter = 20000;
    o->check_every = 10;
    o->train_num = 4;
    o->train_den = 5;
    o->relax = 1.0;
    o->cg_max_iter = 4000;
    o->precision = UOI_FP64;
    o->warm_start = UOI_COLD;
    o->solver = UOI_SOLVER_BATCHED;
}

int uoi_lasso_fit(int32_t n, int32_t p, const double *X, const double *y, const uoi_opts *o,
                  double *beta_out, uint64_t *supp_out, int32_t *jstar_out, uoi_diag *diag) {
    return guarded([&] { return lasso_fit(n, p, X, y, o, beta_out, supp_out, jstar_out, diag); });
}

int uoi_var_fit(int32_t T, int32_t p, int32_t d, const double *series, int32_t block_len,
                const uoi_opts *o, double *A_out, double *mu_out, uint64_t *supp_out,
                int32_t *jstar_out, uoi_diag *diag) {
    return guarded(
        [&] { return var_fit(T, p, d, series, block_len, o, A_out, mu_out, supp_out, jstar_out, diag); });
}

int uoi_lasso_solve_batch(int32_t nb, int32_t p, const double *G, const double *c, const uoi_opts *o,
                          const double *z0, const double *u0, double *z_out, double *u_out,
                          int32_t *iters, double *kkt) {
    return guarded([&] { return solve_batch(nb, p, G, c, o, z0, u0, z_out, u_out, iters, kkt, nullptr, 0); });
}

int uoi_gram(int32_t nb, int32_t m, const int32_t *rows, int32_t p, const double *X, int32_t ldx,
             int32_t pe, const double *Y, int32_t ldy, double *G, double *C, void *stream) {
    return guarded([&] {
        UOI_REQUIRE(nb >= 1 && m >= 1 && p >= 1 && pe >= 0 && ldx >= p, "invalid Gram sizes");
        UOI_REQUIRE(rows && X && G, "NULL pointer");
        UOI_REQUIRE(pe == 0 || (Y && C && ldy >= pe), "pe > 0 needs Y, C and ldy >= pe");
        // the instance for products other than the fits' selection Grams
        const size_t pb = gram_part_bytes(nb, m, p, pe, pe > 0, 1, false);
        void *part = pb ? pool_get(pb) : nullptr;
        launch_gram_f64((hipStream_t)stream, nb, m, rows, nullptr, p, X, ldx, pe, Y, ldy, G,
                        pe ? C : nullptr, nullptr, 1, part, pb);
        UOI_HIP(hipStreamSynchronize((hipStream_t)stream));
        return UOI_OK;
    });
}

int uoi_bootstrap_rows(uint64_t seed, int32_t nb, int32_t n, int32_t *rows, void *stream) {
    return guarded([&] {
        UOI_REQUIRE(nb >= 1 && n >= 1 && rows, "invalid arguments");
        launch_boot_rows((hipStream_t)stream, seed, TAG_LASSO_BOOT, nb, n, rows);
        UOI_HIP(hipStreamSynchronize((hipStream_t)stream));
        return UOI_OK;
    });
}

int uoi_split_rows(uint64_t seed, int32_t nb, int32_t n, int32_t num, int32_t den, int32_t *train,
                   int32_t *eval, void *stream) {
    return guarded([&] {
        UOI_REQUIRE(nb >= 1 && n >= 1 && den > 0 && num > 0 && num < den && train && eval,
                    "invalid arguments");
        int ntr = split_count(n, num, den);
        UOI_REQUIRE(ntr >= 1 && ntr < n, "split leaves an empty side");
        hipStream_t s = (hipStream_t)stream;
        uint8_t *flag = (uint8_t *)pool_get((size_t)nb * n);
        launch_split(s, seed, TAG_LASSO_SPLIT, nb, n, ntr, flag);
        launch_compact_rows(s, nb, n, flag, ntr, train, eval);
        UOI_HIP(hipStreamSynchronize(s));
        return UOI_OK;
    });
}

int uoi_var_boot_rows(uint64_t seed, int32_t nb, int32_t N, int32_t L, int32_t *rows, void *stream) {
    return guarded([&] {
        UOI_REQUIRE(nb >= 1 && N >= 1 && L >= 1 && L <= N && rows, "invalid arguments");
        launch_var_boot_rows((hipStream_t)stream, seed, nb, N, L, rows);
        UOI_HIP(hipStreamSynchronize((hipStream_t)stream));
        return UOI_OK;
    });
}

int uoi_var_split_rows(uint64_t seed, int32_t nb, int32_t N, int32_t L, int32_t num, int32_t den,
                       int32_t *train, int32_t *eval, int32_t *ntr_out, int32_t *nev_out, void *stream) {
    return guarded([&] {
        UOI_REQUIRE(nb >= 1 && N >= 1 && L >= 1 && L <= N && den > 0 && num > 0 && num < den,
                    "invalid arguments");
        UOI_REQUIRE(train && eval && ntr_out && nev_out, "NULL pointer");
        int nblk = (N + L - 1) / L, nbt = split_count(nblk, num, den);
        UOI_REQUIRE(nbt >= 1 && nbt < nblk, "split leaves an empty side");
        hipStream_t s = (hipStream_t)stream;
        char *w = (char *)pool_get((size_t)nb * nblk + 2 * 256 * (size_t)nb + 1024);
        uint8_t *flag = (uint8_t *)w;
        int32_t *cnts = (int32_t *)(w + (((size_t)nb * nblk + 255) & ~size_t(255)));
        launch_split(s, seed, TAG_VAR_SPLIT, nb, nblk, nbt, flag);
        launch_expand_blocks(s, nb, nblk, N, L, flag, train, eval, cnts, cnts + nb);
        UOI_HIP(hipMemcpyAsync(ntr_out, cnts, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
        UOI_HIP(hipMemcpyAsync(nev_out, cnts + nb, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
        UOI_HIP(hipStreamSynchronize(s));
        return UOI_OK;
    });
}

int uoi_spd_inverse(int32_t nb, int32_t p, const double *G, double rho, double *M, void *stream) {
    return guarded([&] {
        UOI_REQUIRE(nb >= 1 && p >= 1 && G && M && rho >= 0.0, "invalid arguments");
        hipStream_t s = (hipStream_t)stream;
        size_t wd = spd_inverse_work_doubles(nb, p);
        double *w = wd ? (double *)pool_get(wd * sizeof(double)) : nullptr;
        spd_inverse_f64(s, nb, p, G, rho, M, w);
        UOI_HIP(hipStreamSynchronize(s));
        return UOI_OK;
    });
}

int uoi_ws_dataset(int32_t nb, int32_t p, int32_t q, int32_t pe, const double *c, const double *lambdas,
                   const double *z, float *X, float *T, void *stream) {
    return guarded([&] {
        UOI_REQUIRE(nb >= 1 && p >= 1 && q >= 1 && pe >= 1 && c && lambdas && z && X && T,
                    "invalid arguments");
        hipStream_t s = (hipStream_t)stream;
        const size_t lb = ((size_t)q * 8 + 255) & ~size_t(255);
        char *w = (char *)pool_get(lb + (size_t)nb * pe * 8 + 256);
        double *lam = (double *)w;
        double *cn = (double *)(w + lb);
        UOI_HIP(hipMemcpyAsync(lam, lambdas, sizeof(double) * q, hipMemcpyHostToDevice, s));
        warm_start_dataset(s, nb, p, q, pe, c, lam, z, X, T, cn);
        UOI_HIP(hipStreamSynchronize(s));
        return UOI_OK;
    });
}

int uoi_lasso_solve_multi(int32_t nb, int32_t p, int32_t pe, const double *G, const double *C,
                          const uoi_opts *o, double *z_out, int32_t *iters, double *kkt) {
    return guarded([&] {
        check_opts(o, false);
        UOI_REQUIRE(nb >= 1 && p >= 1 && pe >= 1 && G && C && z_out, "invalid arguments");
        UOI_REQUIRE(o->warm_start == UOI_COLD, "multi-response solves start cold");
        hipStream_t s = (hipStream_t)o->stream;
        const int q = o->q, R = q * pe;
        AdmmProblem P{nb, p, q, pe, R, G, C, nullptr, o->rho, o->kkt_tol, o->max_iter, o->check_every,
                      nullptr, o->relax};
        P.graphs = (o->flags & UOI_FLAG_EAGER) == 0;
        P.tune = (o->flags & UOI_FLAG_NO_TUNE) == 0;
        const size_t nst = (size_t)nb * p * R;
        auto layout = [&](Arena &a, double *&lam, double *&z, double *&u, int32_t *&its, double *&kk,
                          void *&w) {
            lam = a.take<double>(q);
            z = a.take<double>(nst);
            u = a.take<double>(nst);
            its = a.take<int32_t>((size_t)nb * R);
            kk = a.take<double>((size_t)nb * R);
            w = a.take<char>(admm_work_bytes(P, o->precision, o->solver));
        };
        double *lam, *z, *u, *kk;
        int32_t *its;
        void *w;
        Arena ar;
        layout(ar, lam, z, u, its, kk, w);
        Arena A;
        A.cap = ar.off;
        A.base = (char *)pool_get(ar.off);
        layout(A, lam, z, u, its, kk, w);
        UOI_HIP(hipMemcpyAsync(lam, o->lambdas, sizeof(double) * q, hipMemcpyHostToDevice, s));
        P.lam = lam;
        AdmmOut out{z, u, iters ? iters : its, kkt ? kkt : kk, 0, 0, nullptr, 0, nullptr};
        admm_solve(s, P, o->precision, o->solver, w, false, out, nullptr);
        transpose(s, nb, p, R, z, z_out, true);
        UOI_HIP(hipStreamSynchronize(s));
        admm_finish_stats(out);
        return out.unconverged ? UOI_ENOCONV : UOI_OK;
    });
}

void uoi_release_workspace(void) {
    try {
        pool_release();
    } catch (...) {
    }
}

void uoi_tune_reset(void) {
    try {
        tune_forget();
    } catch (...) {
    }
}

const char *uoi_last_error(void) { return g_last_error.c_str(); }

const char *uoi_version(void) { return "uoi-mi355x 0.1 (gfx950)"; }

}  // extern "C"
