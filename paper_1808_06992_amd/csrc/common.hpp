// Shared host/device helpers of libuoi (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/uoi.h"

namespace uoi {

// ---------------------------------------------------------------------------
// Errors: internal code throws uoi::Error; the ABI layer converts it to a code.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define UOI_HIP(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw ::uoi::Error(e_ == hipErrorOutOfMemory ? UOI_ENOMEM : UOI_EHIP,     \
                               std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

#define UOI_LAUNCH_CHECK() UOI_HIP(hipGetLastError())

#define UOI_REQUIRE(cond, msg)                                  \
    do {                                                        \
        if (!(cond)) throw ::uoi::Error(UOI_EINVAL, (msg));     \
    } while (0)

void set_last_error(const std::string &m);

// Runs an entry point's body: no exception crosses the C ABI; an error becomes
// its status code and the thread's last-error message.
template <class F>
int guarded(F &&f) {
    try {
        set_last_error("");
        return f();
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return UOI_EHIP;
    } catch (...) {
        set_last_error("unknown error");
        return UOI_EHIP;
    }
}

// ---------------------------------------------------------------------------
// Scratch pool: one grow-only device allocation per device, carved by Arena.
// ---------------------------------------------------------------------------
void *pool_get(size_t bytes);  // returns a device buffer of at least `bytes`
void pool_release();
// Pinned host ints for asynchronous readbacks of small results (grow-only, one
// buffer per device, like the pool; calls that overlap on one device race).
// Grow-only pinned host buffers per (device, slot); a slot's buffer is reused by
// the next call that asks for it, so its contents live until then.
enum { kPinnedCounts = 0, kPinnedLists = 1, kPinnedFlag = 2, kPinnedLarge = 3 };
void *pinned_slot(int slot, size_t bytes);
int *pinned_ints(size_t n);  // slot kPinnedCounts
// A second stream of the current device (default priority, non-blocking) with
// two events, for independent kernels that can run beside the caller's stream.
struct AuxStream {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
};
AuxStream &aux_stream();

// Launch sequences replayed as HIP graphs.  graph_launch(s, key, record) launches
// on s the graph of the sequence that record(cs) enqueues on a capture stream cs;
// the sequence is recorded and instantiated the first time its key is seen, and
// the key must determine every argument of every launch in it (pointers,
// sizes, scalars).  Graphs hold kernel launches only (no memset or copy nodes).
// The cache is per device, bounded, and cleared when it fills.
struct GraphKey {
    std::string bytes;
    template <class V>
    GraphKey &add(const V &v) {
        bytes.append(reinterpret_cast<const char *>(&v), sizeof(V));
        return *this;
    }
};
void graph_launch(hipStream_t s, const GraphKey &key, const std::function<void(hipStream_t)> &record);

// Autotuner of launch shapes whose candidates give identical results (tune.hip).
struct TuneResult {
    int choice;    // index of the fastest candidate
    bool ran_all;  // every candidate was just run on the live problem (outputs in place)
};
TuneResult tune_choose(hipStream_t s, const std::string &key, int ncand, const std::function<void(int)> &run,
                       int reps);
int tune_lookup(const std::string &key, int fallback);  // recorded choice, or fallback
void tune_forget();                                     // drop every recorded choice

struct Arena {
    char *base = nullptr;
    size_t off = 0, cap = 0;
    template <class T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        if (base == nullptr) {  // sizing pass
            off += bytes;
            return nullptr;
        }
        if (off + bytes > cap) throw Error(UOI_ENOMEM, "scratch arena overflow");
        T *p = reinterpret_cast<T *>(base + off);
        off += bytes;
        return p;
    }
};

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Device helpers.
// ---------------------------------------------------------------------------
typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

// D(16x16) += A(16x4) * B(4x16).  In both precisions lane l supplies A[l%16][l/16]
// and B[l/16][l%16].  The result layouts differ (measured on gfx950): in float64
// lane l holds D[l/16 + 4t][l%16] in element t, in float32 D[4*(l/16) + t][l%16].
__device__ __forceinline__ dx4 mfma16x16x4(double a, double b, dx4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fx4 mfma16x16x4(float a, float b, fx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row (within the 16x16 block) of element t of lane group lk = l/16.
__device__ __forceinline__ int mfma_row(double, int lk, int t) { return lk + 4 * t; }
__device__ __forceinline__ int mfma_row(float, int lk, int t) { return 4 * lk + t; }

// XCD-aware workgroup order.  The dispatcher deals linear workgroup ids to the 8
// XCDs round robin (id % 8), each XCD with its own L2.  xcd_remap turns the
// linear id into a logical id such that every XCD receives one contiguous range
// of logical ids (a bijection on [0, total) for any total).
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_remap(int L, int total) {
    const int q = total / kNumXcd, r = total % kNumXcd;
    const int x = L % kNumXcd, s = L / kNumXcd;
    return x * q + min(x, r) + s;
}

__device__ __forceinline__ double soft_threshold(double a, double t) {
    return a > t ? a - t : (a < -t ? a + t : 0.0);
}
__device__ __forceinline__ float soft_threshold(float a, float t) {
    return a > t ? a - t : (a < -t ? a + t : 0.0f);
}

// Max of non-negative doubles through their bit patterns (monotone for x >= 0).
__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(addr),
              (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------------------
// Counter-based index streams (SplitMix64 output function, Lemire range map).
// ---------------------------------------------------------------------------
enum : uint32_t { TAG_LASSO_BOOT = 1, TAG_LASSO_SPLIT = 2, TAG_VAR_BOOT = 3, TAG_VAR_SPLIT = 4 };

__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__host__ __device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint32_t tag, uint32_t k,
                                                        uint32_t i) {
    return splitmix64(splitmix64(seed ^ ((uint64_t)tag << 56)) ^ (((uint64_t)k << 32) | i));
}
__host__ __device__ __forceinline__ uint32_t range_map(uint64_t r, uint32_t m) {
#if defined(__HIP_DEVICE_COMPILE__)
    return (uint32_t)__umul64hi(r, (uint64_t)m);
#else
    return (uint32_t)(((unsigned __int128)r * m) >> 64);
#endif
}

inline int split_count(int n, int num, int den) { return (int)(((int64_t)n * num) / den); }
inline int var_block_len_default(int N) {
    int L = 1;
    while ((int64_t)L * L * L < (int64_t)N) ++L;
    return L;
}

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
// index streams
void launch_boot_rows(hipStream_t s, uint64_t seed, uint32_t tag_k0, int nb, int n, int32_t *rows);
void launch_var_boot_rows(hipStream_t s, uint64_t seed, int nb, int N, int L, int32_t *rows);
// Distinct rows of each sample (ascending) with their multiplicities: rows
// [nb][m] drawn from nsrc source rows -> out_rows/out_w [nb][nsrc] (first
// ndist[k] entries valid); cnt is [nb][nsrc] scratch.
void launch_distinct_rows(hipStream_t s, int nb, int nsrc, int m, const int32_t *rows, int32_t *cnt,
                          int32_t *out_rows, int32_t *out_w, int32_t *ndist);
void launch_split(hipStream_t s, uint64_t seed, uint32_t tag, int nb, int cnt, int ntrain,
                  uint8_t *is_train);
void launch_compact_rows(hipStream_t s, int nb, int cnt, const uint8_t *is_train, int ntrain,
                         int32_t *train, int32_t *eval);
void launch_expand_blocks(hipStream_t s, int nb, int nblk, int N, int L, const uint8_t *is_train,
                          int32_t *train, int32_t *eval, int32_t *ntr, int32_t *nev);

// Gram: G[b] = X_r'X_r/m (full symmetric storage), C[b] = X_r'Y_r/m; per-batch row
// counts may be given (mcount != nullptr) with row lists at stride m.  When pe < 32
// and ss != nullptr, ss[b][e] = sum_r Y[r][e]^2 / m comes out of the same product.
// part (part_bytes) holds the partial tiles of the split last round (see
// gram_part_bytes); with nullptr or too little room nothing is split.
void launch_gram_f64(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *mcount,
                     int p, const double *X, int ldx, int pe, const double *Y, int ldy,
                     double *G, double *C, double *ss = nullptr, int role = 0, void *part = nullptr,
                     size_t part_bytes = 0);
// Weighted form over distinct rows: G[b] = sum_r w[b][r] x_r x_r' / div (likewise
// C, ss), rows and weights at stride m, mcount[b] of them.  With w the draw
// multiplicities and div the number of draws this equals the Gram of the sample
// with repeated rows.
void launch_gram_f64_weighted(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *w,
                              const int32_t *mcount, int div, int p, const double *X, int ldx, int pe,
                              const double *Y, int ldy, double *G, double *C, double *ss = nullptr,
                              void *part = nullptr, size_t part_bytes = 0);
// Bytes of partial tiles a product of these sizes splits into on the current
// device (have_c: C is produced; role and weighted name the kernel instance).
size_t gram_part_bytes(int nb, int m, int p, int pe, bool have_c, int role, bool weighted);
// G[b][j][i] = G[b][i][j] for i > j (upper triangle from the lower one)
void launch_symmetrize(hipStream_t s, int nb, int p, double *G);
// sum of squares of Y columns over sampled rows / m:  ss[b*pe + e]
void launch_colsq(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *mcount,
                  int pe, const double *Y, int ldy, double *ss);
// Training-set statistics of nb disjoint training/evaluation splits of the n
// rows, from the evaluation statistics and one full-data product:
// nt_b G_T,b = X'X - ne_b G_E,b (likewise for C).  Counts are the scalars
// nt_c/ne_c, or per split from device arrays nt/ne when those are non-null.
// complement_work_bytes sizes the scratch the full-data product needs.
size_t complement_work_bytes(int n, int p, int pe);
void launch_train_from_eval(hipStream_t s, int nb, int n, int p, const double *X, int ldx, int pe,
                            const double *Y, int ldy, const double *GE, const double *CE,
                            int nt_c, int ne_c, const int32_t *nt, const int32_t *ne, double *GT,
                            double *CT, void *work);

// Batched inverse of G + rho I by blocked Gauss-Jordan sweeps (writes M, and
// its float32 copy M32 when given).
void spd_inverse_f64(hipStream_t s, int nb, int p, const double *G, double rho, double *M,
                     double *work, float *M32 = nullptr);
size_t spd_inverse_work_doubles(int nb, int p);

// Batched products Y_b = A_b V_b with an epilogue (see gemm_epilogues in admm.hip).
void launch_matmul_f64(hipStream_t s, int nb, int p, int R, const double *A, const double *V,
                       double *Y);

// ADMM state, batched FP64 / FP32 and plain.
// training pairs of the warm-start network from solved problems (admm.hip)
void warm_start_dataset(hipStream_t s, int nb, int p, int q, int pe, const double *c, const double *lam,
                        const double *z, float *X, float *T, double *cn);

// warm-start network (mlp.hip)
void mlp_forward(hipStream_t s, uoi_mlp *M, int n, const float *X);
float *mlp_input_buffer(uoi_mlp *M, int n);
const float *mlp_output(const uoi_mlp *M);
int mlp_dims(const uoi_mlp *M, int *n_in, int *n_out);

struct AdmmProblem {
    int nb;              // bootstraps
    int p;               // features
    int q;               // lambdas
    int pe;              // equations per bootstrap (1 for LASSO)
    int R;               // q * pe solves per bootstrap
    const double *G;     // [nb][p][p]
    const double *C;     // [nb][p][pe]
    const double *lam;   // device [q]
    double rho;
    double tol;
    int max_iter;
    int check_every;
    uoi_mlp *mlp;        // warm start by network (LASSO: pe == 1), or nullptr
    double relax;        // over-relaxation alpha (1 = plain scaled ADMM)
    bool no_alloc = false;  // no pinned memory, events or second stream (host waits instead)
    bool graphs = false;    // each chunk of ADMM iterations replayed as one captured graph
    bool tune = false;      // pick launch shapes with the autotuner (else recorded or default)
    int fn32 = 0, fn64 = 0; // column-tile widths of the products (set by admm_solve)
};

// Timing events of the current device, reused across calls (an event may be
// handed out again while its last record is still pending: recording it again
// simply replaces that record).
hipEvent_t event_take();
void event_give(hipEvent_t e);

// Timing of a fit: events are recorded as the work is queued and read only
// after the fit's final synchronisation (resolve), so measuring adds no host
// wait.  Spans write elapsed milliseconds to a float or add to a kernel record.
struct DeferredTiming {
    struct Span {
        hipEvent_t a, b;
        float *ms;       // elapsed time, or
        uoi_kstat *ks;   // accumulated kernel record
        double bytes, flops;
        int launches;
    };
    std::vector<Span> spans;
    std::vector<hipEvent_t> owned;
    hipEvent_t mark(hipStream_t s) {
        hipEvent_t e = event_take();  // pooled: creating events costs host time
        owned.push_back(e);
        UOI_HIP(hipEventRecord(e, s));
        return e;
    }
    void time(hipEvent_t a, hipEvent_t b, float *ms) { spans.push_back(Span{a, b, ms, nullptr, 0, 0, 0}); }
    void kernel(hipEvent_t a, hipEvent_t b, uoi_kstat *k, double bytes, double flops, int launches) {
        spans.push_back(Span{a, b, nullptr, k, bytes, flops, launches});
    }
    void resolve() {  // after the stream has synchronised
        for (const Span &sp : spans) {
            float ms = 0.f;
            UOI_HIP(hipEventElapsedTime(&ms, sp.a, sp.b));
            if (sp.ms) *sp.ms = ms;
            if (sp.ks) {
                sp.ks->ms += ms;
                sp.ks->bytes += sp.bytes;
                sp.ks->flops += sp.flops;
                sp.ks->launches += sp.launches;
            }
        }
        spans.clear();
    }
    ~DeferredTiming() {
        for (hipEvent_t e : owned) event_give(e);
    }
};

struct AdmmOut {
    double *z;           // [nb][p][R]   (feature-major state)
    double *u;           // [nb][p][R]
    int32_t *iters;      // [nb*R]
    double *kkt;         // [nb*R]
    int64_t unconverged; // set by admm_finish_stats once the stream has synchronised
    int max_iters;
    uoi_kstat *kstat;    // [UOI_KSTAT_N] accumulated when non-null (timing runs)
    int64_t warm_used;   // solves started from the network
    int *dstat;          // device: [0] unconverged solves, [1] largest iteration count
    DeferredTiming *dt = nullptr;  // where timing runs record their events (else resolved in place)
};
// Reads the counts that admm_solve left in out.dstat (after the caller's final
// synchronisation of the stream).
void admm_finish_stats(AdmmOut &out);

size_t admm_work_bytes(const AdmmProblem &P, int precision, int solver);
void admm_solve(hipStream_t s, const AdmmProblem &P, int precision, int solver, void *work,
                bool warm, AdmmOut &out, float *stage_ms);

// The batched LASSO solves of uoi_lasso_solve_batch (abi.hip).  With
// scratch_cap > 0, scratch() returns the caller's device buffer of that many
// bytes and nothing is allocated (the allocation-free entry point).
int solve_batch(int nb, int p, const double *G, const double *c, const uoi_opts *o, const double *z0,
                const double *u0, double *z_out, double *u_out, int32_t *iters, double *kkt,
                void *(*scratch)(), size_t scratch_cap);

// per-(b, e) ||c||_inf
void launch_cnorm(hipStream_t s, int nb, int p, int pe, const double *C, double *cn);

// supports: AND over bootstraps of (z != 0);  supp[r][W]
void launch_support_and(hipStream_t s, int nb, int p, int R, const double *z, uint64_t *supp);
// union of the R supports: writes its columns to gidx (increasing) and returns
// their number (synchronises); -1 when p > 65536
int launch_support_union(hipStream_t s, int R, int p, const uint64_t *supp, int *count, int32_t *gidx,
                         std::vector<int32_t> *sizes = nullptr);
// supports in the union's numbering (cs[R][ceil(cnt/64)]) and XU = X[:, gidx]
void launch_compact_design(hipStream_t s, int R, int p, int cnt, const uint64_t *supp, const int32_t *gidx,
                           uint64_t *cs, int n, const double *X, int ldx, double *XU);
// dst[0..p) = 0, dst[gidx[c]] = src[c]
void launch_scatter_cols(hipStream_t s, int p, int cnt, const int32_t *gidx, const double *src, double *dst);

// estimation
struct EstimProblem {
    int nb;                // B2
    int p, pe, q, R;
    const double *GT;      // [nb][p][p] training Grams
    const double *CT;      // [nb][p][pe]
    const double *GE;      // [nb][p][p] evaluation Grams
    const double *CE;      // [nb][p][pe]
    const double *sE;      // [nb][pe] mean squares of the responses on evaluation rows
    const uint64_t *supp;  // [R][W]
    int cg_max_iter;       // iteration cap of the conjugate-gradient refits
    // intercept (optional): training means [nb][p], [nb][pe]; mu [pe] receives the
    // average over splits of the chosen refits' intercepts ybar_T - xbar_T' b
    const double *xT = nullptr, *yT = nullptr;
    double *mu = nullptr;
    bool per_eq = false;   // one support index per (split, equation) instead of per split
};
size_t estim_work_bytes(const EstimProblem &E);
void estimate(hipStream_t s, const EstimProblem &E, void *work, double *beta_out, int32_t *jstar,
              double *losses_out, float *stage_ms, const std::vector<int32_t> *sizes, int *flags_host,
              DeferredTiming *dt = nullptr);

// lag order and intercept of UoI_VAR (center.hip)
void launch_colmeans(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *w,
                     const int32_t *mcount, int div, int P, const double *X, int ldx, int pe,
                     const double *Y, int ldy, double *xbar, double *ybar);
void launch_shift_stats(hipStream_t s, int nb, int P, int pe, double *G, double *C, double *ss,
                        const double *xm, const double *ym, const double *a, const double *b);
void launch_train_means(hipStream_t s, int nb, int P, int pe, int N, const double *xA, const double *yA,
                        const int32_t *nev, const double *xE, const double *yE, double *xT, double *yT);
void launch_var_reorder(hipStream_t s, int q, int p, int d, const uint64_t *supp_in, uint64_t *supp_out,
                        const double *beta, double *A);

// finite check of an array; sets *flag (device int) to 1 on NaN/Inf
void launch_finite_check(hipStream_t s, const double *x, size_t n, int *flag);

}  // namespace uoi
