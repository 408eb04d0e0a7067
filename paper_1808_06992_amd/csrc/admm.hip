// Batched LASSO-ADMM (Eq. (ADMM), Sec. II-E, in the scaled form of Boyd et al.
// 2011, Sec. 6.4) for every (bootstrap, lambda[, equation]) solve of the model
// selection step of Alg. 1 / Alg. 2.
//
// With M = (G + rho I)^{-1} and h = M c cached per bootstrap, one iteration is
//     x = h + rho * M (z - u)          (x-minimisation)
//     z = S_{lambda/rho}(x + u)        (z-minimisation: soft threshold)
//     u = u + x - z                    (dual update)
// All solves of one bootstrap share M, so the x-update of all of them is one
// matrix product M [v_1 .. v_R] (v = z - u): the batched solver runs it on
// MFMA with the threshold and dual update fused into its epilogue.  State is
// feature-major ([bootstrap][feature][solve]) so that a K-step of the product
// reads 16 consecutive solves of one feature row.
//
// Convergence is the relative KKT residual of the LASSO (evaluated in float64
// with the float64 Gram) every `check_every` iterations; a solve that meets the
// tolerance is frozen (its z is the verified iterate) and a tile whose solves
// are all frozen skips its work.  The float32 phase of the mixed path parks
// solves on a KKT estimate that its iteration yields without a product; every
// parked solve is then verified (and finished if needed) in float64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "bgemm.hpp"
#include "common.hpp"

namespace uoi {

// --- epilogue: plain store --------------------------------------------------
template <typename T, int FM, int FN>
struct StoreEpi {
    T *Y;
    int p, R;
    __device__ bool tile_active(int, int, int) const { return true; }
    template <class Acc>
    __device__ void apply(int b, int i_base, int r0, int lr, int lk, Acc (&acc)[FM][FN]) const {
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int c = 0; c < FN; ++c)
                for (int t = 0; t < 4; ++t) {
                    int i = i_base + 16 * a + mfma_row(T(0), lk, t), r = r0 + 16 * c + lr;
                    if (i < p && r < R) Y[((size_t)b * p + i) * R + r] = (T)acc[a][c][t];
                }
    }
};

// --- epilogue: ADMM iteration ----------------------------------------------
// x = h + rho*acc (acc = M v), z = S(x + u, lam/rho), u += x - z, v' = z - u.
template <typename T, int FM, int FN>
struct AdmmEpi {
    const T *h;          // [nb][p][pe]
    T *z, *u, *vout;     // [nb][p][R]
    const uint8_t *state;// [nb][R] 0 = active
    const double *lam;   // [q]
    int p, R, pe;
    T rho, inv_rho, alpha;  // alpha: over-relaxation (1 = none)
    __device__ bool tile_active(int b, int r0, int w) const {
        // one state byte per lane (w <= 64), combined by a ballot: the same answer
        // in every wave of the workgroup
        const int lane = threadIdx.x & 63, r = r0 + lane;
        const bool a = lane < w && r < R && state[(size_t)b * R + min(r, R - 1)] == 0;
        return __ballot(a) != 0ull;
    }
    template <class Acc>
    __device__ void apply(int b, int i_base, int r0, int lr, int lk, Acc (&acc)[FM][FN]) const {
        // All loads of the tile first, unconditionally from clamped (valid)
        // addresses, so that they are in flight together; the state masks only the
        // stores.  Then the threshold / dual update and the stores.
        T hv[FN][FM][4], uv[FN][FM][4], zv[FN][FM][4], thr[FN];
        const bool relaxed = alpha != T(1);
        bool act[FN];
        int rc[FN];
#pragma unroll
        for (int c = 0; c < FN; ++c) {
            const int r = r0 + 16 * c + lr;
            rc[c] = min(r, R - 1);
            act[c] = r < R && state[(size_t)b * R + rc[c]] == 0;
            thr[c] = (T)lam[rc[c] / pe] * inv_rho;
        }
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int ic = min(i_base + 16 * a + mfma_row(T(0), lk, t), p - 1);
#pragma unroll
                for (int c = 0; c < FN; ++c) {
                    const size_t o = ((size_t)b * p + ic) * R + rc[c];
                    uv[c][a][t] = u[o];
                    zv[c][a][t] = relaxed ? z[o] : T(0);
                    hv[c][a][t] = h[((size_t)b * p + ic) * pe + rc[c] % pe];
                }
            }
#pragma unroll
        for (int c = 0; c < FN; ++c) {
            if (!act[c]) continue;
            const int r = r0 + 16 * c + lr;
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int i = i_base + 16 * a + mfma_row(T(0), lk, t);
                    if (i >= p) continue;
                    const size_t o = ((size_t)b * p + i) * R + r;
                    // explicit fused multiply-adds: every instance of the epilogue
                    // rounds the same way, whatever the compiler's contraction choices
                    T x = fma(rho, (T)acc[a][c][t], hv[c][a][t]);
                    if (relaxed) x = fma(alpha, x, (T(1) - alpha) * zv[c][a][t]);
                    const T uo = uv[c][a][t];
                    const T zn = soft_threshold(x + uo, thr[c]);
                    const T un = uo + x - zn;
                    z[o] = zn;
                    u[o] = un;
                    vout[o] = zn - un;
                }
        }
    }
};

// The same iteration in float32 for the split-bfloat16 product: v' = z - u is
// written as the three bfloat16 planes Vp[b][part][r][i] (parts as in
// split_bf16x3; rows i >= p are never written and stay zero).  A lane holds four
// consecutive rows i of one column r, so each part is one 8-byte store.
//
// With vmax set (the last iteration before a check), the iteration also leaves
// a KKT estimate per solve without a product by G: the x-update solves
// (G + rho I) x = c + rho (z - u), so the gradient at x is
//     c - G x = rho (x - z + u)          (z, u before the update)
// and the KKT violation is evaluated with that gradient at the new z (its
// support and signs).  Each entry of the violation is 1-Lipschitz in the
// gradient, and the gradient at z differs from the one at x by G (x - z), so
//     KKT(z) <= max_j v_j + ||G||_inf ||x - z||_inf.
// The epilogue leaves the two maxima per solve (vmax, rmax) and the freeze step
// combines them with ||G||_inf of the bootstrap (weighted, kResidualWeight).
// The float32 phase uses the estimate only to park solves; the float64 phase
// decides convergence with the exact residual.
template <int FN>
struct AdmmEpiBf3 {
    const float *h;      // [nb][p][pe]
    float *z, *u;        // [nb][p][R]
    __bf16 *vp;          // [nb][3][R][ldk]
    const uint8_t *state;
    const double *lam;
    int p, R, pe, ldk;
    float rho, inv_rho, alpha;
    double *vmax;        // [nb][R] per-solve maximum of v (atomic), or null
    double *rmax;        // [nb][R] per-solve maximum of |x - z| (atomic)
    __device__ bool tile_active(int b, int r0, int w) const {
        const int lane = threadIdx.x & 63, r = r0 + lane;
        const bool a = lane < w && r < R && state[(size_t)b * R + min(r, R - 1)] == 0;
        return __ballot(a) != 0ull;
    }
    template <class Acc>
    __device__ void apply(int b, int i_base, int r0, int lr, int lk, Acc (&acc)[1][FN]) const {
        float hv[FN][4], uv[FN][4], zv[FN][4], thr[FN];
        const bool relaxed = alpha != 1.0f;
        bool act[FN];
        int rc[FN];
#pragma unroll
        for (int c = 0; c < FN; ++c) {
            const int r = r0 + 16 * c + lr;
            rc[c] = min(r, R - 1);
            act[c] = r < R && state[(size_t)b * R + rc[c]] == 0;
            thr[c] = (float)lam[rc[c] / pe] * inv_rho;
        }
        const int i4 = i_base + 4 * lk;  // rows i4 .. i4 + 3 of this lane
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ic = min(i4 + t, p - 1);
#pragma unroll
            for (int c = 0; c < FN; ++c) {
                const size_t o = ((size_t)b * p + ic) * R + rc[c];
                uv[c][t] = u[o];
                zv[c][t] = relaxed || vmax ? z[o] : 0.0f;
                hv[c][t] = h[((size_t)b * p + ic) * pe + rc[c] % pe];
            }
        }
        const size_t plane = (size_t)R * ldk;
#pragma unroll
        for (int c = 0; c < FN; ++c) {
            if (!act[c]) continue;
            const int r = r0 + 16 * c + lr;
            float vv[4], kv = 0.0f, rv = 0.0f;
            const float lamf = thr[c] * rho;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = i4 + t;
                // explicit fused multiply-adds (the same rounding in every instance)
                const float x0 = fmaf(rho, acc[0][c][t], hv[c][t]);
                const float x = relaxed ? fmaf(alpha, x0, (1.0f - alpha) * zv[c][t]) : x0;
                const float uo = uv[c][t];
                const float zn = soft_threshold(x + uo, thr[c]);
                const float un = uo + x - zn;
                vv[t] = zn - un;
                if (i < p) {
                    const size_t o = ((size_t)b * p + i) * R + r;
                    z[o] = zn;
                    u[o] = un;
                    if (vmax) {
                        const float g = rho * (x0 - zv[c][t] + uo);
                        const float v = zn != 0.0f ? fabsf(g - (zn > 0.0f ? lamf : -lamf))
                                                   : fmaxf(0.0f, fabsf(g) - lamf);
                        kv = fmaxf(kv, v);
                        rv = fmaxf(rv, fabsf(x0 - zn));
                    }
                }
            }
            if (vmax) {
                // lanes lr, lr+16, lr+32, lr+48 hold the same solve
                kv = fmaxf(kv, __shfl_xor(kv, 16));
                kv = fmaxf(kv, __shfl_xor(kv, 32));
                rv = fmaxf(rv, __shfl_xor(rv, 16));
                rv = fmaxf(rv, __shfl_xor(rv, 32));
                if (lk == 0 && kv > 0.0f) atomic_max_nonneg(&vmax[(size_t)b * R + r], (double)kv);
                if (lk == 0 && rv > 0.0f) atomic_max_nonneg(&rmax[(size_t)b * R + r], (double)rv);
            }
            __bf16 *dst = vp + (size_t)b * 3 * plane + (size_t)r * ldk + i4;
            if (i4 + 3 < p) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    typedef __bf16 bfx4 __attribute__((ext_vector_type(4)));
                    bfx4 w;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const __bf16 a1 = (__bf16)vv[t];
                        const float r1 = vv[t] - (float)a1;
                        const __bf16 a2 = (__bf16)r1;
                        w[t] = q == 0 ? a1 : (q == 1 ? a2 : (__bf16)(r1 - (float)a2));
                    }
                    *(bfx4 *)(dst + q * plane) = w;
                }
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (i4 + t < p) {
                        const __bf16 a1 = (__bf16)vv[t];
                        const float r1 = vv[t] - (float)a1;
                        const __bf16 a2 = (__bf16)r1;
                        dst[t] = a1;
                        dst[plane + t] = a2;
                        dst[2 * plane + t] = (__bf16)(r1 - (float)a2);
                    }
            }
        }
    }
};

// --- epilogue: KKT residual --------------------------------------------------
// acc = (G z)_i; g = c_i - acc; v_i as in the KKT definition; per-solve max over
// i is reduced in the wave and then with an atomic max on the bit pattern.
template <typename T, int FM, int FN>
struct KktEpi {
    const double *C;     // [nb][p][pe]
    const T *z;          // [nb][p][R]
    const uint8_t *state;
    const double *lam;
    double *vmax;        // [nb][R]  (zeroed before the launch)
    int p, R, pe;
    bool only_active;
    __device__ bool tile_active(int b, int r0, int w) const {
        if (!only_active) return true;
        const int lane = threadIdx.x & 63, r = r0 + lane;
        const bool a = lane < w && r < R && state[(size_t)b * R + min(r, R - 1)] == 0;
        return __ballot(a) != 0ull;
    }
    template <class Acc>
    __device__ void apply(int b, int i_base, int r0, int lr, int lk, Acc (&acc)[FM][FN]) const {
        // loads first, unconditionally from clamped addresses (see AdmmEpi)
        double cv[FN][FM][4], zv[FN][FM][4], lm[FN];
        bool rok[FN];
#pragma unroll
        for (int c = 0; c < FN; ++c) {
            const int r = r0 + 16 * c + lr;
            const int rc = min(r, R - 1);
            rok[c] = r < R && !(only_active && state[(size_t)b * R + rc] != 0);
            lm[c] = lam[rc / pe];
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int ic = min(i_base + 16 * a + mfma_row(T(0), lk, t), p - 1);
                    cv[c][a][t] = C[((size_t)b * p + ic) * pe + rc % pe];
                    zv[c][a][t] = (double)z[((size_t)b * p + ic) * R + rc];
                }
        }
#pragma unroll
        for (int c = 0; c < FN; ++c) {
            const int r = r0 + 16 * c + lr;
            double m = 0.0;
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int i = i_base + 16 * a + mfma_row(T(0), lk, t);
                    if (!rok[c] || i >= p) continue;
                    const double g = cv[c][a][t] - (double)acc[a][c][t];
                    const double zi = zv[c][a][t];
                    const double v = zi != 0.0 ? fabs(g - (zi > 0 ? lm[c] : -lm[c])) : fmax(0.0, fabs(g) - lm[c]);
                    m = fmax(m, v);
                }
            // lanes lr, lr+16, lr+32, lr+48 hold the same solve
            m = fmax(m, __shfl_xor(m, 16));
            m = fmax(m, __shfl_xor(m, 32));
            if (rok[c] && lk == 0 && m > 0.0) atomic_max_nonneg(&vmax[(size_t)b * R + r], m);
        }
    }
};

// For the float64 path the Gram product reads z directly; a float32 z is fed to
// the float64 product through this converted copy.
__global__ void k_f32_to_f64(size_t n, const float *__restrict__ a, double *__restrict__ b) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}
__global__ void k_f64_to_f32(size_t n, const double *__restrict__ a, float *__restrict__ b) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// per-(b, e) ||c||_inf.  Block (64 columns e) x (4 row groups); with one column
// all 256 threads share the rows.  Eight rows are loaded per step.
__global__ __launch_bounds__(256) void k_cnorm(int p, int pe, const double *__restrict__ C,
                                               double *__restrict__ cn) {
    __shared__ double red[4][64];
    const int b = blockIdx.y;
    const double *Cb = C + (size_t)b * p * pe;
    if (pe == 1) {
        double m = 0.0;
        for (int i0 = threadIdx.x; i0 < p; i0 += 2048) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = Cb[min(i0 + 256 * u, p - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u) m = fmax(m, fabs(v[u]));  // clamped repeats do not change a max
        }
        m = wave_max(m);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][0] = m;
        __syncthreads();
        if (threadIdx.x == 0)
            cn[b] = fmax(fmax(red[0][0], red[1][0]), fmax(red[2][0], red[3][0]));
        return;
    }
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int e = min(blockIdx.x * 64 + tx, pe - 1);
    double m = 0.0;
    for (int i0 = ty; i0 < p; i0 += 32) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = Cb[(size_t)min(i0 + 4 * u, p - 1) * pe + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) m = fmax(m, fabs(v[u]));
    }
    red[ty][tx] = m;
    __syncthreads();
    if (ty == 0 && blockIdx.x * 64 + tx < pe)
        cn[(size_t)b * pe + blockIdx.x * 64 + tx] = fmax(fmax(red[0][tx], red[1][tx]), fmax(red[2][tx], red[3][tx]));
}

// After a KKT evaluation: freeze solves that meet the tolerance.
// state: 0 active, 1 converged, 2 parked (waits for float64): a float32 solve is
// parked when it meets park_tol, or when it is within stall_tol but its KKT
// residual fell by less than kStallRatio since the previous check (it has
// reached what float32 arithmetic resolves).  kkt[] holds the previous value
// (initialised to a huge number).  iters[] is -1 while a solve is active, -(it+2)
// once it has been parked at iteration it (kept while it is finished in
// float64), and its iteration count once converged.
constexpr double kStallRatio = 0.7;
constexpr double kParkFactor = 5.0;
constexpr double kStallFactor = 30.0;
// The float32 iteration's KKT estimate levels off at the resolution of its
// float32 state (about 3e-8 to 1e-6 relative, depending on |beta| / ||c||_inf),
// so the parking window never goes below these floors: with a tolerance under
// them, solves park at the float32 resolution and the float64 finish carries
// them the rest of the way.  At tolerances of 1e-7 and above the factors rule.
constexpr double kParkFloor = 5e-7;
constexpr double kStallFloor = 3e-5;
// Float64 finish: the length of its first chunk.  Solves parked at 5x the
// tolerance mostly converge within 3 float64 iterations; the later chunks have
// the usual length (2 / 3 / 4 / 10 gave 4.6 / 3.5 / 3.6 / 4.4 ms for the LASSO
// fit's ADMM stage; shorter later chunks slow the long float64 phase of the VAR
// fit).
constexpr int kFinishFirst = 3;
// The float64 finish starts without a check: nearly every bootstrap holds some
// parked solve above the tolerance, so its tile runs anyway, and the check after
// the first chunk decides all of them (0.1 ms less than checking first).
constexpr bool kFinishFirstCheck = false;
// Weight of ||G||_inf ||x - z||_inf in the float32 KKT estimate.  1 gives a
// strict bound, which float32 rounding of x - z keeps above the parking
// threshold for some solves; G (x - z) is far below that worst case in
// practice.  Over 0.05 - 0.3 the LASSO fit was fastest at 0.05 - 0.1 and the
// slowly converging VAR fit at 0.2 - 0.3; without the term (0) the VAR fit
// parks too early and was 40 % slower.
constexpr double kResidualWeight = 0.1;
__global__ void k_freeze(int nb, int R, int pe, double *__restrict__ vmax, double *__restrict__ rmax,
                         const double *__restrict__ gn, const double *__restrict__ zlam,
                         const double *__restrict__ cn, double tol, double park_tol,
                         double stall_tol, int it, int it_base, uint8_t *__restrict__ state,
                         int32_t *__restrict__ iters, double *__restrict__ kkt,
                         int *__restrict__ active, int *__restrict__ active_next) {
    // active[0] = all solves still active, active[1 + b] = those of bootstrap b;
    // the next check's counters and maxima are cleared here, so that no fill
    // kernel is needed between checks
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = s; i < 1 + nb; i += gridDim.x * blockDim.x) active_next[i] = 0;
    bool act = false;
    if (s < nb * R) {
        int b = s / R, r = s % R;
        // an estimate with its residual term (rmax is zero after an exact
        // evaluation); at z = 0 (zlam given) the gradient is c itself, so the
        // residual is max(0, ||c||_inf - lambda) with no product
        const double c = cn[(size_t)b * pe + r % pe];
        const double vm = zlam ? fmax(0.0, c - zlam[r / pe])
                               : vmax[s] + (gn ? kResidualWeight * gn[b] * rmax[s] : 0.0);
        vmax[s] = 0.0;
        rmax[s] = 0.0;
        if (state[s] == 0) {
            double rel = c > 0.0 ? vm / c : vm;
            const double prev = kkt[s];
            kkt[s] = rel;
            const int32_t ip = iters[s];
            if (rel <= tol) {
                // a parked solve counts the iterations up to its parking and those
                // of this sweep (which began at it_base)
                state[s] = 1;
                iters[s] = ip <= -2 ? -ip - 2 + (it - it_base) : it;
            } else if (rel <= park_tol || (rel <= stall_tol && rel > kStallRatio * prev)) {
                state[s] = 2;
                if (ip == -1) iters[s] = -it - 2;  // provisional, still counted as unconverged
            } else {
                act = true;
                atomicAdd(&active[1 + b], 1);
            }
        }
    }
    unsigned long long bal = __ballot(act);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(active, __popcll(bal));
}

__global__ void k_fill_i32(size_t n, int32_t v, int32_t *__restrict__ a) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// stat[0] += solves with a negative (unconverged) count, stat[1] = max count;
// an unconverged count (-1 active, -(it+2) parked) is reported as -1
__global__ void k_iter_stats(int n, int32_t *__restrict__ its, int *__restrict__ stat) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = i < n ? its[i] : 0;
    if (i < n && v < -1) its[i] = -1;
    const unsigned long long bal = __ballot(i < n && v < 0);
    int m = v > 0 ? v : 0;
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) {
        if (bal) atomicAdd(&stat[0], __popcll(bal));
        if (m > 0) atomicMax(&stat[1], m);
    }
}

template <typename T>
__global__ void k_init_state(size_t n, const T *__restrict__ z0, const T *__restrict__ u0,
                             T *__restrict__ z, T *__restrict__ u, T *__restrict__ v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        T a = z0 ? z0[i] : T(0), c = u0 ? u0[i] : T(0);
        z[i] = a;
        u[i] = c;
        v[i] = a - c;
    }
}

// v = z - u after a precision change or a restart
template <typename T>
__global__ void k_refresh_v(size_t n, const T *__restrict__ z, const T *__restrict__ u,
                            T *__restrict__ v0, T *__restrict__ v1) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        T d = z[i] - u[i];
        v0[i] = d;
        v1[i] = d;
    }
}

// v = z - u as the bfloat16 planes of the split product, in both buffers
__global__ void k_refresh_vp(int nb, int p, int R, int ldk, const float *__restrict__ z,
                             const float *__restrict__ u, __bf16 *__restrict__ v0,
                             __bf16 *__restrict__ v1) {
    const size_t n = (size_t)nb * R * p;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int i = (int)(e % p);  // row fastest: the plane stores are contiguous
    const size_t br = e / p;
    const int r = (int)(br % R), b = (int)(br / R);
    const size_t o = ((size_t)b * p + i) * R + r;
    const float d = z[o] - u[o];
    const __bf16 a1 = (__bf16)d;
    const float r1 = d - (float)a1;
    const __bf16 a2 = (__bf16)r1;
    const __bf16 a3 = (__bf16)(r1 - (float)a2);
    const size_t plane = (size_t)R * ldk;
    const size_t q = (size_t)b * 3 * plane + (size_t)r * ldk + i;
    v0[q] = a1; v0[q + plane] = a2; v0[q + 2 * plane] = a3;
    v1[q] = a1; v1[q + plane] = a2; v1[q + 2 * plane] = a3;
}

__global__ void k_unpark(size_t n, uint8_t *__restrict__ state) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && state[i] == 2) state[i] = 0;
}

// ---------------------------------------------------------------------------
// Warm start by the network (LASSO, one response): inputs, prediction, dual
// completion and the per-solve fallback to the cold start.
// ---------------------------------------------------------------------------
// Row (b q + j) pe + e of the network input for response column e of bootstrap b
// at lambda_j:  X[row][0..p) = c_{b,e} / lambda_max_{b,e}, X[row][p] =
// log(lambda_j / lambda_max_{b,e}), with lambda_max_{b,e} = ||c_{b,e}||_inf.
__global__ void k_ws_inputs(int nb, int p, int q, int pe, const double *__restrict__ c,
                            const double *__restrict__ cn, const double *__restrict__ lam,
                            float *__restrict__ X) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t rowlen = (size_t)p + 1;
    if (t >= (size_t)nb * q * pe * rowlen) return;
    const size_t row = t / rowlen;
    const int i = (int)(t % rowlen);
    const int e = (int)(row % pe);
    const size_t bj = row / pe;
    const int b = (int)(bj / q), j = (int)(bj % q);
    const double lm = cn[(size_t)b * pe + e] > 0.0 ? cn[(size_t)b * pe + e] : 1.0;
    double v;
    if (i < p) v = c[((size_t)b * p + i) * pe + e] / lm;
    else v = log(fmax(lam[j], 1e-300) / lm);
    X[t] = (float)v;
}

// z[b][i][j] = S_{theta lambda_j}(Y[(b q + j)][i] * lambda_max_b): the prediction,
// shrunk by theta times the penalty (the regression leaves small values on
// coordinates whose solution is zero).  theta = 1 (kWarmShrink) raised the share
// of accepted starts at p = 200 from 77 % to 88 % and the iterations saved per
// solve from 1.5 to 1.9 (exact counts, KKT 1e-8); 0.1 - 2 were tried.
constexpr double kWarmShrink = 1.0;
__global__ void k_ws_z0(int nb, int p, int q, const float *__restrict__ Y, const double *__restrict__ cn,
                        const double *__restrict__ lam, double theta, double *__restrict__ z) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nb * p * q) return;
    const int j = (int)(t % q);
    const size_t bi = t / q;
    const int i = (int)(bi % p), b = (int)(bi / p);
    z[t] = soft_threshold((double)Y[((size_t)b * q + j) * p + i] * cn[b], theta * lam[j]);
}

// Per solve (b, j): with g = c - G z0, u0 = clip(g/rho, +-lambda/rho).
// The prediction is kept only if it lowers the LASSO objective below that of
// the cold start, F(z) = z'Gz/2 - c'z + lambda |z|_1 with F(0) = 0 (a dense
// prediction violates the KKT conditions on every coordinate that should be
// zero, so the KKT residual is not a fair test of a starting point).
// One workgroup per bootstrap: thread (g, j) of a (256/qj) x qj grid sums the
// coordinates i = g mod (256/qj) of solve j (consecutive threads read
// consecutive solves of a feature row), the partial sums meet in LDS, and the
// same grid then writes u0 or the cold start.
__global__ __launch_bounds__(256) void k_ws_finish(int nb, int p, int q, const double *__restrict__ c,
                                                   const double *__restrict__ Gz,
                                                   const double *__restrict__ lam, double rho,
                                                   double *__restrict__ z, double *__restrict__ u,
                                                   unsigned long long *__restrict__ used) {
    __shared__ double part[256];
    __shared__ int keep[256];
    const int b = blockIdx.x, t = threadIdx.x;
    for (int j0 = 0; j0 < q; j0 += 256) {
        const int qj = min(256, q - j0), G = 256 / qj;
        const int jj = t % qj, g = t / qj, j = j0 + jj;
        const double lm = lam[j];
        double F = 0.0;
        if (g < G)
            for (int i = g; i < p; i += G) {
                const size_t o = ((size_t)b * p + i) * q + j;
                const double zi = z[o];
                F += zi * (0.5 * Gz[o] - c[(size_t)b * p + i]) + lm * fabs(zi);
            }
        part[t] = F;
        __syncthreads();
        if (t < qj) {
            double tot = 0.0;
            for (int h = 0; h < G; ++h) tot += part[h * qj + t];
            keep[t] = tot < 0.0;
        }
        __syncthreads();
        const bool use = keep[jj] != 0;
        if (g < G)
            for (int i = g; i < p; i += G) {
                const size_t o = ((size_t)b * p + i) * q + j;
                if (use) {
                    const double gi = c[(size_t)b * p + i] - Gz[o];
                    u[o] = fmin(fmax(gi / rho, -lm / rho), lm / rho);
                } else {
                    z[o] = 0.0;
                    u[o] = 0.0;
                }
            }
        const unsigned long long bal = __ballot(t < qj && keep[min(t, qj - 1)] != 0);
        if ((t & 63) == 0 && bal) atomicAdd(used, (unsigned long long)__popcll(bal));
        __syncthreads();
    }
}

// Training pairs from solved problems: inputs as k_ws_inputs; targets
// T[row][i] = z[b][j][e][i] / lambda_max_{b,e} (z solve-major, row = (b q + j) pe + e).
__global__ void k_ws_targets(int nb, int p, int q, int pe, const double *__restrict__ cn,
                             const double *__restrict__ z, float *__restrict__ T) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nb * q * pe * p) return;
    const size_t row = t / p;
    const int e = (int)(row % pe);
    const int b = (int)(row / ((size_t)q * pe));
    const double lm = cn[(size_t)b * pe + e] > 0.0 ? cn[(size_t)b * pe + e] : 1.0;
    T[t] = (float)(z[t] / lm);
}

void warm_start_dataset(hipStream_t s, int nb, int p, int q, int pe, const double *c, const double *lam,
                        const double *z, float *X, float *T, double *cn) {
    launch_cnorm(s, nb, p, pe, c, cn);
    size_t nx = (size_t)nb * q * pe * (p + 1), nt = (size_t)nb * q * pe * p;
    hipLaunchKernelGGL(k_ws_inputs, dim3(cdiv(nx, 256)), dim3(256), 0, s, nb, p, q, pe, c, cn, lam, X);
    hipLaunchKernelGGL(k_ws_targets, dim3(cdiv(nt, 256)), dim3(256), 0, s, nb, p, q, pe, cn, z, T);
    UOI_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Plain solver: one workgroup runs one whole solve with matrix-vector products
// (the per-solve organisation of the paper's distributed ADMM, here without
// row sharding).  z, u, v live in LDS; M and G are streamed every iteration.
// ---------------------------------------------------------------------------
constexpr int PLAIN_MAX_ROWS = 16;  // p <= 256 * 16

__global__ __launch_bounds__(256) void k_admm_plain(int p, int pe, int R, const double *__restrict__ M,
                                                    const double *__restrict__ h,
                                                    const double *__restrict__ G,
                                                    const double *__restrict__ C,
                                                    const double *__restrict__ lam,
                                                    const double *__restrict__ cn, double rho,
                                                    double alpha, double tol, int max_iter, int check_every,
                                                    double *__restrict__ zout,
                                                    double *__restrict__ uout,
                                                    int32_t *__restrict__ iters,
                                                    double *__restrict__ kkt) {
    extern __shared__ double sm[];
    double *v = sm, *z = sm + p, *u = sm + 2 * p;
    __shared__ double red[4];
    __shared__ int done_s;
    const int s = blockIdx.x;
    const int b = s / R, r = s % R, e = r % pe;
    const double lm = lam[r / pe], thr = lm / rho;
    const double cnorm = cn[(size_t)b * pe + e];
    const double *Mb = M + (size_t)b * p * p;
    const double *Gb = G + (size_t)b * p * p;
    const int tid = threadIdx.x;
    for (int i = tid; i < p; i += 256) {
        z[i] = zout[((size_t)b * p + i) * R + r];
        u[i] = uout[((size_t)b * p + i) * R + r];
        v[i] = z[i] - u[i];
    }
    __syncthreads();
    int it = 0, status = -1;
    double rel = 0.0;
    for (;;) {
        if (it % check_every == 0 || it == max_iter) {
            // KKT: g = c - G z
            double m = 0.0;
            for (int i = tid; i < p; i += 256) {
                double acc = 0.0;
                for (int k = 0; k < p; ++k) acc += Gb[(size_t)k * p + i] * z[k];
                double g = C[((size_t)b * p + i) * pe + e] - acc;
                double zi = z[i];
                double vv = zi != 0.0 ? fabs(g - (zi > 0 ? lm : -lm)) : fmax(0.0, fabs(g) - lm);
                m = fmax(m, vv);
            }
            m = wave_max(m);
            if ((tid & 63) == 0) red[tid >> 6] = m;
            __syncthreads();
            if (tid == 0) {
                double mm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
                rel = cnorm > 0.0 ? mm / cnorm : mm;
                red[0] = rel;
                done_s = (rel <= tol) ? 1 : (it >= max_iter ? 2 : 0);
            }
            __syncthreads();
            rel = red[0];
            if (done_s) {
                status = done_s == 1 ? it : -1;
                break;
            }
            __syncthreads();
        }
        // x = h + rho M v for my rows, then the threshold and dual update
        double xr[PLAIN_MAX_ROWS];
        int nr = 0;
        for (int i = tid; i < p; i += 256, ++nr) {
            double acc = 0.0;
            for (int k = 0; k < p; ++k) acc += Mb[(size_t)k * p + i] * v[k];
            xr[nr] = h[((size_t)b * p + i) * pe + e] + rho * acc;
        }
        __syncthreads();
        nr = 0;
        for (int i = tid; i < p; i += 256, ++nr) {
            const double xh = alpha * xr[nr] + (1.0 - alpha) * z[i];
            double zn = soft_threshold(xh + u[i], thr);
            double un = u[i] + xh - zn;
            z[i] = zn;
            u[i] = un;
            v[i] = zn - un;
        }
        __syncthreads();
        ++it;
    }
    for (int i = tid; i < p; i += 256) {
        zout[((size_t)b * p + i) * R + r] = z[i];
        uout[((size_t)b * p + i) * R + r] = u[i];
    }
    if (tid == 0) {
        iters[s] = status;
        kkt[s] = rel;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
void launch_matmul_f64(hipStream_t s, int nb, int p, int R, const double *A, const double *V,
                       double *Y) {
    UOI_DISPATCH_FN(R, {
        StoreEpi<double, 1, FN> epi{Y, p, R};
        run_bgemm<double, 1, FN>(s, nb, p, R, A, V, epi);
    });
}

void launch_cnorm(hipStream_t s, int nb, int p, int pe, const double *C, double *cn) {
    hipLaunchKernelGGL(k_cnorm, dim3(cdiv(pe, 64), nb), dim3(256), 0, s, p, pe, C, cn);
    UOI_LAUNCH_CHECK();
}

// gn[b] = ||G_b||_inf = max_j sum_i |G_b[i][j]| (G symmetric: the largest
// absolute column sum).  Block: 64 columns x 4 row groups; the per-block maximum
// goes to gn[b] by an atomic maximum (gn zeroed before).
__global__ __launch_bounds__(256) void k_gnorm(int p, const double *__restrict__ G,
                                               double *__restrict__ gn) {
    __shared__ double red[4][64];
    const int b = blockIdx.y;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + tx, jc = min(j, p - 1);
    const double *Gb = G + (size_t)b * p * p;
    double sum = 0.0;
    for (int i0 = ty; i0 < p; i0 += 32) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = Gb[(size_t)min(i0 + 4 * u, p - 1) * p + jc];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + 4 * u < p) sum += fabs(v[u]);
    }
    red[ty][tx] = sum;
    __syncthreads();
    if (ty == 0) {
        double m = j < p ? red[0][tx] + red[1][tx] + red[2][tx] + red[3][tx] : 0.0;
        m = wave_max(m);
        if (tx == 0) atomic_max_nonneg(&gn[b], m);
    }
}

namespace {
struct AdmmWork {
    double *M, *h, *cn, *vmax, *rmax, *gn;
    uint8_t *state;
    int *active;
    int *stat;  // [0] unconverged solves, [1] largest iteration count
    // float64 iteration buffers
    double *v0, *v1;
    // float32 phase
    float *M32, *h32, *z32, *u32;
    __bf16 *vp0, *vp1;  // float32 phase: v as bfloat16 planes [nb][3][R][ldk]
    int fm32, fm64;     // row blocks per wave of the float32 / float64 products (1 or 2)
    double *z64tmp;
};

// Products with more than one column tile may take two row blocks per wave,
// float32 and float64 alike (the autotuner times both).
inline bool offer_fm2(const AdmmProblem &P) { return P.R > 64 && P.p > 64; }

AdmmWork carve(const AdmmProblem &P, int precision, int solver, Arena &ar) {
    AdmmWork w{};
    w.fm32 = w.fm64 = 1;
    size_t np2 = (size_t)P.nb * P.p * P.p, nst = (size_t)P.nb * P.p * P.R;
    w.M = ar.take<double>(np2);
    w.h = ar.take<double>((size_t)P.nb * P.p * P.pe);
    w.cn = ar.take<double>((size_t)P.nb * P.pe);
    w.vmax = ar.take<double>((size_t)P.nb * P.R);
    w.rmax = ar.take<double>((size_t)P.nb * P.R);
    w.gn = ar.take<double>(P.nb);
    w.state = ar.take<uint8_t>((size_t)P.nb * P.R);
    w.active = ar.take<int>(2 * (1 + P.nb));  // two sets of counters, alternating per check
    w.stat = ar.take<int>(2);
    if (solver == UOI_SOLVER_BATCHED) {
        w.v0 = ar.take<double>(nst);
        w.v1 = ar.take<double>(nst);
        if (precision == UOI_MIXED) {
            w.M32 = ar.take<float>(np2);
            w.h32 = ar.take<float>((size_t)P.nb * P.p * P.pe);
            w.z32 = ar.take<float>(nst);
            w.u32 = ar.take<float>(nst);
            const size_t np3 = (size_t)P.nb * 3 * P.R * bf3_ldk(P.p);
            w.vp0 = ar.take<__bf16>(np3);
            w.vp1 = ar.take<__bf16>(np3);
        }
    }
    return w;
}
}  // namespace

size_t admm_work_bytes(const AdmmProblem &P, int precision, int solver) {
    Arena ar;
    carve(P, precision, solver, ar);
    return ar.off + spd_inverse_work_doubles(P.nb, P.p) * sizeof(double) + 4096;
}

// KKT evaluation of (a subset of) solves followed by the freeze step, and an
// asynchronous copy of the active counts ([0] all, [1 + b] per bootstrap) into
// pinned host memory, marked by an event.  The maxima and the counters of
// buffer `parity` are zero on entry (cleared by the previous check's freeze, or
// at the start of the sweep); this check clears the other buffer.
// With `estimate`, the maxima were left by the last iteration's epilogue (the
// float32 KKT estimate): no product is run, and a solve that meets the
// tolerance is parked rather than converged.  With `zero`, z = 0 (a cold
// start) and the exact residual needs no product either.
template <typename T>
static void check_launch(hipStream_t s, const AdmmProblem &P, const AdmmWork &w, const T *z,
                         bool only_active, double park_tol, double stall_tol, int it, int it_base, AdmmOut &out,
                         int *hact, hipEvent_t ev, int parity, bool estimate, bool zero = false) {
    int *act = w.active + (size_t)parity * (1 + P.nb), *act_next = w.active + (size_t)(parity ^ 1) * (1 + P.nb);
    if (estimate || zero) {
    } else if (std::is_same<T, double>::value) {
        UOI_DISPATCH_FN_RT(P.fn64, {
            if (w.fm64 == 2) {
                KktEpi<double, 2, FN> epi{P.C, (const double *)z, w.state, P.lam, w.vmax, P.p, P.R, P.pe,
                                          only_active};
                run_bgemm<double, 2, FN>(s, P.nb, P.p, P.R, P.G, (const double *)z, epi);
            } else {
                KktEpi<double, 1, FN> epi{P.C, (const double *)z, w.state, P.lam, w.vmax, P.p, P.R, P.pe,
                                          only_active};
                run_bgemm<double, 1, FN>(s, P.nb, P.p, P.R, P.G, (const double *)z, epi);
            }
        });
    } else {
        // float32 z: widen to float64 first so the product is the float64 Gram times z
        size_t n = (size_t)P.nb * P.p * P.R;
        hipLaunchKernelGGL(k_f32_to_f64, dim3(cdiv(n, 256)), dim3(256), 0, s, n, (const float *)z,
                           w.v0);
        UOI_LAUNCH_CHECK();
        UOI_DISPATCH_FN_RT(P.fn64, {
            if (w.fm64 == 2) {
                KktEpi<double, 2, FN> epi{P.C, w.v0, w.state, P.lam, w.vmax, P.p, P.R, P.pe, only_active};
                run_bgemm<double, 2, FN>(s, P.nb, P.p, P.R, P.G, w.v0, epi);
            } else {
                KktEpi<double, 1, FN> epi{P.C, w.v0, w.state, P.lam, w.vmax, P.p, P.R, P.pe, only_active};
                run_bgemm<double, 1, FN>(s, P.nb, P.p, P.R, P.G, w.v0, epi);
            }
        });
    }
    int ns = P.nb * P.R;
    hipLaunchKernelGGL(k_freeze, dim3(cdiv(ns, 256)), dim3(256), 0, s, P.nb, P.R, P.pe, w.vmax, w.rmax,
                       estimate ? (const double *)w.gn : nullptr, zero ? P.lam : nullptr, w.cn,
                       estimate ? -1.0 : P.tol, park_tol, stall_tol, it, it_base, w.state, out.iters, out.kkt, act,
                       act_next);
    UOI_LAUNCH_CHECK();
    UOI_HIP(hipMemcpyAsync(hact, act, sizeof(int) * (1 + P.nb), hipMemcpyDeviceToHost, s));
    if (ev) UOI_HIP(hipEventRecord(ev, s));
}

// Without an event (the allocation-free entry point) the host waits for the
// whole stream, including a chunk queued behind the check.
static int check_wait(hipStream_t s, hipEvent_t ev, const int *hact, int nb, std::vector<int> &act_b) {
    if (ev) UOI_HIP(hipEventSynchronize(ev));
    else UOI_HIP(hipStreamSynchronize(s));
    act_b.assign(hact, hact + 1 + nb);
    return act_b[0];
}

// ADMM iterations in chunks (the first of first_every iterations, the later
// ones of every), each followed by a KKT check.  The
// next chunk is queued before the host reads the previous check (it changes
// only solves that the check left active), so the GPU does not idle while the
// counts travel back; a chunk queued after the last solve froze does no work.
template <typename T>
static int sweep(hipStream_t s, const AdmmProblem &P, const AdmmWork &w, const T *M, const T *h,
                 T *z, T *u, T *va, T *vb, int &it, int it_cap, double park_tol, double stall_tol,
                 AdmmOut &out, bool zero_start, int every, int first_every, bool first_check = true) {
    std::vector<int> act_b;
    // the active counts come back through pinned memory marked by an event; the
    // allocation-free entry point reads them into ordinary host memory instead
    std::vector<int> hact_plain;
    int *hact = nullptr;
    hipEvent_t ev = nullptr;
    if (P.no_alloc) {
        hact_plain.assign(1 + P.nb, 0);
        hact = hact_plain.data();
    } else {
        hact = pinned_ints(1 + P.nb);
        UOI_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    uoi_kstat *ks = out.kstat ? &out.kstat[std::is_same<T, double>::value ? UOI_KSTAT_ADMM64
                                                                           : UOI_KSTAT_ADMM32]
                              : nullptr;
    struct Pending {
        hipEvent_t e0, e1;
        double bytes, flops;
        int n;
        bool used;
    };
    std::vector<Pending> pend;
    // chunk timing goes to the caller's deferred record, else to a local one
    // resolved at the end of the sweep
    DeferredTiming local;
    DeferredTiming *dt = ks ? (out.dt ? out.dt : &local) : nullptr;
    int itq = it;  // iterations queued so far
    // n iterations starting at iteration parity par (the ping-pong buffers of v
    // alternate with the iteration's parity; the last one leaves the KKT estimate)
    const int fnv = std::is_same<T, float>::value ? P.fn32 : P.fn64;
    auto issue = [&](hipStream_t st, int par, int n) {
        for (int t = 0; t < n; ++t) {
            const int odd = (par + t) & 1;
            T *vin = odd ? vb : va;
            T *vout = odd ? va : vb;
            UOI_DISPATCH_FN_RT(fnv, {
                if constexpr (std::is_same<T, float>::value) {
                    __bf16 *pin = odd ? w.vp1 : w.vp0;
                    __bf16 *pout = odd ? w.vp0 : w.vp1;
                    AdmmEpiBf3<FN> epi{h, z, u, pout, w.state, P.lam, P.p, P.R, P.pe, bf3_ldk(P.p),
                                       (float)P.rho, (float)(1.0 / P.rho), (float)P.relax,
                                       t == n - 1 ? w.vmax : nullptr, w.rmax};
                    if (w.fm32 == 2) run_bgemm_bf3<FN, 2>(st, P.nb, P.p, P.R, M, pin, epi);
                    else run_bgemm_bf3<FN, 1>(st, P.nb, P.p, P.R, M, pin, epi);
                } else {
                    if (w.fm64 == 2) {
                        AdmmEpi<T, 2, FN> epi{h, z, u, vout, w.state, P.lam, P.p, P.R, P.pe, (T)P.rho,
                                              (T)(1.0 / P.rho), (T)P.relax};
                        run_bgemm<T, 2, FN>(st, P.nb, P.p, P.R, M, vin, epi);
                    } else {
                        AdmmEpi<T, 1, FN> epi{h, z, u, vout, w.state, P.lam, P.p, P.R, P.pe, (T)P.rho,
                                              (T)(1.0 / P.rho), (T)P.relax};
                        run_bgemm<T, 1, FN>(st, P.nb, P.p, P.R, M, vin, epi);
                    }
                }
            });
        }
    };
    auto run_chunk = [&](int n) {
        Pending pc{nullptr, nullptr, 0.0, 0.0, n, false};
        if (dt) pc.e0 = dt->mark(s);
        const int par = itq & 1;
        if (n > 1 && P.graphs) {
            // the chunk as one graph launch: recorded once per distinct argument set
            // (every pointer and scalar the launches take is in the key)
            GraphKey key;
            key.add(sizeof(T)).add(par).add(n).add(P.fn32).add(P.fn64).add(P.nb).add(P.p).add(P.R).add(P.pe)
                .add(M).add(h).add(z)
                .add(u).add(va).add(vb).add(w.vp0).add(w.vp1).add(w.fm32).add(w.fm64).add(w.state).add(P.lam).add(w.vmax).add(w.rmax)
                .add(P.rho).add(P.relax);
            graph_launch(s, key, [&](hipStream_t cs) { issue(cs, par, n); });
        } else {
            issue(s, par, n);
        }
        itq += n;
        if (dt) pc.e1 = dt->mark(s);
        pend.push_back(pc);
    };
    // algorithmic traffic and work of a chunk run with the active set act_b
    auto account = [&](Pending &pc) {
        double by = 0.0, fl = 0.0;
        for (int b = 0; b < P.nb; ++b)
            if (act_b[1 + b] > 0) {
                by += (double)P.p * P.p * sizeof(T) + 4.0 * P.p * sizeof(T) * act_b[1 + b];
                fl += 2.0 * P.p * P.p * act_b[1 + b];
            }
        pc.bytes = by * pc.n;
        pc.flops = fl * pc.n;
        pc.used = true;
    };
    // cleared once here; each check clears the next one's buffers
    UOI_HIP(hipMemsetAsync(w.vmax, 0, sizeof(double) * (size_t)P.nb * P.R, s));
    UOI_HIP(hipMemsetAsync(w.rmax, 0, sizeof(double) * (size_t)P.nb * P.R, s));
    UOI_HIP(hipMemsetAsync(w.active, 0, sizeof(int) * 2 * (1 + P.nb), s));
    int parity = 0;
    // the first check evaluates the exact residual; the later ones of the float32
    // sweep take the estimate left by the chunk's last iteration.  Without a
    // first check (first_check false) every solve runs the first chunk.
    constexpr bool kEstimate = std::is_same<T, float>::value;
    const int it_base = it;
    int active = 0;
    bool enter = false;
    if (first_check) {
        check_launch<T>(s, P, w, z, true, park_tol, stall_tol, it, it_base, out, hact, ev, parity, false,
                        zero_start);
        parity ^= 1;
        // the first chunk is queued behind the first check as well
        const bool spec0 = it < it_cap;
        if (spec0) run_chunk(std::min(first_every, it_cap - it));
        active = check_wait(s, ev, hact, P.nb, act_b);
        enter = active > 0 && spec0;
    } else {
        act_b.assign(1 + P.nb, P.R);  // for the traffic account: all active
        act_b[0] = P.nb * P.R;
        run_chunk(std::min(first_every, it_cap - it));
        enter = true;
    }
    if (enter) {
        account(pend.back());
        it = itq;
        for (;;) {
            check_launch<T>(s, P, w, z, true, park_tol, stall_tol, it, it_base, out, hact, ev, parity, kEstimate);
            parity ^= 1;
            const bool spec = it < it_cap;
            if (spec) run_chunk(std::min(every, it_cap - it));
            active = check_wait(s, ev, hact, P.nb, act_b);
            if (active == 0 || !spec) break;
            account(pend.back());  // the queued chunk ran with this active set
            it = itq;
        }
    }
    if (dt) {
        for (Pending &pc : pend)
            if (pc.used) dt->kernel(pc.e0, pc.e1, ks, pc.bytes, pc.flops, pc.n);
        if (dt == &local && !pend.empty()) {
            UOI_HIP(hipEventSynchronize(pend.back().e1));
            local.resolve();
        }
    }
    if (ev) UOI_HIP(hipEventDestroy(ev));
    return active;
}

// Mean of the diagonals of nb p x p matrices (one workgroup; fixed summation
// order, so the result does not depend on timing).  The result is written to
// host memory that the device can reach.
__global__ __launch_bounds__(256) void k_mean_diag(int nb, int p, const double *__restrict__ G,
                                                   double *__restrict__ out) {
    __shared__ double part[256];
    const int64_t n = (int64_t)nb * p;
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += 256) {
        const int64_t b = e / p, i = e - b * p;
        acc += G[(b * p + i) * p + i];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0] / (double)n;
}

// The penalty when the caller passes rho = 0: the scale of the data, the mean
// diagonal of the Grams (their average eigenvalue).  On standardised columns it
// is about 1; on a VAR series it is the series' mean square, where rho = 1 is
// far too small for the spectrum and ADMM converges many times more slowly.
// Falls back to 1 for an all-zero design.
constexpr int kPinnedScalar = kPinnedLarge + 1;  // a pinned slot of its own

double data_scaled_rho(hipStream_t s, int nb, int p, const double *G) {
    double *h = (double *)pinned_slot(kPinnedScalar, sizeof(double));
    hipLaunchKernelGGL(k_mean_diag, dim3(1), dim3(256), 0, s, nb, p, G, h);
    UOI_LAUNCH_CHECK();
    UOI_HIP(hipStreamSynchronize(s));
    const double r = *h;
    return std::isfinite(r) && r > 0.0 ? r : 1.0;
}

void admm_solve(hipStream_t s, const AdmmProblem &P0, int precision, int solver, void *work,
                bool warm, AdmmOut &out, float *stage_ms) {
    AdmmProblem P = P0;  // the launch shapes (fn32, fn64) are filled in below
    if (P.rho == 0.0) {
        UOI_REQUIRE(!P.no_alloc, "rho = 0 (scaled to the data) reads a value back: not allocation-free");
        P.rho = data_scaled_rho(s, P.nb, P.p, P.G);
    }
    P.fn32 = P.fn64 = default_fn(P.R);
    Arena ar;
    ar.base = (char *)work;
    ar.cap = (size_t)-1;
    AdmmWork w = carve(P, precision, solver, ar);
    double *spd_work = ar.take<double>(spd_inverse_work_doubles(P.nb, P.p));
    const size_t nst = (size_t)P.nb * P.p * P.R;
    const int ns = P.nb * P.R;

    // stage times: recorded in the caller's deferred record, else resolved here
    DeferredTiming local;
    DeferredTiming *dt = stage_ms ? (out.dt ? out.dt : &local) : nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (dt) ev[0] = dt->mark(s);

    // ||G||_inf per bootstrap for the float32 KKT estimate: one pass over G on the
    // second stream, beside the factorization
    const bool mixed = solver != UOI_SOLVER_PLAIN && precision != UOI_FP64;
    // (the allocation-free entry point creates no second stream: same stream)
    AuxStream *ax = P.no_alloc ? nullptr : &aux_stream();
    if (mixed) {
        hipStream_t gs = s;
        if (ax) {
            UOI_HIP(hipEventRecord(ax->e0, s));
            UOI_HIP(hipStreamWaitEvent(ax->s, ax->e0, 0));
            gs = ax->s;
        }
        UOI_HIP(hipMemsetAsync(w.gn, 0, sizeof(double) * P.nb, gs));
        hipLaunchKernelGGL(k_gnorm, dim3(cdiv(P.p, 64), P.nb), dim3(256), 0, gs, P.p, P.G, w.gn);
        UOI_LAUNCH_CHECK();
        if (ax) UOI_HIP(hipEventRecord(ax->e1, ax->s));
    }
    // factor: M = (G + rho I)^{-1}, h = M C, and ||c||_inf per equation
    {
        // matrices per pass of the blocked sweep (1, 2 or 3 passes over the batch):
        // every matrix is swept the same way whatever the pass, so the candidates
        // give identical results and the autotuner times them on the live batch
        const size_t pp = (size_t)P.p * P.p;
        const int ncand = P.nb >= 16 && P.p > 88 ? 3 : 1;
        auto run_spd = [&](int c) {
            const int ch = (P.nb + c) / (c + 1);
            for (int b0 = 0; b0 < P.nb; b0 += ch)
                spd_inverse_f64(s, std::min(ch, P.nb - b0), P.p, P.G + b0 * pp, P.rho, w.M + b0 * pp, spd_work,
                                w.M32 ? w.M32 + b0 * pp : nullptr);  // M32: mixed only
        };
        const std::string key = "spd_passes/nb" + std::to_string(P.nb) + "/p" + std::to_string(P.p);
        if (P.tune && ncand > 1) {
            const TuneResult r = tune_choose(s, key, ncand, run_spd, 1);
            if (!r.ran_all) run_spd(r.choice);
        } else {
            run_spd(ncand > 1 ? std::min(tune_lookup(key, 0), ncand - 1) : 0);
        }
    }
    launch_matmul_f64(s, P.nb, P.p, P.pe, w.M, P.C, w.h);
    launch_cnorm(s, P.nb, P.p, P.pe, P.C, w.cn);
    if (dt) ev[1] = dt->mark(s);

    UOI_HIP(hipMemsetAsync(w.state, 0, ns, s));
    UOI_HIP(hipMemsetAsync(out.kkt, 0x7f, sizeof(double) * ns, s));  // "previous" KKT: huge
    hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(ns, 256)), dim3(256), 0, s, (size_t)ns, -1, out.iters);
    UOI_LAUNCH_CHECK();
    out.dstat = w.stat;
    out.warm_used = 0;
    if (P.mlp) {
        UOI_REQUIRE(!P.no_alloc, "the allocation-free entry point starts cold");
        // network start for every (bootstrap, lambda); falls back to cold per solve
        int nin = 0, nout = 0;
        mlp_dims(P.mlp, &nin, &nout);
        UOI_REQUIRE(P.pe == 1 && nin == P.p + 1 && nout == P.p,
                    "warm-start network must have input p+1 and output p (LASSO only)");
        const int n = P.nb * P.q;
        float *Xs = mlp_input_buffer(P.mlp, n);
        size_t nx = (size_t)n * (P.p + 1);
        hipLaunchKernelGGL(k_ws_inputs, dim3(cdiv(nx, 256)), dim3(256), 0, s, P.nb, P.p, P.q, 1, P.C, w.cn,
                           P.lam, Xs);
        UOI_LAUNCH_CHECK();
        mlp_forward(s, P.mlp, n, Xs);
        hipLaunchKernelGGL(k_ws_z0, dim3(cdiv(nst, 256)), dim3(256), 0, s, P.nb, P.p, P.q,
                           mlp_output(P.mlp), w.cn, P.lam, kWarmShrink, out.z);
        UOI_LAUNCH_CHECK();
        double *Gz = w.v0 ? w.v0 : out.u;  // scratch of the state size
        UOI_DISPATCH_FN(P.R, {
            StoreEpi<double, 1, FN> epi{Gz, P.p, P.R};
            run_bgemm<double, 1, FN>(s, P.nb, P.p, P.R, P.G, out.z, epi);
        });
        UOI_HIP(hipMemsetAsync(w.active, 0, sizeof(unsigned long long), s));
        if (Gz == out.u) {
            // plain solver: no spare state buffer; the completion reads Gz before writing u
            UOI_REQUIRE(false, "warm start by network needs the batched solver");
        }
        hipLaunchKernelGGL(k_ws_finish, dim3(P.nb), dim3(256), 0, s, P.nb, P.p, P.q, P.C, Gz,
                           P.lam, P.rho, out.z, out.u, (unsigned long long *)w.active);
        UOI_LAUNCH_CHECK();
        unsigned long long used = 0;
        UOI_HIP(hipMemcpyAsync(&used, w.active, sizeof(used), hipMemcpyDeviceToHost, s));
        UOI_HIP(hipStreamSynchronize(s));
        out.warm_used = (int64_t)used;
        warm = true;
    } else if (!warm) {
        UOI_HIP(hipMemsetAsync(out.z, 0, sizeof(double) * nst, s));
        UOI_HIP(hipMemsetAsync(out.u, 0, sizeof(double) * nst, s));
    }
    // Column-tile width of the batched products (16 FN solves per workgroup).
    // Candidates: every width except one that needs as many column tiles as a
    // narrower width with more padding columns (same tiles, more wasted work):
    // FN = 1, 2, 3 at R = 48, all four at R = 5760 (the VAR fits).  Fewer tiles
    // re-read M less often, more tiles give more workgroups; the tuner decides.  The
    // accumulation order of every output, and the epilogue's rounding (explicit
    // fused multiply-adds), are the same for every width, so the autotuner times
    // them on the live operands, each iteration with its real epilogue writing
    // scratch state (float32: into the idle float64 buffer; float64: into the
    // ping-pong buffers, which the refresh after the choice overwrites).  The
    // float64 choice is made with every solve active (before the float64 sweep,
    // or after the parked solves are released).
    // With more than one column tile, the candidates come twice: one row block per
    // wave (candidates 0 .. n - 1), then two (from n on; the same accumulation
    // order, so the same results).  The choice sets w.fm32 or w.fm64.
    auto pick_fn = [&](bool f32) -> int {
        std::vector<int> cand, fm;
        for (int f = 1; f <= 4; ++f) {
            const long tf = cdiv(P.R, 16 * f), wf = tf * 16 * f - P.R;
            bool dominated = false;
            for (int g = 1; g < f; ++g) {
                const long tg = cdiv(P.R, 16 * g), wg = tg * 16 * g - P.R;
                if (tg == tf && wg < wf) dominated = true;
            }
            if (!dominated) cand.push_back(f);
        }
        fm.assign(cand.size(), 1);
        if (offer_fm2(P)) {
            const size_t n0 = cand.size();
            for (size_t c = 0; c < n0; ++c) {
                cand.push_back(cand[c]);
                fm.push_back(2);
            }
        }
        const std::string key = std::string(f32 ? "admm32_fn" : "admm64_fn") + "/nb" + std::to_string(P.nb) +
                                "/p" + std::to_string(P.p) + "/R" + std::to_string(P.R);
        const int nc = (int)cand.size();
        auto chosen = [&](int c) {
            (f32 ? w.fm32 : w.fm64) = fm[c];
            return cand[c];
        };
        if (!P.tune || nc == 1) return chosen(std::min(std::max(tune_lookup(key, 0), 0), nc - 1));
        const size_t nst_ = (size_t)P.nb * P.p * P.R;
        const TuneResult r = tune_choose(s, key, nc, [&](int c) {
            UOI_DISPATCH_FN_RT(cand[c], {
                if (f32) {
                    // scratch state: z and u in the (idle) float64 buffer, v into the
                    // plane buffer the first iteration overwrites anyway
                    float *zs = (float *)w.v0, *us = (float *)w.v0 + nst_;
                    AdmmEpiBf3<FN> e{w.h32, zs, us, w.vp1, w.state, P.lam, P.p, P.R, P.pe, bf3_ldk(P.p),
                                     (float)P.rho, (float)(1.0 / P.rho), (float)P.relax, nullptr, w.rmax};
                    if (fm[c] == 2) run_bgemm_bf3<FN, 2>(s, P.nb, P.p, P.R, w.M32, w.vp0, e);
                    else run_bgemm_bf3<FN, 1>(s, P.nb, P.p, P.R, w.M32, w.vp0, e);
                } else {
                    // (z in v0, u and the next v both in v1: scratch)
                    if (fm[c] == 2) {
                        AdmmEpi<double, 2, FN> e{w.h, w.v0, w.v1, w.v1, w.state, P.lam, P.p, P.R, P.pe, P.rho,
                                                 1.0 / P.rho, P.relax};
                        run_bgemm<double, 2, FN>(s, P.nb, P.p, P.R, w.M, out.z, e);
                    } else {
                        AdmmEpi<double, 1, FN> e{w.h, w.v0, w.v1, w.v1, w.state, P.lam, P.p, P.R, P.pe, P.rho,
                                                 1.0 / P.rho, P.relax};
                        run_bgemm<double, 1, FN>(s, P.nb, P.p, P.R, w.M, out.z, e);
                    }
                }
            });
        }, 5);
        return chosen(r.choice);
    };
    int it = 0, active = 0;
    if (solver == UOI_SOLVER_PLAIN) {
        size_t lds = sizeof(double) * 3 * (size_t)P.p;
        UOI_REQUIRE(P.p <= 256 * PLAIN_MAX_ROWS && lds <= 160 * 1024, "plain solver: p too large");
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (out.kstat) {
            UOI_HIP(hipEventCreate(&e0));
            UOI_HIP(hipEventCreate(&e1));
            UOI_HIP(hipEventRecord(e0, s));
        }
        hipLaunchKernelGGL(k_admm_plain, dim3(ns), dim3(256), lds, s, P.p, P.pe, P.R, w.M, w.h, P.G,
                           P.C, P.lam, w.cn, P.rho, P.relax, P.tol, P.max_iter, P.check_every, out.z,
                           out.u, out.iters, out.kkt);
        UOI_LAUNCH_CHECK();
        if (out.kstat) {
            UOI_HIP(hipEventRecord(e1, s));
            UOI_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            UOI_HIP(hipEventElapsedTime(&ms, e0, e1));
            UOI_HIP(hipEventDestroy(e0));
            UOI_HIP(hipEventDestroy(e1));
            std::vector<int32_t> its(ns);
            UOI_HIP(hipMemcpy(its.data(), out.iters, sizeof(int32_t) * ns, hipMemcpyDeviceToHost));
            uoi_kstat &k = out.kstat[UOI_KSTAT_PLAIN];
            double pp = (double)P.p * P.p;
            for (int v : its) {
                double n = v < 0 ? P.max_iter : v;
                double checks = std::floor(n / P.check_every) + 1.0;
                k.bytes += (n + checks) * pp * sizeof(double);
                k.flops += (n + checks) * 2.0 * pp;
            }
            k.ms += ms;
            k.launches += 1;
        }
    } else if (precision == UOI_FP64) {
        P.fn64 = pick_fn(false);  // (its scratch output is overwritten by the refresh below)
        hipLaunchKernelGGL(k_refresh_v<double>, dim3(cdiv(nst, 256)), dim3(256), 0, s, nst, out.z,
                           out.u, w.v0, w.v1);
        UOI_LAUNCH_CHECK();
        active = sweep<double>(s, P, w, w.M, w.h, out.z, out.u, w.v0, w.v1, it, P.max_iter, P.tol, 0.0,
                               out, !warm, P.check_every, P.check_every);
    } else {
        // float32 phase: operator and state in float32, first KKT check in
        // float64, later ones on the iteration's estimate; solves whose estimate
        // reaches kParkFactor x the tolerance, or stalls within kStallFactor x
        // the tolerance, are parked, then verified and finished in float64.
        // (the float32 copy of M was written by the factorization)
        if (ax) UOI_HIP(hipStreamWaitEvent(s, ax->e1, 0));  // ||G||_inf (started beside the factor)
        size_t nh = (size_t)P.nb * P.p * P.pe;
        hipLaunchKernelGGL(k_f64_to_f32, dim3(cdiv(nh, 256)), dim3(256), 0, s, nh, w.h, w.h32);
        // v planes: zero (rows past p stay zero), then v = z - u (zero at a cold start)
        const int ldk = bf3_ldk(P.p);
        const size_t np3 = (size_t)P.nb * 3 * P.R * ldk;
        UOI_HIP(hipMemsetAsync(w.vp0, 0, sizeof(__bf16) * np3, s));
        UOI_HIP(hipMemsetAsync(w.vp1, 0, sizeof(__bf16) * np3, s));
        if (warm) {
            hipLaunchKernelGGL(k_f64_to_f32, dim3(cdiv(nst, 256)), dim3(256), 0, s, nst, out.z, w.z32);
            hipLaunchKernelGGL(k_f64_to_f32, dim3(cdiv(nst, 256)), dim3(256), 0, s, nst, out.u, w.u32);
            hipLaunchKernelGGL(k_refresh_vp, dim3(cdiv(nst, 256)), dim3(256), 0, s, P.nb, P.p, P.R, ldk,
                               w.z32, w.u32, w.vp0, w.vp1);
        } else {
            UOI_HIP(hipMemsetAsync(w.z32, 0, sizeof(float) * nst, s));
            UOI_HIP(hipMemsetAsync(w.u32, 0, sizeof(float) * nst, s));
        }
        UOI_LAUNCH_CHECK();
        P.fn32 = pick_fn(true);
        // max_iter bounds the two phases together: the float32 phase may take at
        // most half of it (solves still active then go on in float64), and the
        // float64 finish runs up to max_iter on the shared iteration counter, so
        // no solve's count (float32 iterations up to its parking plus those of
        // the finish) exceeds max_iter.
        const int cap32 = P.max_iter - P.max_iter / 2;
        active = sweep<float>(s, P, w, w.M32, w.h32, w.z32, w.u32, nullptr, nullptr, it, cap32,
                              std::max(P.tol * kParkFactor, kParkFloor),
                              std::max(P.tol * kStallFactor, kStallFloor), out, !warm, P.check_every,
                              P.check_every);
        // widen the state and finish parked / active solves in float64
        hipLaunchKernelGGL(k_f32_to_f64, dim3(cdiv(nst, 256)), dim3(256), 0, s, nst, w.z32, out.z);
        hipLaunchKernelGGL(k_f32_to_f64, dim3(cdiv(nst, 256)), dim3(256), 0, s, nst, w.u32, out.u);
        hipLaunchKernelGGL(k_unpark, dim3(cdiv(ns, 256)), dim3(256), 0, s, (size_t)ns, w.state);
        P.fn64 = pick_fn(false);
        hipLaunchKernelGGL(k_refresh_v<double>, dim3(cdiv(nst, 256)), dim3(256), 0, s, nst, out.z,
                           out.u, w.v0, w.v1);
        UOI_LAUNCH_CHECK();
        int it64 = it;
        active = sweep<double>(s, P, w, w.M, w.h, out.z, out.u, w.v0, w.v1, it64, P.max_iter,
                               P.tol, 0.0, out, false, P.check_every, std::min(P.check_every, kFinishFirst),
                               kFinishFirstCheck);
        it = it64;
    }
    if (dt) {
        ev[2] = dt->mark(s);
        dt->time(ev[0], ev[1], &stage_ms[0]);
        dt->time(ev[1], ev[2], &stage_ms[1]);
        if (dt == &local) {
            UOI_HIP(hipEventSynchronize(ev[2]));
            local.resolve();
        }
    }
    // unconverged solves and the largest iteration count, read by admm_finish_stats
    UOI_HIP(hipMemsetAsync(w.stat, 0, 2 * sizeof(int), s));
    hipLaunchKernelGGL(k_iter_stats, dim3(cdiv(ns, 256)), dim3(256), 0, s, ns, out.iters, w.stat);
    UOI_LAUNCH_CHECK();
    (void)active;
}

void admm_finish_stats(AdmmOut &out) {
    int h[2] = {0, 0};
    if (out.dstat) UOI_HIP(hipMemcpy(h, out.dstat, sizeof(h), hipMemcpyDeviceToHost));
    out.unconverged = h[0];
    out.max_iters = h[1];
}

}  // namespace uoi
