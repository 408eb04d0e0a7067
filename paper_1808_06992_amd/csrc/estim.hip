// Model estimation of Alg. 1 / Alg. 2: for every estimation split k and every
// support S_j (per equation e for VAR) the least-squares refit on the training
// rows, its loss on the evaluation rows, the best support per split and the
// average of the chosen refits (Eq. (union)).
//
// The paper runs OLS as ADMM with lambda = 0; here the same minimiser is
// computed directly in float64 from the training normal equations
// G_T[S,S] b = c_T[S]:
//   - |S| <= kSmall: one workgroup per (split, support) gathers G_T[S,S] into
//     LDS, factors it by Cholesky and solves (supports of uneven size run side by
//     side, each workgroup sized by its own support);
//   - kSmall < |S| <= kMid: one workgroup per (split, support) runs a
//     left-looking blocked Cholesky, reading G_T[S,S] straight from G_T and
//     keeping the factor in global scratch (L2-resident), with c_T[S] carried as
//     an extra row so that the forward solve comes out of the factorization;
//   - larger supports: conjugate gradients on the masked operator, batched over
//     all (split, support) pairs of a split so that every iteration is one MFMA
//     product with G_T (the same kernel as the ADMM x-update).
// The evaluation loss is the mean squared residual on the evaluation rows,
// expanded through the evaluation Gram: L = s_E - 2 b'c_E + b'G_E b.
#include <algorithm>
#include <vector>

#include "bgemm.hpp"
#include "common.hpp"

namespace uoi {

namespace {
constexpr int kSmall = 80;   // in-LDS Cholesky up to this support size
constexpr int kMid = 256;    // blocked Cholesky with the factor in global scratch up to this size
constexpr int kPW = 16;      // panel width of the blocked Cholesky
constexpr size_t kMidScratch = (size_t)256 << 20;  // bytes of factor storage per launch
constexpr double kCgTol = 1e-13;
}

// Orders the LDS accesses of one wave across its lanes (stores before it are
// seen by loads after it): per lane, the compiler may otherwise move a load
// above another lane's store.
__device__ __forceinline__ void lane_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void k_popcount(int R, int W, const uint64_t *__restrict__ supp, int32_t *__restrict__ cnt) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    int c = 0;
    for (int w = 0; w < W; ++w) c += __popcll(supp[(size_t)r * W + w]);
    cnt[r] = c;
}

// List the members of support r into idx (LDS); returns the size.
__device__ int support_members(const uint64_t *__restrict__ sw, int W, int *idx) {
    __shared__ int woff[1025];
    // word offsets (W <= 1024 checked on the host): wave 0 loads 64 words at a time,
    // all in flight, and prefix-sums their popcounts across the wave
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int base = 0;
        for (int w0 = 0; w0 < W; w0 += 64) {
            const int w = w0 + lane;
            const uint64_t x = sw[min(w, W - 1)];  // clamped: the count is masked below
            const int c = w < W ? __popcll(x) : 0;
            int incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            if (w < W) woff[w] = base + incl - c;
            base += __shfl(incl, 63);
        }
        if (lane == 0) woff[W] = base;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
        uint64_t x = sw[w];
        int o = woff[w];
        while (x) {
            int bit = __ffsll((unsigned long long)x) - 1;
            idx[o++] = w * 64 + bit;
            x &= x - 1;
        }
    }
    __syncthreads();
    return woff[W];
}

// Loss on the evaluation rows through the evaluation Gram, for b on members idx.
__device__ double eval_loss(int s, const int *idx, const double *bv, const double *GEb,
                            const double *CEb, int p, int pe, int e, double sE) {
    __shared__ double red[8];
    double part = 0.0;
    {   // b' G_E b over the members; thread (ty, tx) of a (blockDim/16) x 16 grid
        const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15, ny = blockDim.x >> 4;
        for (int a = ty; a < s; a += ny) {
            const double *row = GEb + (size_t)idx[a] * p;
            double ra = 0.0;
            for (int c = tx; c < s; c += 16) ra += row[idx[c]] * bv[c];
            part += bv[a] * ra;
        }
    }
    for (int a = threadIdx.x; a < s; a += blockDim.x) part -= 2.0 * bv[a] * CEb[(size_t)idx[a] * pe + e];
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
    __syncthreads();
    return sE + tot;
}

// Small supports: gather, Cholesky, solve, loss.  Grid (R, nb); one workgroup per
// (support r, split k); supports above kSmall are skipped here.
__global__ __launch_bounds__(256) void k_ols_small(int p, int pe, int R, int W,
                                                   const uint64_t *__restrict__ supp,
                                                   const int32_t *__restrict__ cnt,
                                                   const double *__restrict__ GT,
                                                   const double *__restrict__ CT,
                                                   const double *__restrict__ GE,
                                                   const double *__restrict__ CE,
                                                   const double *__restrict__ sE,
                                                   double *__restrict__ Fit, double *__restrict__ loss,
                                                   int *__restrict__ bad) {
    extern __shared__ double Ls[];  // s x s
    __shared__ int idx[kSmall];
    __shared__ double bv[kSmall];
    __shared__ int fail;
    const int r = blockIdx.x, k = blockIdx.y;
    if (cnt[r] > kSmall) return;
    const int e = r % pe;
    const double *GTb = GT + (size_t)k * p * p;
    const double *CTb = CT + (size_t)k * p * pe;
    const int s = support_members(supp + (size_t)r * W, W, idx);
    if (threadIdx.x == 0) fail = 0;
    for (int t0 = threadIdx.x; t0 < s * s; t0 += 1024) {  // four gathers in flight
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = min(t0 + 256 * u, s * s - 1);
            v[u] = GTb[(size_t)idx[t / s] * p + idx[t % s]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (t0 + 256 * u < s * s) Ls[t0 + 256 * u] = v[u];
    }
    for (int a = threadIdx.x; a < s; a += 256) bv[a] = CTb[(size_t)idx[a] * pe + e];
    __syncthreads();
    // right-looking Cholesky, lower triangle
    for (int j = 0; j < s; ++j) {
        if (threadIdx.x == 0) {
            double d = Ls[j * s + j];
            if (!(d > 0.0)) { fail = 1; d = 1.0; }
            Ls[j * s + j] = sqrt(d);
        }
        __syncthreads();
        const double dj = Ls[j * s + j];
        for (int i = j + 1 + threadIdx.x; i < s; i += 256) Ls[i * s + j] /= dj;
        __syncthreads();
        {   // trailing update of the lower triangle; thread (ty, tx) of a 16 x 16 grid
            const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
            for (int i = j + 1 + ty; i < s; i += 16) {
                const double lij = Ls[i * s + j];
                for (int c = j + 1 + tx; c <= i; c += 16) Ls[i * s + c] -= lij * Ls[c * s + j];
            }
        }
        __syncthreads();
    }
    // L y = c (column sweep), then L' b = y (row sweep)
    for (int j = 0; j < s; ++j) {
        if (threadIdx.x == 0) bv[j] /= Ls[j * s + j];
        __syncthreads();
        for (int i = j + 1 + threadIdx.x; i < s; i += 256) bv[i] -= Ls[i * s + j] * bv[j];
        __syncthreads();
    }
    for (int j = s - 1; j >= 0; --j) {
        if (threadIdx.x == 0) bv[j] /= Ls[j * s + j];
        __syncthreads();
        for (int i = threadIdx.x; i < j; i += 256) bv[i] -= Ls[j * s + i] * bv[j];
        __syncthreads();
    }
    double *F = Fit + ((size_t)k * R + r) * p;
    for (int i = threadIdx.x; i < p; i += 256) F[i] = 0.0;
    __syncthreads();
    for (int a = threadIdx.x; a < s; a += 256) F[idx[a]] = bv[a];
    double L = eval_loss(s, idx, bv, GE + (size_t)k * p * p, CE + (size_t)k * p * pe, p, pe, e,
                         sE[(size_t)k * pe + e]);
    if (threadIdx.x == 0) {
        loss[(size_t)k * R + r] = L;
        if (fail) atomicOr(bad, 1);
    }
}

// Mid-size supports.  Grid: one workgroup per listed system (split k, support r).
// The factor of the bordered matrix [G_T[S,S]; c_T[S]'] is stored column-major
// with leading dimension s+1 (column t holds rows t..s; row s is L^{-1} c).
__global__ __launch_bounds__(256) void k_ols_mid(int p, int pe, int R, int W,
                                                 const uint64_t *__restrict__ supp,
                                                 const int2 *__restrict__ sys,
                                                 const size_t *__restrict__ off,
                                                 double *__restrict__ Lbase,
                                                 const double *__restrict__ GT,
                                                 const double *__restrict__ CT,
                                                 const double *__restrict__ GE,
                                                 const double *__restrict__ CE,
                                                 const double *__restrict__ sE,
                                                 double *__restrict__ Fit, double *__restrict__ loss,
                                                 int *__restrict__ bad) {
    constexpr int LDP = kPW + 1;
    __shared__ int idx[kMid];
    __shared__ double Pn[(kMid + 1) * LDP];  // panel rows kb..s, kPW columns
    __shared__ double Lp[64][LDP];           // staged rows kb..kb+kPW of the factor
    __shared__ double xv[kMid + 1];
    __shared__ double red[8][33];
    __shared__ double colb[kPW], rdiag[kPW];
    __shared__ int fail;
    const int tid = threadIdx.x;
    const int k = sys[blockIdx.x].x, r = sys[blockIdx.x].y;
    const int e = r % pe;
    const int s = support_members(supp + (size_t)r * W, W, idx);  // kSmall < s <= kMid (host)
    const int ld = s + 1;
    double *L = Lbase + off[blockIdx.x];
    const double *GTb = GT + (size_t)k * p * p;
    const double *CTb = CT + (size_t)k * p * pe;
    if (tid == 0) fail = 0;
    for (int kb = 0; kb < s; kb += kPW) {
        const int nbk = min(kPW, s - kb);
        const int m = s + 1 - kb;  // panel rows kb..s (row s is the right-hand side)
        {   // all loads of the panel first (clamped, unconditional), then the stores
            constexpr int MAXQ = ((kMid + 1) * kPW + 255) / 256;
            double pv[MAXQ];
#pragma unroll
            for (int u = 0; u < MAXQ; ++u) {
                const int q = tid + 256 * u;
                const int c = min(q / m, nbk - 1), i = min(q % m, m - 1);
                const int gi = kb + i, gc = idx[kb + c];
                pv[u] = gi < s ? GTb[(size_t)gc * p + idx[gi]] : CTb[(size_t)gc * pe + e];
            }
#pragma unroll
            for (int u = 0; u < MAXQ; ++u) {
                const int q = tid + 256 * u;
                if (q < m * kPW) {
                    const int c = q / m, i = q % m;
                    Pn[i * LDP + c] = c < nbk ? pv[u] : 0.0;
                }
            }
        }
        __syncthreads();
        // left-looking: subtract the contribution of the factored columns 0..kb
        for (int t0 = 0; t0 < kb; t0 += 64) {
            const int nt = min(64, kb - t0);
            for (int q = tid; q < 64 * kPW; q += 256) {
                const int t = q / kPW, c = q % kPW;
                Lp[t][c] = (t < nt && c < nbk) ? L[(size_t)(t0 + t) * ld + kb + c] : 0.0;
            }
            __syncthreads();
            for (int i = tid; i < m; i += 256) {
                double acc[kPW];
#pragma unroll
                for (int c = 0; c < kPW; ++c) acc[c] = Pn[i * LDP + c];
                for (int t = 0; t < nt; t += 8) {
                    // eight factor entries in flight at once; columns past nt are read
                    // clamped (finite) and meet zero rows of Lp
                    double a[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) a[u] = L[(size_t)(t0 + min(t + u, nt - 1)) * ld + kb + i];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
#pragma unroll
                        for (int c = 0; c < kPW; ++c) acc[c] -= a[u] * Lp[t + u][c];
                }
#pragma unroll
                for (int c = 0; c < kPW; ++c) Pn[i * LDP + c] = acc[c];
            }
            __syncthreads();
        }
        // factor the panel: its nbk x nbk top block by one wave in registers,
        // then every row below (and the right-hand side row) by a forward
        // substitution against that block, one row per thread
        if (tid < 64) {
            const int c = tid & 15, r0 = tid >> 4;  // column c, rows r0 + 4a
            double v[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int r = r0 + 4 * a;
                v[a] = (r < nbk && c < nbk) ? Pn[r * LDP + c] : (r == c ? 1.0 : 0.0);  // identity padding
            }
#pragma unroll
            for (int j = 0; j < kPW; ++j) {
                lane_sync();  // the previous step's reads are done
                if (c == j) {
#pragma unroll
                    for (int a = 0; a < 4; ++a) colb[r0 + 4 * a] = v[a];  // column j
                }
                lane_sync();
                double d = colb[j];
                if (!(d > 0.0)) {
                    if (j < nbk && tid == 0) fail = 1;
                    d = 1.0;
                }
                const double sd = sqrt(d), rsd = 1.0 / sd;
                if (tid == 0) rdiag[j] = rsd;
                const double lc = colb[c] * rsd;  // L[c][j]
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int r = r0 + 4 * a;
                    const double lr = colb[r] * rsd;  // L[r][j]
                    if (c == j) v[a] = r == j ? sd : (r > j ? lr : v[a]);
                    else if (c > j && r >= c) v[a] = fma(-lr, lc, v[a]);
                }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int r = r0 + 4 * a;
                if (r < nbk && c <= r) Pn[r * LDP + c] = v[a];
            }
        }
        __syncthreads();
        for (int i = nbk + tid; i < m; i += 256) {
            double l[kPW];
#pragma unroll
            for (int c = 0; c < kPW; ++c) l[c] = c < nbk ? Pn[i * LDP + c] : 0.0;
#pragma unroll
            for (int c = 0; c < kPW; ++c) {
                if (c < nbk) {
                    double t = l[c];
#pragma unroll
                    for (int c2 = 0; c2 < c; ++c2) t = fma(-l[c2], Pn[c * LDP + c2], t);
                    l[c] = t * rdiag[c];
                }
            }
#pragma unroll
            for (int c = 0; c < kPW; ++c)
                if (c < nbk) Pn[i * LDP + c] = l[c];
        }
        __syncthreads();
        for (int q = tid; q < m * nbk; q += 256) {
            const int c = q / m, i = q % m;
            if (i >= c) L[(size_t)(kb + c) * ld + kb + i] = Pn[i * LDP + c];
        }
        __syncthreads();
    }
    // backward solve L' x = y with y = row s of the factor, in blocks of 32 from the end
    for (int t = tid; t < s; t += 256) xv[t] = L[(size_t)t * ld + s];
    __syncthreads();
    constexpr int LB = 33;
    double *Lb = Pn;  // (the panel buffer is free now) Lb[u][j] = L[t0 + u][t0 + j], u > j, and the diagonal at u = j
    for (int t1 = s; t1 > 0; t1 -= 32) {
        const int t0 = max(0, t1 - 32);
        {   // xv[t] -= sum_{i >= t1} L[i][t] x_i for t in [t0, t1)
            const int tt = tid & 31, g = tid >> 5;
            const int t = t0 + tt;
            double part = 0.0;
            if (t < t1)
                for (int i0 = t1 + g; i0 < s; i0 += 32) {
                    double lv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) lv[u] = L[(size_t)t * ld + min(i0 + 8 * u, s - 1)];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (i0 + 8 * u < s) part += lv[u] * xv[i0 + 8 * u];
                }
            red[g][tt] = part;
        }
        // the diagonal block into LDS (column j of the factor holds rows j.. contiguously)
        for (int q = tid; q < 32 * 32; q += 256) {
            const int j = q >> 5, u = q & 31;
            const bool in = t0 + u < t1 && t0 + j < t1 && u >= j;
            Lb[u * LB + j] = in ? L[(size_t)(t0 + j) * ld + t0 + u] : 0.0;
        }
        __syncthreads();
        if (tid < 64) {
            // one wave, lane j holding x_{t0+j}: from the block's end, x_t is final
            // once the columns after it are applied; it is divided by L[t][t] and
            // broadcast, and every row j < t subtracts L[t][j] x_t
            const int j = tid & 31;
            double xr = 0.0;
            if (tid < 32 && t0 + j < t1) {
                double sacc = 0.0;
                for (int g = 0; g < 8; ++g) sacc += red[g][j];
                xr = xv[t0 + j] - sacc;
            }
            for (int u = t1 - 1 - t0; u >= 0; --u) {
                const long long xb = __double_as_longlong(xr);
                const int lo = __builtin_amdgcn_readlane((int)xb, u);
                const int hi = __builtin_amdgcn_readlane((int)(xb >> 32), u);
                const double xt = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo) / Lb[u * LB + u];
                if (j == u) xr = xt;
                else if (j < u) xr = fma(-Lb[u * LB + j], xt, xr);
            }
            if (tid < 32 && t0 + j < t1) xv[t0 + j] = xr;
        }
        __syncthreads();
    }
    double *F = Fit + ((size_t)k * R + r) * p;
    for (int i = tid; i < p; i += 256) F[i] = 0.0;
    __syncthreads();
    for (int a = tid; a < s; a += 256) F[idx[a]] = xv[a];
    double Lo = eval_loss(s, idx, xv, GE + (size_t)k * p * p, CE + (size_t)k * p * pe, p, pe, e,
                          sE[(size_t)k * pe + e]);
    if (tid == 0) {
        loss[(size_t)k * R + r] = Lo;
        if (fail) atomicOr(bad, 1);
    }
}

// ---------------------------------------------------------------------------
// Conjugate gradients for the large supports (columns c < nL of each split,
// support Lidx[c]); vectors are [k][p][nL], the mask is the support bitmask.
// ---------------------------------------------------------------------------
struct CgEpi {
    const uint64_t *supp;
    const int32_t *Lidx;
    const uint8_t *state;
    const double *P;
    double *AP, *pAp;
    int p, nL, W;
    __device__ bool tile_active(int b, int r0, int w) const {
        const int lane = threadIdx.x & 63, r = r0 + lane;
        const bool a = lane < w && r < nL && state[(size_t)b * nL + min(r, nL - 1)] == 0;
        return __ballot(a) != 0ull;
    }
    template <class Acc, int FM, int FN>
    __device__ void apply_impl(int b, int i_base, int r0, int lr, int lk, Acc (&acc)[FM][FN]) const {
        for (int c = 0; c < FN; ++c) {
            int r = r0 + 16 * c + lr;
            const int rc = min(r, nL - 1);
            bool ok = r < nL && state[(size_t)b * nL + rc] == 0;
            const uint64_t *sw = supp + (size_t)Lidx[rc] * W;
            double pv[FM][4];
            bool mk[FM][4];
            for (int a = 0; a < FM; ++a)  // loads before the stores of AP, from clamped addresses
                for (int t = 0; t < 4; ++t) {
                    int i = i_base + 16 * a + mfma_row(0.0, lk, t);
                    const int ic = min(i, p - 1);
                    bool in = ok && i < p;
                    mk[a][t] = in && ((sw[ic >> 6] >> (ic & 63)) & 1ull);
                    pv[a][t] = in ? P[((size_t)b * p + ic) * nL + rc] : 0.0;
                }
            double part = 0.0;
            for (int a = 0; a < FM; ++a)
                for (int t = 0; t < 4; ++t) {
                    int i = i_base + 16 * a + mfma_row(0.0, lk, t);
                    if (!ok || i >= p) continue;
                    double ap = mk[a][t] ? (double)acc[a][c][t] : 0.0;
                    AP[((size_t)b * p + i) * nL + r] = ap;
                    part += pv[a][t] * ap;
                }
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            if (ok && lk == 0) atomicAdd(&pAp[(size_t)b * nL + r], part);
        }
    }
    template <class Acc, int FM, int FN>
    __device__ void apply(int b, int i_base, int r0, int lr, int lk, Acc (&acc)[FM][FN]) const {
        apply_impl<Acc, FM, FN>(b, i_base, r0, lr, lk, acc);
    }
};

__global__ void k_cg_init(int nb, int p, int pe, int nL, int W, const uint64_t *__restrict__ supp,
                          const int32_t *__restrict__ Lidx, const double *__restrict__ CT,
                          double *__restrict__ X, double *__restrict__ Rv, double *__restrict__ P,
                          double *__restrict__ rr) {
    int c = blockIdx.x * 64 + (threadIdx.x & 63);
    int i0 = blockIdx.y * 16 + (threadIdx.x >> 6) * 4;
    int k = blockIdx.z;
    if (c >= nL) return;
    int rsup = Lidx[c], e = rsup % pe;
    const uint64_t *sw = supp + (size_t)rsup * W;
    double part = 0.0;
    for (int i = i0; i < min(p, i0 + 4); ++i) {
        bool m = (sw[i >> 6] >> (i & 63)) & 1ull;
        double v = m ? CT[((size_t)k * p + i) * pe + e] : 0.0;
        size_t o = ((size_t)k * p + i) * nL + c;
        X[o] = 0.0;
        Rv[o] = v;
        P[o] = v;
        part += v * v;
    }
    atomicAdd(&rr[(size_t)k * nL + c], part);
}

__global__ void k_cg_update(int p, int nL, const uint8_t *__restrict__ state,
                            const double *__restrict__ rr, const double *__restrict__ pAp,
                            const double *__restrict__ P, const double *__restrict__ AP,
                            double *__restrict__ X, double *__restrict__ Rv, double *__restrict__ rrn) {
    int c = blockIdx.x * 64 + (threadIdx.x & 63);
    int i0 = blockIdx.y * 16 + (threadIdx.x >> 6) * 4;
    int k = blockIdx.z;
    if (c >= nL) return;
    size_t sc = (size_t)k * nL + c;
    if (state[sc]) return;
    double den = pAp[sc];
    double alpha = den > 0.0 ? rr[sc] / den : 0.0;
    double pv[4], xv[4], rv[4], av[4];
    const int n = min(p, i0 + 4) - i0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        size_t o = ((size_t)k * p + i0 + t) * nL + c;
        bool in = t < n;
        pv[t] = in ? P[o] : 0.0;
        xv[t] = in ? X[o] : 0.0;
        rv[t] = in ? Rv[o] : 0.0;
        av[t] = in ? AP[o] : 0.0;
    }
    double part = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t >= n) continue;
        size_t o = ((size_t)k * p + i0 + t) * nL + c;
        X[o] = xv[t] + alpha * pv[t];
        double r = rv[t] - alpha * av[t];
        Rv[o] = r;
        part += r * r;
    }
    atomicAdd(&rrn[sc], part);
}

__global__ void k_cg_dir(int p, int nL, const uint8_t *__restrict__ state,
                         const double *__restrict__ rr, const double *__restrict__ rrn,
                         const double *__restrict__ Rv, double *__restrict__ P) {
    int c = blockIdx.x * 64 + (threadIdx.x & 63);
    int i0 = blockIdx.y * 16 + (threadIdx.x >> 6) * 4;
    int k = blockIdx.z;
    if (c >= nL) return;
    size_t sc = (size_t)k * nL + c;
    if (state[sc]) return;
    double beta = rr[sc] > 0.0 ? rrn[sc] / rr[sc] : 0.0;
    for (int i = i0; i < min(p, i0 + 4); ++i) {
        size_t o = ((size_t)k * p + i) * nL + c;
        P[o] = Rv[o] + beta * P[o];
    }
}

__global__ void k_cg_scalars(int n, double tol2, uint8_t *__restrict__ state, double *__restrict__ rr,
                             double *__restrict__ rrn, const double *__restrict__ rr0,
                             double *__restrict__ pAp, int *__restrict__ active) {
    int sc = blockIdx.x * blockDim.x + threadIdx.x;
    bool act = false;
    if (sc < n && !state[sc]) {
        double v = rrn[sc];
        rr[sc] = v;
        if (v <= tol2 * rr0[sc]) state[sc] = 1;
        else act = true;
    }
    if (sc < n) {
        rrn[sc] = 0.0;
        pAp[sc] = 0.0;
    }
    unsigned long long bal = __ballot(act);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(active, __popcll(bal));
}

// Systems still active when conjugate gradients reached its iteration cap:
// *count += their number.
__global__ void k_count_active(int n, const uint8_t *__restrict__ state, int *__restrict__ count) {
    const int sc = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long bal = __ballot(sc < n && state[sc] == 0);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(count, __popcll(bal));
}

// Scatter the CG solutions into the dense fits and compute their losses.
__global__ __launch_bounds__(256) void k_cg_finish(int p, int pe, int R, int nL, int W,
                                                   const uint64_t *__restrict__ supp,
                                                   const int32_t *__restrict__ Lidx,
                                                   const double *__restrict__ X,
                                                   const double *__restrict__ GE,
                                                   const double *__restrict__ CE,
                                                   const double *__restrict__ sE,
                                                   double *__restrict__ Fit, double *__restrict__ loss) {
    extern __shared__ double dyn[];
    int *idx = reinterpret_cast<int *>(dyn);
    double *bv = dyn + (p + 1) / 2 + 1;
    const int c = blockIdx.x, k = blockIdx.y;
    const int rsup = Lidx[c], e = rsup % pe;
    const int s = support_members(supp + (size_t)rsup * W, W, idx);
    for (int a = threadIdx.x; a < s; a += 256) bv[a] = X[((size_t)k * p + idx[a]) * nL + c];
    __syncthreads();
    double *F = Fit + ((size_t)k * R + rsup) * p;
    for (int i = threadIdx.x; i < p; i += 256) F[i] = 0.0;
    __syncthreads();
    for (int a = threadIdx.x; a < s; a += 256) F[idx[a]] = bv[a];
    double L = eval_loss(s, idx, bv, GE + (size_t)k * p * p, CE + (size_t)k * p * pe, p, pe, e,
                         sE[(size_t)k * pe + e]);
    if (threadIdx.x == 0) loss[(size_t)k * R + rsup] = L;
}

// L[k][j] = sum_e loss[k][j*pe + e]; jstar[k] = first argmin over j.
__global__ void k_argmin(int q, int pe, const double *__restrict__ loss, double *__restrict__ Lq,
                         int32_t *__restrict__ jstar) {
    const int k = blockIdx.x;
    for (int j = threadIdx.x; j < q; j += blockDim.x) {
        double s = 0.0;
        for (int e = 0; e < pe; ++e) s += loss[((size_t)k * q + j) * pe + e];
        Lq[(size_t)k * q + j] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int best = 0;
        for (int j = 1; j < q; ++j)
            if (Lq[(size_t)k * q + j] < Lq[(size_t)k * q + best]) best = j;
        jstar[k] = best;
    }
}

// beta*[e][i] = (1/nb) sum_k Fit[k][jstar_k*pe + e][i]
// j* of split k for equation e: one per split, or one per (split, equation)
__device__ __forceinline__ int chosen(const int32_t *jstar, bool per_eq, int pe, int k, int e) {
    return per_eq ? jstar[(size_t)k * pe + e] : jstar[k];
}

// Per-equation choice: jstar[k][e] = first argmin over j of loss[k][j pe + e].
__global__ void k_argmin_eq(int q, int pe, int R, const double *__restrict__ loss, int32_t *__restrict__ jstar) {
    const int k = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= pe) return;
    const double *L = loss + (size_t)k * R + e;
    int best = 0;
    for (int j = 1; j < q; ++j)
        if (L[(size_t)j * pe] < L[(size_t)best * pe]) best = j;
    jstar[(size_t)k * pe + e] = best;
}

__global__ void k_average(int nb, int p, int pe, int R, bool per_eq, const double *__restrict__ Fit,
                          const int32_t *__restrict__ jstar, double *__restrict__ out) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)pe * p) return;
    int e = (int)(t / p), i = (int)(t % p);
    double s = 0.0;
    for (int k = 0; k < nb; ++k)
        s += Fit[((size_t)k * R + (size_t)chosen(jstar, per_eq, pe, k, e) * pe + e) * p + i];
    out[t] = s / nb;
}

// mu[e] = (1/nb) sum_k (yT[k][e] - xT[k]' Fit[k][jstar_k pe + e]): the intercepts of
// the chosen refits averaged like their coefficients.  One workgroup per equation.
__global__ __launch_bounds__(256) void k_intercept(int nb, int p, int pe, int R, bool per_eq,
                                                   const double *__restrict__ Fit,
                                                   const int32_t *__restrict__ jstar,
                                                   const double *__restrict__ xT,
                                                   const double *__restrict__ yT, double *__restrict__ mu) {
    __shared__ double red[4];
    const int e = blockIdx.x;
    double acc = 0.0;
    for (int k = 0; k < nb; ++k) {
        const double *f = Fit + ((size_t)k * R + (size_t)chosen(jstar, per_eq, pe, k, e) * pe + e) * p;
        const double *x = xT + (size_t)k * p;
        for (int i = threadIdx.x; i < p; i += 256) acc -= x[i] * f[i];
        if (threadIdx.x == 0) acc += yT[(size_t)k * pe + e];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) mu[e] = (red[0] + red[1] + red[2] + red[3]) / nb;
}

// ---------------------------------------------------------------------------
namespace {
size_t mid_scratch_doubles(const EstimProblem &E) {
    const int sm = std::min(E.p, kMid);
    const size_t worst = (size_t)E.nb * E.R * (size_t)(sm + 1) * sm;
    return std::min(worst, kMidScratch / sizeof(double));
}
struct EstimWork {
    int2 *sys;
    size_t *off;
    double *Lmid;
    int32_t *cnt, *Lidx;
    double *Fit, *loss, *Lq;
    double *X, *Rv, *P, *AP, *rr, *rr0, *rrn, *pAp;
    uint8_t *state;
    int *flags;  // [0] bad factor, [1] active count, [2] refits CG left unconverged
};
EstimWork carve(const EstimProblem &E, int nL, Arena &ar) {
    EstimWork w{};
    w.cnt = ar.take<int32_t>(E.R);  // first: the popcounts are written here before the carve
    w.Lidx = ar.take<int32_t>(std::max(nL, 1));
    w.Fit = ar.take<double>((size_t)E.nb * E.R * E.p);
    w.loss = ar.take<double>((size_t)E.nb * E.R);
    w.Lq = ar.take<double>((size_t)E.nb * E.q);
    size_t nv = (size_t)E.nb * E.p * std::max(nL, 1);
    size_t ns = (size_t)E.nb * std::max(nL, 1);
    w.X = ar.take<double>(nv);
    w.Rv = ar.take<double>(nv);
    w.P = ar.take<double>(nv);
    w.AP = ar.take<double>(nv);
    w.rr = ar.take<double>(ns);
    w.rr0 = ar.take<double>(ns);
    w.rrn = ar.take<double>(ns);
    w.pAp = ar.take<double>(ns);
    w.state = ar.take<uint8_t>(ns);
    w.flags = ar.take<int>(3);
    const size_t nsys = (size_t)E.nb * E.R;
    w.sys = ar.take<int2>(nsys);
    w.off = ar.take<size_t>(nsys);
    w.Lmid = E.p > kSmall ? ar.take<double>(mid_scratch_doubles(E)) : nullptr;
    return w;
}
}  // namespace

size_t estim_work_bytes(const EstimProblem &E) {
    // worst case: every support is large
    Arena ar;
    carve(E, E.R, ar);
    return ar.off + 4096;
}

// sizes: the support sizes when the caller already read them back (saves a
// host round trip); the device copy is formed here either way.  flags_host
// (two ints of pinned memory): the singular-refit flag and the number of refits
// that conjugate gradients left above its tolerance are copied there, and the
// caller reads them after synchronising the stream.  dt: where the stage times
// are recorded (resolved by the caller), else resolved here.
void estimate(hipStream_t s, const EstimProblem &E, void *work, double *beta_out, int32_t *jstar,
              double *losses_out, float *stage_ms, const std::vector<int32_t> *sizes, int *flags_host,
              DeferredTiming *dt) {
    const int W = (E.p + 63) / 64;
    UOI_REQUIRE(W <= 1024, "estimation: p must be <= 65536");
    // support sizes decide the solver of every column (they do not depend on k)
    Arena pre;
    pre.base = (char *)work;
    pre.cap = (size_t)-1;
    int32_t *cnt = pre.take<int32_t>(E.R);
    hipLaunchKernelGGL(k_popcount, dim3(cdiv(E.R, 256)), dim3(256), 0, s, E.R, W, E.supp, cnt);
    UOI_LAUNCH_CHECK();
    std::vector<int32_t> hc(E.R);
    if (sizes && (int)sizes->size() == E.R) {
        hc = *sizes;
    } else {
        UOI_HIP(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * E.R, hipMemcpyDeviceToHost, s));
        UOI_HIP(hipStreamSynchronize(s));
    }
    std::vector<int32_t> lidx, mids;
    int smax = 0;
    for (int r = 0; r < E.R; ++r) {
        if (hc[r] > kMid) lidx.push_back(r);
        else if (hc[r] > kSmall) mids.push_back(r);
        else smax = std::max(smax, (int)hc[r]);
    }
    const int nL = (int)lidx.size();
    Arena ar;
    ar.base = (char *)work;
    ar.cap = (size_t)-1;
    EstimWork w = carve(E, nL, ar);
    if (nL) {
        int32_t *pl = (int32_t *)pinned_slot(kPinnedLarge, sizeof(int32_t) * nL);
        std::copy(lidx.begin(), lidx.end(), pl);
        UOI_HIP(hipMemcpyAsync(w.Lidx, pl, sizeof(int32_t) * nL, hipMemcpyHostToDevice, s));
    }
    UOI_HIP(hipMemsetAsync(w.flags, 0, 3 * sizeof(int), s));

    // stage times: recorded in the caller's deferred record, else resolved here
    DeferredTiming local;
    DeferredTiming *dtm = stage_ms ? (dt ? dt : &local) : nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    if (dtm) ev[0] = dtm->mark(s);
    // small supports, on a second stream beside the mid-size ones (they write
    // disjoint systems' results; the mid-size launch ends with a few long systems)
    AuxStream &ax = aux_stream();
    UOI_HIP(hipEventRecord(ax.e0, s));
    UOI_HIP(hipStreamWaitEvent(ax.s, ax.e0, 0));
    size_t lds = sizeof(double) * (size_t)smax * smax;
    hipLaunchKernelGGL(k_ols_small, dim3(E.R, E.nb), dim3(256), lds, ax.s, E.p, E.pe, E.R, W, E.supp,
                       w.cnt, E.GT, E.CT, E.GE, E.CE, E.sE, w.Fit, w.loss, w.flags);
    UOI_LAUNCH_CHECK();
    UOI_HIP(hipEventRecord(ax.e1, ax.s));
    // mid-size supports: blocked Cholesky per (split, support), in chunks that fit
    // the factor scratch
    if (!mids.empty()) {
        const size_t cap = mid_scratch_doubles(E);
        // the system lists of all chunks go to disjoint parts of one pinned
        // buffer, so no copy waits for the host and no list is overwritten early
        const size_t nmid = mids.size() * (size_t)E.nb;
        char *pin = (char *)pinned_slot(kPinnedLists, (sizeof(int2) + sizeof(size_t)) * nmid);
        int2 *psys = (int2 *)pin;
        size_t *poff = (size_t *)(pin + sizeof(int2) * nmid);
        size_t pused = 0;
        std::vector<int2> sys;
        std::vector<size_t> off;
        size_t used = 0;
        auto flush = [&]() {
            if (sys.empty()) return;
            std::copy(sys.begin(), sys.end(), psys + pused);
            std::copy(off.begin(), off.end(), poff + pused);
            UOI_HIP(hipMemcpyAsync(w.sys, psys + pused, sizeof(int2) * sys.size(), hipMemcpyHostToDevice, s));
            UOI_HIP(hipMemcpyAsync(w.off, poff + pused, sizeof(size_t) * off.size(), hipMemcpyHostToDevice, s));
            pused += sys.size();
            hipLaunchKernelGGL(k_ols_mid, dim3((unsigned)sys.size()), dim3(256), 0, s, E.p, E.pe, E.R, W,
                               E.supp, w.sys, w.off, w.Lmid, E.GT, E.CT, E.GE, E.CE, E.sE, w.Fit, w.loss,
                               w.flags);
            UOI_LAUNCH_CHECK();
            // (the next chunk's copies into w.sys / w.off follow this launch on the
            // stream, so the device lists are not overwritten early)
            sys.clear();
            off.clear();
            used = 0;
        };
        // largest systems first: the launch lasts as long as its slowest
        // workgroup, so the long ones must not start in a late round
        std::stable_sort(mids.begin(), mids.end(), [&](int a, int b) { return hc[a] > hc[b]; });
        for (int r : mids)
            for (int k = 0; k < E.nb; ++k) {
                const size_t need = (size_t)(hc[r] + 1) * hc[r];
                if (used + need > cap) flush();
                sys.push_back(make_int2(k, r));
                off.push_back(used);
                used += need;
            }
        flush();
    }
    UOI_HIP(hipStreamWaitEvent(s, ax.e1, 0));
    // large supports by batched conjugate gradients
    if (nL) {
        size_t ns = (size_t)E.nb * nL;
        UOI_HIP(hipMemsetAsync(w.rr, 0, sizeof(double) * ns, s));
        UOI_HIP(hipMemsetAsync(w.rrn, 0, sizeof(double) * ns, s));
        UOI_HIP(hipMemsetAsync(w.pAp, 0, sizeof(double) * ns, s));
        UOI_HIP(hipMemsetAsync(w.state, 0, ns, s));
        dim3 eg(cdiv(nL, 64), cdiv(E.p, 16), E.nb);
        hipLaunchKernelGGL(k_cg_init, eg, dim3(256), 0, s, E.nb, E.p, E.pe, nL, W, E.supp, w.Lidx,
                           E.CT, w.X, w.Rv, w.P, w.rr);
        UOI_HIP(hipMemcpyAsync(w.rr0, w.rr, sizeof(double) * ns, hipMemcpyDeviceToDevice, s));
        UOI_LAUNCH_CHECK();
        CgEpi epi{E.supp, w.Lidx, w.state, w.P, w.AP, w.pAp, E.p, nL, W};
        for (int it = 0; it < E.cg_max_iter; ++it) {
            UOI_DISPATCH_FN(nL, run_bgemm<double, 1, FN>(s, E.nb, E.p, nL, E.GT, w.P, epi));
            hipLaunchKernelGGL(k_cg_update, eg, dim3(256), 0, s, E.p, nL, w.state, w.rr, w.pAp, w.P, w.AP,
                               w.X, w.Rv, w.rrn);
            hipLaunchKernelGGL(k_cg_dir, eg, dim3(256), 0, s, E.p, nL, w.state, w.rr, w.rrn, w.Rv, w.P);
            hipLaunchKernelGGL(k_cg_scalars, dim3(cdiv(ns, 256)), dim3(256), 0, s, (int)ns,
                               kCgTol * kCgTol, w.state, w.rr, w.rrn, w.rr0, w.pAp, w.flags + 1);
            UOI_LAUNCH_CHECK();
            if (it % 8 == 7) {
                int active = 0;
                UOI_HIP(hipMemcpyAsync(&active, w.flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
                UOI_HIP(hipStreamSynchronize(s));
                if (active == 0) break;
            }
            UOI_HIP(hipMemsetAsync(w.flags + 1, 0, sizeof(int), s));
        }
        // systems that reached the cap above the tolerance are counted (the fit
        // reports them as not converged); their current iterates are still used
        hipLaunchKernelGGL(k_count_active, dim3(cdiv(ns, 256)), dim3(256), 0, s, (int)ns, w.state, w.flags + 2);
        UOI_LAUNCH_CHECK();
        size_t lds2 = sizeof(double) * ((size_t)(E.p + 1) / 2 + 1 + E.p);
        UOI_REQUIRE(lds2 <= 64 * 1024, "estimation: p too large for the CG finish kernel");
        hipLaunchKernelGGL(k_cg_finish, dim3(nL, E.nb), dim3(256), lds2, s, E.p, E.pe, E.R, nL, W,
                           E.supp, w.Lidx, w.X, E.GE, E.CE, E.sE, w.Fit, w.loss);
        UOI_LAUNCH_CHECK();
    }
    if (dtm) ev[1] = dtm->mark(s);
    // (the summed losses and their argmin are formed in both modes; with a choice
    // per equation jstar holds [nb][pe] and the losses reported are per equation)
    if (E.per_eq)
        hipLaunchKernelGGL(k_argmin_eq, dim3(cdiv(E.pe, 64), E.nb), dim3(64), 0, s, E.q, E.pe, E.R, w.loss, jstar);
    else
        hipLaunchKernelGGL(k_argmin, dim3(E.nb), dim3(64), 0, s, E.q, E.pe, w.loss, w.Lq, jstar);
    hipLaunchKernelGGL(k_average, dim3(cdiv((size_t)E.pe * E.p, 256)), dim3(256), 0, s, E.nb, E.p, E.pe,
                       E.R, E.per_eq, w.Fit, jstar, beta_out);
    UOI_LAUNCH_CHECK();
    if (E.mu) {
        hipLaunchKernelGGL(k_intercept, dim3(E.pe), dim3(256), 0, s, E.nb, E.p, E.pe, E.R, E.per_eq, w.Fit, jstar,
                           E.xT,
                           E.yT, E.mu);
        UOI_LAUNCH_CHECK();
    }
    if (losses_out && E.per_eq)
        UOI_HIP(hipMemcpyAsync(losses_out, w.loss, sizeof(double) * E.nb * E.R, hipMemcpyDeviceToDevice, s));
    else if (losses_out)
        UOI_HIP(hipMemcpyAsync(losses_out, w.Lq, sizeof(double) * E.nb * E.q, hipMemcpyDeviceToDevice, s));
    if (dtm) {
        ev[2] = dtm->mark(s);
        dtm->time(ev[0], ev[1], &stage_ms[0]);
        dtm->time(ev[1], ev[2], &stage_ms[1]);
        if (dtm == &local) {
            UOI_HIP(hipEventSynchronize(ev[2]));
            local.resolve();
        }
    }
    // [0] singular-refit flag, [1] refits left unconverged by conjugate gradients
    UOI_HIP(hipMemcpyAsync(flags_host, w.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    UOI_HIP(hipMemcpyAsync(flags_host + 1, w.flags + 2, sizeof(int), hipMemcpyDeviceToHost, s));
}

}  // namespace uoi
