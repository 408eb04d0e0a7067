// Lag order d and intercept of UoI_VAR (Alg. 2 for the VAR(d) model of Eq. (5),
// in the regression form of Eq. (6)-(7), returning A_1..A_d and mu).
//
// Design of regression row r (response x_{r+d}): the library reads the d lagged
// observations as one contiguous slice of the row-major series, series[r ..
// r+d-1], i.e. its columns run from lag d to lag 1 (the reverse of Eq. (7)'s
// block order); the fit maps coefficients and support bits to Eq. (7)'s order
// on output (k_var_reorder).
//
// Intercept: the model x_t = mu + sum_l A_l x_{t-l} + u_t with mu unpenalised.
// Profiling mu out of a least-squares term centres the sample, so every
// statistic is taken about a shift (a, b) of the design and response columns:
// for a sample with Gram G = mean x x', cross-products C = mean x y', mean
// squares s = mean y^2 and means (xbar, ybar),
//     G_ab = mean (x - a)(x - a)' = G - xbar a' - a xbar' + a a'
//     C_ab = mean (x - a)(y - b)' = C - xbar b' - a ybar' + a b'
//     s_ab = mean (y - b)^2       = s - 2 ybar b + b^2.
// Selection: every bootstrap sample about its own means (a = xbar).  Estimation:
// the training statistics about the training means, and the evaluation
// statistics about the TRAINING means too, so that the usual loss s - 2 b'c +
// b'Gb of the refits is the mean squared residual y - mu - x'b on the
// evaluation rows with the refit's intercept mu = ybar_T - xbar_T' b.
#include "common.hpp"

namespace uoi {

// xbar[b][c] = sum_a w_a X[r_a][c] / div_b (c < P), likewise ybar with Y, over the
// rows r_a = rows[b m + a], a < mcount[b] (or m); rows == nullptr means the rows
// 0 .. m-1, w == nullptr unit weights, div <= 0 the row count.  Block: 64
// columns x 4 row groups, eight rows loaded per step.
__global__ __launch_bounds__(256) void k_colmeans(int m, const int32_t *__restrict__ rows,
                                                  const int32_t *__restrict__ w,
                                                  const int32_t *__restrict__ mcount, int div, int P,
                                                  const double *__restrict__ X, int ldx, int pe,
                                                  const double *__restrict__ Y, int ldy,
                                                  double *__restrict__ xbar, double *__restrict__ ybar) {
    __shared__ double red[4][64];
    const int b = blockIdx.y, tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + tx, cc = min(c, P + pe - 1);
    const double *src = cc < P ? X + cc : Y + (cc - P);
    const size_t ld = cc < P ? (size_t)ldx : (size_t)ldy;
    const int mb = mcount ? mcount[b] : m;
    const int32_t *rb = rows ? rows + (size_t)b * m : nullptr;
    const int32_t *wb = w ? w + (size_t)b * m : nullptr;
    double acc = 0.0;
    for (int a0 = ty; a0 < mb; a0 += 32) {
        int r[8];
        double wt[8], v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int a = min(a0 + 4 * u, mb - 1);
            r[u] = rb ? rb[a] : a;
            wt[u] = a0 + 4 * u < mb ? (wb ? (double)wb[a] : 1.0) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[(size_t)r[u] * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += wt[u] * v[u];
    }
    red[ty][tx] = acc;
    __syncthreads();
    if (ty == 0 && c < P + pe) {
        const double tot = red[0][tx] + red[1][tx] + red[2][tx] + red[3][tx];
        const double mean = tot / (double)(div > 0 ? div : mb);
        if (c < P) xbar[(size_t)b * P + c] = mean;
        else ybar[(size_t)b * pe + (c - P)] = mean;
    }
}

// Statistics about the shift (a, b): see the file comment.  G [nb][P][P],
// C [nb][P][pe], s [nb][pe] (nullable); xm, ym the sample means, a, bv the shift.
__global__ void k_shift_stats(int P, int pe, double *__restrict__ G, double *__restrict__ C,
                              double *__restrict__ s, const double *__restrict__ xm,
                              const double *__restrict__ ym, const double *__restrict__ a,
                              const double *__restrict__ bv) {
    const int k = blockIdx.y;
    const double *xk = xm + (size_t)k * P, *ak = a + (size_t)k * P;
    const double *yk = ym + (size_t)k * pe, *bk = bv + (size_t)k * pe;
    const size_t nG = (size_t)P * P, nC = (size_t)P * pe, n = nG + nC + (s ? pe : 0);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        if (t < nG) {
            const int i = (int)(t / P), j = (int)(t % P);
            G[(size_t)k * nG + t] += -xk[i] * ak[j] - ak[i] * xk[j] + ak[i] * ak[j];
        } else if (t < nG + nC) {
            const size_t u = t - nG;
            const int i = (int)(u / pe), e = (int)(u % pe);
            C[(size_t)k * nC + u] += -xk[i] * bk[e] - ak[i] * yk[e] + ak[i] * bk[e];
        } else {
            const int e = (int)(t - nG - nC);
            s[(size_t)k * pe + e] += -2.0 * yk[e] * bk[e] + bk[e] * bk[e];
        }
    }
}

// Training means from the full-data means and the evaluation means (the split
// partitions the N rows): xT = (N xA - ne xE) / (N - ne), likewise for y.
__global__ void k_train_means(int P, int pe, int N, const double *__restrict__ xA,
                              const double *__restrict__ yA, const int32_t *__restrict__ nev,
                              const double *__restrict__ xE, const double *__restrict__ yE,
                              double *__restrict__ xT, double *__restrict__ yT) {
    const int k = blockIdx.y;
    const double ne = (double)nev[k], nt = (double)(N - nev[k]);
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < P + pe; c += gridDim.x * blockDim.x) {
        if (c < P) xT[(size_t)k * P + c] = ((double)N * xA[c] - ne * xE[(size_t)k * P + c]) / nt;
        else yT[(size_t)k * pe + c - P] = ((double)N * yA[c - P] - ne * yE[(size_t)k * pe + c - P]) / nt;
    }
}

// Output in Eq. (7)'s order: A[l][e][m] = beta[e][(d-1-l) p + m] (lag l+1), and
// support bit l p + m of equation e = internal bit (d-1-l) p + m.
__global__ void k_var_reorder(int q, int p, int d, const uint64_t *__restrict__ sin,
                              uint64_t *__restrict__ sout, const double *__restrict__ beta,
                              double *__restrict__ A) {
    const int P = d * p, W = (P + 63) / 64;
    const size_t nA = (size_t)d * p * p, nS = (size_t)q * p * W;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nA + nS;
         t += (size_t)gridDim.x * blockDim.x) {
        if (t < nA) {
            const int l = (int)(t / ((size_t)p * p)), e = (int)((t / p) % p), m = (int)(t % p);
            A[t] = beta[(size_t)e * P + (size_t)(d - 1 - l) * p + m];
        } else {
            const size_t u = t - nA;
            const size_t je = u / W;
            const int wd = (int)(u % W);
            const uint64_t *src = sin + je * W;
            uint64_t word = 0;
            for (int x = wd * 64; x < min(P, wd * 64 + 64); ++x) {
                const int l = x / p, m = x % p, xi = (d - 1 - l) * p + m;
                word |= ((src[xi >> 6] >> (xi & 63)) & 1ull) << (x & 63);
            }
            sout[u] = word;
        }
    }
}

void launch_colmeans(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *w,
                     const int32_t *mcount, int div, int P, const double *X, int ldx, int pe,
                     const double *Y, int ldy, double *xbar, double *ybar) {
    hipLaunchKernelGGL(k_colmeans, dim3(cdiv(P + pe, 64), nb), dim3(256), 0, s, m, rows, w, mcount, div, P,
                       X, ldx, pe, Y, ldy, xbar, ybar);
    UOI_LAUNCH_CHECK();
}

void launch_shift_stats(hipStream_t s, int nb, int P, int pe, double *G, double *C, double *ss,
                        const double *xm, const double *ym, const double *a, const double *b) {
    const size_t n = (size_t)P * P + (size_t)P * pe + (ss ? pe : 0);
    hipLaunchKernelGGL(k_shift_stats, dim3(std::min<size_t>(cdiv(n, 256), 1024), nb), dim3(256), 0, s, P, pe,
                       G, C, ss, xm, ym, a, b);
    UOI_LAUNCH_CHECK();
}

void launch_train_means(hipStream_t s, int nb, int P, int pe, int N, const double *xA, const double *yA,
                        const int32_t *nev, const double *xE, const double *yE, double *xT, double *yT) {
    hipLaunchKernelGGL(k_train_means, dim3(cdiv(P + pe, 256), nb), dim3(256), 0, s, P, pe, N, xA, yA, nev, xE,
                       yE, xT, yT);
    UOI_LAUNCH_CHECK();
}

void launch_var_reorder(hipStream_t s, int q, int p, int d, const uint64_t *supp_in, uint64_t *supp_out,
                        const double *beta, double *A) {
    const size_t n = (size_t)d * p * p + (size_t)q * p * ((d * p + 63) / 64);
    hipLaunchKernelGGL(k_var_reorder, dim3(std::min<size_t>(cdiv(n, 256), 4096)), dim3(256), 0, s, q, p, d,
                       supp_in, supp_out, beta, A);
    UOI_LAUNCH_CHECK();
}

}  // namespace uoi
