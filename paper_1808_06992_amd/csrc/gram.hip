// Gram of sampled rows on float64 MFMA: G_b = X_r'X_r / m and C_b = X_r'Y_r / m.
//
// These are the normal-equation statistics of the bootstrap samples T^k of
// Alg. 1 / Alg. 2; the bootstrap is a row gather inside the kernel, so no
// resampled copy of X is ever written.  The product dominates the paper's
// single-node profile (its matrix multiplication inside LASSO-ADMM, Sec. IV-A.1).
//
// Work decomposition: 64x64 output tiles; G is symmetric, so only tiles on or
// below the diagonal are computed and each is written to both halves.  A tile
// streams the sampled rows in chunks of 16 through LDS; 4 waves each own a
// 32x32 quadrant as 2x2 MFMA 16x16x4 blocks.
#include "common.hpp"

namespace uoi {

namespace {
constexpr int GT = 64;   // tile edge
constexpr int GK = 16;   // rows per LDS chunk
}

__global__ __launch_bounds__(256) void k_gram_f64(int m, const int32_t *__restrict__ rows,
                                                  const int32_t *__restrict__ mcount, int p,
                                                  const double *__restrict__ X, int ldx, int pe,
                                                  const double *__restrict__ Y, int ldy,
                                                  double *__restrict__ G, double *__restrict__ C,
                                                  int T, int Tc) {
    __shared__ double As[GK][GT];
    __shared__ double Bs[GK][GT];
    const int b = blockIdx.y;
    int tile = blockIdx.x;
    const int ntri = T * (T + 1) / 2;
    int ti, tj;
    bool isC;
    if (tile < ntri) {
        // tile -> (ti, tj) with tj <= ti, row-major over the lower triangle
        ti = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
        while (ti * (ti + 1) / 2 > tile) --ti;
        tj = tile - ti * (ti + 1) / 2;
        isC = false;
    } else {
        tile -= ntri;
        ti = tile / Tc;
        tj = tile % Tc;
        isC = true;
    }
    const int i0 = ti * GT, j0 = tj * GT;
    const int mb = mcount ? mcount[b] : m;
    const int32_t *rb = rows + (size_t)b * m;
    const double *Bsrc = isC ? Y : X;
    const int ldb = isC ? ldy : ldx;
    const int nb_cols = isC ? pe : p;

    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int lr = lane & 15, lk = lane >> 4;

    dx4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) acc[a][c] = dx4{0, 0, 0, 0};

    for (int k0 = 0; k0 < mb; k0 += GK) {
        // stage 16 gathered rows: columns [i0, i0+64) of X and [j0, j0+64) of X or Y
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int e = threadIdx.x + 256 * t;
            int kk = e >> 6, cc = e & 63;
            double va = 0.0, vb = 0.0;
            if (k0 + kk < mb) {
                size_t r = (size_t)rb[k0 + kk];
                if (i0 + cc < p) va = X[r * ldx + i0 + cc];
                if (j0 + cc < nb_cols) vb = Bsrc[r * ldb + j0 + cc];
            }
            As[kk][cc] = va;
            Bs[kk][cc] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < GK / 4; ++s) {
            double a0 = As[4 * s + lk][wm * 32 + lr];
            double a1 = As[4 * s + lk][wm * 32 + 16 + lr];
            double b0 = Bs[4 * s + lk][wn * 32 + lr];
            double b1 = Bs[4 * s + lk][wn * 32 + 16 + lr];
            acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
            acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
            acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
            acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }

    const double inv = 1.0 / (double)mb;
    for (int fm = 0; fm < 2; ++fm)
        for (int fn = 0; fn < 2; ++fn)
            for (int t = 0; t < 4; ++t) {
                int i = i0 + wm * 32 + fm * 16 + mfma_row(0.0, lk, t);
                int j = j0 + wn * 32 + fn * 16 + lr;
                double v = acc[fm][fn][t] * inv;
                if (isC) {
                    if (i < p && j < pe) C[((size_t)b * p + i) * pe + j] = v;
                } else if (i < p && j < p) {
                    G[((size_t)b * p + i) * p + j] = v;
                    G[((size_t)b * p + j) * p + i] = v;
                }
            }
}

// ss[b][e] = sum over sampled rows of Y[r][e]^2 / m
__global__ __launch_bounds__(256) void k_colsq(int m, const int32_t *__restrict__ rows,
                                               const int32_t *__restrict__ mcount, int pe,
                                               const double *__restrict__ Y, int ldy,
                                               double *__restrict__ ss) {
    __shared__ double part[4][64];
    int b = blockIdx.y;
    int e = blockIdx.x * 64 + (threadIdx.x & 63);
    int ph = threadIdx.x >> 6;
    int mb = mcount ? mcount[b] : m;
    const int32_t *rb = rows + (size_t)b * m;
    double acc = 0.0;
    if (e < pe)
        for (int k = ph; k < mb; k += 4) {
            double v = Y[(size_t)rb[k] * ldy + e];
            acc += v * v;
        }
    part[ph][threadIdx.x & 63] = acc;
    __syncthreads();
    if (ph == 0 && e < pe) {
        double s = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                   part[3][threadIdx.x];
        ss[(size_t)b * pe + e] = s / (double)mb;
    }
}

void launch_gram_f64(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *mcount,
                     int p, const double *X, int ldx, int pe, const double *Y, int ldy,
                     double *G, double *C) {
    int T = (int)cdiv(p, GT);
    int Tc = (C != nullptr && pe > 0) ? (int)cdiv(pe, GT) : 0;
    int tiles = T * (T + 1) / 2 + T * Tc;
    hipLaunchKernelGGL(k_gram_f64, dim3(tiles, nb), dim3(256), 0, s, m, rows, mcount, p, X, ldx,
                       pe, Y, ldy, G, C, T, Tc);
    UOI_LAUNCH_CHECK();
}

void launch_colsq(hipStream_t s, int nb, int m, const int32_t *rows, const int32_t *mcount,
                  int pe, const double *Y, int ldy, double *ss) {
    hipLaunchKernelGGL(k_colsq, dim3(cdiv(pe, 64), nb), dim3(256), 0, s, m, rows, mcount, pe, Y,
                       ldy, ss);
    UOI_LAUNCH_CHECK();
}

}  // namespace uoi
