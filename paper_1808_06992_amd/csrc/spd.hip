// Batched inverse M = (G + rho I)^{-1} in float64 for the ADMM x-update.
//
// The paper factors (X'X + rho I) once and applies it with triangular solves
// every iteration (its "triangular solve" routine, Sec. IV-A.1).  Here the
// inverse is formed once per bootstrap so that every ADMM iteration becomes a
// matrix product.  It is computed by the symmetric sweep operator (block
// Gauss-Jordan): sweeping pivot block K of a symmetric A with Q = A_KK^{-1}
//     A_ij <- A_ij - A_iK Q A_Kj   (i, j not in K)
//     A_iK <- A_iK Q,  A_Kj <- Q A_Kj,  A_KK <- -Q
// and sweeping every block leaves -A^{-1}.  Pivots are Schur complements of
// an SPD matrix, so no pivoting is needed.
//
// Per block step: (1) one workgroup per matrix sweeps the kb x kb pivot block in
// LDS (Q = A_KK^{-1}); (2) a row-parallel MFMA kernel forms W = A_:K Q and keeps
// the old panel A_:K; (3) a tiled MFMA kernel applies the rank-kb update to the
// whole matrix.
#include "common.hpp"

namespace uoi {

namespace {
constexpr int NB = 64;     // pivot block
constexpr int SMALL = 88;  // whole-matrix in-LDS sweep up to this size (LDS <= 64 KB)
}

// Unblocked symmetric sweep of an n x n matrix held in LDS (row stride ld).
// Leaves -A^{-1} in place.  256 threads; thread (ty, tx) = (tid/16, tid%16)
// owns rows ty + 16a and columns tx + 16c (n <= 16 MB).
template <int MB>  // rows / columns per thread: n <= 16 * MB
__device__ void lds_sweep(double *A, int n, int ld) {
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    for (int k = 0; k < n; ++k) {
        const double pinv = 1.0 / A[k * ld + k];
        // off-pivot update; it reads row and column k only, so every operand is
        // loaded before any store of this phase
        double ak[MB], rk[MB], v[MB][MB];
#pragma unroll
        for (int a = 0; a < MB; ++a) {
            const int i = ty + 16 * a, j = tx + 16 * a;
            ak[a] = i < n ? A[i * ld + k] * pinv : 0.0;
            rk[a] = j < n ? A[k * ld + j] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int c = 0; c < MB; ++c) {
                const int i = ty + 16 * a, j = tx + 16 * c;
                v[a][c] = (i < n && j < n) ? A[i * ld + j] : 0.0;
            }
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int c = 0; c < MB; ++c) {
                const int i = ty + 16 * a, j = tx + 16 * c;
                if (i < n && j < n && i != k && j != k) A[i * ld + j] = v[a][c] - ak[a] * rk[c];
            }
        __syncthreads();
        // pivot row / column scaling and the pivot itself
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            if (i != k) {
                const double x = A[i * ld + k] * pinv;
                A[i * ld + k] = x;
                A[k * ld + i] = x;
            } else {
                A[k * ld + k] = -pinv;
            }
        }
        __syncthreads();
    }
}

// Whole-matrix inverse for p <= SMALL: M = (G + rho I)^{-1}.
__global__ __launch_bounds__(256) void k_inv_small(int p, const double *__restrict__ G, double rho,
                                                   double *__restrict__ M) {
    extern __shared__ double A[];
    const int b = blockIdx.x;
    const double *Gb = G + (size_t)b * p * p;
    for (int e = threadIdx.x; e < p * p; e += 256) {
        int i = e / p, j = e % p;
        A[e] = Gb[e] + (i == j ? rho : 0.0);
    }
    __syncthreads();
    lds_sweep<6>(A, p, p);
    double *Mb = M + (size_t)b * p * p;
    for (int e = threadIdx.x; e < p * p; e += 256) Mb[e] = -A[e];
}

// M = G + rho I (the matrix that the blocked sweep works on in place)
__global__ void k_shift_copy(size_t n, int p, const double *__restrict__ G, double rho,
                             double *__restrict__ M) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) {
        size_t w = e % ((size_t)p * p);
        int i = (int)(w / p), j = (int)(w % p);
        M[e] = G[e] + (i == j ? rho : 0.0);
    }
}

__global__ void k_negate(size_t n, double *__restrict__ M) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) M[e] = -M[e];
}

// (1) Q = A_KK^{-1} for pivot block [k0, k0+kb) (one workgroup per matrix).
__global__ __launch_bounds__(256) void k_pivot(int p, int k0, int kb, const double *__restrict__ A,
                                               double *__restrict__ Q) {
    constexpr int LD = NB + 1;
    __shared__ double S[NB * LD];
    const int b = blockIdx.x;
    const double *Ab = A + (size_t)b * p * p;
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        int i = e / NB, j = e % NB;
        if (i < kb && j < kb) S[i * LD + j] = Ab[(size_t)(k0 + i) * p + k0 + j];
    }
    __syncthreads();
    lds_sweep<4>(S, kb, LD);  // S = -Q
    double *Qb = Q + (size_t)b * NB * NB;
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        int i = e / NB, j = e % NB;
        Qb[e] = (i < kb && j < kb) ? -S[i * LD + j] : 0.0;  // stored NB x NB, zero padded
    }
}

// (2) Panel for rows [i0, i0+64): Old = A[i, K], W = A[i, K] Q on MFMA.
__global__ __launch_bounds__(256) void k_panel(int p, int k0, int kb, const double *__restrict__ A,
                                               const double *__restrict__ Q, double *__restrict__ W,
                                               double *__restrict__ Old) {
    constexpr int LD = 64 + 1;
    __shared__ double As[NB * LD];  // As[t][r] = A[i0 + r][k0 + t]
    __shared__ double Qs[NB * LD];  // Qs[t][c] = Q[t][c]
    const int b = blockIdx.y;
    const int i0 = blockIdx.x * 64;
    const double *Ab = A + (size_t)b * p * p;
    const double *Qb = Q + (size_t)b * NB * NB;
    double *Ob = Old + (size_t)b * p * NB;
    // Only the lower-triangle 128-tiles (and whole diagonal tiles) of A are kept up to
    // date, so rows in a tile above the pivot's tile read A[i][K] as A[K][i].
    const bool above = (i0 / 128) < (k0 / 128);
    for (int e = threadIdx.x; e < 64 * NB; e += 256) {
        int r, t;
        if (above) { t = e / 64; r = e % 64; }   // coalesced along i
        else { r = e / NB; t = e % NB; }          // coalesced along k
        double v = 0.0;
        if (i0 + r < p && t < kb)
            v = above ? Ab[(size_t)(k0 + t) * p + i0 + r] : Ab[(size_t)(i0 + r) * p + k0 + t];
        As[t * LD + r] = v;
        if (i0 + r < p) Ob[(size_t)(i0 + r) * NB + t] = v;
    }
    for (int e = threadIdx.x; e < NB * NB; e += 256) Qs[(e / NB) * LD + e % NB] = Qb[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int lr = lane & 15, lk = lane >> 4;
    dx4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) acc[a][c] = dx4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) {
        double a0 = As[(4 * s + lk) * LD + wm * 32 + lr];
        double a1 = As[(4 * s + lk) * LD + wm * 32 + 16 + lr];
        double b0 = Qs[(4 * s + lk) * LD + wn * 32 + lr];
        double b1 = Qs[(4 * s + lk) * LD + wn * 32 + 16 + lr];
        acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
        acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
        acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
        acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
    double *Wb = W + (size_t)b * p * NB;
    for (int fm = 0; fm < 2; ++fm)
        for (int fn = 0; fn < 2; ++fn)
            for (int t = 0; t < 4; ++t) {
                int r = wm * 32 + fm * 16 + mfma_row(0.0, lk, t), c = wn * 32 + fn * 16 + lr;
                if (i0 + r < p) Wb[(size_t)(i0 + r) * NB + c] = acc[fm][fn][t];
            }
}

// (3) Rank-kb update of a 128x128 tile of A (tiles on or below the diagonal only;
// the sweep keeps A symmetric, the upper triangle is filled in at the end):
//   i,j not in K: A_ij -= W_i . Old_j ;  i not in K, j in K: A_ij = W_i[j-k0]
//   i in K, j not in K: A_ij = W_j[i-k0] ;  i, j in K: A_ij = -Q
// W and Old are staged through LDS in quarters of the pivot index, transposed
// (pivot-index-major, padded rows) so that the MFMA operand reads are conflict
// free; each wave owns a 64x64 quadrant as 4x4 MFMA blocks.
__global__ __launch_bounds__(256, 2) void k_update(int p, int k0, int kb, double *__restrict__ A,
                                                   const double *__restrict__ W,
                                                   const double *__restrict__ Old,
                                                   const double *__restrict__ Q) {
    constexpr int QK = 16, LD = 128 + 1;
    __shared__ double Ws[QK * LD];
    __shared__ double Os[QK * LD];
    int tile, by0, b;
    xcd_tile(tile, by0, b);  // all tiles of one matrix on one XCD: W, Old stay in its L2
    // tile -> (ti, tj), tj <= ti: only the lower triangle (and whole diagonal tiles)
    int ti = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
    while (ti * (ti + 1) / 2 > tile) --ti;
    const int tj = tile - ti * (ti + 1) / 2;
    const int i0 = ti * 128, j0 = tj * 128;
    const double *Wb = W + (size_t)b * p * NB;
    const double *Ob = Old + (size_t)b * p * NB;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int lr = lane & 15, lk = lane >> 4;
    dx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = dx4{0, 0, 0, 0};
    const int nq = (kb + QK - 1) / QK;
    for (int h = 0; h < nq; ++h) {
        for (int e = threadIdx.x; e < 128 * QK; e += 256) {
            int r = e / QK, t = e % QK;
            Ws[t * LD + r] = (i0 + r < p) ? Wb[(size_t)(i0 + r) * NB + h * QK + t] : 0.0;
            Os[t * LD + r] = (j0 + r < p) ? Ob[(size_t)(j0 + r) * NB + h * QK + t] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < QK / 4; ++s) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = Ws[(4 * s + lk) * LD + wm * 64 + 16 * a + lr];
#pragma unroll
            for (int a = 0; a < 4; ++a) bv[a] = Os[(4 * s + lk) * LD + wn * 64 + 16 * a + lr];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] = mfma16x16x4(av[a], bv[c], acc[a][c]);
        }
        __syncthreads();
    }
    double *Ab = A + (size_t)b * p * p;
    const double *Qb = Q + (size_t)b * NB * NB;
    const bool plain = !(i0 < k0 + kb && i0 + 128 > k0) && !(j0 < k0 + kb && j0 + 128 > k0);
#pragma unroll
    for (int fm = 0; fm < 4; ++fm) {
        // read-modify-write one 16-row band: loads first, then stores
        double old[4][4];
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = i0 + wm * 64 + fm * 16 + mfma_row(0.0, lk, t);
                const int j = j0 + wn * 64 + fn * 16 + lr;
                old[fn][t] = (i < p && j < p) ? Ab[(size_t)i * p + j] : 0.0;
            }
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = i0 + wm * 64 + fm * 16 + mfma_row(0.0, lk, t);
                const int j = j0 + wn * 64 + fn * 16 + lr;
                if (i >= p || j >= p) continue;
                double v = old[fn][t] - acc[fm][fn][t];             // A_ij - A_iK Q A_Kj
                if (!plain) {
                    const bool iK = i >= k0 && i < k0 + kb, jK = j >= k0 && j < k0 + kb;
                    if (iK && jK) v = -Qb[(i - k0) * NB + (j - k0)];      // -Q
                    else if (jK) v = Wb[(size_t)i * NB + (j - k0)];       // A_iK Q
                    else if (iK) v = Wb[(size_t)j * NB + (i - k0)];       // Q A_Kj = (A_jK Q)'
                }
                Ab[(size_t)i * p + j] = v;
            }
    }
}

size_t spd_inverse_work_doubles(int nb, int p) {
    if (p <= SMALL) return 0;
    return (size_t)nb * NB * NB + 2 * (size_t)nb * p * NB;
}

void spd_inverse_f64(hipStream_t s, int nb, int p, const double *G, double rho, double *M,
                     double *work) {
    if (p <= SMALL) {
        size_t lds = sizeof(double) * (size_t)p * p;
        hipLaunchKernelGGL(k_inv_small, dim3(nb), dim3(256), lds, s, p, G, rho, M);
        UOI_LAUNCH_CHECK();
        return;
    }
    double *Q = work;
    double *W = Q + (size_t)nb * NB * NB;
    double *Old = W + (size_t)nb * p * NB;
    size_t n = (size_t)nb * p * p;
    hipLaunchKernelGGL(k_shift_copy, dim3(cdiv(n, 256)), dim3(256), 0, s, n, p, G, rho, M);
    UOI_LAUNCH_CHECK();
    const int T = (int)cdiv(p, 128);
    for (int k0 = 0; k0 < p; k0 += NB) {
        int kb = std::min(NB, p - k0);
        hipLaunchKernelGGL(k_pivot, dim3(nb), dim3(256), 0, s, p, k0, kb, M, Q);
        hipLaunchKernelGGL(k_panel, dim3(cdiv(p, 64), nb), dim3(256), 0, s, p, k0, kb, M, Q, W, Old);
        hipLaunchKernelGGL(k_update, dim3(T * (T + 1) / 2, 1, nb), dim3(256), 0, s, p, k0, kb, M, W, Old, Q);
        UOI_LAUNCH_CHECK();
    }
    launch_symmetrize(s, nb, p, M);
    hipLaunchKernelGGL(k_negate, dim3(cdiv(n, 256)), dim3(256), 0, s, n, M);
    UOI_LAUNCH_CHECK();
}

}  // namespace uoi
