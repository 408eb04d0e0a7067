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
// Per block step: (1) one workgroup per matrix sweeps the kb x kb pivot block
// in LDS; (2) a row-parallel kernel forms W = A_:K Q and keeps the old panel
// A_:K; (3) a tiled MFMA kernel applies the rank-kb update to the whole matrix.
#include "common.hpp"

namespace uoi {

namespace {
constexpr int NB = 64;     // pivot block
constexpr int SMALL = 88;  // whole-matrix in-LDS sweep up to this size (LDS <= 64 KB)
}

// Unblocked symmetric sweep of an n x n matrix held in LDS (row stride ld).
// Leaves -A^{-1} in place.
__device__ void lds_sweep(double *A, int n, int ld) {
    for (int k = 0; k < n; ++k) {
        const double pinv = 1.0 / A[k * ld + k];
        // update the off-pivot part first: it reads row/column k only
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            int i = e / n, j = e % n;
            if (i != k && j != k) A[i * ld + j] -= A[i * ld + k] * A[k * ld + j] * pinv;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if (i != k) {
                A[i * ld + k] *= pinv;
                A[k * ld + i] = A[i * ld + k];
            }
        __syncthreads();
        if (threadIdx.x == 0) A[k * ld + k] = -pinv;
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
    lds_sweep(A, p, p);
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

// (1) Q = A_KK^{-1} (stored as +Q) for pivot block [k0, k0+kb).
__global__ __launch_bounds__(256) void k_pivot(int p, int k0, int kb, const double *__restrict__ A,
                                               double *__restrict__ Q) {
    __shared__ double S[NB * NB];
    const int b = blockIdx.x;
    const double *Ab = A + (size_t)b * p * p;
    for (int e = threadIdx.x; e < kb * kb; e += 256) {
        int i = e / kb, j = e % kb;
        S[i * kb + j] = Ab[(size_t)(k0 + i) * p + k0 + j];
    }
    __syncthreads();
    lds_sweep(S, kb, kb);
    double *Qb = Q + (size_t)b * NB * NB;
    for (int e = threadIdx.x; e < kb * kb; e += 256) Qb[e] = -S[e];
}

// (2) W[i] = A[i, K] Q and Old[i] = A[i, K] for every row i (row-major, width NB).
__global__ __launch_bounds__(256) void k_panel(int p, int k0, int kb, const double *__restrict__ A,
                                               const double *__restrict__ Q, double *__restrict__ W,
                                               double *__restrict__ Old) {
    __shared__ double Qs[NB * NB];
    const int b = blockIdx.y;
    const double *Qb = Q + (size_t)b * NB * NB;
    for (int e = threadIdx.x; e < kb * kb; e += 256) Qs[e] = Qb[e];
    __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= p) return;
    const double *row = A + ((size_t)b * p + i) * p + k0;
    double *Wr = W + ((size_t)b * p + i) * NB;
    double *Or = Old + ((size_t)b * p + i) * NB;
    double a[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        a[t] = t < kb ? row[t] : 0.0;
        Or[t] = a[t];
    }
    for (int j = 0; j < NB; ++j) {
        double acc = 0.0;
        if (j < kb) {
#pragma unroll
            for (int t = 0; t < NB; ++t) acc += a[t] * (t < kb ? Qs[t * kb + j] : 0.0);
        }
        Wr[j] = acc;
    }
}

// (3) Rank-kb update of a 64x64 tile of A:
//   i,j not in K: A_ij -= W_i . Old_j ;  i not in K, j in K: A_ij = W_i[j-k0]
//   i in K, j not in K: A_ij = W_j[i-k0] ;  i, j in K: A_ij = -Q
__global__ __launch_bounds__(256) void k_update(int p, int k0, int kb, double *__restrict__ A,
                                                const double *__restrict__ W,
                                                const double *__restrict__ Old,
                                                const double *__restrict__ Q) {
    // pivot-index-major staging: Ws[t][r] = W[i0 + r][t], Os[t][r] = Old[j0 + r][t]
    __shared__ double Ws[NB][64];
    __shared__ double Os[NB][64];
    const int b = blockIdx.z;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const double *Wb = W + (size_t)b * p * NB;
    const double *Ob = Old + (size_t)b * p * NB;
    for (int e = threadIdx.x; e < 64 * NB; e += 256) {
        int r = e / NB, t = e % NB;
        Ws[t][r] = (i0 + r < p) ? Wb[(size_t)(i0 + r) * NB + t] : 0.0;
        Os[t][r] = (j0 + r < p) ? Ob[(size_t)(j0 + r) * NB + t] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int lr = lane & 15, lk = lane >> 4;
    dx4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) acc[a][c] = dx4{0, 0, 0, 0};
    for (int s = 0; s < NB / 4; ++s) {
        double a0 = Ws[4 * s + lk][wm * 32 + lr];
        double a1 = Ws[4 * s + lk][wm * 32 + 16 + lr];
        double b0 = Os[4 * s + lk][wn * 32 + lr];
        double b1 = Os[4 * s + lk][wn * 32 + 16 + lr];
        acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
        acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
        acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
        acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
    double *Ab = A + (size_t)b * p * p;
    const double *Qb = Q + (size_t)b * NB * NB;
    for (int fm = 0; fm < 2; ++fm)
        for (int fn = 0; fn < 2; ++fn)
            for (int t = 0; t < 4; ++t) {
                int il = wm * 32 + fm * 16 + mfma_row(0.0, lk, t), jl = wn * 32 + fn * 16 + lr;
                int i = i0 + il, j = j0 + jl;
                if (i >= p || j >= p) continue;
                bool iK = i >= k0 && i < k0 + kb, jK = j >= k0 && j < k0 + kb;
                double *dst = Ab + (size_t)i * p + j;
                if (!iK && !jK) *dst -= acc[fm][fn][t];        // A_ij - A_iK Q A_Kj
                else if (!iK) *dst = Ws[j - k0][il];             // A_iK Q
                else if (!jK) *dst = Wb[(size_t)j * NB + (i - k0)];  // Q A_Kj = (A_jK Q)'
                else *dst = -Qb[(i - k0) * kb + (j - k0)];       // -Q
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
    for (int k0 = 0; k0 < p; k0 += NB) {
        int kb = std::min(NB, p - k0);
        hipLaunchKernelGGL(k_pivot, dim3(nb), dim3(256), 0, s, p, k0, kb, M, Q);
        hipLaunchKernelGGL(k_panel, dim3(cdiv(p, 256), nb), dim3(256), 0, s, p, k0, kb, M, Q, W, Old);
        hipLaunchKernelGGL(k_update, dim3(cdiv(p, 64), cdiv(p, 64), nb), dim3(256), 0, s, p, k0, kb,
                           M, W, Old, Q);
        UOI_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_negate, dim3(cdiv(n, 256)), dim3(256), 0, s, n, M);
    UOI_LAUNCH_CHECK();
}

}  // namespace uoi
