// Batched inverse M = (G + rho I)^{-1} in float64 for the ADMM x-update.
//
// The paper factors (X'X + rho I) once and applies it with triangular solves
// every iteration (the triangular-solve routine of its profile, Sec. IV-A.1).  Here the
// inverse is formed once per bootstrap so that every ADMM iteration becomes a
// matrix product.  It is computed by the symmetric sweep operator (block
// Gauss-Jordan): sweeping pivot block K of a symmetric A with Q = A_KK^{-1}
//     A_ij <- A_ij - A_iK Q A_Kj   (i, j not in K)
//     A_iK <- A_iK Q,  A_Kj <- Q A_Kj,  A_KK <- -Q
// and sweeping every block leaves -A^{-1}.  Pivots are Schur complements of
// an SPD matrix, so no pivoting is needed.
//
// Per 64-wide block step: (1) one workgroup per matrix sweeps the pivot block
// in registers (Q = A_KK^{-1}), inside the previous step's update after the
// first step; (2) a row-parallel MFMA kernel forms W = A_:K Q
// and keeps the old panel A_:K, both stored pivot-index-major; (3) an MFMA kernel
// applies the rank-64 update to the 64x64 tiles on and below the diagonal (the
// sweep keeps A symmetric).  The first step reads G and adds rho on the
// diagonal, so no shifted copy is made; the last step stores the negated result
// in both triangles.
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

// (1) Q = A_KK^{-1} of the pivot block [k0, k0+kb) of one matrix, by one
// workgroup of 256 threads.  Thread (ty, tx) = (tid / 64, tid % 64) keeps rows
// ty + 4a (a < 16) of column tx in registers for all 64 steps (the block is
// padded with the identity beyond kb, which leaves the kb x kb part unchanged);
// step k publishes the old pivot row and column through LDS, double-buffered
// by step parity so that one barrier per step suffices.  LDS reads are
// broadcasts or unit-stride.  The first block step reads G and adds the shift
// rho on the diagonal.
__device__ void pivot_block(int p, int k0, int kb, const double *__restrict__ Ab, double shift,
                            double *__restrict__ Qb) {
    __shared__ double rowb[2][NB], colb[2][NB];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double v[16];
#pragma unroll
    for (int a = 0; a < 16; ++a) {  // loads from clamped addresses, all in flight together
        const int i = ty + 4 * a;
        v[a] = Ab[(size_t)(k0 + min(i, kb - 1)) * p + k0 + min(tx, kb - 1)];
    }
#pragma unroll
    for (int a = 0; a < 16; ++a) {
        const int i = ty + 4 * a;
        v[a] = (i < kb && tx < kb) ? v[a] + (i == tx ? shift : 0.0) : (i == tx ? 1.0 : 0.0);
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int buf = k & 1;
        if (ty == (k & 3)) rowb[buf][tx] = v[k >> 2];
        if (tx == k) {
#pragma unroll
            for (int a = 0; a < 16; ++a) colb[buf][ty + 4 * a] = v[a];
        }
        __syncthreads();
        const double pinv = 1.0 / rowb[buf][k];
        const double rk = rowb[buf][tx];
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            const int i = ty + 4 * a;
            const double aik = colb[buf][i] * pinv;
            double nv;
            if (i != k && tx != k) nv = v[a] - aik * rk;   // A_ij - A_ik A_kj / A_kk
            else if (i != k) nv = aik;                     // column k
            else if (tx != k) nv = rk * pinv;              // row k
            else nv = -pinv;                               // pivot
            v[a] = nv;
        }
    }
#pragma unroll
    for (int a = 0; a < 16; ++a) {
        const int i = ty + 4 * a;
        Qb[i * NB + tx] = (i < kb && tx < kb) ? -v[a] : 0.0;  // zero padded
    }
}

// The first pivot block (later ones are inverted inside the preceding update).
__global__ __launch_bounds__(256) void k_pivot(int p, int k0, int kb, const double *__restrict__ src,
                                               double shift, double *__restrict__ Q) {
    const int b = blockIdx.x;
    pivot_block(p, k0, kb, src + (size_t)b * p * p, shift, Q + (size_t)b * NB * NB);
}

// (2) Panel for rows [i0, i0+64): Old = A[i, K] and W = A[i, K] Q (MFMA), both
// stored pivot-index-major (Wt[t][i], Ot[t][i], t < NB) so that the update reads
// them as unit-stride MFMA operands.  Only the lower-triangle 64-tiles of A are
// current, so rows above the pivot block read A[i][K] as A[K][i].
__global__ __launch_bounds__(256) void k_panel(int p, int k0, int kb, const double *__restrict__ src,
                                               double shift, const double *__restrict__ Q,
                                               double *__restrict__ Wt, double *__restrict__ Ot) {
    constexpr int LD = 64 + 1;
    __shared__ double As[NB * LD];  // As[t][r] = A[i0 + r][k0 + t]; later W staged as [c][r]
    __shared__ double Qs[NB * LD];  // Qs[t][c] = Q[t][c]
    const int b = blockIdx.y;
    const int i0 = blockIdx.x * 64;
    const double *Ab = src + (size_t)b * p * p;
    const double *Qb = Q + (size_t)b * NB * NB;
    double *Wb = Wt + (size_t)b * p * NB;
    double *Ob = Ot + (size_t)b * p * NB;
    const bool above = i0 < k0;
    // all loads of the panel first (clamped, unconditional), then the stores
    constexpr int PER = 64 * NB / 256;
    double pv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q;
        int r, t;
        if (above) { t = e / 64; r = e % 64; }   // coalesced along i
        else { r = e / NB; t = e % NB; }          // coalesced along k
        const int gi = min(i0 + r, p - 1), gk = min(k0 + t, p - 1);
        pv[q] = above ? Ab[(size_t)gk * p + gi] : Ab[(size_t)gi * p + gk];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + 256 * q;
        int r, t;
        if (above) { t = e / 64; r = e % 64; }
        else { r = e / NB; t = e % NB; }
        const bool ok = i0 + r < p && t < kb;
        As[t * LD + r] = ok ? pv[q] + (i0 + r == k0 + t ? shift : 0.0) : 0.0;
    }
    {
        double qv[NB * NB / 256];
#pragma unroll
        for (int q = 0; q < NB * NB / 256; ++q) qv[q] = Qb[threadIdx.x + 256 * q];
#pragma unroll
        for (int q = 0; q < NB * NB / 256; ++q) {
            const int e = threadIdx.x + 256 * q;
            Qs[(e / NB) * LD + e % NB] = qv[q];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * NB; e += 256) {
        const int t = e / 64, r = e % 64;
        if (i0 + r < p) Ob[(size_t)t * p + i0 + r] = As[t * LD + r];
    }
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
    __syncthreads();  // As is reused to stage W as [c][r]
    for (int fm = 0; fm < 2; ++fm)
        for (int fn = 0; fn < 2; ++fn)
            for (int t = 0; t < 4; ++t) {
                int r = wm * 32 + fm * 16 + mfma_row(0.0, lk, t), c = wn * 32 + fn * 16 + lr;
                As[c * LD + r] = acc[fm][fn][t];
            }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * NB; e += 256) {
        const int c = e / 64, r = e % 64;
        if (i0 + r < p) Wb[(size_t)c * p + i0 + r] = As[c * LD + r];
    }
}

// (3) Rank-kb update of one 64x64 tile on or below the diagonal:
//   i,j not in K: A_ij -= W_i . Old_j ;  i not in K, j in K: A_ij = W_i[j-k0]
//   i in K, j not in K: A_ij = W_j[i-k0] ;  i, j in K: A_ij = -Q
// Each wave owns a 32x32 quadrant (2x2 MFMA blocks).  The tile's old values are
// requested first; the operands W_i[t] and Old_j[t] are read straight from the
// pivot-index-major panels (unit stride along i, L2-resident), with no LDS and no
// barrier.  Step 0 reads G (+ rho on the diagonal) and writes M.
__global__ __launch_bounds__(256) void k_update(int p, int k0, int kb, const double *__restrict__ src,
                                                double shift, double *__restrict__ dst,
                                                const double *__restrict__ Wt,
                                                const double *__restrict__ Ot,
                                                const double *__restrict__ Q,
                                                double *__restrict__ Qnext, float *__restrict__ M32) {
    // Workgroup -> (matrix, tile).  When another pivot block follows, the first nb
    // workgroups (dispatched first) take the diagonal tile of that block, one per
    // matrix, and invert it once stored, while the other tiles are updated.  The
    // remaining tiles are dealt so that all tiles of one matrix run on the same
    // XCD: the panels then stay in its L2.
    const int ntri = gridDim.x, nb = gridDim.z;
    const int L = blockIdx.x + ntri * blockIdx.z;
    const int kt = k0 / 64;
    const bool next = k0 + NB < p;
    const int dtile = (kt + 1) * (kt + 2) / 2 + kt + 1;  // tile index of (kt+1, kt+1)
    int tile, b;
    bool pivot = false;
    if (!next) {
        const int id = xcd_remap(L, nb * ntri);
        b = id / ntri;
        tile = id - b * ntri;
    } else if (L < nb) {
        b = L;
        tile = dtile;
        pivot = true;
    } else {
        const int id = xcd_remap(L - nb, nb * (ntri - 1));
        b = id / (ntri - 1);
        tile = id - b * (ntri - 1);
        tile += tile >= dtile;
    }
    int ti = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
    while (ti * (ti + 1) / 2 > tile) --ti;
    const int tj = tile - ti * (ti + 1) / 2;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    const int lr = lane & 15, lk = lane >> 4;
    const int ib = ti * 64 + wm * 32, jb = tj * 64 + wn * 32;  // quadrant origin
    const double *Ab = src + (size_t)b * p * p;
    double old[2][2][4];
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
        for (int fn = 0; fn < 2; ++fn)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                // clamped (valid) addresses: values outside the matrix are never stored
                const int i = min(ib + fm * 16 + mfma_row(0.0, lk, t), p - 1);
                const int j = min(jb + fn * 16 + lr, p - 1);
                old[fm][fn][t] = Ab[(size_t)i * p + j] + (i == j ? shift : 0.0);
            }
    const double *Wb = Wt + (size_t)b * p * NB;
    const double *Ob = Ot + (size_t)b * p * NB;
    // operand rows past p only reach outputs that are not stored: read clamped
    const int ia0 = min(ib + lr, p - 1), ia1 = min(ib + 16 + lr, p - 1);
    const int jb0 = min(jb + lr, p - 1), jb1 = min(jb + 16 + lr, p - 1);
    dx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = dx4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) {
        const int t = 4 * s + lk;  // rows t >= kb of the panels are zero
        const size_t o = (size_t)t * p;
        const double a0 = Wb[o + ia0], a1 = Wb[o + ia1];
        const double b0 = Ob[o + jb0], b1 = Ob[o + jb1];
        acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
        acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
        acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
        acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
    double *Db = dst + (size_t)b * p * p;
    const double *Qb = Q + (size_t)b * NB * NB;
    const bool plain = ti != kt && tj != kt;
    // After the last block step the values are final: M = -(swept matrix) is
    // stored in both triangles (the upper one as the exact mirror of the lower one,
    // transposed through LDS so that its stores are coalesced), with its float32
    // copy when M32 is given.
    extern __shared__ double tr[];  // [64][65], last step only
    float *Fb = M32 ? M32 + (size_t)b * p * p : nullptr;
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
        for (int fn = 0; fn < 2; ++fn)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = ib + fm * 16 + mfma_row(0.0, lk, t), j = jb + fn * 16 + lr;
                if (i >= p || j >= p) continue;
                double v = old[fm][fn][t] - acc[fm][fn][t];
                if (!plain) {
                    const bool iK = i >= k0 && i < k0 + kb, jK = j >= k0 && j < k0 + kb;
                    if (iK && jK) v = -Qb[(i - k0) * NB + (j - k0)];        // -Q
                    else if (jK) v = Wb[(size_t)(j - k0) * p + i];          // A_iK Q
                    else if (iK) v = Wb[(size_t)(i - k0) * p + j];          // Q A_Kj = (A_jK Q)'
                }
                if (next) {
                    Db[(size_t)i * p + j] = v;
                } else {
                    tr[(i - ti * 64) * 65 + (j - tj * 64)] = -v;
                    if (ti > tj || j <= i) {
                        Db[(size_t)i * p + j] = -v;
                        if (Fb) Fb[(size_t)i * p + j] = (float)-v;
                    }
                }
            }
    if (!next) {
        __syncthreads();
        // mirror: (r, c) of the transposed tile = (c, r) of this one; on a diagonal
        // tile only the strict upper part
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int r = e >> 6, c = e & 63;
            const int gi = tj * 64 + r, gj = ti * 64 + c;
            if (gi < p && gj < p && (ti > tj || gi < gj)) {
                const double v = tr[c * 65 + r];
                Db[(size_t)gi * p + gj] = v;
                if (Fb) Fb[(size_t)gi * p + gj] = (float)v;
            }
        }
        return;
    }
    if (pivot) {
        __syncthreads();  // the tile's stores are visible to the whole workgroup
        pivot_block(p, k0 + NB, min(NB, p - k0 - NB), Db, 0.0, Qnext + (size_t)b * NB * NB);
    }
}

__global__ void k_narrow(size_t n, const double *__restrict__ a, float *__restrict__ b) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

size_t spd_inverse_work_doubles(int nb, int p) {
    if (p <= SMALL) return 0;
    return 2 * (size_t)nb * NB * NB + 2 * (size_t)nb * p * NB;
}

void spd_inverse_f64(hipStream_t s, int nb, int p, const double *G, double rho, double *M,
                     double *work, float *M32) {
    if (p <= SMALL) {
        size_t lds = sizeof(double) * (size_t)p * p;
        hipLaunchKernelGGL(k_inv_small, dim3(nb), dim3(256), lds, s, p, G, rho, M);
        if (M32) {
            const size_t n = (size_t)nb * p * p;
            hipLaunchKernelGGL(k_narrow, dim3(cdiv(n, 256)), dim3(256), 0, s, n, M, M32);
        }
        UOI_LAUNCH_CHECK();
        return;
    }
    // Q of step K lives in buffer K % 2: the update of step K inverts the next
    // pivot block into the other buffer while its own tiles still read Q.
    double *Qbuf[2] = {work, work + (size_t)nb * NB * NB};
    double *Wt = work + 2 * (size_t)nb * NB * NB;
    double *Ot = Wt + (size_t)nb * p * NB;
    const int T = (int)cdiv(p, 64);
    hipLaunchKernelGGL(k_pivot, dim3(nb), dim3(256), 0, s, p, 0, std::min(NB, p), G, rho, Qbuf[0]);
    for (int k0 = 0, K = 0; k0 < p; k0 += NB, ++K) {
        const int kb = std::min(NB, p - k0);
        // the first step reads G + rho I and writes every lower tile of M
        const double *src = k0 == 0 ? G : M;
        const double sh = k0 == 0 ? rho : 0.0;
        double *Q = Qbuf[K & 1];
        hipLaunchKernelGGL(k_panel, dim3(T, nb), dim3(256), 0, s, p, k0, kb, src, sh, Q, Wt, Ot);
        // the last step also writes the upper triangle and the float32 copy
        const bool last = k0 + NB >= p;
        const size_t lds = last ? sizeof(double) * 64 * 65 : 0;
        hipLaunchKernelGGL(k_update, dim3(T * (T + 1) / 2, 1, nb), dim3(256), lds, s, p, k0, kb, src, sh, M,
                           Wt, Ot, Q, Qbuf[(K + 1) & 1], last ? M32 : nullptr);
        UOI_LAUNCH_CHECK();
    }
}

}  // namespace uoi
