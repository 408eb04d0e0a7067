// Batched product Y_b = A_b V_b with a fused epilogue, on MFMA 16x16x4
// (float64 or float32).  A_b is a symmetric p x p matrix (an inverse or a Gram,
// one per bootstrap), V_b is p x R row-major (R solves side by side).  This is
// the x-update of every ADMM iteration, the KKT gradient G z, and the
// conjugate-gradient product of the refits.
//
// Workgroup: 4 waves stacked along rows; wave w owns rows
// [i0 + 16*FM*w, +16*FM) and all 16*FN columns of the tile, as FM x FN MFMA
// accumulators.  The reduction runs over k in chunks of KC = 32:
//   - V[k0:k0+32, cols] is staged in LDS (double buffered) and shared by the
//     4 waves;
//   - A[i][k] is read as A[k][i] (symmetry), so a wave's operand for one MFMA
//     step is 4 rows x 16 consecutive entries, loaded straight into registers;
//     the loads of chunk c+1 are issued before the MFMAs of chunk c.
// One barrier per chunk.  Every A element is read once per launch; V is read
// once per row tile.  (Measured alternatives: 64-row chunks, or a three-stage
// register ring, both cost occupancy on float64 and ran slower.)
// Workgroups are remapped so that all tiles of one matrix run on the same XCD:
// the V block of a matrix is then re-read from that XCD's L2 instead of from
// the fabric (the dispatcher deals workgroups to the 8 XCDs round robin).
#pragma once
#include <type_traits>

#include "common.hpp"

namespace uoi {

template <typename T>
struct AccT {
    typedef typename std::conditional<std::is_same<T, double>::value, dx4, fx4>::type type;
};

constexpr int BG_KC = 32;

template <typename T, int FM, int FN, class Epi>
__global__ __launch_bounds__(256) void k_bgemm(int p, int R, const T *__restrict__ A,
                                               const T *__restrict__ V, Epi epi) {
    typedef typename AccT<T>::type acc_t;
    constexpr int TN = 16 * FN;
    __shared__ T Vs[2][BG_KC][TN];
    int bx, by, b;
    xcd_tile(bx, by, b);
    const int r0 = bx * TN;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int i_base = by * (64 * FM) + wid * (16 * FM);
    const int lr = lane & 15, lk = lane >> 4;
    if (!epi.tile_active(b, r0, TN)) return;  // uniform over the workgroup

    const T *Ab = A + (size_t)b * p * p;
    const T *Vb = V + (size_t)b * p * R;

    acc_t acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int c = 0; c < FN; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[a][c][t] = 0;

    int icol[FM];
    bool iok[FM];
#pragma unroll
    for (int a = 0; a < FM; ++a) {
        icol[a] = i_base + 16 * a + lr;
        iok[a] = icol[a] < p;
    }

    // All loads are issued unconditionally from clamped (valid, finite) addresses
    // and masked only where the values are used, so that the loads of a chunk stay
    // in flight together: rows of V past p are zeroed when staged (which also
    // cancels the clamped A rows past p), columns past R and rows of A past p only
    // reach outputs that the epilogue discards.
    // V chunk loader: KC*TN values over 256 threads
    constexpr int VPT = (BG_KC * TN + 255) / 256;
    T vreg[VPT];
    auto load_v = [&](int k0) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int e = min(tid + 256 * q, BG_KC * TN - 1);
            const int kk = min(k0 + e / TN, p - 1), cc = min(r0 + e % TN, R - 1);
            vreg[q] = Vb[(size_t)kk * R + cc];
        }
    };
    auto store_v = [&](int buf, int k0) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int e = tid + 256 * q;
            if (e < BG_KC * TN) Vs[buf][e / TN][e % TN] = k0 + e / TN < p ? vreg[q] : T(0);
        }
    };
    int icl[FM];
#pragma unroll
    for (int a = 0; a < FM; ++a) icl[a] = min(icol[a], p - 1);
    T areg[BG_KC / 4][FM];
    auto load_a = [&](int k0) {
#pragma unroll
        for (int s = 0; s < BG_KC / 4; ++s) {
            const int k = min(k0 + 4 * s + lk, p - 1);
#pragma unroll
            for (int a = 0; a < FM; ++a) areg[s][a] = Ab[(size_t)k * p + icl[a]];
        }
    };

    const int nchunk = (p + BG_KC - 1) / BG_KC;
    load_v(0);
    load_a(0);
    store_v(0, 0);
    __syncthreads();
    for (int c = 0; c < nchunk; ++c) {
        const int cur = c & 1;
        const bool more = c + 1 < nchunk;
        T acur[BG_KC / 4][FM];
#pragma unroll
        for (int s = 0; s < BG_KC / 4; ++s)
#pragma unroll
            for (int a = 0; a < FM; ++a) acur[s][a] = areg[s][a];
        if (more) {  // prefetch chunk c+1 while chunk c is multiplied
            load_v((c + 1) * BG_KC);
            load_a((c + 1) * BG_KC);
        }
#pragma unroll
        for (int s = 0; s < BG_KC / 4; ++s)
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int cc = 0; cc < FN; ++cc) {
                    const T bv = Vs[cur][4 * s + lk][16 * cc + lr];
                    acc[a][cc] = mfma16x16x4(acur[s][a], bv, acc[a][cc]);
                }
        if (more) store_v(cur ^ 1, (c + 1) * BG_KC);
        __syncthreads();
    }
    if (i_base < p) epi.apply(b, i_base, r0, lr, lk, acc);
}

template <typename T, int FM, int FN, class Epi>
inline void run_bgemm(hipStream_t s, int nb, int p, int R, const T *A, const T *V, const Epi &epi) {
    dim3 grid(cdiv(R, 16 * FN), cdiv(p, 64 * FM), nb);
    hipLaunchKernelGGL((k_bgemm<T, FM, FN, Epi>), grid, dim3(256), 0, s, p, R, A, V, epi);
    UOI_LAUNCH_CHECK();
}

// Column-block width: the smallest multiple of 16 that covers R, up to 64.
#define UOI_DISPATCH_FN(R, ...)                                   \
    do {                                                          \
        if ((R) <= 16) { constexpr int FN = 1; __VA_ARGS__; }      \
        else if ((R) <= 32) { constexpr int FN = 2; __VA_ARGS__; } \
        else if ((R) <= 48) { constexpr int FN = 3; __VA_ARGS__; } \
        else { constexpr int FN = 4; __VA_ARGS__; }                \
    } while (0)

}  // namespace uoi
