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

// Logical (column tile x, row tile y, matrix z) of a product workgroup.  z is
// slowest, so the tiles of one matrix stay on one XCD (xcd_remap), and y is
// fastest: the workgroups resident together on an XCD then cover a few column
// strips of V over every row strip of A.  A column strip of V is fetched from
// beyond the L2 about once per product, and A (far smaller than V when there
// are many columns) is the operand that is fetched again.  With x fastest, the
// strips of V were fetched once per row tile.
__device__ __forceinline__ void bg_tile(int &x, int &y, int &z) {
    const int gx = gridDim.x, gy = gridDim.y;
    const int total = gx * gy * gridDim.z;
    const int L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int id = xcd_remap(L, total);
    z = id / (gx * gy);
    const int rem = id - z * gx * gy;
    x = rem / gy;
    y = rem - x * gy;
}

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
    bg_tile(bx, by, b);
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

// ---------------------------------------------------------------------------
// Float32 product on bfloat16 MFMA (16x16x32).  Every float32 operand x is
// split as x = x1 + x2 + x3 + r, each part the bfloat16 rounding (to nearest)
// of what the previous parts leave, so |x2| <= 2^-8 |x|, |x3| <= 2^-16 |x| and
// |r| <= 2^-24 |x|; the differences are exact in float32.  The six part
// products of order 2^-16 and above (a1b1, a1b2, a2b1, a1b3, a2b2, a3b1) give A V
// to float32 accuracy: the dropped ones are below 2^-23 relative.  bfloat16
// keeps the float32 exponent range, so no scaling is needed.  The six MFMAs of
// a 32-deep step cost about a third of the eight float32 16x16x4 steps they
// replace, which leaves the float32 ADMM iteration bound by reading A.
//
// Layout as k_bgemm (4 waves x 16 FM rows, 16*FN columns, KC = 32): lane (lr, lk)
// reads eight entries of row i = i_base + 16 a + lr of A (= column i, by
// symmetry; a < FM) as two 16-byte loads and splits them in registers.  V arrives
// already split, as three bfloat16 planes Vp[b][part][r][k] with k contiguous
// and rows k >= p zero up to bf3_ldk(p) (the producing epilogue writes them; it
// splits each element once instead of once per row block); a chunk is copied to
// LDS (double buffered) in 16-byte pieces, so that each MFMA operand is one
// 16-byte LDS read.
typedef __bf16 bfx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split_bf16x3(const float (&x)[8], bfx8 &p1, bfx8 &p2, bfx8 &p3) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 a = (__bf16)x[e];
        const float r1 = x[e] - (float)a;
        const __bf16 b = (__bf16)r1;
        const float r2 = r1 - (float)b;
        p1[e] = a;
        p2[e] = b;
        p3[e] = (__bf16)r2;
    }
}

constexpr int BF3_KC = 32;  // k per chunk
constexpr int BF3_D = 4;    // register ring depth (chunks in flight)
// k extent of a V plane row: the chunks the product reads, rounded to the ring
inline int bf3_ldk(int p) {
    const int nchunk = (p + BF3_KC - 1) / BF3_KC;
    return ((nchunk + BF3_D - 1) / BF3_D * BF3_D + BF3_D) * BF3_KC;
}

__device__ __forceinline__ fx4 mfma16x16x32(bfx8 a, bfx8 b, fx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// FM row blocks of 16 per wave (a workgroup covers 64 FM rows): with FM = 2 each
// V operand read from LDS feeds twice the MFMAs and each V strip is fetched by
// half as many workgroups.  Its register ring is two chunks deep and its
// registers are held to three waves per SIMD (measured best of depths 2 to 4,
// with and without the bound).
template <int FN, int FM, bool VEC4, class Epi>
__global__ __launch_bounds__(256, FM == 2 ? 3 : 1) void k_bgemm_bf3(int p, int R, const float *__restrict__ A,
                                                   const __bf16 *__restrict__ Vp, int ldk, Epi epi) {
    constexpr int TN = 16 * FN;
    constexpr int KC = BF3_KC;
    constexpr int KP = KC + 8;  // k stride of an LDS plane row (bfloat16), 16-byte aligned
    __shared__ __attribute__((aligned(16))) __bf16 Vs[2][3][TN][KP];
    int bx, by, b;
    bg_tile(bx, by, b);
    const int r0 = bx * TN;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int i_base = by * (64 * FM) + wid * (16 * FM);
    const int lr = lane & 15, lk = lane >> 4;
    if (!epi.tile_active(b, r0, TN)) return;  // uniform over the workgroup

    const float *Ab = A + (size_t)b * p * p;
    fx4 acc[FM][1][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int c = 0; c < FN; ++c) acc[a][0][c] = fx4{0.f, 0.f, 0.f, 0.f};

    // All loads come from valid addresses: the V planes hold zeros at rows p ..
    // ldk - 1, which cancel the clamped A values they meet; rows of A past p and
    // columns past R only reach outputs that the epilogue discards.
    // The loop body has no branch around a load: the compiler can then keep the
    // loads of several chunks in flight (a load under a branch makes it wait for
    // every earlier one).
    const float *arows[FM];
#pragma unroll
    for (int a = 0; a < FM; ++a) arows[a] = Ab + (size_t)min(i_base + 16 * a + lr, p - 1) * p;
    // Lane group lk takes k = 4 lk .. 4 lk + 3 and 16 + 4 lk .. 16 + 4 lk + 3 of a
    // chunk (elements 0-3 and 4-7 of its MFMA operand), so that each of the two
    // loads covers 64 contiguous bytes of a row; V is laid out in LDS in the same
    // order.
    auto load_a = [&](float (&an)[8], const float *arow, int k0) {
        const int k = k0 + 4 * lk;
        if (VEC4) {  // rows of A 16-byte aligned (p % 4 == 0)
            const fx4 x0 = *(const fx4 *)(arow + min(k, p - 4));
            const fx4 x1 = *(const fx4 *)(arow + min(k + 16, p - 4));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                an[e] = x0[e];
                an[4 + e] = x1[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                an[e] = arow[min(k + e, p - 1)];
                an[4 + e] = arow[min(k + 16 + e, p - 1)];
            }
        }
    };
    // V: thread tid < 4 TN copies rows k0 + 8 og .. + 7 of tile column cv, three
    // planes (the four threads of a column read its 64 contiguous bytes); the
    // other threads load a copy and store nothing
    const bool vst = tid < 4 * TN;
    const int cv = min(tid >> 2, TN - 1), og = tid & 3;
    const size_t plane = (size_t)R * ldk;
    const __bf16 *vcol = Vp + (size_t)b * 3 * plane + (size_t)min(r0 + cv, R - 1) * ldk + 8 * og;
    typedef bfx8 vraw[3];
    auto load_v = [&](vraw &vn, int k0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) vn[q] = *(const bfx8 *)(vcol + q * plane + k0);
    };
    // rows 8 og .. 8 og + 3 and 8 og + 4 .. 8 og + 7 go to the operand positions
    // of the lane groups that take them (see load_a)
    const int s0 = 8 * ((2 * og) & 3) + 4 * (og >> 1);
    auto store_v = [&](int buf, const vraw &vn) {
        if (vst) {
            typedef __bf16 bfx4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                *(bfx4 *)&Vs[buf][q][cv][s0] = bfx4{vn[q][0], vn[q][1], vn[q][2], vn[q][3]};
                *(bfx4 *)&Vs[buf][q][cv][s0 + 8] = bfx4{vn[q][4], vn[q][5], vn[q][6], vn[q][7]};
            }
        }
    };

    // Raw chunks travel through a register ring D deep: the loads of chunk c + D
    // are issued when chunk c is multiplied, so memory latency is covered by D - 1
    // chunks of work (the MFMAs alone are too short to cover it).  The chunk loop
    // is unrolled by D so that ring slots are static registers, and runs over a
    // multiple of D chunks: chunks past p are staged as zeros.
    constexpr int D = FM == 2 ? 2 : BF3_D;  // (bf3_ldk pads for the deepest ring)
    const int nchunk = (p + KC - 1) / KC;
    float an[D][FM][8];
    vraw vn[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        load_v(vn[d], d * KC);
#pragma unroll
        for (int a = 0; a < FM; ++a) load_a(an[d][a], arows[a], d * KC);
    }
    bfx8 a1[FM], a2[FM], a3[FM];
    store_v(0, vn[0]);
#pragma unroll
    for (int a = 0; a < FM; ++a) split_bf16x3(an[0][a], a1[a], a2[a], a3[a]);
    __syncthreads();
    for (int c = 0; c < nchunk; c += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int cc = c + d;
            // slot d was staged at the end of the previous chunk
            load_v(vn[d], (cc + D) * KC);
#pragma unroll
            for (int a = 0; a < FM; ++a) load_a(an[d][a], arows[a], (cc + D) * KC);
            const int cur = cc & 1;
#pragma unroll
            for (int q = 0; q < FN; ++q) {
                const bfx8 b1 = *(const bfx8 *)&Vs[cur][0][16 * q + lr][8 * lk];
                const bfx8 b2 = *(const bfx8 *)&Vs[cur][1][16 * q + lr][8 * lk];
                const bfx8 b3 = *(const bfx8 *)&Vs[cur][2][16 * q + lr][8 * lk];
#pragma unroll
                for (int a = 0; a < FM; ++a) {
                    fx4 t = acc[a][0][q];
                    t = mfma16x16x32(a3[a], b1, t);  // small terms first
                    t = mfma16x16x32(a2[a], b2, t);
                    t = mfma16x16x32(a1[a], b3, t);
                    t = mfma16x16x32(a2[a], b1, t);
                    t = mfma16x16x32(a1[a], b2, t);
                    acc[a][0][q] = mfma16x16x32(a1[a], b1, t);
                }
            }
            store_v(cur ^ 1, vn[(d + 1) % D]);
#pragma unroll
            for (int a = 0; a < FM; ++a) split_bf16x3(an[(d + 1) % D][a], a1[a], a2[a], a3[a]);
            __syncthreads();
        }
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
        if (i_base + 16 * a < p) epi.apply(b, i_base + 16 * a, r0, lr, lk, acc[a]);
}

// Vp: three bfloat16 planes [nb][3][R][ldk], ldk = bf3_ldk(p), zero at rows >= p.
template <int FN, int FM = 1, class Epi>
inline void run_bgemm_bf3(hipStream_t s, int nb, int p, int R, const float *A, const __bf16 *Vp,
                          const Epi &epi) {
    dim3 grid(cdiv(R, 16 * FN), cdiv(p, 64 * FM), nb);
    const int ldk = bf3_ldk(p);
    if (p % 4 == 0 && ((uintptr_t)A & 15) == 0)
        hipLaunchKernelGGL((k_bgemm_bf3<FN, FM, true, Epi>), grid, dim3(256), 0, s, p, R, A, Vp, ldk, epi);
    else
        hipLaunchKernelGGL((k_bgemm_bf3<FN, FM, false, Epi>), grid, dim3(256), 0, s, p, R, A, Vp, ldk, epi);
    UOI_LAUNCH_CHECK();
}

// Column-block width chosen at run time (1..4 blocks of 16 columns).
#define UOI_DISPATCH_FN_RT(fnv, ...)                               \
    do {                                                          \
        switch (fnv) {                                            \
        case 1: { constexpr int FN = 1; __VA_ARGS__; break; }     \
        case 2: { constexpr int FN = 2; __VA_ARGS__; break; }     \
        case 3: { constexpr int FN = 3; __VA_ARGS__; break; }     \
        default: { constexpr int FN = 4; __VA_ARGS__; break; }    \
        }                                                         \
    } while (0)
inline int default_fn(int R) { return R <= 16 ? 1 : R <= 32 ? 2 : R <= 48 ? 3 : 4; }

// Column-block width: the smallest multiple of 16 that covers R, up to 64.
#define UOI_DISPATCH_FN(R, ...)                                   \
    do {                                                          \
        if ((R) <= 16) { constexpr int FN = 1; __VA_ARGS__; }      \
        else if ((R) <= 32) { constexpr int FN = 2; __VA_ARGS__; } \
        else if ((R) <= 48) { constexpr int FN = 3; __VA_ARGS__; } \
        else { constexpr int FN = 4; __VA_ARGS__; }                \
    } while (0)

}  // namespace uoi
