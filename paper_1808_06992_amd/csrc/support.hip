// Supports and their intersection (Eq. (intersection), Alg. 1 model selection):
// S_j^k = {i : z_i != 0} of the ADMM estimate, S_j = AND over bootstraps k.
// Supports are bitmasks of W = ceil(p/64) uint64 words, bit i of word i/64.
#include "common.hpp"

namespace uoi {

// supp[r][w] starts as the mask of valid bits; then one thread per (bootstrap
// b, solve r, word w) folds the bits of z[b][64w .. 64w+63][r] != 0 in with a
// 64-bit atomic AND.  Threads run along r, so every read of z is a coalesced row
// segment, and the 64 feature reads of a thread are independent.
__global__ void k_support_init(int R, int p, uint64_t *__restrict__ supp) {
    int W = (p + 63) / 64;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)R * W) return;
    int w = (int)(t % W);
    int nbits = min(64, p - 64 * w);
    supp[t] = nbits == 64 ? ~0ull : ((1ull << nbits) - 1ull);
}

__global__ void k_support_and(int p, int R, const double *__restrict__ z, uint64_t *__restrict__ supp) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    int w = blockIdx.y;
    int b = blockIdx.z;
    int W = gridDim.y;
    if (r >= R) return;
    int lo = w * 64, hi = min(p, lo + 64);
    const double *zb = z + (size_t)b * p * R;
    uint64_t word = 0;
#pragma unroll 16
    for (int i = lo; i < hi; ++i)
        if (zb[(size_t)i * R + r] != 0.0) word |= 1ull << (i - lo);
    uint64_t full = (hi - lo == 64) ? ~0ull : ((1ull << (hi - lo)) - 1ull);
    if (word != full) atomicAnd(reinterpret_cast<unsigned long long *>(&supp[(size_t)r * W + w]),
                                (unsigned long long)word);
}

// Union U of the supports of all R solves and its compact numbering: gidx[c] is
// the column of compact column c (increasing), *count = |U|.  The refits of the
// estimation step only read statistics of columns in some support, so they can
// run on X[:, U].  One workgroup; W <= 1024 words.  With sizes, sizes[r] =
// |S_r| as well.
__global__ __launch_bounds__(1024) void k_support_union(int R, int W, const uint64_t *__restrict__ supp,
                                                        int *__restrict__ count, int32_t *__restrict__ gidx,
                                                        int32_t *__restrict__ sizes) {
    __shared__ int base[1024];
    const int t = threadIdx.x;
    if (sizes)
        for (int r = t; r < R; r += 1024) {
            int c = 0;
            for (int w = 0; w < W; ++w) c += __popcll(supp[(size_t)r * W + w]);
            sizes[r] = c;
        }
    uint64_t u = 0;
    if (t < W)
        for (int r = 0; r < R; ++r) u |= supp[(size_t)r * W + t];
    const int pc = t < W ? __popcll(u) : 0;
    base[t] = pc;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan
        const int v = t >= d ? base[t - d] : 0;
        __syncthreads();
        base[t] += v;
        __syncthreads();
    }
    if (t == 1023) *count = base[1023];
    int c = base[t] - pc;
    while (u) {
        gidx[c++] = 64 * t + __ffsll((unsigned long long)u) - 1;
        u &= u - 1;
    }
}

// Support r in the compact numbering: bit c of cs[r] = bit gidx[c] of supp[r].
__global__ void k_support_compact(int R, int W, int Wc, int cnt, const uint64_t *__restrict__ supp,
                                  const int32_t *__restrict__ gidx, uint64_t *__restrict__ cs) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)R * Wc) return;
    const int r = (int)(t / Wc), w = (int)(t % Wc);
    const uint64_t *sr = supp + (size_t)r * W;
    uint64_t word = 0;
    const int nbit = min(64, cnt - 64 * w);
    for (int b = 0; b < nbit; ++b) {
        const int i = gidx[64 * w + b];
        word |= ((sr[i >> 6] >> (i & 63)) & 1ull) << b;
    }
    cs[t] = word;
}

// XU[r][c] = X[r][gidx[c]]
__global__ void k_gather_cols(int n, int ldx, int pc, const double *__restrict__ X,
                              const int32_t *__restrict__ gidx, double *__restrict__ XU) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)n * pc) return;
    const size_t r = t / pc;
    const int c = (int)(t % pc);
    XU[t] = X[r * ldx + gidx[c]];
}

// dst[gidx[c]] = src[c] (dst zeroed by the caller)
__global__ void k_scatter_cols(int pc, const int32_t *__restrict__ gidx, const double *__restrict__ src,
                               double *__restrict__ dst) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < pc) dst[gidx[c]] = src[c];
}

int launch_support_union(hipStream_t s, int R, int p, const uint64_t *supp, int *count, int32_t *gidx,
                         std::vector<int32_t> *sizes) {
    const int W = (p + 63) / 64;
    if (W > 1024) return -1;
    // count[0] = |U|; with sizes, count[1 + r] = |S_r|, read back in the same copy
    hipLaunchKernelGGL(k_support_union, dim3(1), dim3(1024), 0, s, R, W, supp, count, gidx,
                       sizes ? count + 1 : nullptr);
    UOI_LAUNCH_CHECK();
    std::vector<int32_t> h(sizes ? 1 + R : 1);
    UOI_HIP(hipMemcpyAsync(h.data(), count, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, s));
    UOI_HIP(hipStreamSynchronize(s));
    if (sizes) sizes->assign(h.begin() + 1, h.end());
    return h[0];
}

void launch_compact_design(hipStream_t s, int R, int p, int cnt, const uint64_t *supp, const int32_t *gidx,
                           uint64_t *cs, int n, const double *X, int ldx, double *XU) {
    const int W = (p + 63) / 64, Wc = (cnt + 63) / 64;
    hipLaunchKernelGGL(k_support_compact, dim3(cdiv((size_t)R * Wc, 256)), dim3(256), 0, s, R, W, Wc, cnt,
                       supp, gidx, cs);
    hipLaunchKernelGGL(k_gather_cols, dim3(cdiv((size_t)n * cnt, 256)), dim3(256), 0, s, n, ldx, cnt, X, gidx,
                       XU);
    UOI_LAUNCH_CHECK();
}

void launch_scatter_cols(hipStream_t s, int p, int cnt, const int32_t *gidx, const double *src, double *dst) {
    UOI_HIP(hipMemsetAsync(dst, 0, sizeof(double) * p, s));
    hipLaunchKernelGGL(k_scatter_cols, dim3(cdiv(cnt, 256)), dim3(256), 0, s, cnt, gidx, src, dst);
    UOI_LAUNCH_CHECK();
}

void launch_support_and(hipStream_t s, int nb, int p, int R, const double *z, uint64_t *supp) {
    int W = (p + 63) / 64;
    hipLaunchKernelGGL(k_support_init, dim3(cdiv((size_t)R * W, 256)), dim3(256), 0, s, R, p, supp);
    hipLaunchKernelGGL(k_support_and, dim3(cdiv(R, 64), W, nb), dim3(64), 0, s, p, R, z, supp);
    UOI_LAUNCH_CHECK();
}

}  // namespace uoi
