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

void launch_support_and(hipStream_t s, int nb, int p, int R, const double *z, uint64_t *supp) {
    int W = (p + 63) / 64;
    hipLaunchKernelGGL(k_support_init, dim3(cdiv((size_t)R * W, 256)), dim3(256), 0, s, R, p, supp);
    hipLaunchKernelGGL(k_support_and, dim3(cdiv(R, 64), W, nb), dim3(64), 0, s, p, R, z, supp);
    UOI_LAUNCH_CHECK();
}

}  // namespace uoi
