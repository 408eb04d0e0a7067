// Supports and their intersection (Eq. (intersection), Alg. 1 model selection):
// S_j^k = {i : z_i != 0} of the ADMM estimate, S_j = AND over bootstraps k.
// Supports are bitmasks of W = ceil(p/64) uint64 words, bit i of word i/64.
#include "common.hpp"

namespace uoi {

// supp[r][w] = AND_b (bits of z[b][64w .. 64w+63][r] != 0); threads run along r so
// every read of z is a coalesced row segment.
__global__ void k_support_and(int nb, int p, int R, const double *__restrict__ z,
                              uint64_t *__restrict__ supp) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    int w = blockIdx.y;
    int W = gridDim.y;
    if (r >= R) return;
    int lo = w * 64, hi = min(p, lo + 64);
    uint64_t word = (hi - lo == 64) ? ~0ull : ((1ull << (hi - lo)) - 1ull);
    for (int b = 0; b < nb && word; ++b) {
        const double *zb = z + (size_t)b * p * R;
        for (int i = lo; i < hi; ++i)
            if (zb[(size_t)i * R + r] == 0.0) word &= ~(1ull << (i - lo));
    }
    supp[(size_t)r * W + w] = word;
}

void launch_support_and(hipStream_t s, int nb, int p, int R, const double *z, uint64_t *supp) {
    int W = (p + 63) / 64;
    hipLaunchKernelGGL(k_support_and, dim3(cdiv(R, 256), W), dim3(256), 0, s, nb, p, R, z, supp);
    UOI_LAUNCH_CHECK();
}

}  // namespace uoi
