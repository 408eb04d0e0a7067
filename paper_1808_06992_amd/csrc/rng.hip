// Index streams of the bootstrap and train/evaluation samples (Alg. 1 "generate
// bootstrap sample", Alg. 2 block bootstrap of Sec. III-A.2).  Keys are a
// counter-based SplitMix64 of (seed, tag, bootstrap, position); draws use a
// multiply-shift range map, so every index is a pure function of its position.
#include "common.hpp"

namespace uoi {

// rows[k][i] = range_map(key(seed, LASSO_BOOT, k, i), n): n draws with replacement.
__global__ void k_boot_rows(uint64_t seed, int n, int32_t *__restrict__ rows) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int k = blockIdx.y;
    if (i < n)
        rows[(size_t)k * n + i] = (int32_t)range_map(stream_key(seed, TAG_LASSO_BOOT, k, i), (uint32_t)n);
}

// Moving-block bootstrap: row i belongs to block i/L, whose start is drawn in [0, N-L].
__global__ void k_var_boot_rows(uint64_t seed, int N, int L, int32_t *__restrict__ rows) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int k = blockIdx.y;
    if (i < N) {
        int b = i / L;
        uint32_t start = range_map(stream_key(seed, TAG_VAR_BOOT, k, b), (uint32_t)(N - L + 1));
        rows[(size_t)k * N + i] = (int32_t)start + (i - b * L);
    }
}

// Train/eval split: item i of bootstrap k is a training item when fewer than
// ntrain items precede it in (key, index) order.  Keys of a 256-item tile are
// generated into LDS and compared by every thread.
__global__ __launch_bounds__(256) void k_split_rank(uint64_t seed, uint32_t tag, int cnt, int ntrain,
                                                    uint8_t *__restrict__ is_train) {
    __shared__ uint64_t tile[256];
    int i = blockIdx.x * 256 + threadIdx.x;
    int k = blockIdx.y;
    uint64_t mine = i < cnt ? stream_key(seed, tag, k, i) : 0;
    int before = 0;
    for (int t0 = 0; t0 < cnt; t0 += 256) {
        int j = t0 + threadIdx.x;
        tile[threadIdx.x] = j < cnt ? stream_key(seed, tag, k, j) : ~0ull;
        __syncthreads();
        int lim = min(256, cnt - t0);
        for (int t = 0; t < lim; ++t) {
            uint64_t kj = tile[t];
            int j2 = t0 + t;
            before += (kj < mine) || (kj == mine && j2 < i);
        }
        __syncthreads();
    }
    if (i < cnt) is_train[(size_t)k * cnt + i] = before < ntrain ? 1 : 0;
}

// The same split for up to kSortMax items: one block per sample sorts the
// (key, index) pairs in LDS (bitonic network) and flags the first ntrain.
constexpr int kSortMax = 8192;
__global__ __launch_bounds__(1024) void k_split_sort(uint64_t seed, uint32_t tag, int cnt, int np2,
                                                     int ntrain, uint8_t *__restrict__ is_train) {
    extern __shared__ unsigned long long sm[];
    unsigned long long *key = sm;
    int *ix = reinterpret_cast<int *>(sm + np2);
    const int k = blockIdx.x;
    for (int i = threadIdx.x; i < np2; i += blockDim.x) {
        key[i] = i < cnt ? stream_key(seed, tag, k, i) : ~0ull;
        ix[i] = i;
    }
    for (int size = 2; size <= np2; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int t = threadIdx.x; t < (np2 >> 1); t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1)), j = i + stride;
                const bool up = (i & size) == 0;
                const unsigned long long ki = key[i], kj = key[j];
                const int ii = ix[i], ij = ix[j];
                const bool gt = ki > kj || (ki == kj && ii > ij);
                if (gt == up) {
                    key[i] = kj; key[j] = ki;
                    ix[i] = ij; ix[j] = ii;
                }
            }
        }
    __syncthreads();
    for (int pos = threadIdx.x; pos < cnt; pos += blockDim.x)
        is_train[(size_t)k * cnt + ix[pos]] = pos < ntrain ? 1 : 0;
}

// Stable compaction of items into ascending train / eval lists (one block per bootstrap).
__global__ __launch_bounds__(256) void k_compact(int cnt, int ntrain, const uint8_t *__restrict__ is_train,
                                                 int32_t *__restrict__ train, int32_t *__restrict__ eval) {
    __shared__ int wtot[4];
    __shared__ int base_s[2];
    int k = blockIdx.x;
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint8_t *f = is_train + (size_t)k * cnt;
    int32_t *tr = train + (size_t)k * ntrain;
    int32_t *ev = eval + (size_t)k * (cnt - ntrain);
    if (threadIdx.x == 0) base_s[0] = base_s[1] = 0;
    __syncthreads();
    for (int c0 = 0; c0 < cnt; c0 += 256) {
        int i = c0 + threadIdx.x;
        bool valid = i < cnt;
        bool t = valid && f[i];
        unsigned long long bal = __ballot(t);
        int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[wid] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wid) woff += wtot[w];
            tot += wtot[w];
        }
        int nvalid = min(256, cnt - c0);
        int bt = base_s[0], be = base_s[1];
        if (valid) {
            int pt = woff + pre;  // training items before me in this chunk
            if (t) tr[bt + pt] = i;
            else ev[be + (threadIdx.x - pt)] = i;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            base_s[0] = bt + tot;
            base_s[1] = be + (nvalid - tot);
        }
        __syncthreads();
    }
}

// VAR split: blocks [bL, min((b+1)L, N)) flagged as training are expanded to rows
// in ascending order; row lists of bootstrap k start at k*N.
__global__ __launch_bounds__(256) void k_expand_blocks(int nblk, int N, int L,
                                                       const uint8_t *__restrict__ is_train,
                                                       int32_t *__restrict__ train,
                                                       int32_t *__restrict__ eval,
                                                       int32_t *__restrict__ ntr,
                                                       int32_t *__restrict__ nev) {
    __shared__ int off_s[1024];
    __shared__ int base_s[2];
    int k = blockIdx.x;
    const uint8_t *f = is_train + (size_t)k * nblk;
    int32_t *tr = train + (size_t)k * N;
    int32_t *ev = eval + (size_t)k * N;
    if (threadIdx.x == 0) base_s[0] = base_s[1] = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nblk; c0 += 1024) {
        int nc = min(1024, nblk - c0);
        if (threadIdx.x == 0) {
            int a = base_s[0], e = base_s[1];
            for (int t = 0; t < nc; ++t) {
                int b = c0 + t;
                int sz = min(L, N - b * L);
                if (f[b]) { off_s[t] = a; a += sz; }
                else { off_s[t] = e; e += sz; }
            }
            base_s[0] = a;
            base_s[1] = e;
        }
        __syncthreads();
        for (int t = 0; t < nc; ++t) {
            int b = c0 + t;
            int sz = min(L, N - b * L);
            int32_t *dst = f[b] ? tr : ev;
            for (int r = threadIdx.x; r < sz; r += 256) dst[off_s[t] + r] = b * L + r;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ntr[k] = base_s[0];
        nev[k] = base_s[1];
    }
}

// Multiplicities of the source rows in a sample: cnt[k][r] = number of draws of
// row r (cnt zeroed by the caller).
__global__ void k_count_rows(int nsrc, int m, const int32_t *__restrict__ rows, int32_t *__restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int k = blockIdx.y;
    if (i < m) atomicAdd(&cnt[(size_t)k * nsrc + rows[(size_t)k * m + i]], 1);
}

// Distinct rows of each sample in ascending order with their multiplicities
// (one block per sample): out_rows[k][0..nd), out_w[k][0..nd), nd = ndist[k].
__global__ __launch_bounds__(256) void k_distinct_rows(int nsrc, const int32_t *__restrict__ cnt,
                                                       int32_t *__restrict__ out_rows,
                                                       int32_t *__restrict__ out_w,
                                                       int32_t *__restrict__ ndist) {
    __shared__ int wtot[4];
    __shared__ int base_s;
    const int k = blockIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int32_t *c = cnt + (size_t)k * nsrc;
    int32_t *orow = out_rows + (size_t)k * nsrc;
    int32_t *ow = out_w + (size_t)k * nsrc;
    if (threadIdx.x == 0) base_s = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nsrc; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const int ci = i < nsrc ? c[i] : 0;
        const bool t = ci > 0;
        const unsigned long long bal = __ballot(t);
        const int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[wid] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wid) woff += wtot[w];
            tot += wtot[w];
        }
        const int base = base_s;
        if (t) {
            orow[base + woff + pre] = i;
            ow[base + woff + pre] = ci;
        }
        __syncthreads();
        if (threadIdx.x == 0) base_s = base + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) ndist[k] = base_s;
}

__global__ void k_finite(const double *__restrict__ x, size_t n, int *flag) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < n; i += stride) bad |= !isfinite(x[i]);
    if (bad) atomicOr(flag, 1);
}

void launch_boot_rows(hipStream_t s, uint64_t seed, uint32_t, int nb, int n, int32_t *rows) {
    hipLaunchKernelGGL(k_boot_rows, dim3(cdiv(n, 256), nb), dim3(256), 0, s, seed, n, rows);
    UOI_LAUNCH_CHECK();
}

void launch_distinct_rows(hipStream_t s, int nb, int nsrc, int m, const int32_t *rows, int32_t *cnt,
                          int32_t *out_rows, int32_t *out_w, int32_t *ndist) {
    UOI_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)nb * nsrc, s));
    hipLaunchKernelGGL(k_count_rows, dim3(cdiv(m, 256), nb), dim3(256), 0, s, nsrc, m, rows, cnt);
    hipLaunchKernelGGL(k_distinct_rows, dim3(nb), dim3(256), 0, s, nsrc, cnt, out_rows, out_w, ndist);
    UOI_LAUNCH_CHECK();
}

void launch_var_boot_rows(hipStream_t s, uint64_t seed, int nb, int N, int L, int32_t *rows) {
    hipLaunchKernelGGL(k_var_boot_rows, dim3(cdiv(N, 256), nb), dim3(256), 0, s, seed, N, L, rows);
    UOI_LAUNCH_CHECK();
}

void launch_split(hipStream_t s, uint64_t seed, uint32_t tag, int nb, int cnt, int ntrain,
                  uint8_t *is_train) {
    if (cnt <= kSortMax) {
        int np2 = 2;
        while (np2 < cnt) np2 <<= 1;
        const size_t lds = (size_t)np2 * (sizeof(unsigned long long) + sizeof(int));
        hipLaunchKernelGGL(k_split_sort, dim3(nb), dim3(1024), lds, s, seed, tag, cnt, np2, ntrain,
                           is_train);
    } else {
        hipLaunchKernelGGL(k_split_rank, dim3(cdiv(cnt, 256), nb), dim3(256), 0, s, seed, tag, cnt,
                           ntrain, is_train);
    }
    UOI_LAUNCH_CHECK();
}

void launch_compact_rows(hipStream_t s, int nb, int cnt, const uint8_t *is_train, int ntrain,
                         int32_t *train, int32_t *eval) {
    hipLaunchKernelGGL(k_compact, dim3(nb), dim3(256), 0, s, cnt, ntrain, is_train, train, eval);
    UOI_LAUNCH_CHECK();
}

void launch_expand_blocks(hipStream_t s, int nb, int nblk, int N, int L, const uint8_t *is_train,
                          int32_t *train, int32_t *eval, int32_t *ntr, int32_t *nev) {
    hipLaunchKernelGGL(k_expand_blocks, dim3(nb), dim3(256), 0, s, nblk, N, L, is_train, train, eval,
                       ntr, nev);
    UOI_LAUNCH_CHECK();
}

void launch_finite_check(hipStream_t s, const double *x, size_t n, int *flag) {
    unsigned g = (unsigned)std::min<size_t>(1024, (n + 255) / 256);
    if (g == 0) return;
    hipLaunchKernelGGL(k_finite, dim3(g), dim3(256), 0, s, x, n, flag);
    UOI_LAUNCH_CHECK();
}

}  // namespace uoi
