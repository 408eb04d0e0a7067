// Warm-start network: a 3-layer ReLU MLP trained and run on the GPU with
// bfloat16 operands and float32 accumulation (MFMA 16x16x32 bf16).
//
// Not part of the paper: the paper's ADMM starts cold.  The network maps one
// LASSO problem of the selection sweep (bootstrap statistics c, penalty
// lambda) to a starting point for ADMM:
//     input  [c / lambda_max, log(lambda / lambda_max)]      (p + 1 values)
//     output z / lambda_max                                  (p values)
// with lambda_max = ||c||_inf of the bootstrap.  The dual variable is then
// completed from z (see admm.hip), and a solve whose predicted start is worse
// than the cold start falls back to the cold start.
//
// Layers y = x W' + b, W stored (out, in) row-major; master weights float32,
// GEMM operands (inputs, weights, hidden activations, back-propagated
// gradients) bfloat16 with round-to-nearest-even; loss = mean squared error;
// optimiser Adam (Kingma and Ba, 2015).
#include <cmath>
#include <vector>

#include "common.hpp"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct uoi_mlp {
    int n_in, hid, n_out;
    int64_t nparam;
    int64_t oW1, ob1, oW2, ob2, oW3, ob3;  // offsets into the flat parameter vector
    float *theta, *grad, *m, *v;           // float32 master weights, gradient, Adam moments
    bf16 *W1, *W2, *W3;                    // bfloat16 copies used by the GEMMs
    int64_t step;
    int cap;                               // activation buffers sized for this batch
    bf16 *X0, *H1, *H2, *dY, *dA1, *dA2;
    float *Y, *Xs;                         // network output; float32 staging of inputs
    double *loss;
};

namespace uoi {

// D(16x16) += A(16x32) B(32x16) in bf16 with float32 accumulation.  Lane l
// supplies A[l%16][8*(l/16) + e] and B[8*(l/16) + e][l%16], e < 8, and holds
// D[4*(l/16) + t][l%16] in element t (measured on gfx950).
__device__ __forceinline__ fx4 mfma_bf16(bf16x8 a, bf16x8 b, fx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// C(M x N) = op(A) op(B): TA -> A stored K x M (lda), else M x K; TB -> B stored
// N x K (ldb), else K x N.  64x64 tiles, 4 waves of 32x32, k-chunks of 32
// staged in LDS as [row][k] so each lane reads its 8 consecutive k at once.
template <bool TA, bool TB, class Epi>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const bf16 *__restrict__ A,
                                                   int lda, const bf16 *__restrict__ B, int ldb, Epi epi) {
    constexpr int LD = 40;  // padded row (80 bytes: keeps 16-byte alignment)
    __shared__ __attribute__((aligned(16))) bf16 As[64 * LD];
    __shared__ __attribute__((aligned(16))) bf16 Bs[64 * LD];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1, lr = lane & 15, lk = lane >> 4;
    fx4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) acc[a][c] = fx4{0, 0, 0, 0};
    const bf16 zero = (bf16)0.0f;
    for (int k0 = 0; k0 < K; k0 += 32) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            int i, k;
            if (!TA) { i = e >> 5; k = e & 31; }
            else { k = e >> 6; i = e & 63; }
            bf16 va = zero;
            if (i0 + i < M && k0 + k < K) va = TA ? A[(size_t)(k0 + k) * lda + i0 + i] : A[(size_t)(i0 + i) * lda + k0 + k];
            As[i * LD + k] = va;
            int j, kb;
            if (TB) { j = e >> 5; kb = e & 31; }
            else { kb = e >> 6; j = e & 63; }
            bf16 vb = zero;
            if (j0 + j < N && k0 + kb < K) vb = TB ? B[(size_t)(j0 + j) * ldb + k0 + kb] : B[(size_t)(k0 + kb) * ldb + j0 + j];
            Bs[j * LD + kb] = vb;
        }
        __syncthreads();
        bf16x8 av[2], bv[2];
        for (int a = 0; a < 2; ++a) av[a] = *reinterpret_cast<const bf16x8 *>(&As[(wm * 32 + 16 * a + lr) * LD + 8 * lk]);
        for (int c = 0; c < 2; ++c) bv[c] = *reinterpret_cast<const bf16x8 *>(&Bs[(wn * 32 + 16 * c + lr) * LD + 8 * lk]);
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 2; ++c) acc[a][c] = mfma_bf16(av[a], bv[c], acc[a][c]);
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c)
            for (int t = 0; t < 4; ++t) {
                const int i = i0 + wm * 32 + 16 * a + 4 * lk + t, j = j0 + wn * 32 + 16 * c + lr;
                if (i < M && j < N) epi(i, j, acc[a][c][t]);
            }
}

// hidden layer: out = bf16(relu(v + b[j]))
struct EpiHidden {
    const float *b;
    bf16 *out;
    int ld;
    __device__ void operator()(int i, int j, float v) const {
        float x = v + b[j];
        out[(size_t)i * ld + j] = (bf16)(x > 0.f ? x : 0.f);
    }
};
// output layer: out = v + b[j] (float32)
struct EpiOut {
    const float *b;
    float *out;
    int ld;
    __device__ void operator()(int i, int j, float v) const { out[(size_t)i * ld + j] = v + b[j]; }
};
// back-propagated gradient through a ReLU: out = bf16(v * [h > 0])
struct EpiMask {
    const bf16 *h;
    bf16 *out;
    int ld;
    __device__ void operator()(int i, int j, float v) const {
        float hv = (float)h[(size_t)i * ld + j];
        out[(size_t)i * ld + j] = (bf16)(hv > 0.f ? v : 0.f);
    }
};
// weight gradient (float32)
struct EpiStore {
    float *out;
    int ld;
    __device__ void operator()(int i, int j, float v) const { out[(size_t)i * ld + j] = v; }
};

template <bool TA, bool TB, class Epi>
static void gemm(hipStream_t s, int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb,
                 const Epi &epi) {
    hipLaunchKernelGGL((k_gemm_bf16<TA, TB, Epi>), dim3(cdiv(N, 64), cdiv(M, 64)), dim3(256), 0, s, M, N,
                       K, A, lda, B, ldb, epi);
    UOI_LAUNCH_CHECK();
}

__global__ void k_f32_to_bf16(size_t n, const float *__restrict__ a, bf16 *__restrict__ b) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (bf16)a[i];
}

// d = y - t; dY = bf16(2 d / (n m)); loss accumulates sum d^2 (float64)
__global__ void k_mse(size_t nm, const float *__restrict__ Y, const float *__restrict__ T,
                      bf16 *__restrict__ dY, double *__restrict__ loss) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (i < nm) {
        float d = Y[i] - T[i];
        dY[i] = (bf16)(2.0f * d / (float)nm);
        s = (double)d * (double)d;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, s);
}

// g[j] = sum_i d[i][j]  (bias gradient)
__global__ void k_colsum(int n, int m, const bf16 *__restrict__ d, float *__restrict__ g) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += (float)d[(size_t)i * m + j];
    g[j] = s;
}

__global__ void k_adam(size_t n, float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float c1, float c2) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static void refresh_bf16(hipStream_t s, uoi_mlp *M) {
    size_t n1 = (size_t)M->hid * M->n_in, n2 = (size_t)M->hid * M->hid, n3 = (size_t)M->n_out * M->hid;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(cdiv(n1, 256)), dim3(256), 0, s, n1, M->theta + M->oW1, M->W1);
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(cdiv(n2, 256)), dim3(256), 0, s, n2, M->theta + M->oW2, M->W2);
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(cdiv(n3, 256)), dim3(256), 0, s, n3, M->theta + M->oW3, M->W3);
    UOI_LAUNCH_CHECK();
}

static void ensure_cap(uoi_mlp *M, int n) {
    if (n <= M->cap) return;
    UOI_HIP(hipDeviceSynchronize());
    for (void *p : {(void *)M->X0, (void *)M->H1, (void *)M->H2, (void *)M->dY, (void *)M->dA1,
                    (void *)M->dA2, (void *)M->Y, (void *)M->Xs})
        if (p) (void)hipFree(p);
    const size_t c = (size_t)n;
    UOI_HIP(hipMalloc(&M->X0, c * M->n_in * sizeof(bf16)));
    UOI_HIP(hipMalloc(&M->H1, c * M->hid * sizeof(bf16)));
    UOI_HIP(hipMalloc(&M->H2, c * M->hid * sizeof(bf16)));
    UOI_HIP(hipMalloc(&M->dY, c * M->n_out * sizeof(bf16)));
    UOI_HIP(hipMalloc(&M->dA1, c * M->hid * sizeof(bf16)));
    UOI_HIP(hipMalloc(&M->dA2, c * M->hid * sizeof(bf16)));
    UOI_HIP(hipMalloc(&M->Y, c * M->n_out * sizeof(float)));
    UOI_HIP(hipMalloc(&M->Xs, c * M->n_in * sizeof(float)));
    M->cap = n;
}

// forward pass of n rows of X (float32, device); result in M->Y
void mlp_forward(hipStream_t s, uoi_mlp *M, int n, const float *X) {
    ensure_cap(M, n);
    size_t nx = (size_t)n * M->n_in;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(cdiv(nx, 256)), dim3(256), 0, s, nx, X, M->X0);
    UOI_LAUNCH_CHECK();
    gemm<false, true>(s, n, M->hid, M->n_in, M->X0, M->n_in, M->W1, M->n_in,
                      EpiHidden{M->theta + M->ob1, M->H1, M->hid});
    gemm<false, true>(s, n, M->hid, M->hid, M->H1, M->hid, M->W2, M->hid,
                      EpiHidden{M->theta + M->ob2, M->H2, M->hid});
    gemm<false, true>(s, n, M->n_out, M->hid, M->H2, M->hid, M->W3, M->hid,
                      EpiOut{M->theta + M->ob3, M->Y, M->n_out});
}

// forward + backward; gradient into M->grad, sum of squared errors into M->loss
static void mlp_backward(hipStream_t s, uoi_mlp *M, int n, const float *X, const float *T) {
    mlp_forward(s, M, n, X);
    size_t nm = (size_t)n * M->n_out;
    UOI_HIP(hipMemsetAsync(M->loss, 0, sizeof(double), s));
    hipLaunchKernelGGL(k_mse, dim3(cdiv(nm, 256)), dim3(256), 0, s, nm, M->Y, T, M->dY, M->loss);
    UOI_LAUNCH_CHECK();
    float *g = M->grad;
    // output layer
    gemm<true, false>(s, M->n_out, M->hid, n, M->dY, M->n_out, M->H2, M->hid, EpiStore{g + M->oW3, M->hid});
    hipLaunchKernelGGL(k_colsum, dim3(cdiv(M->n_out, 256)), dim3(256), 0, s, n, M->n_out, M->dY, g + M->ob3);
    gemm<false, false>(s, n, M->hid, M->n_out, M->dY, M->n_out, M->W3, M->hid, EpiMask{M->H2, M->dA2, M->hid});
    // second hidden layer
    gemm<true, false>(s, M->hid, M->hid, n, M->dA2, M->hid, M->H1, M->hid, EpiStore{g + M->oW2, M->hid});
    hipLaunchKernelGGL(k_colsum, dim3(cdiv(M->hid, 256)), dim3(256), 0, s, n, M->hid, M->dA2, g + M->ob2);
    gemm<false, false>(s, n, M->hid, M->hid, M->dA2, M->hid, M->W2, M->hid, EpiMask{M->H1, M->dA1, M->hid});
    // first hidden layer
    gemm<true, false>(s, M->hid, M->n_in, n, M->dA1, M->hid, M->X0, M->n_in, EpiStore{g + M->oW1, M->n_in});
    hipLaunchKernelGGL(k_colsum, dim3(cdiv(M->hid, 256)), dim3(256), 0, s, n, M->hid, M->dA1, g + M->ob1);
    UOI_LAUNCH_CHECK();
}

// mean squared error of the last backward pass (synchronises the stream)
static double mlp_last_loss(hipStream_t s, uoi_mlp *M, int n) {
    double l = 0.0;
    UOI_HIP(hipMemcpyAsync(&l, M->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    UOI_HIP(hipStreamSynchronize(s));
    return l / ((double)n * M->n_out);
}

}  // namespace uoi

using namespace uoi;

template <class F>
static int mlp_guard(F &&f) {
    try {
        set_last_error("");
        return f();
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return UOI_EHIP;
    }
}

extern "C" {

int uoi_mlp_create(int32_t n_in, int32_t hidden, int32_t n_out, uoi_mlp **out) {
    return mlp_guard([&] {
        UOI_REQUIRE(out && n_in >= 1 && hidden >= 1 && n_out >= 1, "invalid network sizes");
        uoi_mlp *M = new uoi_mlp{};
        M->n_in = n_in; M->hid = hidden; M->n_out = n_out;
        int64_t o = 0;
        M->oW1 = o; o += (int64_t)hidden * n_in;
        M->ob1 = o; o += hidden;
        M->oW2 = o; o += (int64_t)hidden * hidden;
        M->ob2 = o; o += hidden;
        M->oW3 = o; o += (int64_t)n_out * hidden;
        M->ob3 = o; o += n_out;
        M->nparam = o;
        try {
            UOI_HIP(hipMalloc(&M->theta, o * sizeof(float)));
            UOI_HIP(hipMalloc(&M->grad, o * sizeof(float)));
            UOI_HIP(hipMalloc(&M->m, o * sizeof(float)));
            UOI_HIP(hipMalloc(&M->v, o * sizeof(float)));
            UOI_HIP(hipMalloc(&M->W1, (size_t)hidden * n_in * sizeof(bf16)));
            UOI_HIP(hipMalloc(&M->W2, (size_t)hidden * hidden * sizeof(bf16)));
            UOI_HIP(hipMalloc(&M->W3, (size_t)n_out * hidden * sizeof(bf16)));
            UOI_HIP(hipMalloc(&M->loss, sizeof(double)));
            UOI_HIP(hipMemset(M->theta, 0, o * sizeof(float)));
            UOI_HIP(hipMemset(M->m, 0, o * sizeof(float)));
            UOI_HIP(hipMemset(M->v, 0, o * sizeof(float)));
            refresh_bf16(nullptr, M);
            UOI_HIP(hipDeviceSynchronize());
        } catch (...) {
            uoi_mlp_destroy(M);
            throw;
        }
        *out = M;
        return UOI_OK;
    });
}

void uoi_mlp_destroy(uoi_mlp *M) {
    if (!M) return;
    (void)hipDeviceSynchronize();
    for (void *p : {(void *)M->theta, (void *)M->grad, (void *)M->m, (void *)M->v, (void *)M->W1, (void *)M->W2,
                    (void *)M->W3, (void *)M->loss, (void *)M->X0, (void *)M->H1, (void *)M->H2, (void *)M->dY,
                    (void *)M->dA1, (void *)M->dA2, (void *)M->Y, (void *)M->Xs})
        if (p) (void)hipFree(p);
    delete M;
}

int64_t uoi_mlp_num_params(const uoi_mlp *M) { return M ? M->nparam : -1; }

int uoi_mlp_set_params(uoi_mlp *M, const float *theta, void *stream) {
    return mlp_guard([&] {
        UOI_REQUIRE(M && theta, "NULL argument");
        hipStream_t s = (hipStream_t)stream;
        UOI_HIP(hipMemcpyAsync(M->theta, theta, M->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
        UOI_HIP(hipMemsetAsync(M->m, 0, M->nparam * sizeof(float), s));
        UOI_HIP(hipMemsetAsync(M->v, 0, M->nparam * sizeof(float), s));
        M->step = 0;
        refresh_bf16(s, M);
        UOI_HIP(hipStreamSynchronize(s));
        return UOI_OK;
    });
}

int uoi_mlp_get_params(const uoi_mlp *M, float *theta, void *stream) {
    return mlp_guard([&] {
        UOI_REQUIRE(M && theta, "NULL argument");
        hipStream_t s = (hipStream_t)stream;
        UOI_HIP(hipMemcpyAsync(theta, M->theta, M->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
        UOI_HIP(hipStreamSynchronize(s));
        return UOI_OK;
    });
}

int uoi_mlp_forward(uoi_mlp *M, int32_t n, const float *X, float *Y, void *stream) {
    return mlp_guard([&] {
        UOI_REQUIRE(M && X && Y && n >= 1, "invalid arguments");
        hipStream_t s = (hipStream_t)stream;
        mlp_forward(s, M, n, X);
        UOI_HIP(hipMemcpyAsync(Y, M->Y, (size_t)n * M->n_out * sizeof(float), hipMemcpyDeviceToDevice, s));
        UOI_HIP(hipStreamSynchronize(s));
        return UOI_OK;
    });
}

int uoi_mlp_loss_grad(uoi_mlp *M, int32_t n, const float *X, const float *T, float *grad, double *loss,
                      void *stream) {
    return mlp_guard([&] {
        UOI_REQUIRE(M && X && T && n >= 1, "invalid arguments");
        hipStream_t s = (hipStream_t)stream;
        mlp_backward(s, M, n, X, T);
        if (grad) UOI_HIP(hipMemcpyAsync(grad, M->grad, M->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
        double l = mlp_last_loss(s, M, n);
        if (loss) *loss = l;
        return UOI_OK;
    });
}

int uoi_mlp_train_step(uoi_mlp *M, int32_t n, const float *X, const float *T, float lr, double *loss,
                       void *stream) {
    return mlp_guard([&] {
        UOI_REQUIRE(M && X && T && n >= 1 && lr > 0.f, "invalid arguments");
        hipStream_t s = (hipStream_t)stream;
        mlp_backward(s, M, n, X, T);
        M->step += 1;
        float c1 = 1.f - powf(0.9f, (float)M->step), c2 = 1.f - powf(0.999f, (float)M->step);
        hipLaunchKernelGGL(k_adam, dim3(cdiv(M->nparam, 256)), dim3(256), 0, s, (size_t)M->nparam, M->theta,
                           M->grad, M->m, M->v, lr, c1, c2);
        UOI_LAUNCH_CHECK();
        refresh_bf16(s, M);
        // the loss is read back (a stream synchronisation) only when asked for
        if (loss) *loss = mlp_last_loss(s, M, n);
        return UOI_OK;
    });
}

}  // extern "C"

namespace uoi {
float *mlp_input_buffer(uoi_mlp *M, int n) {
    ensure_cap(M, n);
    return M->Xs;
}
int mlp_dims(const uoi_mlp *M, int *n_in, int *n_out) {
    *n_in = M->n_in;
    *n_out = M->n_out;
    return 0;
}
const float *mlp_output(const uoi_mlp *M) { return M->Y; }
}  // namespace uoi
