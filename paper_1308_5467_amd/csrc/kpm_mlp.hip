// Learned damping network (replaces the Jackson factors of Appendix A,
// eq. (jackson), at degree 127): 128 -> 256 -> 256 -> 128, GELU hidden
// layers, sigmoid head with g_0 := 1, FP32.
//
//   forward   z1 = x W1 + b1, h1 = gelu(z1); z2 = h1 W2 + b2, h2 = gelu(z2);
//             z3 = h2 W3 + b3, g = sigmoid(z3) (g_0 = 1)
//   loss      phi = (g * x) K^T  (K: 200 x 128 blur operator: the Gaussian-
//             blurred density of eq. (tdosFinal) at 200 midpoints of [-1, 1]
//             per unit g_k mu_k), L = mean_n dt sum_i |phi - target|
//             (eq. (err2), p = 1, on the regularised density of eq. (blurphi))
//   backward  dphi = sign(e) dt / N; dz3 = ((dphi K) * x) g (1 - g) (0 at k = 0);
//             dW3 = h2^T dz3, dh2 = dz3 W3^T, dz2 = dh2 gelu'(z2), ... ;
//             bias gradients are column sums
//   update    Adam
//
// Every product is one tiled FP32 GEMM kernel (64 x 64 output tile per
// 256-thread workgroup, 16-deep LDS stages, 4 x 4 outputs per thread) with
// a fused epilogue; each output is accumulated by one thread in a fixed
// order, so results are bitwise reproducible.  The whole network costs a
// few GFLOP per epoch at a batch of 8192, far below the moment computation,
// so the GEMMs are plain vector FMA rather than matrix-core code.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "kpm_internal.h"

namespace kpm {

constexpr int NIN = 128, NH = 256, NOUT = 128, NPTS = 200;
constexpr int64_t P_W1 = 0, P_B1 = P_W1 + NIN * NH, P_W2 = P_B1 + NH, P_B2 = P_W2 + NH * NH,
                  P_W3 = P_B2 + NH, P_B3 = P_W3 + NH * NOUT, P_TOTAL = P_B3 + NOUT;

__device__ __forceinline__ float gelu_f(float u) { return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float u) {
    return 0.5f * (1.0f + erff(u * 0.70710678118654752f)) + u * expf(-0.5f * u * u) * 0.3989422804014327f;
}
__device__ __forceinline__ float sigmoid_f(float u) { return 1.0f / (1.0f + expf(-u)); }

// ---------------------------------------------------------------- epilogues
struct EpiStore {  // C = acc
    float* C;
    int ldc;
    __device__ void operator()(int r, int c, float acc) const { C[(int64_t)r * ldc + c] = acc; }
};
struct EpiBiasGelu {  // Z = acc + b, H = gelu(Z)
    const float* bias;
    float* Z;
    float* H;
    int ld;
    __device__ void operator()(int r, int c, float acc) const {
        const float z = acc + bias[c];
        Z[(int64_t)r * ld + c] = z;
        H[(int64_t)r * ld + c] = gelu_f(z);
    }
};
struct EpiBiasSigmoid {  // G = sigmoid(acc + b), G[:, 0] = 1
    const float* bias;
    float* G;
    int ld;
    __device__ void operator()(int r, int c, float acc) const {
        G[(int64_t)r * ld + c] = c == 0 ? 1.0f : sigmoid_f(acc + bias[c]);
    }
};
struct EpiLoss {  // e = acc - T; dphi = sign(e) * scale; absE = |e|
    const float* T;
    float* dphi;
    float* absE;
    float scale;
    int ld;
    __device__ void operator()(int r, int c, float acc) const {
        const float e = acc - T[(int64_t)r * ld + c];
        dphi[(int64_t)r * ld + c] = e > 0.0f ? scale : (e < 0.0f ? -scale : 0.0f);
        absE[(int64_t)r * ld + c] = fabsf(e);
    }
};
struct EpiDz3 {  // dz3 = acc * x * g (1 - g), 0 at k = 0
    const float* X;
    const float* G;
    float* D;
    int ld;
    __device__ void operator()(int r, int c, float acc) const {
        const int64_t i = (int64_t)r * ld + c;
        const float g = G[i];
        D[i] = c == 0 ? 0.0f : acc * X[i] * g * (1.0f - g);
    }
};
struct EpiGeluGrad {  // D = acc * gelu'(Z)
    const float* Z;
    float* D;
    int ld;
    __device__ void operator()(int r, int c, float acc) const {
        const int64_t i = (int64_t)r * ld + c;
        D[i] = acc * gelu_grad_f(Z[i]);
    }
};

// C[M x N] = op(A) op(B); op(A)(i, k) = TA ? A[k*lda + i] : A[i*lda + k];
// op(B)(k, j) = TB ? B[j*ldb + k] : B[k*ldb + j].
constexpr int BM = 64, BN = 64, BK = 16;
template <bool TA, bool TB, typename Epi>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                                                   const float* __restrict__ B, int ldb, Epi epi) {
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + e * 256;
            int i, k;
            if (TA) { k = idx / BM; i = idx % BM; }
            else { i = idx / BK; k = idx % BK; }
            const int gi = i0 + i, gk = k0 + k;
            float v = 0.0f;
            if (gi < M && gk < K) v = TA ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk];
            As[k][i] = v;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + e * 256;
            int j, k;
            if (TB) { j = idx / BK; k = idx % BK; }
            else { k = idx / BN; j = idx % BN; }
            const int gj = j0 + j, gk = k0 + k;
            float v = 0.0f;
            if (gj < N && gk < K) v = TB ? B[(int64_t)gj * ldb + gk] : B[(int64_t)gk * ldb + gj];
            Bs[k][j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BK; ++k) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[k][ty * 4 + u];
                b[u] = Bs[k][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = i0 + ty * 4 + u, c = j0 + tx * 4 + v;
            if (r < M && c < N) epi(r, c, acc[u][v]);
        }
}

template <bool TA, bool TB, typename Epi>
static hipError_t gemm(hipStream_t s, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
                       Epi epi) {
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
    gemm_kernel<TA, TB, Epi><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, epi);
    return hipGetLastError();
}

// out[j] (+)= sum over rows of D[r*ld + j], accumulated in FP64, rows in order.
__global__ void colsum_kernel(const float* __restrict__ D, int rows, int cols, int ld, float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += (double)D[(int64_t)r * ld + j];
    out[j] = (float)s;
}

// loss[0] = sum of |e| (FP64, fixed order: per-thread strided sums, then a tree).
__global__ __launch_bounds__(256) void sum_abs_kernel(const float* __restrict__ absE, int64_t count, double scale,
                                                      float* __restrict__ loss_out, double* __restrict__ acc_out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) s += (double)absE[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double l = sh[0] * scale;
        if (loss_out) loss_out[0] = (float)l;
        if (acc_out) acc_out[0] += l;
    }
}

// K[i][k] = (1/Q) sum_q w_k cos(k th_q) g_sigma(t_i - cos th_q), th_q = (q + 1/2) pi / Q,
// w_0 = 1, w_k = 2, t_i = -1 + (i + 1/2) 2/npts.  Computed in FP64, stored FP32.
__global__ void blur_operator_kernel(int nmom, int npts, double sigma, int Q, float* __restrict__ Kop) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nmom * npts) return;
    const int i = idx / nmom, k = idx - i * nmom;
    const double t = -1.0 + (i + 0.5) * (2.0 / npts);
    const double norm = 1.0 / sqrt(2.0 * M_PI * sigma * sigma);
    double s = 0.0;
    for (int q = 0; q < Q; ++q) {
        const double th = (q + 0.5) * M_PI / Q;
        const double dtq = t - cos(th);
        s += cos(k * th) * exp(-dtq * dtq / (2.0 * sigma * sigma));
    }
    Kop[idx] = (float)(s * norm * (k == 0 ? 1.0 : 2.0) / Q);
}

__global__ void adam_kernel(int64_t P, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__device__ __forceinline__ uint64_t mlp_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Weights uniform in [-s, s] (s = 1/sqrt(fan-in); the output layer 0.1/sqrt(256))
// from SplitMix64 output (index + 1) of `seed`; hidden biases 0; output bias
// logit of the Jackson factors of degree 127 so that training starts from
// Jackson damping.
__global__ void mlp_init_kernel(uint64_t seed, float* __restrict__ p) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P_TOTAL;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t z = mlp_mix(seed + (uint64_t)(i + 1) * 0x9e3779b97f4a7c15ull);
        const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        float val;
        if (i < P_B1) val = (float)((2.0 * u - 1.0) / sqrt((double)NIN));
        else if (i < P_W2) val = 0.0f;
        else if (i < P_B2) val = (float)((2.0 * u - 1.0) / sqrt((double)NH));
        else if (i < P_W3) val = 0.0f;
        else if (i < P_B3) val = (float)(0.1 * (2.0 * u - 1.0) / sqrt((double)NH));
        else {
            const int k = (int)(i - P_B3);
            const int Mj = NOUT - 1;
            const double a = M_PI / (Mj + 2);
            double gj = ((1.0 - (double)k / (Mj + 2)) * sin(a) * cos(k * a) + cos(a) * sin(k * a) / (Mj + 2)) / sin(a);
            gj = fmin(fmax(gj, 1e-4), 1.0 - 1e-4);
            val = (float)log(gj / (1.0 - gj));
        }
        p[i] = val;
    }
}

__global__ void gather_rows_kernel(const float* __restrict__ src, int cols, const int32_t* __restrict__ idx,
                                   int nrows, float* __restrict__ dst) {
    const int64_t total = (int64_t)nrows * cols;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / cols, c = t - r * cols;
        dst[t] = src[(int64_t)idx[r] * cols + c];
    }
}

// ---------------------------------------------------------------- network passes
struct MlpBufs {  // activations for a batch of N rows
    float *z1, *h1, *z2, *h2, *g, *dphi, *absE, *d3, *d2, *d1;
};

// Forward pass of a few rows (inference on one moment vector): one
// workgroup per row keeps the activations in LDS and runs the three layers
// in one launch; thread t owns output column t of each layer and reads
// column t of the weights (coalesced over the workgroup), 32 weights in
// flight per thread ahead of the FMA chain.  Each output is
// the same k-ordered FMA chain plus bias as in the tiled GEMM, so the
// result is bitwise that of the batched path.
constexpr int kSmallRows = 16;
__global__ __launch_bounds__(NH) void forward_small_kernel(const float* __restrict__ x, const float* __restrict__ p,
                                                           float* __restrict__ g) {
    __shared__ float xs[NIN], h1[NH], h2[NH];
    const int t = threadIdx.x;
    const int64_t row = blockIdx.x;
    if (t < NIN) xs[t] = x[row * NIN + t];
    __syncthreads();
    const float* __restrict__ W1 = p + P_W1;
    const float* __restrict__ W2 = p + P_W2;
    const float* __restrict__ W3 = p + P_W3;
    float acc = 0.0f;
#pragma unroll 32
    for (int k = 0; k < NIN; ++k) acc = fmaf(xs[k], W1[k * NH + t], acc);
    h1[t] = gelu_f(acc + p[P_B1 + t]);
    __syncthreads();
    acc = 0.0f;
#pragma unroll 32
    for (int k = 0; k < NH; ++k) acc = fmaf(h1[k], W2[k * NH + t], acc);
    h2[t] = gelu_f(acc + p[P_B2 + t]);
    __syncthreads();
    if (t < NOUT) {
        acc = 0.0f;
#pragma unroll 32
        for (int k = 0; k < NH; ++k) acc = fmaf(h2[k], W3[k * NOUT + t], acc);
        g[row * NOUT + t] = t == 0 ? 1.0f : sigmoid_f(acc + p[P_B3 + t]);
    }
}

static hipError_t forward(hipStream_t s, int N, const float* x, const float* p, const MlpBufs& b) {
    hipError_t e;
    if ((e = gemm<false, false>(s, N, NH, NIN, x, NIN, p + P_W1, NH, EpiBiasGelu{p + P_B1, b.z1, b.h1, NH})))
        return e;
    if ((e = gemm<false, false>(s, N, NH, NH, b.h1, NH, p + P_W2, NH, EpiBiasGelu{p + P_B2, b.z2, b.h2, NH})))
        return e;
    return gemm<false, false>(s, N, NOUT, NH, b.h2, NH, p + P_W3, NOUT, EpiBiasSigmoid{p + P_B3, b.g, NOUT});
}

__global__ void mul_kernel(int64_t n, const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ o) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        o[i] = a[i] * b[i];
}

hipError_t mlp_mul(hipStream_t s, int64_t n, const float* a, const float* b, float* o) {
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    mul_kernel<<<(int)std::max<int64_t>(blocks, 1), 256, 0, s>>>(n, a, b, o);
    return hipGetLastError();
}

// Loss and gradients for a batch; grads[P_TOTAL]; loss_out (device float) and
// loss_acc (device double accumulator) optional.
static hipError_t loss_grad(hipStream_t s, int N, const float* x, const float* target, const float* Kop,
                            const float* p, const MlpBufs& b, float* grads, float* loss_out, double* loss_acc,
                            float* xg) {
    hipError_t e;
    if ((e = forward(s, N, x, p, b))) return e;
    const float dt = 2.0f / NPTS;
    // xg = g * x (the damped moments), then phi = xg K^T with the loss epilogue
    if ((e = mlp_mul(s, (int64_t)N * NOUT, b.g, x, xg))) return e;
    if ((e = gemm<false, true>(s, N, NPTS, NOUT, xg, NOUT, Kop, NOUT,
                               EpiLoss{target, b.dphi, b.absE, dt / (float)N, NPTS})))
        return e;
    sum_abs_kernel<<<1, 256, 0, s>>>(b.absE, (int64_t)N * NPTS, (double)dt / N, loss_out, loss_acc);
    // dz3 = ((dphi K) * x) g (1 - g)
    if ((e = gemm<false, false>(s, N, NOUT, NPTS, b.dphi, NPTS, Kop, NOUT, EpiDz3{x, b.g, b.d3, NOUT}))) return e;
    // layer 3
    if ((e = gemm<true, false>(s, NH, NOUT, N, b.h2, NH, b.d3, NOUT, EpiStore{grads + P_W3, NOUT}))) return e;
    colsum_kernel<<<(NOUT + 127) / 128, 128, 0, s>>>(b.d3, N, NOUT, NOUT, grads + P_B3);
    if ((e = gemm<false, true>(s, N, NH, NOUT, b.d3, NOUT, p + P_W3, NOUT, EpiGeluGrad{b.z2, b.d2, NH}))) return e;
    // layer 2
    if ((e = gemm<true, false>(s, NH, NH, N, b.h1, NH, b.d2, NH, EpiStore{grads + P_W2, NH}))) return e;
    colsum_kernel<<<(NH + 127) / 128, 128, 0, s>>>(b.d2, N, NH, NH, grads + P_B2);
    if ((e = gemm<false, true>(s, N, NH, NH, b.d2, NH, p + P_W2, NH, EpiGeluGrad{b.z1, b.d1, NH}))) return e;
    // layer 1
    if ((e = gemm<true, false>(s, NIN, NH, N, x, NIN, b.d1, NH, EpiStore{grads + P_W1, NH}))) return e;
    colsum_kernel<<<(NH + 127) / 128, 128, 0, s>>>(b.d1, N, NH, NH, grads + P_B1);
    return hipGetLastError();
}

}  // namespace kpm

using namespace kpm;

// ---------------------------------------------------------------- host side
namespace {

struct MlpWork {
    MlpBufs b;
    float* xg = nullptr;
    int cap = 0;
};

kpm_status mlp_params(kpm_ctx* ctx, float** p) {
    if (!ctx->mlp_params.p) {
        if (hipMalloc(&ctx->mlp_params.p, P_TOTAL * sizeof(float)) != hipSuccess) {
            ctx->mlp_params.p = nullptr;
            return kpm_fail(ctx, KPM_ERR_ALLOC, "hipMalloc for the network parameters failed");
        }
        ctx->mlp_params.cap = P_TOTAL * sizeof(float);
    }
    *p = (float*)ctx->mlp_params.p;
    return KPM_OK;
}

kpm_status mlp_work(kpm_ctx* ctx, int N, MlpWork* w) {
    const size_t per_row = (size_t)(6 * NH + 3 * NOUT + 2 * NPTS) * sizeof(float);
    void* base;
    kpm_status st = kpm_ws(ctx, "mlp_act", per_row * (size_t)N + 4096, &base);
    if (st != KPM_OK) return st;
    float* f = (float*)base;
    auto take = [&](size_t cols) {
        float* r = f;
        f += cols * (size_t)N;
        return r;
    };
    w->b.z1 = take(NH);
    w->b.h1 = take(NH);
    w->b.z2 = take(NH);
    w->b.h2 = take(NH);
    w->b.g = take(NOUT);
    w->b.d3 = take(NOUT);
    w->xg = take(NOUT);
    w->b.dphi = take(NPTS);
    w->b.absE = take(NPTS);
    w->b.d2 = take(NH);
    w->b.d1 = take(NH);
    w->cap = N;
    return KPM_OK;
}

kpm_status blur_op(kpm_ctx* ctx, float sigma, float** K) {
    void* k;
    kpm_status st = kpm_ws(ctx, "mlp_blur", (size_t)NPTS * NOUT * sizeof(float), &k);
    if (st != KPM_OK) return st;
    // The operator is rebuilt whenever this context has not built it for
    // this sigma in this buffer (the cache lives in the context, so a new
    // context never trusts memory it has not written).
    if (ctx->mlp_blur_sigma != sigma || ctx->mlp_blur_buf != k) {
        blur_operator_kernel<<<(NPTS * NOUT + 127) / 128, 128, 0, ctx->stream>>>(NOUT, NPTS, (double)sigma, 8192,
                                                                               (float*)k);
        KPM_HIP(ctx, hipGetLastError());
        ctx->mlp_blur_sigma = sigma;
        ctx->mlp_blur_buf = k;
    }
    *K = (float*)k;
    return KPM_OK;
}

kpm_status upload(kpm_ctx* ctx, const char* role, const float* host, size_t count, float** dev) {
    void* d;
    kpm_status st = kpm_ws(ctx, role, count * sizeof(float), &d);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(d, host, count * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    *dev = (float*)d;
    return KPM_OK;
}

kpm_status need_model(kpm_ctx* ctx) {
    if (!ctx->mlp_ready) return kpm_fail(ctx, KPM_ERR_NOMODEL, "no network parameters set (init, set or load first)");
    return KPM_OK;
}

}  // namespace

extern "C" int64_t kpm_mlp_param_count(void) { return P_TOTAL; }

extern "C" kpm_status kpm_mlp_set_params(kpm_ctx* ctx, const float* params) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!params) return kpm_fail(ctx, KPM_ERR_ARG, "params is NULL");
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    float* p;
    kpm_status st = mlp_params(ctx, &p);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipMemcpyAsync(p, params, P_TOTAL * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->mlp_ready = true;
    return KPM_OK;
}

extern "C" kpm_status kpm_mlp_get_params(kpm_ctx* ctx, float* params) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (!params) return kpm_fail(ctx, KPM_ERR_ARG, "params is NULL");
    kpm_status st = need_model(ctx);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    KPM_HIP(ctx, hipMemcpyAsync(params, ctx->mlp_params.p, P_TOTAL * sizeof(float), hipMemcpyDeviceToHost,
                                ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KPM_OK;
}

extern "C" kpm_status kpm_mlp_init(kpm_ctx* ctx, uint64_t seed) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    float* p;
    kpm_status st = mlp_params(ctx, &p);
    if (st != KPM_OK) return st;
    mlp_init_kernel<<<256, 256, 0, ctx->stream>>>(seed, p);
    KPM_HIP(ctx, hipGetLastError());
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->mlp_ready = true;
    return KPM_OK;
}

extern "C" kpm_status kpm_mlp_forward(kpm_ctx* ctx, int N, const float* x, float* g) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (N < 1 || N > (1 << 22) || !x || !g) return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    kpm_status st = need_model(ctx);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    MlpWork w;
    float* xd;
    if ((st = mlp_work(ctx, N, &w)) != KPM_OK) return st;
    if ((st = upload(ctx, "mlp_x", x, (size_t)N * NIN, &xd)) != KPM_OK) return st;
    if (N <= kSmallRows) {
        forward_small_kernel<<<N, NH, 0, ctx->stream>>>(xd, (const float*)ctx->mlp_params.p, w.b.g);
        KPM_HIP(ctx, hipGetLastError());
    } else {
        KPM_HIP(ctx, forward(ctx->stream, N, xd, (const float*)ctx->mlp_params.p, w.b));
    }
    KPM_HIP(ctx, hipMemcpyAsync(g, w.b.g, (size_t)N * NOUT * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KPM_OK;
}

extern "C" kpm_status kpm_mlp_loss_grad(kpm_ctx* ctx, int N, const float* x, const float* target, float sigma,
                                        float* loss, float* grads) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (N < 1 || N > (1 << 22) || !x || !target || !loss || !grads || !(sigma > 0.0f))
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    kpm_status st = need_model(ctx);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    MlpWork w;
    float *xd, *td, *Kop;
    void *gd, *ld;
    if ((st = mlp_work(ctx, N, &w)) != KPM_OK) return st;
    if ((st = upload(ctx, "mlp_x", x, (size_t)N * NIN, &xd)) != KPM_OK) return st;
    if ((st = upload(ctx, "mlp_t", target, (size_t)N * NPTS, &td)) != KPM_OK) return st;
    if ((st = blur_op(ctx, sigma, &Kop)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_grad", P_TOTAL * sizeof(float), &gd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_loss", 64, &ld)) != KPM_OK) return st;
    KPM_HIP(ctx, loss_grad(ctx->stream, N, xd, td, Kop, (const float*)ctx->mlp_params.p, w.b, (float*)gd,
                           (float*)ld, nullptr, w.xg));
    KPM_HIP(ctx, hipMemcpyAsync(grads, gd, P_TOTAL * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipMemcpyAsync(loss, ld, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return KPM_OK;
}

extern "C" kpm_status kpm_mlp_train(kpm_ctx* ctx, int N, const float* x, const float* target, float sigma,
                                    int epochs, int batch, float lr, uint64_t seed, float* loss_per_epoch) {
    if (!ctx) return KPM_ERR_ARG;
    ctx->err.clear();
    if (N < 1 || N > (1 << 22) || !x || !target || !(sigma > 0.0f) || epochs < 0 || batch < 1 || !(lr > 0.0f))
        return kpm_fail(ctx, KPM_ERR_ARG, "bad argument");
    kpm_status st = need_model(ctx);
    if (st != KPM_OK) return st;
    KPM_HIP(ctx, hipSetDevice(ctx->device));
    batch = std::min(batch, N);
    MlpWork w;
    float *xd, *td, *Kop;
    void *gd, *md, *vd, *xb, *tb, *idx, *lacc;
    if ((st = mlp_work(ctx, batch, &w)) != KPM_OK) return st;
    if ((st = upload(ctx, "mlp_xall", x, (size_t)N * NIN, &xd)) != KPM_OK) return st;
    if ((st = upload(ctx, "mlp_tall", target, (size_t)N * NPTS, &td)) != KPM_OK) return st;
    if ((st = blur_op(ctx, sigma, &Kop)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_grad", P_TOTAL * sizeof(float), &gd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_adam_m", P_TOTAL * sizeof(float), &md)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_adam_v", P_TOTAL * sizeof(float), &vd)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_xb", (size_t)batch * NIN * sizeof(float), &xb)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_tb", (size_t)batch * NPTS * sizeof(float), &tb)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_idx", (size_t)N * 4, &idx)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_lacc", (size_t)std::max(epochs, 1) * 8, &lacc)) != KPM_OK) return st;
    KPM_HIP(ctx, hipMemsetAsync(md, 0, P_TOTAL * sizeof(float), ctx->stream));
    KPM_HIP(ctx, hipMemsetAsync(vd, 0, P_TOTAL * sizeof(float), ctx->stream));
    KPM_HIP(ctx, hipMemsetAsync(lacc, 0, (size_t)std::max(epochs, 1) * 8, ctx->stream));
    float* p = (float*)ctx->mlp_params.p;
    std::vector<int32_t> order(N);
    std::vector<int> nb_of_epoch(epochs);
    uint64_t rng = seed;
    auto next = [&]() {  // SplitMix64 sequence
        uint64_t z = (rng += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    int t = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = 0; i < N; ++i) order[i] = i;
        for (int i = N - 1; i > 0; --i) std::swap(order[i], order[(int)(next() % (uint64_t)(i + 1))]);
        // the index array is uploaded per epoch; wait for the previous epoch's gathers first
        KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
        KPM_HIP(ctx, hipMemcpyAsync(idx, order.data(), (size_t)N * 4, hipMemcpyHostToDevice, ctx->stream));
        int nb = 0;
        for (int b0 = 0; b0 < N; b0 += batch) {
            const int nr = std::min(batch, N - b0);
            const int32_t* ib = (const int32_t*)idx + b0;
            gather_rows_kernel<<<256, 256, 0, ctx->stream>>>(xd, NIN, ib, nr, (float*)xb);
            gather_rows_kernel<<<256, 256, 0, ctx->stream>>>(td, NPTS, ib, nr, (float*)tb);
            KPM_HIP(ctx, loss_grad(ctx->stream, nr, (float*)xb, (float*)tb, Kop, p, w.b, (float*)gd, nullptr,
                                   (double*)lacc + ep, w.xg));
            ++t;
            const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
            adam_kernel<<<256, 256, 0, ctx->stream>>>(P_TOTAL, p, (float*)gd, (float*)md, (float*)vd, lr, 0.9f,
                                                      0.999f, 1e-8f, c1, c2);
            KPM_HIP(ctx, hipGetLastError());
            ++nb;
        }
        nb_of_epoch[ep] = nb;
    }
    std::vector<double> la(std::max(epochs, 1));
    KPM_HIP(ctx, hipMemcpyAsync(la.data(), lacc, la.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    KPM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (loss_per_epoch)
        for (int ep = 0; ep < epochs; ++ep) loss_per_epoch[ep] = (float)(la[ep] / nb_of_epoch[ep]);
    return KPM_OK;
}

extern "C" kpm_status kpm_mlp_save(kpm_ctx* ctx, const char* path) {
    if (!ctx) return KPM_ERR_ARG;
    if (!path) return kpm_fail(ctx, KPM_ERR_ARG, "path is NULL");
    std::vector<float> p(P_TOTAL);
    kpm_status st = kpm_mlp_get_params(ctx, p.data());
    if (st != KPM_OK) return st;
    FILE* f = fopen(path, "wb");
    if (!f) return kpm_fail(ctx, KPM_ERR_ARG, std::string("cannot open ") + path);
    const char magic[8] = {'K', 'P', 'M', 'M', 'L', 'P', '1', '\0'};
    const int64_t count = P_TOTAL;
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&count, 8, 1, f) == 1 &&
              fwrite(p.data(), sizeof(float), P_TOTAL, f) == (size_t)P_TOTAL;
    ok = (fclose(f) == 0) && ok;
    return ok ? KPM_OK : kpm_fail(ctx, KPM_ERR_ARG, std::string("write failed: ") + path);
}

extern "C" kpm_status kpm_mlp_load(kpm_ctx* ctx, const char* path) {
    if (!ctx) return KPM_ERR_ARG;
    if (!path) return kpm_fail(ctx, KPM_ERR_ARG, "path is NULL");
    FILE* f = fopen(path, "rb");
    if (!f) return kpm_fail(ctx, KPM_ERR_ARG, std::string("cannot open ") + path);
    char magic[8];
    int64_t count = 0;
    std::vector<float> p(P_TOTAL);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "KPMMLP1", 8) == 0 && fread(&count, 8, 1, f) == 1 &&
              count == P_TOTAL && fread(p.data(), sizeof(float), P_TOTAL, f) == (size_t)P_TOTAL;
    fclose(f);
    if (!ok) return kpm_fail(ctx, KPM_ERR_ARG, std::string("not a damping-network file: ") + path);
    return kpm_mlp_set_params(ctx, p.data());
}

namespace {
// x[k] = mu[k] as float for k <= M, 0 above (one row of network input).
__global__ __launch_bounds__(NIN) void learned_input_kernel(const double* __restrict__ mu, int M,
                                                            float* __restrict__ x) {
    const int k = threadIdx.x;
    x[k] = k <= M ? (float)mu[k] : 0.0f;
}
// g[k] = network output k (g[0] = 1) for k <= M.
__global__ __launch_bounds__(NOUT) void learned_output_kernel(const float* __restrict__ gf, int M,
                                                              double* __restrict__ g) {
    const int k = threadIdx.x;
    if (k <= M) g[k] = k == 0 ? 1.0 : (double)gf[k];
}
}  // namespace

// The same damping factors as kpm_learned_damping from device moments into
// device factors, enqueued on the context's stream without a wait.
kpm_status kpm_learned_damping_device(kpm_ctx* ctx, int M, const double* mu_dev, double* g_dev) {
    if (M < 0 || M > NOUT - 1) return kpm_fail(ctx, KPM_ERR_ARG, "learned damping is defined for M <= 127");
    kpm_status st = need_model(ctx);
    if (st != KPM_OK) return st;
    MlpWork w;
    void* xd;
    if ((st = mlp_work(ctx, 1, &w)) != KPM_OK) return st;
    if ((st = kpm_ws(ctx, "mlp_x", (size_t)NIN * sizeof(float), &xd)) != KPM_OK) return st;
    learned_input_kernel<<<1, NIN, 0, ctx->stream>>>(mu_dev, M, (float*)xd);
    KPM_HIP(ctx, hipGetLastError());
    forward_small_kernel<<<1, NH, 0, ctx->stream>>>((const float*)xd, (const float*)ctx->mlp_params.p, w.b.g);
    KPM_HIP(ctx, hipGetLastError());
    learned_output_kernel<<<1, NOUT, 0, ctx->stream>>>(w.b.g, M, g_dev);
    KPM_HIP(ctx, hipGetLastError());
    return KPM_OK;
}

// Degree M <= 127: the network reads mu_0..mu_M with zeros above (the
// truncation it is trained with) and g_0..g_M are returned.
kpm_status kpm_learned_damping(kpm_ctx* ctx, int M, const double* mu, double* g) {
    if (M < 0 || M > NOUT - 1) return kpm_fail(ctx, KPM_ERR_ARG, "learned damping is defined for M <= 127");
    float x[NIN], gf[NOUT];
    for (int k = 0; k < NIN; ++k) x[k] = k <= M ? (float)mu[k] : 0.0f;
    kpm_status st = kpm_mlp_forward(ctx, 1, x, gf);
    if (st != KPM_OK) return st;
    for (int k = 0; k <= M; ++k) g[k] = gf[k];
    g[0] = 1.0;
    return KPM_OK;
}
