// Surrogate network kernels: a multilayer perceptron n_in -> width (SiLU) x
// depth -> 1 that predicts the sweep's figure of merit, trained with AdamW on
// the mean squared error.
//
// The hidden layers' products are dense contractions and run on MFMA in the
// BF16 mode (v_mfma_f32_16x16x32_bf16: operands rounded to BF16 on load, FP32
// accumulate); the FP32 mode runs the same products with FP32 FMAs (used to
// check gradients tightly).  The 1-wide head, the loss, the bias gradients and
// the optimiser are FP32 elementwise / fixed-order reductions.
#include "gbd_internal.h"

#include <math.h>

namespace gbd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoid(z); }
__device__ inline float dsilu(float z) {
    const float s = sigmoid(z);
    return s * (1.0f + z * (1.0f - s));
}

__device__ inline void epilogue(const MlpGemm &g, int m, int n, float acc) {
    const int64_t o = (int64_t)m * g.N + n;
    if (g.epi == 0) {
        const float z = acc + (g.bias ? g.bias[n] : 0.0f);
        g.C[o] = z;
        if (g.H) g.H[o] = silu(z);
    } else if (g.epi == 1) {
        g.C[o] = acc * dsilu(g.zmul[o]);
    } else {
        g.C[o] = acc;
    }
}

// One workgroup of 4 wavefronts per 16 x 16 output tile, the K axis split
// between them: wavefront w takes K steps of 32 w KS ... + KS - 1 of every
// round of 4 KS steps, all their loads issued before the products (these
// products are small, K <= 256 in training: load latency decides, not
// throughput), and the four partial tiles are added in the order w = 0 ... 3
// through LDS.  Operand layout of the 16x16x32 BF16 MFMA: lane l supplies
// A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16], i = 0..7, and
// receives D[4 (l / 16) + i][l % 16], i = 0..3.  Every access is
// bounds-checked (zero padding of M, N and K).
template <int KS>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(MlpGemm g) {
    __shared__ floatx4 part[4][64];
    const int tm = blockIdx.y * 16, tn = blockIdx.x * 16;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, kg = lane >> 4;
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const int m = tm + r, n = tn + r;
    for (int k0 = 32 * KS * w; k0 < g.K; k0 += 32 * KS * 4) {
        bf16x8 va[KS], vb[KS];
#pragma unroll
        for (int s = 0; s < KS; s++)
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int k = k0 + 32 * s + kg * 8 + i;
                const float a = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0.0f;
                const float b = (n < g.N && k < g.K) ? g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn] : 0.0f;
                va[s][i] = (__bf16)a;
                vb[s][i] = (__bf16)b;
            }
#pragma unroll
        for (int s = 0; s < KS; s++) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va[s], vb[s], acc, 0, 0, 0);
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
        const floatx4 t = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int mm = tm + kg * 4 + i, nn = tn + r;
            if (mm < g.M && nn < g.N) epilogue(g, mm, nn, t[i]);
        }
    }
}

__global__ void __launch_bounds__(256) gemm_f32_kernel(MlpGemm g) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)g.M * g.N) return;
    const int m = (int)(t / g.N), n = (int)(t - (int64_t)m * g.N);
    float acc = 0.0f;
    for (int k = 0; k < g.K; k++)
        acc = fmaf(g.A[(int64_t)m * g.sam + (int64_t)k * g.sak], g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn], acc);
    epilogue(g, m, n, acc);
}

__global__ void __launch_bounds__(256) gather_kernel(const float *__restrict__ X, const float *__restrict__ y,
                                                     const int32_t *__restrict__ idx, int B, int n_in,
                                                     float *__restrict__ Xb, float *__restrict__ yb) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int64_t r = idx ? idx[b] : b;
    for (int i = 0; i < n_in; i++) Xb[(int64_t)b * n_in + i] = X[r * n_in + i];
    if (y) yb[b] = y[r];
}

// yhat[b] = sum_i H[b][i] w[i] + w0: a wavefront per row, lane l taking
// columns l, l + 64, ... (coalesced), then a fixed shuffle tree
__global__ void __launch_bounds__(256) head_forward_kernel(const float *__restrict__ H, const float *__restrict__ w,
                                                           const float *__restrict__ w0, int B, int W,
                                                           float *__restrict__ yhat) {
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (b >= B) return;  // uniform per wavefront
    float acc = 0.0f;
    for (int i = lane; i < W; i += 64) acc = fmaf(H[(int64_t)b * W + i], w[i], acc);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) yhat[b] = acc + w0[0];
}

// g[b] = 2 (yhat - y) / B and the loss mean((yhat - y)^2), one workgroup
__global__ void __launch_bounds__(256) loss_kernel(const float *__restrict__ yhat, const float *__restrict__ y, int B,
                                                   float *__restrict__ g, float *__restrict__ loss) {
    __shared__ float part[256];
    float s = 0.0f;
    for (int b = threadIdx.x; b < B; b += 256) {
        const float d = yhat[b] - y[b];
        g[b] = 2.0f * d / (float)B;
        s = fmaf(d, d, s);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) loss[0] = part[0] / (float)B;
}

// Column sums over a batch, in parallel and in a fixed order: a block of
// 256 threads takes 32 columns, thread (c, r) sums rows r, r + 8, ... of
// column c (coalesced across c), and the 8 partial sums of a column are
// added in order r = 0 ... 7.  out[i] = sum_b wgt[b] X[b][i] for i < W (wgt
// null: weight 1), and with bias_col also out[W] = sum_b wgt[b].
constexpr int kSumCols = 32, kSumRows = 8;
__device__ inline void column_sums(const float *__restrict__ X, const float *__restrict__ wgt, int B, int W,
                                   bool bias_col, float *__restrict__ out) {
    __shared__ float part[kSumRows][kSumCols];
    const int c = threadIdx.x % kSumCols, r = threadIdx.x / kSumCols;
    const int i = blockIdx.x * kSumCols + c;
    float acc = 0.0f;
    if (i < W) {
        for (int b = r; b < B; b += kSumRows) acc = fmaf(wgt ? wgt[b] : 1.0f, X[(int64_t)b * W + i], acc);
    } else if (bias_col && i == W) {
        for (int b = r; b < B; b += kSumRows) acc += wgt ? wgt[b] : 1.0f;
    }
    part[r][c] = acc;
    __syncthreads();
    if (r == 0 && (i < W || (bias_col && i == W))) {
        float s = part[0][c];
#pragma unroll
        for (int k = 1; k < kSumRows; k++) s += part[k][c];
        out[i] = s;
    }
}

// head gradients: dw[i] = sum_b g[b] H[b][i] (i < W), dw0 = sum_b g[b] (i == W)
__global__ void __launch_bounds__(kSumCols * kSumRows) head_grad_kernel(const float *__restrict__ g,
                                                                        const float *__restrict__ H, int B, int W,
                                                                        float *__restrict__ dw) {
    column_sums(H, g, B, W, true, dw);
}

// dZ[b][i] = g[b] w[i] SiLU'(Z[b][i]) for the last hidden layer
__global__ void __launch_bounds__(256) head_back_kernel(const float *__restrict__ g, const float *__restrict__ w,
                                                        const float *__restrict__ Z, int B, int W,
                                                        float *__restrict__ dZ) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * W) return;
    const int b = (int)(t / W), i = (int)(t - (int64_t)b * W);
    dZ[t] = g[b] * w[i] * dsilu(Z[t]);
}

// db[o] = sum_b dZ[b][o]
__global__ void __launch_bounds__(kSumCols * kSumRows) colsum_kernel(const float *__restrict__ dZ, int B, int W,
                                                                     float *__restrict__ db) {
    column_sums(dZ, nullptr, B, W, false, db);
}

__global__ void __launch_bounds__(256) adamw_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                    float *__restrict__ m, float *__restrict__ v, int64_t n, float lr,
                                                    float b1, float b2, float eps, float wd, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] = p[i] - lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
}

// acc[0] += v[0] (one running loss sum in step order)
__global__ void __launch_bounds__(64) accum_kernel(float *__restrict__ acc, const float *__restrict__ v) {
    if (threadIdx.x == 0) acc[0] += v[0];
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_mlp_gemm(int bf16, const MlpGemm &g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (bf16) {
        dim3 grid((g.N + 15) / 16, (g.M + 15) / 16);
        if (g.K <= 128)
            gemm_bf16_kernel<1><<<grid, 256, 0, s>>>(g);
        else
            gemm_bf16_kernel<2><<<grid, 256, 0, s>>>(g);
    } else {
        gemm_f32_kernel<<<blocks_for((int64_t)g.M * g.N, 256), 256, 0, s>>>(g);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_gather(const float *X, const float *y, const int32_t *idx, int B, int n_in, float *Xb, float *yb,
                             hipStream_t s) {
    if (B <= 0) return hipSuccess;
    gather_kernel<<<blocks_for(B, 256), 256, 0, s>>>(X, y, idx, B, n_in, Xb, yb);
    return hipGetLastError();
}

hipError_t launch_mlp_head_forward(const float *H, const float *w, const float *w0, int B, int W, float *yhat,
                                   hipStream_t s) {
    if (B <= 0) return hipSuccess;
    head_forward_kernel<<<blocks_for(B, 4), 256, 0, s>>>(H, w, w0, B, W, yhat);
    return hipGetLastError();
}

hipError_t launch_mlp_head_backward(const float *yhat, const float *y, const float *H, const float *w, const float *Z,
                                    int B, int W, float *g, float *loss, float *dw, float *dZ, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    loss_kernel<<<1, 256, 0, s>>>(yhat, y, B, g, loss);
    head_grad_kernel<<<blocks_for(W + 1, kSumCols), kSumCols * kSumRows, 0, s>>>(g, H, B, W, dw);
    head_back_kernel<<<blocks_for((int64_t)B * W, 256), 256, 0, s>>>(g, w, Z, B, W, dZ);
    return hipGetLastError();
}

hipError_t launch_mlp_colsum(const float *dZ, int B, int W, float *db, hipStream_t s) {
    if (W <= 0) return hipSuccess;
    colsum_kernel<<<blocks_for(W, kSumCols), kSumCols * kSumRows, 0, s>>>(dZ, B, W, db);
    return hipGetLastError();
}

hipError_t launch_mlp_adamw(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                            float eps, float wd, float c1, float c2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    adamw_kernel<<<blocks_for(n, 256), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, wd, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_accum(float *acc, const float *v, hipStream_t s) {
    accum_kernel<<<1, 64, 0, s>>>(acc, v);
    return hipGetLastError();
}

}  // namespace gbd
