// Issue-rate probe: the rates at which one gfx950 CU issues the instruction
// classes the evaluation kernels are made of, measured rather than taken
// from unit counts.  Each thread runs `iters` rounds of 16 independent
// dependency chains of one class (so latency is hidden by the chains and by
// the other wavefronts), over a grid of 8 workgroups of 256 threads per CU;
// the benchmark converts the time into lane-instructions per CU per clock.
//
//   class 0  v_fma_f32          (FP32 multiply-add, unpacked)
//   class 1  v_fma_f64          (FP64 multiply-add)
//   class 2  v_sin_f32          (transcendental unit)
//   class 3  v_exp_f32          (transcendental unit)
//   class 4  v_mfma_f32_16x16x4_f32   (4 chains per wavefront)
//   class 5  v_mfma_f32_16x16x32_f16  (4 chains per wavefront)
//   class 6  v_mfma_f64_16x16x4_f64   (4 chains per wavefront)
//   class 7  v_fmac_f32         (FP32 multiply-add, two-operand encoding)
//   class 8  v_mul_f32          (FP32 multiply)
//   class 9  classes 5 and 0 together: per round 4 v_mfma_f32_16x16x32_f16
//            (4 chains) and 16 v_fma_f32 (16 chains), all independent, so
//            its time against the two classes' shows how far the matrix and
//            vector instructions of one SIMD overlap
#include "../../include/gbd.h"
#include "gbd_internal.h"

namespace gbd {

namespace {

typedef float pf4 __attribute__((ext_vector_type(4)));
typedef double pd4 __attribute__((ext_vector_type(4)));
typedef _Float16 ph8 __attribute__((ext_vector_type(8)));

template <int CLS>
__global__ void __launch_bounds__(256) issue_probe_kernel(int iters, float x, float y, float *__restrict__ sink) {
    float acc = 0.0f;
    if constexpr (CLS == 7 || CLS == 8) {
        // per-thread multiplier and addend in VGPRs: the two-operand forms
        const float b = x + 1e-7f * (float)(threadIdx.x & 7), c = y + 1e-7f * (float)(threadIdx.x & 3);
        float a[16];
#pragma unroll
        for (int k = 0; k < 16; k++) a[k] = x + 0.001f * (k + threadIdx.x);
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int k = 0; k < 16; k++) {
                if constexpr (CLS == 7) a[k] = fmaf(b, c, a[k]);
                if constexpr (CLS == 8) a[k] = a[k] * b;
            }
        }
#pragma unroll
        for (int k = 0; k < 16; k++) acc += a[k];
    } else if constexpr (CLS == 0 || CLS == 2 || CLS == 3) {
        float a[16];
#pragma unroll
        for (int k = 0; k < 16; k++) a[k] = x + 0.001f * (k + threadIdx.x);
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int k = 0; k < 16; k++) {
                if constexpr (CLS == 0) a[k] = fmaf(a[k], x, y);
                if constexpr (CLS == 2) a[k] = __builtin_amdgcn_sinf(a[k]);
                if constexpr (CLS == 3) a[k] = __builtin_amdgcn_exp2f(-a[k]);  // a -> 2^-a stays in (0, 1]
            }
        }
#pragma unroll
        for (int k = 0; k < 16; k++) acc += a[k];
    } else if constexpr (CLS == 1) {
        double a[16];
#pragma unroll
        for (int k = 0; k < 16; k++) a[k] = (double)x + 0.001 * (k + threadIdx.x);
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int k = 0; k < 16; k++) a[k] = fma(a[k], (double)x, (double)y);
        }
#pragma unroll
        for (int k = 0; k < 16; k++) acc += (float)a[k];
    } else if constexpr (CLS == 4) {
        pf4 c[4];
#pragma unroll
        for (int k = 0; k < 4; k++) c[k] = pf4{0.0f, 0.0f, 0.0f, 0.0f};
        const float a = x + 0.001f * threadIdx.x, b = y;
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int k = 0; k < 4; k++) c[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[k], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 4; k++) acc += c[k][0] + c[k][1] + c[k][2] + c[k][3];
    } else if constexpr (CLS == 5) {
        pf4 c[4];
#pragma unroll
        for (int k = 0; k < 4; k++) c[k] = pf4{0.0f, 0.0f, 0.0f, 0.0f};
        ph8 a, b;
#pragma unroll
        for (int t = 0; t < 8; t++) {
            a[t] = (_Float16)(x + 0.001f * t);
            b[t] = (_Float16)y;
        }
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int k = 0; k < 4; k++) c[k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c[k], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 4; k++) acc += c[k][0] + c[k][1] + c[k][2] + c[k][3];
    } else if constexpr (CLS == 9) {
        pf4 c[4];
#pragma unroll
        for (int k = 0; k < 4; k++) c[k] = pf4{0.0f, 0.0f, 0.0f, 0.0f};
        ph8 a, b;
#pragma unroll
        for (int t = 0; t < 8; t++) {
            a[t] = (_Float16)(x + 0.001f * t);
            b[t] = (_Float16)y;
        }
        float v[16];
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = x + 0.001f * (k + threadIdx.x);
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int k = 0; k < 4; k++) c[k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c[k], 0, 0, 0);
#pragma unroll
            for (int k = 0; k < 16; k++) v[k] = fmaf(v[k], x, y);
        }
#pragma unroll
        for (int k = 0; k < 4; k++) acc += c[k][0] + c[k][1] + c[k][2] + c[k][3];
#pragma unroll
        for (int k = 0; k < 16; k++) acc += v[k];
    } else {
        pd4 c[4];
#pragma unroll
        for (int k = 0; k < 4; k++) c[k] = pd4{0.0, 0.0, 0.0, 0.0};
        const double a = (double)x + 0.001 * threadIdx.x, b = (double)y;
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int k = 0; k < 4; k++) c[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[k], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < 4; k++) acc += (float)(c[k][0] + c[k][1] + c[k][2] + c[k][3]);
    }
    // y is 0 at run time: the store never happens, but the compiler cannot know
    if (y > 1e30f) sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace

hipError_t launch_issue_probe(int cls, int blocks, int iters, float *sink, hipStream_t s) {
    switch (cls) {
        case 0: issue_probe_kernel<0><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        case 1: issue_probe_kernel<1><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        case 2: issue_probe_kernel<2><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        case 3: issue_probe_kernel<3><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        case 4: issue_probe_kernel<4><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        case 5: issue_probe_kernel<5><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        case 6: issue_probe_kernel<6><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        case 7: issue_probe_kernel<7><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        case 8: issue_probe_kernel<8><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        case 9: issue_probe_kernel<9><<<blocks, 256, 0, s>>>(iters, 0.999f, 0.0f, sink); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gbd
