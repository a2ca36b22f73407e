// Separable (matrix) form of the mixed-precision evaluation.
//
// When no beamlet's phasor on the plane has a cross term (p4 = l4 = 0, as
// for every rotationally symmetric system evaluated on a plane normal to the
// axis: each 2x2 block of its ray-transfer matrix is a multiple of the
// identity, so the complex curvature is too), the coherent sum of the
// sum-of-Gaussians equation factors over the plane's two axes:
//   E(a_i, b_r) = sum_j U_j(a_i) V_j(b_r),
//   U_j(a) = 2^(m0 + m1 da + m3 da^2) e^(2 pi i (p0 + p1 da + p3 da^2)),
//   V_j(b) = 2^(m2 db + m5 db^2)      e^(2 pi i (p2 db + p5 db^2)),
// with da = a - a_rho, db = b - b_rho: a complex matrix product over the
// beamlet index, evaluated here on FP32 MFMA (v_mfma_f32_16x16x4_f32).  Each
// factor is formed like the direct form's phasor (FP64 phase reduced to turns,
// FP32 log2-amplitude from the pixel's own offset, hardware sin/cos/exp2), so
// every beamlet-pixel term is the same product as in the other forms.
//
// Tiling: a wavefront owns a 64 x 64 pixel tile as 4 x 4 blocks of 16 x 16
// and walks its segment of beamlets four at a time (the MFMA's K = 4): lane l
// forms U and V of beamlet j0 + l / 16 at the 4 + 4 coordinates l % 16 + 16 b
// it feeds the MFMA, so the factors cost 8 phasors per lane per 4 beamlets
// against 64 MFMAs (16 blocks x {Re, Im} x 2 real products).  Accumulators
// stay in FP32 over the segment; segments are summed in FP64 by the reduction.
#include "gbd_device.h"

namespace gbd {

namespace {

using namespace dev;

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kSepBlocks = 4;  // 16-pixel blocks per wavefront along each axis

// One factor: 2^(L) e^(2 pi i T), T = c0 + d (c1 + c2 d) in FP64 (turns),
// L = l0 + df (l1 + l2 df) in FP32 from the pixel's own offset.
__device__ inline void factor(double d, float df, double c0, double c1, double c2, float l0, float l1, float l2,
                              float &re, float &im) {
    const double T = c0 + d * (c1 + c2 * d);
    const float ph = (float)__builtin_amdgcn_fract(T);
    const float m = __builtin_amdgcn_exp2f(l0 + df * (l1 + l2 * df));
    re = m * __builtin_amdgcn_cosf(ph);
    im = m * __builtin_amdgcn_sinf(ph);
}

template <int WX, int WY>
__global__ void __launch_bounds__(64 * WX * WY) eval_sep_kernel(EvalGeom g, const Rec32 *__restrict__ rec,
                                                                 float4 *__restrict__ partial,
                                                                 float2 *__restrict__ out) {
    constexpr int NB = kSepBlocks;
    const int w = work_item(blockIdx.x, gridDim.x);
    if (w >= g.work) return;
    const int tiles = g.tiles_x * g.tiles_y;
    const int seg = w / tiles;
    const int t = w - seg * tiles;
    const int ty = t / g.tiles_x, tx = t - ty * g.tiles_x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wx = wv % WX, wy = wv / WX;
    const int x0 = (tx * WX + wx) * 16 * NB, y0 = (ty * WY + wy) * 16 * NB;
    const int li = lane & 15, lk = lane >> 4;

    // plane coordinates this lane evaluates its factors at; a coordinate off
    // the grid gets the amplitude exponent -inf (factor 0), so no branches
    double ax[NB], by[NB];
    float axf[NB], byf[NB], mx[NB], my[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int ix = x0 + 16 * b + li, iy = y0 + 16 * b + li;
        mx[b] = ix < g.nx ? 0.0f : -INFINITY;
        my[b] = iy < g.ny ? 0.0f : -INFINITY;
        ax[b] = g.a0 + ix * g.dx;
        by[b] = g.b0 + iy * g.dy;
        axf[b] = (float)ax[b];
        byf[b] = (float)by[b];
    }

    // accR/accI[p][q]: rows of the product are y (A operand = V), columns x (B = U)
    f4 accR[NB][NB], accI[NB][NB];
#pragma unroll
    for (int p = 0; p < NB; p++)
#pragma unroll
        for (int q = 0; q < NB; q++) accR[p][q] = accI[p][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};

    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
    for (int64_t j0 = jb; j0 < je; j0 += 4) {
        const int64_t j = j0 + lk;
        const Rec32 *rp = rec + (j < je ? j : jb);
        const float dead = j < je ? 0.0f : -INFINITY;  // past the segment end: factor 0
        const double arho = rp->arho, brho = rp->brho;
        const double p0 = rp->p[0], p1 = rp->p[1], p2 = rp->p[2], p3 = rp->p[3], p5 = rp->p[5];
        const float m0 = rp->m[0] + dead, m1 = rp->m[1], m2 = rp->m[2], m3 = rp->m[3], m5 = rp->m[5];
        const float arf = rp->arho_f, brf = rp->brho_f;
        float ur[NB], ui[NB], vr[NB], vi[NB], vn[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) {
            factor(ax[b] - arho, axf[b] - arf, p0, p1, p3, m0 + mx[b], m1, m3, ur[b], ui[b]);
            factor(by[b] - brho, byf[b] - brf, 0.0, p2, p5, my[b], m2, m5, vr[b], vi[b]);
            vn[b] = -vi[b];
        }
        // Re += Vr Ur - Vi Ui ; Im += Vr Ui + Vi Ur
#pragma unroll
        for (int p = 0; p < NB; p++)
#pragma unroll
            for (int q = 0; q < NB; q++) {
                accR[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vr[p], ur[q], accR[p][q], 0, 0, 0);
                accI[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vr[p], ui[q], accI[p][q], 0, 0, 0);
            }
#pragma unroll
        for (int p = 0; p < NB; p++)
#pragma unroll
            for (int q = 0; q < NB; q++) {
                accR[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vn[p], ui[q], accR[p][q], 0, 0, 0);
                accI[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vi[p], ur[q], accI[p][q], 0, 0, 0);
            }
    }

    // D[row][col] of a 16 x 16 block: lane l holds rows 4 (l / 16) + e, column l % 16
    const int64_t M = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int p = 0; p < NB; p++)
#pragma unroll
        for (int q = 0; q < NB; q++) {
            const int ix = x0 + 16 * q + li;
            if (ix >= g.nx) continue;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int iy = y0 + 16 * p + 4 * lk + e;
                if (iy >= g.ny) continue;
                const int64_t px = (int64_t)iy * g.nx + ix;
                if (g.nseg == 1)
                    out[px] = make_float2(accR[p][q][e], accI[p][q][e]);
                else
                    partial[(int64_t)seg * M + px] = make_float4(accR[p][q][e], accI[p][q][e], 0.0f, 0.0f);
            }
        }
}

}  // namespace

hipError_t launch_eval_sep(const EvalGeom &g, const Rec32 *rec, float4 *partial, float2 *out, hipStream_t s) {
    const int grid = (g.work + 7) / 8 * 8;
    eval_sep_kernel<kSepWavesX, kSepWavesY><<<grid, 64 * kSepWavesX * kSepWavesY, 0, s>>>(g, rec, partial, out);
    return hipGetLastError();
}

}  // namespace gbd
