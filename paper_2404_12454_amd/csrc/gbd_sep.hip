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
// feeds the MFMA U and V of beamlet j0 + l / 16 at the coordinates l % 16 + 16 b
// of its 4 + 4 blocks, 64 MFMAs per step (16 blocks x {Re, Im} x 2 real
// products).  Four wavefronts (2 x 2 tiles) share the factors through LDS, so
// each lane forms 4 phasors per step instead of 8: on gfx950 VALU and MFMA
// issue from one SIMD do not overlap, so every VALU instruction per MFMA is
// time lost from the matrix pipe.  The record fields of a step are loaded
// two steps ahead (the loop is unrolled by two).  Accumulators stay in FP32
// over the segment; segments are summed in FP64 by the reduction.  The host
// sizes segments so that every one is non-empty (jb < je <= N).
//
// Higher-order (elegant Hermite-Gaussian) beamlets without cross terms keep
// the factorisation: their Hermite-Gaussian factor is a product of one
// polynomial in da and one in db, folded into U and V.
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

// A higher-order beamlet's per-axis Hermite-Gaussian factor (no cross
// terms): the factor times c0 + g (c1 + c2 g), g = G d along the axis.
__device__ inline void hg_axis(float df, float gr0, float gi0, float c0r, float c0i, float c1, float c2, float &re,
                               float &im) {
    const float gr = gr0 * df, gi = gi0 * df;
    const float tr = fmaf(c2, gr, c1), ti = c2 * gi;
    const float pr = c0r + (gr * tr - gi * ti), pi = c0i + (gr * ti + gi * tr);
    const float r = re * pr - im * pi;
    im = re * pi + im * pr;
    re = r;
}

// The record fields one lane's factors need; a beamlet index past the
// segment end gets the amplitude exponent -inf (factor 0).  With HG also
// the diagonal of G and the per-axis polynomial coefficients.
struct Fields {
    double arho, brho, p0, p1, p2, p3, p5;
    float m0, m1, m2, m3, m5, arf, brf;
    float mbias;  // 0, or -inf past the segment end (applied when the factor is formed, so the loads
                  // are not waited for before then)
    float gxr, gxi, cx0r, cx0i, cx1, cx2;
    float gyr, gyi, cy0r, cy0i, cy1, cy2;
};
template <bool HG>
__device__ inline Fields load_fields(const Rec32 *__restrict__ rec, const RecHG32 *__restrict__ hg, int64_t j,
                                     int64_t jb, int64_t je) {
    const int64_t jj = j < je ? j : jb;
    const Rec32 *rp = rec + jj;
    Fields f;
    if constexpr (HG) {
        const RecHG32 *h = hg + jj;
        f.gxr = h->g[0][0][0];
        f.gxi = h->g[0][0][1];
        f.cx0r = h->cx0[0];
        f.cx0i = h->cx0[1];
        f.cx1 = h->cx1;
        f.cx2 = h->cx2;
        f.gyr = h->g[1][1][0];
        f.gyi = h->g[1][1][1];
        f.cy0r = h->cy0[0];
        f.cy0i = h->cy0[1];
        f.cy1 = h->cy1;
        f.cy2 = h->cy2;
    }
    f.arho = rp->arho;
    f.brho = rp->brho;
    f.p0 = rp->p[0];
    f.p1 = rp->p[1];
    f.p2 = rp->p[2];
    f.p3 = rp->p[3];
    f.p5 = rp->p[5];
    f.m0 = rp->m[0];
    f.mbias = j < je ? 0.0f : -INFINITY;
    f.m1 = rp->m[1];
    f.m2 = rp->m[2];
    f.m3 = rp->m[3];
    f.m5 = rp->m[5];
    f.arf = rp->arho_f;
    f.brf = rp->brho_f;
    return f;
}

template <int WX, int WY, bool HG>
__global__ void __launch_bounds__(64 * WX * WY) eval_sep_kernel(EvalGeom g, const Rec32 *__restrict__ rec,
                                                                 const RecHG32 *__restrict__ hg,
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

    // Factor sharing: U over this workgroup's x range wx is needed by the two
    // wavefronts (wx, 0), (wx, 1), V over y range wy by (0, wy), (1, wy).
    // Wavefront (wx, wy) forms U blocks 2 wy, 2 wy + 1 of range wx and V blocks
    // 2 wx, 2 wx + 1 of range wy and publishes them in LDS (double-buffered,
    // one barrier per step); each lane's value sits where the same lane of the
    // partner wavefront reads it (same beamlet and in-block position).
    static_assert(WX == 2 && WY == 2, "factor sharing assumes 2 x 2 wavefronts");
    __shared__ float2 lu[2][2][NB][64], lv[2][2][NB][64];  // [buffer][range][block][lane]
    double ax[2], by[2];
    float axf[2], byf[2], mx[2], my[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int ix = x0 + 16 * (2 * wy + h) + li, iy = y0 + 16 * (2 * wx + h) + li;
        mx[h] = ix < g.nx ? 0.0f : -INFINITY;
        my[h] = iy < g.ny ? 0.0f : -INFINITY;
        ax[h] = g.a0 + ix * g.dx;
        by[h] = g.b0 + iy * g.dy;
        axf[h] = (float)ax[h];
        byf[h] = (float)by[h];
    }
    auto publish = [&](const Fields &f, int buf) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            float ur, ui, vr, vi;
            const float dxf = axf[h] - f.arf, dyf = byf[h] - f.brf;
            factor(ax[h] - f.arho, dxf, f.p0, f.p1, f.p3, f.m0 + (f.mbias + mx[h]), f.m1, f.m3, ur, ui);
            factor(by[h] - f.brho, dyf, 0.0, f.p2, f.p5, my[h], f.m2, f.m5, vr, vi);
            if constexpr (HG) {
                hg_axis(dxf, f.gxr, f.gxi, f.cx0r, f.cx0i, f.cx1, f.cx2, ur, ui);
                hg_axis(dyf, f.gyr, f.gyi, f.cy0r, f.cy0i, f.cy1, f.cy2, vr, vi);
            }
            lu[buf][wx][2 * wy + h][lane] = make_float2(ur, ui);
            lv[buf][wy][2 * wx + h][lane] = make_float2(vr, vi);
        }
    };

    // accR/accI[p][q]: rows of the product are y (A operand = V), columns x (B = U)
    f4 accR[NB][NB], accI[NB][NB];
#pragma unroll
    for (int p = 0; p < NB; p++)
#pragma unroll
        for (int q = 0; q < NB; q++) accR[p][q] = accI[p][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};

    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
    // record fields of the steps two and three ahead live in fa / fb in turn
    // (the loop is unrolled by two), so a load is consumed two steps after
    // it is issued and no register copies tie the loads to the current step
    publish(load_fields<HG>(rec, hg, jb + lk, jb, je), 0);
    Fields fa = load_fields<HG>(rec, hg, jb + 4 + lk, jb, je);
    Fields fb = load_fields<HG>(rec, hg, jb + 8 + lk, jb, je);
    __syncthreads();
    int buf = 0;
    auto step = [&](int64_t j0, Fields &f) {
        float ur[NB], ui[NB], vr[NB], vi[NB], vn[NB];
        auto read_step = [&]() {
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const float2 u = lu[buf][wx][b][lane], v = lv[buf][wy][b][lane];
                ur[b] = u.x;
                ui[b] = u.y;
                vr[b] = v.x;
                vi[b] = v.y;
                vn[b] = -v.y;
            }
        };
        // this step's factors (published before the last barrier) are read
        // before the next step's factor arithmetic, so that the LDS latency
        // passes under it; with the higher-order factors the registers this
        // holds would halve the occupancy, so there they are read after it
        if constexpr (!HG) read_step();
        if (j0 + 4 < je) publish(f, buf ^ 1);
        f = load_fields<HG>(rec, hg, j0 + 12 + lk, jb, je);
        if constexpr (HG) read_step();
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
        __syncthreads();
        buf ^= 1;
    };
    for (int64_t j0 = jb; j0 < je; j0 += 8) {
        step(j0, fa);
        if (j0 + 4 < je) step(j0 + 4, fb);
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

hipError_t launch_eval_sep(const EvalGeom &g, const Rec32 *rec, const RecHG32 *hg, float4 *partial, float2 *out,
                           hipStream_t s) {
    const int grid = (g.work + 7) / 8 * 8;
    if (hg)
        eval_sep_kernel<kSepWavesX, kSepWavesY, true>
            <<<grid, 64 * kSepWavesX * kSepWavesY, 0, s>>>(g, rec, hg, partial, out);
    else
        eval_sep_kernel<kSepWavesX, kSepWavesY, false>
            <<<grid, 64 * kSepWavesX * kSepWavesY, 0, s>>>(g, rec, nullptr, partial, out);
    return hipGetLastError();
}

}  // namespace gbd
