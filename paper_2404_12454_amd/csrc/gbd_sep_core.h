// Core of the separable (matrix) form, shared by the single-instance kernel
// and the batched sweep: the MFMA accumulation of one 2 x 2-wavefront pixel
// tile over a range of beamlets (see gbd_sep.hip for the method).
#pragma once

#include "gbd_device.h"

namespace gbd {
namespace sep {

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

// Plane grid of one evaluation.
struct SepGeom {
    int32_t nx, ny;
    double a0, b0, dx, dy;
};

// LDS factor buffers of one workgroup: [buffer][range][block][lane].
template <int NB>
struct SepLds {
    float2 lu[2][2][NB][64], lv[2][2][NB][64];
};

// Accumulates beamlets [jb, je) (je > jb) of rec (and hg) into accR / accI
// for the wavefront's 64 x 64 pixels of workgroup tile (tx, ty).  All
// threads of the workgroup call it together; it leaves the LDS buffers free
// (its last step ends with a barrier).
template <int WX, int WY, bool HG>
__device__ inline void sep_accumulate(const SepGeom &g, const Rec32 *__restrict__ rec,
                                      const RecHG32 *__restrict__ hg, int64_t jb, int64_t je, int tx, int ty,
                                      SepLds<kSepBlocks> &L, f4 (&accR)[kSepBlocks][kSepBlocks],
                                      f4 (&accI)[kSepBlocks][kSepBlocks]) {
    constexpr int NB = kSepBlocks;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wx = wv % WX, wy = wv / WX;
    const int x0 = (tx * WX + wx) * 16 * NB, y0 = (ty * WY + wy) * 16 * NB;
    const int li = lane & 15, lk = lane >> 4;
    auto &lu = L.lu;
    auto &lv = L.lv;

    // Factor sharing: U over this workgroup's x range wx is needed by the two
    // wavefronts (wx, 0), (wx, 1), V over y range wy by (0, wy), (1, wy).
    // Wavefront (wx, wy) forms U blocks 2 wy, 2 wy + 1 of range wx and V blocks
    // 2 wx, 2 wx + 1 of range wy and publishes them in LDS (double-buffered,
    // one barrier per step); each lane's value sits where the same lane of the
    // partner wavefront reads it (same beamlet and in-block position).
    static_assert(WX == 2 && WY == 2, "factor sharing assumes 2 x 2 wavefronts");
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
#pragma unroll
    for (int p = 0; p < NB; p++)
#pragma unroll
        for (int q = 0; q < NB; q++) accR[p][q] = accI[p][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};

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

}

}  // namespace sep
}  // namespace gbd
