// Core of the separable (matrix) form, shared by the single-instance kernel
// and the batched sweep: the MFMA accumulation of one workgroup's pixel tile
// (128 x 128 on FP32 MFMA, 256 x 128 in FP16 halves) over a range of
// beamlets (see gbd_sep.hip for the method).
#pragma once

#include <type_traits>

#include "gbd_device.h"

namespace gbd {
namespace sep {

using namespace dev;

typedef float f4 __attribute__((ext_vector_type(4)));

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

// The accumulation in three real products (Gauss's form of the complex
// product).  With U = ur + i ui and V = vr + i vi, the real products
// P1 = vr ur, P2 = vi ui and P3 = (vr + vi)(ur + ui) give Re(V U) = P1 - P2
// and Im(V U) = P3 - P1 - P2: three MFMA products per block and step instead
// of four, the factor sums formed once by the wavefront that publishes the
// factor.  The three sums take 12 accumulator VGPRs per 16 x 16 block, so a
// wavefront owns 64 x 32 pixels (4 x 2 blocks) and a workgroup 2 x 4
// wavefronts (128 x 128 pixels); U over x range wx is needed by the 4
// wavefronts (wx, *), V over y range wy by the 2 wavefronts (*, wy), so each
// lane forms one U and one V factor per quad of beamlets.
constexpr int k3WX = 2, k3WY = 4;  // wavefronts per workgroup along x and y
constexpr int k3BX = 4, k3BY = 2;  // 16-pixel blocks per wavefront along x and y
// Quads of beamlets per pass between barriers, and the LDS slot of a factor:
// fundamental beamlets keep (re, im, re + im, 0) in a float4, four quads per
// pass; higher-order beamlets, whose factors cost more VALU, pay more for
// each barrier and take eight quads per pass in the same 128 KiB, the factor
// as (re, im) with re + im formed by the reader (the same FP32 sum either
// way).  Measured on 51,468 x 512^2: fundamental 0.780 ms (four quads) against
// 0.799 ms (eight), higher-order 1.029 ms against 0.966 ms.
template <bool HG>
struct Sep3Cfg {
    static constexpr int quads = HG ? 8 : 4;
    using slot = typename std::conditional<HG, float2, float4>::type;
};

template <bool HG>
struct Sep3Lds {
    // [buffer][quad][range][block][lane]
    typename Sep3Cfg<HG>::slot lu[2][Sep3Cfg<HG>::quads][k3WX][k3BX][64], lv[2][Sep3Cfg<HG>::quads][k3WY][k3BY][64];
};

// Accumulates beamlets [jb, je) (je > jb) into accR / accI (rows y, columns
// x) for the wavefront's 64 x 32 pixels of workgroup tile (tx, ty); all
// threads of the workgroup call it together; it leaves the LDS buffers free.
// Each pass between barriers takes Q quads of beamlets (Q MFMA K-steps of
// 4, Sep3Cfg), so the barrier and the LDS round trip are paid once per 24 Q
// MFMAs;
// while a quad's products run, the lane forms its factors of the same quad
// of the next pass, whose record fields were loaded two quads earlier.  A
// quad past je publishes zero U factors and adds nothing.
template <bool HG>
__device__ inline void sep_accumulate_3m(const SepGeom &g, const Rec32 *__restrict__ rec,
                                         const RecHG32 *__restrict__ hg, int64_t jb, int64_t je, int tx, int ty,
                                         Sep3Lds<HG> &L, f4 (&accR)[k3BY][k3BX], f4 (&accI)[k3BY][k3BX]) {
    constexpr int Q = Sep3Cfg<HG>::quads;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wx = wv % k3WX, wy = wv / k3WX;
    const int x0 = (tx * k3WX + wx) * 16 * k3BX, y0 = (ty * k3WY + wy) * 16 * k3BY;
    const int li = lane & 15, lk = lane >> 4;
    auto &lu = L.lu;
    auto &lv = L.lv;

    // this wavefront forms U block wy of x range wx and V block wx of y range wy
    const int ix = x0 + 16 * wy + li, iy = y0 + 16 * wx + li;
    const float mx = ix < g.nx ? 0.0f : -INFINITY, my = iy < g.ny ? 0.0f : -INFINITY;
    const double ax = g.a0 + ix * g.dx, by = g.b0 + iy * g.dy;
    const float axf = (float)ax, byf = (float)by;
    auto publish = [&](const Fields &f, int buf, int qd) {
        float ur, ui, vr, vi;
        const float dxf = axf - f.arf, dyf = byf - f.brf;
        factor(ax - f.arho, dxf, f.p0, f.p1, f.p3, f.m0 + (f.mbias + mx), f.m1, f.m3, ur, ui);
        factor(by - f.brho, dyf, 0.0, f.p2, f.p5, my, f.m2, f.m5, vr, vi);
        if constexpr (HG) {
            hg_axis(dxf, f.gxr, f.gxi, f.cx0r, f.cx0i, f.cx1, f.cx2, ur, ui);
            hg_axis(dyf, f.gyr, f.gyi, f.cy0r, f.cy0i, f.cy1, f.cy2, vr, vi);
        }
        if constexpr (HG) {
            lu[buf][qd][wx][wy][lane] = make_float2(ur, ui);
            lv[buf][qd][wy][wx][lane] = make_float2(vr, vi);
        } else {
            lu[buf][qd][wx][wy][lane] = make_float4(ur, ui, ur + ui, 0.0f);
            lv[buf][qd][wy][wx][lane] = make_float4(vr, vi, vr + vi, 0.0f);
        }
    };

    f4 a1[k3BY][k3BX], a2[k3BY][k3BX], a3[k3BY][k3BX];
#pragma unroll
    for (int p = 0; p < k3BY; p++)
#pragma unroll
        for (int q = 0; q < k3BX; q++) a1[p][q] = a2[p][q] = a3[p][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};

    static_assert(Q % 2 == 0, "the two-slot field ring needs an even number of quads per pass");
    constexpr int P = 4 * Q;  // beamlets per pass
#pragma unroll
    for (int qd = 0; qd < Q; qd++) publish(load_fields<HG>(rec, hg, jb + 4 * qd + lk, jb, je), 0, qd);
    // the next pass's first two quads (fn[qd % 2] holds its quad qd)
    Fields fn[2] = {load_fields<HG>(rec, hg, jb + P + lk, jb, je), load_fields<HG>(rec, hg, jb + P + 4 + lk, jb, je)};
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += P) {
        const bool more = j0 + P < je;
#pragma unroll
        for (int qd = 0; qd < Q; qd++) {
            float ur[k3BX], ui[k3BX], us[k3BX], vr[k3BY], vi[k3BY], vs[k3BY];
#pragma unroll
            for (int b = 0; b < k3BX; b++) {
                const auto u = lu[buf][qd][wx][b][lane];
                ur[b] = u.x;
                ui[b] = u.y;
                if constexpr (HG)
                    us[b] = u.x + u.y;
                else
                    us[b] = u.z;
            }
#pragma unroll
            for (int b = 0; b < k3BY; b++) {
                const auto v = lv[buf][qd][wy][b][lane];
                vr[b] = v.x;
                vi[b] = v.y;
                if constexpr (HG)
                    vs[b] = v.x + v.y;
                else
                    vs[b] = v.z;
            }
            if (more) {
                publish(fn[qd % 2], buf ^ 1, qd);
                fn[qd % 2] = load_fields<HG>(rec, hg, j0 + P + 4 * (qd + 2) + lk, jb, je);
            }
#pragma unroll
            for (int p = 0; p < k3BY; p++)
#pragma unroll
                for (int q = 0; q < k3BX; q++) {
                    a1[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vr[p], ur[q], a1[p][q], 0, 0, 0);
                    a2[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vi[p], ui[q], a2[p][q], 0, 0, 0);
                    a3[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(vs[p], us[q], a3[p][q], 0, 0, 0);
                }
        }
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int p = 0; p < k3BY; p++)
#pragma unroll
        for (int q = 0; q < k3BX; q++) {
            accR[p][q] = a1[p][q] - a2[p][q];
            accI[p][q] = a3[p][q] - a1[p][q] - a2[p][q];
        }
}

// ---------------------------------------------------------------------------
// The same contraction on FP16 MFMA (v_mfma_f32_16x16x32_f16: 16 x 16 x 32
// per instruction in a quarter of the issue time of FP32's 16 x 16 x 4).
// Every factor x (FP32) is split into FP16 halves x = hi + lo + r,
// hi = fp16(x), lo = fp16(x - hi), |r| <= 2^-22 |x| for |x| >= 2^-3 (lo
// normal) and |r| <= 2^-25 below; products of halves are exact in FP32, and
//   V U = Vh Uh + Vh Ul + Vl Uh  (+ Vl Ul, at most 2^-22 |V U|, left out)
// so a term carries the two splits' errors and the dropped product:
// within 2^-20.4 of itself.
//
// K layout: the 32 K slots of one instruction are 16 beamlets x (re, im):
// lane group l / 16 supplies beamlets 4 (l / 16) ... + 3 of a pass of 16,
// two slots each, so every operand register holds one beamlet's packed
// (re, im) pair and no value appears twice in an operand:
//   B_h = (Ur_h, Ui_h), B_l = (Ur_l, Ui_l)                     (U, columns)
//   A_h = (Vr_h, -Vi_h), A_l = (Vr_l, -Vi_l)  ->  Re: A B = Vr Ur - Vi Ui
//   W_h = (Vi_h, Vr_h),  W_l = (Vi_l, Vr_l)   ->  Im: W B = Vi Ur + Vr Ui
// and a pass of 16 beamlets takes 3 instructions (hh, hl, lh) per sum and
// block, 8 accumulator VGPRs per block.  The factors are formed, split and
// packed once, by the lane that publishes them to LDS; the readers load
// each operand with one 16-byte read.
//
// FP16's range (largest 65504, spacing 2^-24 below 2^-14) is met by scaling:
// beamlet j's U by 2^(E - u_j), its V by 2^(scale - E + u_j) (E =
// kSepHalfExp, u_j its U modulus bound over the grid, 2^scale the common
// factor), so every factor is below 2^E and a term's error stays below
// 2^-20 of itself or 2^-38 of the largest term, whichever is larger.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// (re, im) as two packed FP16 pairs: hi = (fp16(re), fp16(im)), lo the
// rounded remainders (round to nearest even throughout)
__device__ inline void split_halves(float re, float im, uint32_t &hi, uint32_t &lo) {
    // re and im as the FP32 values they are (not re-formed from the product
    // that made them, which could round hi differently in its two uses)
    asm("" : "+v"(re), "+v"(im));
    hi = __builtin_bit_cast(uint32_t, h2{(_Float16)re, (_Float16)im});
    // lo = fp16(x - hi) in one mixed-precision fused multiply-add per half
    // (FP32 x, FP16 hi from the packed pair, one rounding to FP16): the low
    // half of lo from re and hi's low half, its high half from im and hi's
    // high half (op_sel picks the half, op_sel_hi marks the FP16 source)
    asm("v_fma_mixlo_f16 %0, %1, 1.0, -%2 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %0, %3, 1.0, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "=&v"(lo)
        : "v"(re), "v"(hi), "v"(im));
}

// split_halves of (re, -im): the conjugate's halves, the negation folded
// into the conversions' source modifiers
__device__ inline void split_halves_conj(float re, float im, uint32_t &hi, uint32_t &lo) {
    asm("" : "+v"(re), "+v"(im));
    hi = __builtin_bit_cast(uint32_t, h2{(_Float16)re, (_Float16)(-im)});
    asm("v_fma_mixlo_f16 %0, %1, 1.0, -%2 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %0, -%3, 1.0, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "=&v"(lo)
        : "v"(re), "v"(hi), "v"(im));
}

// (a, b) -> (-b, a) of a packed FP16 pair, exactly (a product by 1.0 whose
// low result takes the negated high half and high result the low half;
// FP16 denormals are kept)
__device__ inline uint32_t rot_halves(uint32_t v) {
    uint32_t w;
    asm("v_pk_mul_f16 %0, %1, 1.0 op_sel:[1,0] op_sel_hi:[0,0] neg_lo:[1,0]" : "=v"(w) : "v"(v));
    return w;
}

// Workgroup tiles: WX x WY wavefronts of BX x BY 16 x 16 blocks.  In the
// FP16 halves form a lane forms, per quad of beamlets, UB = BX / WY factors
// U (its wavefront shares its x range with WY - 1 others) and VB = BY / WX
// factors V.
//   HTileLarge (the FP16 halves form, single evaluations and the batched
//     sweep): 4 x 2 wavefronts of 64 x 64 pixels (256 x 128 per workgroup,
//     133 KiB of LDS); per lane and quad 2 U + 1 V beside the products of 4
//     blocks.  The k3 layout (2 x 4 of 64 x 32, 1 U + 1 V beside 2 blocks)
//     took a third more factor arithmetic per pair in this form (0.442
//     against 0.339 ms on 51,468 beamlets x 512^2 pixels); the FP32 form
//     keeps it (Sep3Tile).
template <int WX_, int WY_, int BX_, int BY_>
struct HTile {
    static constexpr int WX = WX_, WY = WY_, BX = BX_, BY = BY_;
    static constexpr int UB = BX / WY, VB = BY / WX;
    static_assert(BX % WY == 0 && BY % WX == 0 && BX * BY % 4 == 0, "FP16 halves tile");
};
using HTileLarge = HTile<4, 2, 4, 4>;
using Sep3Tile = HTile<k3WX, k3WY, k3BX, k3BY>;  // the FP32 form's workgroup (dimensions only)

// LDS per buffer: U (hi, lo) and V (A_h, A_l, W_h, W_l) words of one pass of
// 16 beamlets, double-buffered so the next pass's factors are written while
// this pass's products run.  A pixel's 16 beamlets fill a row of 16 words
// as 4 groups of 4 (one 16-byte operand each), the groups of row r stored
// in the order g ^ swz(r), swz(r) = ((r >> 1) & 3) ^ ((r >> 3) & 1).  Then
// the 16 lanes of a lane group (rows 0 ... 15, one group each) read from 16
// distinct 4-bank groups of a 64-bank LDS, and any 8 consecutive lanes from
// 8 distinct ones of a 32-bank one; a wavefront's 64 single-word writes
// (row l % 16, word l / 16 of one group) hit 64 distinct banks of 64.
__device__ inline int swz(int r) { return ((r >> 1) & 3) ^ ((r >> 3) & 1); }

// Records staged in LDS a pass ahead: the 22 words of a Rec32 that the
// factors need, 24 to a record (6 16-byte reads), 16 records a pass.
constexpr int kStageWords = 24, kStageUsed = 22;
// staged word w holds Rec32 word kStageSrc[w]:
//   0-7  arho, p0, p1, p3 (FP64, U)    8-13  brho, p2, p5 (FP64, V)
//   14-16 m0, m1, m3 (U)   17-18 m2, m5 (V)   19-20 arho_f, brho_f   21 pad (the U bound)
__device__ constexpr int kStageSrc[kStageUsed] = {0, 1, 4, 5, 6, 7, 10, 11, 2, 3, 8, 9, 14, 15,
                                                  16, 17, 19, 18, 21, 22, 23, 27};
static_assert(sizeof(Rec32) == 60 * 4 && kStageWords % 4 == 0, "staged record layout");
// A record past the segment's end is staged as m0 = -inf (staged word
// kStagedM0), its U bound u = -1e30 (kStagedU) and zeros in its other words:
// its U factors 2^(m0 + 14 - u) and V factors 2^(scale - 14 + u) are both
// exactly zero (a finite V there could leave FP16's range, and 0 x inf is NaN).
constexpr int kStagedM0 = 14, kStagedU = 21;
constexpr uint32_t kPadU = 0xf149f2cau;  // -1e30f
static_assert(kStageSrc[kStagedM0] == offsetof(Rec32, m) / 4, "staged m0 word");
static_assert(kStageSrc[kStagedU] == offsetof(Rec32, pad) / 4, "staged U bound word");
// Higher-order beamlets: 12 words of each RecHG32 (the diagonal of G and the
// per-axis polynomial coefficients), staged beside the record words by the
// first 16 x 12 threads: staged word w holds RecHG32 word kStageSrcHG[w]:
//   0-5 g_xx (re, im), cx0 (re, im), cx1, cx2     6-11 g_yy, cy0, cy1, cy2
constexpr int kStageHG = 12;
__device__ constexpr int kStageSrcHG[kStageHG] = {0, 1, 8, 9, 12, 13, 6, 7, 10, 11, 14, 15};
static_assert(sizeof(RecHG32) == 24 * 4, "staged higher-order record layout");

template <class T>
struct SepHLdsT {
    // [buffer][range][block][part][pixel in block][beamlet in pass, swizzled]
    uint32_t lu[2][T::WX][T::BX][2][16][16];
    uint32_t lv[2][T::WY][T::BY][4][16][16];
    // [buffer][beamlet in pass][staged word]; rows 16 ... take the idle
    // threads' words (every thread stores: a guarded store would let the
    // compiler sink the load into the guard, next to the store)
    static constexpr int kRows = (64 * T::WX * T::WY + kStageUsed - 1) / kStageUsed;
    uint32_t rs[2][kRows][kStageWords];
    // higher-order words, [buffer][beamlet in pass][staged word] likewise
    static constexpr int kRowsHG = (64 * T::WX * T::WY + kStageHG - 1) / kStageHG;
    uint32_t rh[2][kRowsHG][kStageHG];
};
static_assert(sizeof(SepHLdsT<HTileLarge>) <= 163840, "the large tile's LDS exceeds a workgroup's 160 KiB");
static_assert(64 * HTileLarge::WX * HTileLarge::WY >= 16 * kStageUsed,
              "a workgroup stages a pass's records one word per thread");

__device__ inline h8 operand(const uint32_t *p) { return __builtin_bit_cast(h8, *reinterpret_cast<const uint4 *>(p)); }

// As sep_accumulate_3m (segment walk) in FP16 halves, tile T; accR / accI
// hold the field times 2^scale.  HG: higher-order beamlets without cross
// terms, each factor times its axis polynomial (hg_axis, as in the FP32
// form) before the split.  The hi x hi,
// hi x lo and lo x hi products of every block in that order each pass (lo
// x lo, at most 2^-22 of a term, is left out).  The record words reach LDS
// two passes before their factors are used: during pass p each thread loads
// one word of pass p + 2's records and writes it before the pass's barrier,
// and the factors of pass p + 1, formed during pass p, read pass p + 1's.
// Every pass forms the next one's factors, the last one too (past the end:
// zero factors nobody reads), so the loop body has no branch.
template <class T, bool HG = false>
__device__ inline void sep_accumulate_h(const SepGeom &g, const Rec32 *__restrict__ rec,
                                        const RecHG32 *__restrict__ hg, int64_t jb, int64_t je, int tx, int ty,
                                        int scale, SepHLdsT<T> &L, f4 (&accR)[T::BY][T::BX],
                                        f4 (&accI)[T::BY][T::BX]) {
    constexpr int WX = T::WX, WY = T::WY, BX = T::BX, BY = T::BY, UB = T::UB, VB = T::VB;
    constexpr int Q = 4;                 // quads of beamlets per pass (one pass of 16 between barriers)
    constexpr int PERQ = BX * BY / Q;    // blocks whose products run beside one quad's factors
    constexpr int P = 4 * Q;             // beamlets per pass
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wx = wv % WX, wy = wv / WX;
    const int x0 = (tx * WX + wx) * 16 * BX, y0 = (ty * WY + wy) * 16 * BY;
    const int li = lane & 15, lk = lane >> 4;
    const int sw = swz(li);
    auto &lu = L.lu;
    auto &lv = L.lv;
    auto &rs = L.rs;
    auto &rh = L.rh;

    // this wavefront forms U blocks wy UB ... + UB - 1 of x range wx and V
    // blocks wx VB ... + VB - 1 of y range wy (unmasked past the grid's edge,
    // as in sep_accumulate_3m; there the factors may even leave FP16's range,
    // which reaches only outputs that are not stored)
    double ax[UB], by[VB];
    float axf[UB], byf[VB];
#pragma unroll
    for (int u = 0; u < UB; u++) {
        const int ix = x0 + 16 * (wy * UB + u) + li;
        ax[u] = g.a0 + ix * g.dx;
        axf[u] = (float)ax[u];
    }
#pragma unroll
    for (int v = 0; v < VB; v++) {
        const int iy = y0 + 16 * (wx * VB + v) + li;
        by[v] = g.b0 + iy * g.dy;
        byf[v] = (float)by[v];
    }
    const float E = (float)kSepHalfExp, sc = (float)scale;
    const Rec32 *__restrict__ srec = rec + jb;
    const RecHG32 *__restrict__ shg = HG ? hg + jb : nullptr;
    const int n = (int)(je - jb);

    // staging: thread t moves word kStageSrc[t % 22] of record t / 22 (the
    // threads past 16 x 22 load words of later records, clamped, and store
    // them into rows nobody reads); past the segment's end it stores the pad
    // word instead (m0 = -inf, u = -1e30, else 0), which zeroes that
    // beamlet's U and V factors
    const int st = threadIdx.x, sr = st / kStageUsed, sc_w = st - sr * kStageUsed, sw_src = kStageSrc[sc_w];
    const uint32_t pad_w = sc_w == kStagedM0 ? 0xff800000u : sc_w == kStagedU ? kPadU : 0u;
    // and, for higher-order beamlets, word kStageSrcHG[t % 12] of record t / 12
    const int hr = st / kStageHG, hc = st - hr * kStageHG, hw_src = HG ? kStageSrcHG[hc] : 0;
    struct Staged {
        uint32_t w, h;
    };
    auto stage_load = [&](int i0) {  // words of the pass starting at beamlet i0
        const int i = i0 + sr;
        Staged v;
        const uint32_t w = reinterpret_cast<const uint32_t *>(srec + (i < n ? i : 0))[sw_src];
        // the word masked and the pad merged by bit operations, so the load
        // stays unconditional (a select on it becomes a branch in the loop)
        const uint32_t keep = 0u - (uint32_t)(i < n);
        v.w = (w & keep) | (pad_w & ~keep);
        v.h = 0u;
        if constexpr (HG) {
            const int ih = i0 + hr;
            v.h = reinterpret_cast<const uint32_t *>(shg + (ih < n ? ih : 0))[hw_src];
        }
        return v;
    };
    auto stage_store = [&](int sbuf, const Staged &v) {
        rs[sbuf][sr][sc_w] = v.w;
        if constexpr (HG) rh[sbuf][hr][hc] = v.h;
    };

    // quad qd of a pass: beamlet b = 4 qd + lk, the pass's records in rs[sbuf]
    auto publish = [&](int sbuf, int i0, int buf, int qd) {
        const int b = 4 * qd + lk;
        const uint32_t *r = rs[sbuf][b];
        uint4 w[6];
#pragma unroll
        for (int k = 0; k < 6; k++) w[k] = reinterpret_cast<const uint4 *>(r)[k];
        auto f64 = [&](int k) {
            const uint4 &q = w[k >> 2];
            const uint32_t lo = (k & 3) == 0 ? q.x : q.z, hi = (k & 3) == 0 ? q.y : q.w;
            return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
        };
        auto f32 = [&](int k) {
            const uint4 &q = w[k >> 2];
            const uint32_t v = (k & 3) == 0 ? q.x : (k & 3) == 1 ? q.y : (k & 3) == 2 ? q.z : q.w;
            return __builtin_bit_cast(float, v);
        };
        const double arho = f64(0), p0 = f64(2), p1 = f64(4), p3 = f64(6);
        const double brho = f64(8), p2 = f64(10), p5 = f64(12);
        const float m0 = f32(14), m1 = f32(15), m3 = f32(16), m2 = f32(17), m5 = f32(18);
        const float arf = f32(19), brf = f32(20), u = f32(21);
        // (a beamlet past the segment's end was staged with m0 = -inf)
        const float lu0 = m0 + (E - u), lv0 = (sc - E) + u;
        const int col = 4 * (qd ^ sw) + lk;
        float hx[6], hy[6];
        if constexpr (HG) {
            const uint4 *hq = reinterpret_cast<const uint4 *>(rh[sbuf][b]);
            const uint4 q0 = hq[0], q1 = hq[1], q2 = hq[2];
            const uint32_t hw[12] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
#pragma unroll
            for (int k = 0; k < 6; k++) {
                hx[k] = __builtin_bit_cast(float, hw[k]);
                hy[k] = __builtin_bit_cast(float, hw[6 + k]);
            }
        }
#pragma unroll
        for (int k = 0; k < UB; k++) {
            float ur, ui;
            factor(ax[k] - arho, axf[k] - arf, p0, p1, p3, lu0, m1, m3, ur, ui);
            if constexpr (HG) hg_axis(axf[k] - arf, hx[0], hx[1], hx[2], hx[3], hx[4], hx[5], ur, ui);
            uint32_t uh, ul;
            split_halves(ur, ui, uh, ul);
            lu[buf][wx][wy * UB + k][0][li][col] = uh;
            lu[buf][wx][wy * UB + k][1][li][col] = ul;
        }
#pragma unroll
        for (int k = 0; k < VB; k++) {
            float vr, vi;
            factor(by[k] - brho, byf[k] - brf, 0.0, p2, p5, lv0, m2, m5, vr, vi);
            if constexpr (HG) hg_axis(byf[k] - brf, hy[0], hy[1], hy[2], hy[3], hy[4], hy[5], vr, vi);
            // A = (Vr, -Vi) halves; W = (Vi, Vr) = rot_halves(A)
            uint32_t ah, al;
            split_halves_conj(vr, vi, ah, al);
            const int blk = wx * VB + k;
            lv[buf][wy][blk][0][li][col] = ah;
            lv[buf][wy][blk][1][li][col] = al;
            lv[buf][wy][blk][2][li][col] = rot_halves(ah);
            lv[buf][wy][blk][3][li][col] = rot_halves(al);
        }
    };

#pragma unroll
    for (int p = 0; p < BY; p++)
#pragma unroll
        for (int q = 0; q < BX; q++) accR[p][q] = accI[p][q] = f4{0.0f, 0.0f, 0.0f, 0.0f};

    // passes 0 and 1's records, then pass 0's factors
    {
        const Staged w0 = stage_load(0), w1 = stage_load(P);
        stage_store(0, w0);
        stage_store(1, w1);
    }
    __syncthreads();
#pragma unroll
    for (int qd = 0; qd < Q; qd++) publish(0, 0, 0, qd);
    __syncthreads();
    const int rd = 4 * (lk ^ sw);  // this lane's operand group in a row
    int buf = 0;
    for (int i0 = 0; i0 < n; i0 += P) {
        // pass p = i0 / P: factors in buf, records of pass p + 1 in rs[buf ^ 1]
        const Staged wnext = stage_load(i0 + 2 * P);
        // keep the load here, a pass before its use (the scheduler would
        // otherwise sink it to the store and wait on it there)
        __builtin_amdgcn_sched_barrier(0);
        h8 bh[BX], bl[BX];
#pragma unroll
        for (int q = 0; q < BX; q++) {
            bh[q] = operand(&lu[buf][wx][q][0][li][rd]);
            bl[q] = operand(&lu[buf][wx][q][1][li][rd]);
        }
        h8 ah, al, wh, wl;
        // the next pass's quads, formed between this pass's products
#pragma unroll
        for (int k = 0; k < Q; k++) {
            publish(buf ^ 1, i0 + P, buf ^ 1, k);
            // blocks PERQ k ... + PERQ - 1 in row-major order; a block row's
            // V operands are read at its first block
#pragma unroll
            for (int i = 0; i < PERQ; i++) {
                const int m = PERQ * k + i, p = m / BX, q = m % BX;
                if (q == 0 || i == 0) {
                    ah = operand(&lv[buf][wy][p][0][li][rd]);
                    al = operand(&lv[buf][wy][p][1][li][rd]);
                    wh = operand(&lv[buf][wy][p][2][li][rd]);
                    wl = operand(&lv[buf][wy][p][3][li][rd]);
                }
                accR[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[q], accR[p][q], 0, 0, 0);
                accI[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wh, bh[q], accI[p][q], 0, 0, 0);
                accR[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[q], accR[p][q], 0, 0, 0);
                accI[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wh, bl[q], accI[p][q], 0, 0, 0);
                accR[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[q], accR[p][q], 0, 0, 0);
                accI[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wl, bh[q], accI[p][q], 0, 0, 0);
            }
        }
        // pass p + 2's records into the buffer pass p - 1 read
        stage_store(buf, wnext);
        __syncthreads();
        buf ^= 1;
    }
}

}  // namespace sep
}  // namespace gbd
