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
// Tiling (the core in gbd_sep_core.h): a wavefront owns a 64 x 32 pixel
// tile as 4 x 2 blocks of 16 x 16 and walks its segment of beamlets four at a
// time (the MFMA's K = 4): lane l feeds the MFMA U and V of beamlet j0 + l / 16
// at the coordinates l % 16 + 16 b of its blocks.  The complex product takes
// three real MFMA products (Gauss's form), 24 MFMAs per quad of beamlets.
// Eight wavefronts (2 x 4 tiles, 128 x 128 pixels) share the factors through
// LDS, so each lane forms 2 phasors per quad instead of 6: on gfx950 VALU and
// MFMA issue from one SIMD do not overlap, so every VALU instruction per
// MFMA is time lost from the matrix pipe.  Four quads (eight with
// higher-order factors) pass between barriers, and the record fields are
// loaded two quads ahead.  Accumulators stay in
// FP32 over the segment; segments are summed in FP64 by the reduction.  The
// host sizes segments so that every one is non-empty (jb < je <= N).
//
// Higher-order (elegant Hermite-Gaussian) beamlets without cross terms keep
// the factorisation: their Hermite-Gaussian factor is a product of one
// polynomial in da and one in db, folded into U and V.
#include "gbd_sep_core.h"

namespace gbd {

namespace {

using namespace sep;

template <bool HG>
__global__ void __launch_bounds__(64 * k3WX * k3WY) eval_sep_kernel(EvalGeom g, const Rec32 *__restrict__ rec,
                                                                     const RecHG32 *__restrict__ hg,
                                                                     float2 *__restrict__ partial,
                                                                     float2 *__restrict__ out, StatusPost sp) {
    __shared__ Sep3Lds<HG> L;
    if (sp.post && blockIdx.x == 0 && threadIdx.x == 0) post_status(sp);
    const int w = work_item(blockIdx.x, gridDim.x);
    if (w >= g.work) return;
    const int tiles = g.tiles_x * g.tiles_y;
    const int seg = w / tiles;
    const int t = w - seg * tiles;
    const int ty = t / g.tiles_x, tx = t - ty * g.tiles_x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wx = wv % k3WX, wy = wv / k3WX;
    const int x0 = (tx * k3WX + wx) * 16 * k3BX, y0 = (ty * k3WY + wy) * 16 * k3BY;
    const int li = lane & 15, lk = lane >> 4;
    const SepGeom sg{g.nx, g.ny, g.a0, g.b0, g.dx, g.dy};
    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
    f4 accR[k3BY][k3BX], accI[k3BY][k3BX];
    sep_accumulate_3m<HG>(sg, rec, hg, jb, je, tx, ty, L, accR, accI);

    // D[row][col] of a 16 x 16 block: lane l holds rows 4 (l / 16) + e, column l % 16
    const int64_t M = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int p = 0; p < k3BY; p++)
#pragma unroll
        for (int q = 0; q < k3BX; q++) {
            const int ix = x0 + 16 * q + li;
            if (ix >= g.nx) continue;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int iy = y0 + 16 * p + 4 * lk + e;
                if (iy >= g.ny) continue;
                const int64_t px = (int64_t)iy * g.nx + ix;
                const float2 v = make_float2(accR[p][q][e], accI[p][q][e]);
                if (g.nseg == 1)
                    out[px] = v;
                else
                    partial[(int64_t)seg * M + px] = v;
            }
        }
}

// FP16 halves form (fundamental beamlets): the same stores from tiles of
// T (HTileLarge: 4 x 2 wavefronts of 64 x 64 pixels), the accumulators
// descaled by 2^-scale (exact: a power of two).
template <class T, bool HG>
__global__ void __launch_bounds__(64 * T::WX * T::WY) eval_seph_kernel(EvalGeom g, const Rec32 *__restrict__ rec,
                                                                        const RecHG32 *__restrict__ hg, int scale,
                                                                        float2 *__restrict__ partial,
                                                                        float2 *__restrict__ out, StatusPost sp) {
    __shared__ SepHLdsT<T> L;
    if (sp.post && blockIdx.x == 0 && threadIdx.x == 0) post_status(sp);
    const int w = work_item(blockIdx.x, gridDim.x);
    if (w >= g.work) return;
    const int tiles = g.tiles_x * g.tiles_y;
    const int seg = w / tiles;
    const int t = w - seg * tiles;
    const int ty = t / g.tiles_x, tx = t - ty * g.tiles_x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wx = wv % T::WX, wy = wv / T::WX;
    const int x0 = (tx * T::WX + wx) * 16 * T::BX, y0 = (ty * T::WY + wy) * 16 * T::BY;
    const int li = lane & 15, lk = lane >> 4;
    const SepGeom sg{g.nx, g.ny, g.a0, g.b0, g.dx, g.dy};
    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
    f4 accR[T::BY][T::BX], accI[T::BY][T::BX];
    sep_accumulate_h<T, HG>(sg, rec, hg, jb, je, tx, ty, scale, L, accR, accI);

    const int64_t M = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int p = 0; p < T::BY; p++)
#pragma unroll
        for (int q = 0; q < T::BX; q++) {
            const int ix = x0 + 16 * q + li;
            if (ix >= g.nx) continue;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int iy = y0 + 16 * p + 4 * lk + e;
                if (iy >= g.ny) continue;
                const int64_t px = (int64_t)iy * g.nx + ix;
                const float2 v = make_float2(ldexpf(accR[p][q][e], -scale), ldexpf(accI[p][q][e], -scale));
                if (g.nseg == 1)
                    out[px] = v;
                else
                    partial[(int64_t)seg * M + px] = v;
            }
        }
}

}  // namespace

hipError_t launch_eval_seph(const EvalGeom &g, const Rec32 *rec, const RecHG32 *hg, int scale, float2 *partial,
                            float2 *out, hipStream_t s, hipEvent_t t0, hipEvent_t t1, const StatusPost &sp) {
    using T = HTileLarge;
    static_assert(T::WX == kSepHWavesX && T::WY == kSepHWavesY && 16 * T::BX == kSepHTile && 16 * T::BY == kSepHTile,
                  "FP16 halves tiles: host and kernel disagree");
    const dim3 grid((g.work + 7) / 8 * 8), block(64 * T::WX * T::WY);
    if (hg)
        return launch_timed(eval_seph_kernel<T, true>, grid, block, s, t0, t1, g, rec, hg, scale, partial, out, sp);
    return launch_timed(eval_seph_kernel<T, false>, grid, block, s, t0, t1, g, rec, hg, scale, partial, out, sp);
}

hipError_t launch_eval_sep(const EvalGeom &g, const Rec32 *rec, const RecHG32 *hg, float2 *partial, float2 *out,
                           hipStream_t s, hipEvent_t t0, hipEvent_t t1, const StatusPost &sp) {
    static_assert(k3WX == kSepWavesX && k3WY == kSepWavesY && 16 * k3BX == kSepTileX && 16 * k3BY == kSepTileY,
                  "separable form: host and kernel tiles");
    const dim3 grid((g.work + 7) / 8 * 8), block(64 * k3WX * k3WY);
    if (hg) return launch_timed(eval_sep_kernel<true>, grid, block, s, t0, t1, g, rec, hg, partial, out, sp);
    return launch_timed(eval_sep_kernel<false>, grid, block, s, t0, t1, g, rec, hg, partial, out, sp);
}

}  // namespace gbd
