// Separable (matrix) form in FP64: where no beamlet's phasor has a cross
// term the coherent sum factors over the plane's two axes,
//   E(a_i, b_r) = sum_j U_j(a_i) V_j(b_r),
//   U_j(a) = e^(l0 + l1 da + l3 da^2) e^(2 pi i (p0 + p1 da + p3 da^2)),
//   V_j(b) = e^(l2 db + l5 db^2)      e^(2 pi i (p2 db + p5 db^2)),
// a complex matrix product over the beamlet index on FP64 MFMA
// (v_mfma_f64_16x16x4_f64, FP64 products and sums).  Each factor is the FP64
// form's phasor (phase reduced to turns; exp and the turn-phase sine and
// cosine by cexp_turns64, within a few units in the last place of the device
// library's exp and sincospi), so every beamlet-pixel term is the same
// product as in the other FP64 forms up to rounding.  Higher-order beamlets
// without cross terms fold their per-axis Hermite-Gaussian polynomial into U
// and V.
//
// Tiling: a 16 x 16 block of FP64 accumulators takes 8 VGPRs per lane and
// part (Re, Im), so a wavefront owns 64 x 32 pixels (4 x 2 blocks, 128
// accumulator VGPRs) and walks its segment four beamlets per quad (the
// MFMA's K = 4), 32 MFMAs per quad.  Eight wavefronts (2 x 4, a 128 x 128
// pixel workgroup tile, one workgroup per CU) share the factors through
// double-buffered LDS: U over an x range is needed by 4 wavefronts, V over a
// y range by 2, so a lane forms one U and one V factor per quad instead of 6.
// Q quads pass between barriers; a lane forms its factors of the same quad
// of the next pass while a quad's products run, from record fields loaded
// one quad earlier.  Operand layout as in the FP32 form: lane l supplies
// V_{j0 + l/16} at row l % 16 of its block as the A operand and U_{j0 + l/16}
// at column l % 16 as the B operand; unlike the FP32 instruction it holds
// rows l / 16 + 4 e, e = 0..3, column l % 16 of each result block (found by a
// lane-layout probe and fixed by the parity tests).  Segments are summed in
// FP64 by the reduction; the host sizes them so that every one is non-empty.
#include "gbd_device.h"

namespace gbd {

namespace {

using namespace dev;

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kBX = 4, kBY = 2;  // 16-pixel blocks per wavefront along x and y
constexpr int kWX = 2, kWY = 4;  // wavefronts per workgroup along x and y
constexpr int kQ = 4;            // quads of beamlets per pass between barriers

struct Fields64 {
    double arho, brho, p0, p1, p2, p3, p5, l0, l1, l2, l3, l5;
    double lbias;  // 0, or -inf past the segment end (factor 0)
    // higher-order beamlets: G's diagonal and the per-axis polynomials
    double gxr, gxi, cx0r, cx0i, cx1, cx2;
    double gyr, gyi, cy0r, cy0i, cy1, cy2;
};

template <bool HG>
__device__ inline Fields64 load_fields64(const Rec64 *__restrict__ rec, const RecHG64 *__restrict__ hg, int64_t j,
                                         int64_t jb, int64_t je) {
    const int64_t jj = j < je ? j : jb;
    const Rec64 *rp = rec + jj;
    Fields64 f;
    if constexpr (HG) {
        const RecHG64 *h = hg + jj;
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
    f.l0 = rp->l[0];
    f.l1 = rp->l[1];
    f.l2 = rp->l[2];
    f.l3 = rp->l[3];
    f.l5 = rp->l[5];
    f.lbias = j < je ? 0.0 : -INFINITY;
    return f;
}

// The factor times a higher-order beamlet's axis polynomial c0 + g (c1 + c2 g),
// g = G d (no cross terms: G diagonal), FP64.
__device__ inline double2 hg_axis64(double2 u, double d, double gr0, double gi0, double c0r, double c0i, double c1,
                                   double c2) {
    const double gr = gr0 * d, gi = gi0 * d;
    const double tr = fma(c2, gr, c1), ti = c2 * gi;
    const double pr = c0r + (gr * tr - gi * ti), pi = c0i + (gr * ti + gi * tr);
    return make_double2(u.x * pr - u.y * pi, u.x * pi + u.y * pr);
}

// e^(g0 + d (g1 + g2 d)) e^(2 pi i (c0 + d (c1 + c2 d))), FP64
__device__ inline double2 factor64(double d, double c0, double c1, double c2, double g0, double g1, double g2) {
    double T = c0 + d * (c1 + c2 * d);
    T -= rint(T);
    return cexp_turns64(g0 + d * (g1 + g2 * d), T);
}

struct Lds64 {
    double2 lu[2][kQ][kWX][kBX][64], lv[2][kQ][kWY][kBY][64];  // [buffer][quad][range][block][lane]
};

template <bool HG>
__global__ void __launch_bounds__(64 * kWX * kWY) eval_sep64_kernel(EvalGeom g, const Rec64 *__restrict__ rec,
                                                                     const RecHG64 *__restrict__ hg,
                                                                     double2 *__restrict__ partial,
                                                                     double2 *__restrict__ out, StatusPost sp) {
    __shared__ Lds64 L;
    if (sp.post && blockIdx.x == 0 && threadIdx.x == 0) post_status(sp);
    auto &lu = L.lu;
    auto &lv = L.lv;
    const int w = work_item(blockIdx.x, gridDim.x);
    if (w >= g.work) return;
    const int tiles = g.tiles_x * g.tiles_y;
    const int seg = w / tiles;
    const int t = w - seg * tiles;
    const int ty = t / g.tiles_x, tx = t - ty * g.tiles_x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wx = wv % kWX, wy = wv / kWX;
    const int x0 = (tx * kWX + wx) * 16 * kBX, y0 = (ty * kWY + wy) * 16 * kBY;
    const int li = lane & 15, lk = lane >> 4;

    // this wavefront forms U block wy of x range wx and V block wx of y range wy
    const int ix = x0 + 16 * wy + li, iyv = y0 + 16 * wx + li;
    const double ax = g.a0 + ix * g.dx, lx = ix < g.nx ? 0.0 : -INFINITY;
    const double by = g.b0 + iyv * g.dy, ly = iyv < g.ny ? 0.0 : -INFINITY;
    auto publish = [&](const Fields64 &f, int buf, int qd) {
        const double da = ax - f.arho, db = by - f.brho;
        double2 u = factor64(da, f.p0, f.p1, f.p3, f.l0 + (f.lbias + lx), f.l1, f.l3);
        double2 v = factor64(db, 0.0, f.p2, f.p5, ly, f.l2, f.l5);
        if constexpr (HG) {
            u = hg_axis64(u, da, f.gxr, f.gxi, f.cx0r, f.cx0i, f.cx1, f.cx2);
            v = hg_axis64(v, db, f.gyr, f.gyi, f.cy0r, f.cy0i, f.cy1, f.cy2);
        }
        lu[buf][qd][wx][wy][lane] = u;
        lv[buf][qd][wy][wx][lane] = v;
    };

    // accR/accI[p][q]: rows of the product are y (A operand = V), columns x (B = U)
    d4 accR[kBY][kBX], accI[kBY][kBX];
#pragma unroll
    for (int p = 0; p < kBY; p++)
#pragma unroll
        for (int q = 0; q < kBX; q++) accR[p][q] = accI[p][q] = d4{0.0, 0.0, 0.0, 0.0};

    constexpr int P = 4 * kQ;  // beamlets per pass
    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
#pragma unroll
    for (int qd = 0; qd < kQ; qd++) publish(load_fields64<HG>(rec, hg, jb + 4 * qd + lk, jb, je), 0, qd);
    Fields64 fn = load_fields64<HG>(rec, hg, jb + P + lk, jb, je);  // the next pass's first quad
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += P) {
        const bool more = j0 + P < je;
#pragma unroll
        for (int qd = 0; qd < kQ; qd++) {
            double ur[kBX], ui[kBX], vr[kBY], vi[kBY], vn[kBY];
#pragma unroll
            for (int b = 0; b < kBX; b++) {
                const double2 u = lu[buf][qd][wx][b][lane];
                ur[b] = u.x;
                ui[b] = u.y;
            }
#pragma unroll
            for (int b = 0; b < kBY; b++) {
                const double2 v = lv[buf][qd][wy][b][lane];
                vr[b] = v.x;
                vi[b] = v.y;
                vn[b] = -v.y;
            }
            if (more) {
                publish(fn, buf ^ 1, qd);
                fn = load_fields64<HG>(rec, hg, j0 + P + 4 * (qd + 1) + lk, jb, je);
            }
            // Re += Vr Ur - Vi Ui ; Im += Vr Ui + Vi Ur
#pragma unroll
            for (int p = 0; p < kBY; p++)
#pragma unroll
                for (int q = 0; q < kBX; q++) {
                    accR[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(vr[p], ur[q], accR[p][q], 0, 0, 0);
                    accI[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(vr[p], ui[q], accI[p][q], 0, 0, 0);
                }
#pragma unroll
            for (int p = 0; p < kBY; p++)
#pragma unroll
                for (int q = 0; q < kBX; q++) {
                    accR[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(vn[p], ui[q], accR[p][q], 0, 0, 0);
                    accI[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(vi[p], ur[q], accI[p][q], 0, 0, 0);
                }
        }
        __syncthreads();
        buf ^= 1;
    }

    const int64_t M = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int p = 0; p < kBY; p++)
#pragma unroll
        for (int q = 0; q < kBX; q++) {
            const int ixo = x0 + 16 * q + li;
            if (ixo >= g.nx) continue;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int iy = y0 + 16 * p + lk + 4 * e;
                if (iy >= g.ny) continue;
                const int64_t px = (int64_t)iy * g.nx + ixo;
                const double2 v = make_double2(accR[p][q][e], accI[p][q][e]);
                if (g.nseg == 1)
                    out[px] = v;
                else
                    partial[(int64_t)seg * M + px] = v;
            }
        }
}

}  // namespace

hipError_t launch_eval_sep64(const EvalGeom &g, const Rec64 *rec, const RecHG64 *hg, double2 *partial, double2 *out,
                             hipStream_t s, hipEvent_t t0, hipEvent_t t1, const StatusPost &sp) {
    static_assert(kWX == kSep64WavesX && kWY == kSep64WavesY && 16 * kBY == kSepRows64 && 16 * kBX == kSepTileX,
                  "FP64 separable form: host and kernel tiles");
    const dim3 grid((g.work + 7) / 8 * 8), block(64 * kWX * kWY);
    if (hg) return launch_timed(eval_sep64_kernel<true>, grid, block, s, t0, t1, g, rec, hg, partial, out, sp);
    return launch_timed(eval_sep64_kernel<false>, grid, block, s, t0, t1, g, rec, hg, partial, out, sp);
}

}  // namespace gbd
