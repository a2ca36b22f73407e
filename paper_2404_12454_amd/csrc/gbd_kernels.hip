// gfx950 kernels of plane-evaluation Gaussian beamlet decomposition,
// single-instance form.
//
//  setup_kernel   O(N), FP64: one beamlet per lane.  Complex-curvature law and
//                 eigenvalue-branch amplitude (Sec. 4.1 Gaussian solution,
//                 Appendix C closed-form 2x2 algebra), base ray (Appendix A
//                 ab/cd laws), hit point on the detector plane, misalignment
//                 phase (Appendix A tilt-phase equation in completed-square
//                 form), and the per-beamlet phasor coefficients on the plane.
//  eval_*_kernel  O(N M): every pixel sums every beamlet's phasor (Sec. 1
//                 sum-of-Gaussians equation evaluated with the Sec. 3
//                 plane-evaluation expression).  A transcendental-bound VALU
//                 workload (no contraction, so no MFMA).
//  reduce_kernel  fixed-order sum of the per-segment partial fields.
#include "gbd_device.h"

namespace gbd {

namespace {

using namespace dev;

__global__ void __launch_bounds__(256) setup_kernel(BeamletsDev b, PlaneGeom pl, double gturns,
                                                    Rec64 *__restrict__ r64, Rec32 *__restrict__ r32,
                                                    RecHG64 *__restrict__ h64, RecHG32 *__restrict__ h32,
                                                    RecCut64 *__restrict__ c64, RecCut32 *__restrict__ c32,
                                                    uint32_t *__restrict__ status,
                                                    uint32_t *__restrict__ status_next) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) {  // the next setup's flag and peak words (not used by this one)
        status_next[0] = 0u;
        status_next[1] = 0u;
    }
    float peak = -INFINITY;
    uint32_t flag = 0;
    if (j < b.n) flag = setup_one(b, pl, gturns, j, r64, r32, h64, h32, c64, c32, false, &peak);
    // status[0]: the flags OR-ed; status[1]: the largest term modulus of any
    // beamlet over the grid, as ceil(log2) + 2048 clamped to [1, 4095] (0:
    // none).  One atomic of each per workgroup: the words are shared by the
    // whole grid, so per-lane atomics serialise (an informational flag such as
    // FLAG_STEEP is set by most beamlets)
    uint32_t key = isfinite(peak) ? (uint32_t)fminf(fmaxf(ceilf(peak) + 2048.0f, 1.0f), 4095.0f) : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        key = max(key, (uint32_t)__shfl_xor((int)key, o));
        flag |= (uint32_t)__shfl_xor((int)flag, o);
    }
    __shared__ uint32_t wflag[4], wkey[4];
    if ((threadIdx.x & 63) == 0) {
        wflag[threadIdx.x >> 6] = flag;
        wkey[threadIdx.x >> 6] = key;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t f = 0, k = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) {
            f |= wflag[w];
            k = max(k, wkey[w]);
        }
        if (f) atomicOr(status, f);
        if (k) atomicMax(status + 1, k);
    }
}

// The setup's status words and a sequence number posted to the host by a
// kernel of their own (post_status).
__global__ void __launch_bounds__(64) status_post_kernel(StatusPost sp) {
    if (threadIdx.x == 0) post_status(sp);
}

// The rotor forms' sigma^(k^2) tables, k = 1..16, from the FP64 records on
// rows dy apart: FP64 (q64) or rounded into the Rec32 records (r32).  Thread
// t of a block computes entry t % 16 of beamlet 16 (block) + t / 16, so each
// beamlet's table is written contiguously.
__global__ void __launch_bounds__(256) sigma_kernel(int64_t n, double dy, const Rec64 *__restrict__ rec,
                                                    RecSq64 *__restrict__ q64, Rec32 *__restrict__ r32) {
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const int k = (threadIdx.x & 15) + 1;
    if (j >= n) return;
    const double2 v = rotor_sigma(rec[j].p[5], rec[j].l[5], dy, k);
    if (q64) {
        q64[j].sq[k - 1][0] = v.x;
        q64[j].sq[k - 1][1] = v.y;
    } else {
        r32[j].sq[k - 1][0] = (float)v.x;
        r32[j].sq[k - 1][1] = (float)v.y;
    }
}

// Mixed form.  Each lane owns ROWS pixels of one detector column; a
// wavefront spans 64 consecutive columns (coalesced stores); WAVES
// wavefronts stack in y; the workgroup sums one segment of beamlets.
// FORM: 0 direct, 1 stepped, 2 rotor accumulation; HG (direct and rotor
// forms): higher-order beamlets, records hg.
template <int ROWS, int WAVES, int FORM, bool HG = false>
__global__ void __launch_bounds__(64 * WAVES) eval_mixed_kernel(EvalGeom g, const Rec32 *__restrict__ rec,
                                                                float4 *__restrict__ partial,
                                                                float2 *__restrict__ out,
                                                                const RecHG32 *__restrict__ hg = nullptr) {
    static_assert(!HG || FORM == 0 || FORM == 2, "higher-order beamlets: direct or rotor form");
    __shared__ Rec32 tile[kMixedTile];
    __shared__ RecHG32 htile[HG ? kMixedTile : 1];
    const int w = work_item(blockIdx.x, gridDim.x);
    if (w >= g.work) return;
    const int tiles = g.tiles_x * g.tiles_y;
    const int seg = w / tiles;
    const int t = w - seg * tiles;
    const int ty = t / g.tiles_x, tx = t - ty * g.tiles_x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ix = tx * 64 + lane;
    const int iy0 = (ty * WAVES + wv) * ROWS;
    const double a = g.a0 + ix * g.dx;
    const double b0 = g.b0 + iy0 * g.dy;

    float s_re[ROWS], s_im[ROWS], c_re[ROWS], c_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) s_re[k] = s_im[k] = c_re[k] = c_im[k] = 0.0f;
    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
    if constexpr (FORM == 2)
        mixed_accumulate_rotor<ROWS, 64 * WAVES, HG>(tile, rec, jb, je, a, b0, g.dy, s_re, s_im, c_re, c_im, htile,
                                                     hg);
    else if constexpr (FORM == 1)
        mixed_accumulate_step<ROWS, 64 * WAVES>(tile, rec, jb, je, a, b0, g.dy, s_re, s_im, c_re, c_im);
    else
        mixed_accumulate<ROWS, 64 * WAVES, HG>(tile, rec, jb, je, a, b0, g.dy, s_re, s_im, c_re, c_im, htile, hg);

    if (ix >= g.nx) return;
    const int64_t M = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int k = 0; k < ROWS; k++) {
        const int iy = iy0 + k;
        if (iy < g.ny) {
            const int64_t p = (int64_t)iy * g.nx + ix;
            if (g.nseg == 1)
                out[p] = make_float2(s_re[k] - c_re[k], s_im[k] - c_im[k]);
            else
                partial[(int64_t)seg * M + p] = make_float4(s_re[k], s_im[k], c_re[k], c_im[k]);
        }
    }
}

// FP64 form: the same phasor in FP64 throughout (sincospi and exp from the
// device math library), plain FP64 accumulation; HG: times each beamlet's
// Hermite-Gaussian factor.
template <int ROWS, int WAVES, bool HG = false>
__global__ void __launch_bounds__(64 * WAVES) eval_fp64_kernel(EvalGeom g, const Rec64 *__restrict__ rec,
                                                               double2 *__restrict__ partial,
                                                               double2 *__restrict__ out,
                                                               const RecHG64 *__restrict__ hg = nullptr) {
    constexpr int CH = 64;  // records per LDS tile (8 KiB, and 12 KiB of factors)
    __shared__ Rec64 tile[CH];
    __shared__ RecHG64 htile[HG ? CH : 1];
    const int w = work_item(blockIdx.x, gridDim.x);
    if (w >= g.work) return;
    const int tiles = g.tiles_x * g.tiles_y;
    const int seg = w / tiles;
    const int t = w - seg * tiles;
    const int ty = t / g.tiles_x, tx = t - ty * g.tiles_x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ix = tx * 64 + lane;
    const int iy0 = (ty * WAVES + wv) * ROWS;
    const double a = g.a0 + ix * g.dx;
    const double b0 = g.b0 + iy0 * g.dy;
    const double dy = g.dy, dy2 = g.dy * g.dy;

    double acc_re[ROWS], acc_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) acc_re[k] = acc_im[k] = 0.0;

    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
    for (int64_t j0 = jb; j0 < je; j0 += CH) {
        const int cnt = (int)min((int64_t)CH, je - j0);
        __syncthreads();
        {
            const double2 *src = reinterpret_cast<const double2 *>(rec + j0);
            double2 *dst = reinterpret_cast<double2 *>(tile);
            for (int i = threadIdx.x; i < cnt * 8; i += 64 * WAVES) dst[i] = src[i];
            if constexpr (HG) {
                const double2 *hs = reinterpret_cast<const double2 *>(hg + j0);
                double2 *hd = reinterpret_cast<double2 *>(htile);
                for (int i = threadIdx.x; i < cnt * (int)(sizeof(RecHG64) / 16); i += 64 * WAVES) hd[i] = hs[i];
            }
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; jj++) {
            const Rec64 &r = tile[jj];
            const double da = a - r.arho, db = b0 - r.brho;
            const double q = r.p[2] + r.p[4] * da;
            const double T0 = r.p[0] + da * (r.p[1] + r.p[3] * da) + db * (q + r.p[5] * db);
            const double T1 = dy * (q + 2.0 * r.p[5] * db);
            const double T2 = r.p[5] * dy2;
            const double ql = r.l[2] + r.l[4] * da;
            const double Vc = r.l[0] + da * (r.l[1] + r.l[3] * da);
#pragma unroll
            for (int k = 0; k < ROWS; k++) {
                const double th = T0 + (double)k * (T1 + (double)k * T2);
                const double rr = th - rint(th);
                double s, c;
                sincospi(2.0 * rr, &s, &c);
                const double dbk = fma((double)k, dy, db);
                const double m = exp(Vc + dbk * (ql + r.l[5] * dbk));
                if constexpr (HG) {
                    const cd P = hg_factor(htile[jj], da, dbk);
                    const double er = m * c, ei = m * s;
                    acc_re[k] += er * P.re - ei * P.im;
                    acc_im[k] += er * P.im + ei * P.re;
                } else {
                    acc_re[k] = fma(m, c, acc_re[k]);
                    acc_im[k] = fma(m, s, acc_im[k]);
                }
            }
        }
    }
    if (ix >= g.nx) return;
    const int64_t M = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int k = 0; k < ROWS; k++) {
        const int iy = iy0 + k;
        if (iy < g.ny) {
            const int64_t p = (int64_t)iy * g.nx + ix;
            const double2 v = make_double2(acc_re[k], acc_im[k]);
            if (g.nseg == 1)
                out[p] = v;
            else
                partial[(int64_t)seg * M + p] = v;
        }
    }
}

// FP64 rotor form: the mixed rotor recurrence E(h + k) = E(h) rho^k sigma^(k^2)
// in FP64 throughout (anchor at the lane's middle row h from the FP64 phase
// and ln-amplitude quadratics, rho and 1/rho from the row slopes, sigma^(k^2)
// from the FP64 table sigma_kernel fills), so a further row costs two complex
// FP64 multiply-adds instead of an exp and a sincospi (the anchor's by
// exp_cw64 and cis_turns64; the FP64 direct form keeps the device library's,
// an independent check of them).  HG: higher-order
// beamlets, each term times the Hermite-Gaussian factor's degree-4 row
// polynomial (as in the mixed rotor form), records hg.  The anchor is flushed
// below e^-700 and the ln-amplitude slope capped at +-40 per row: with the
// curvature bound of well-sampled grids (|ln-amplitude curvature| <= 0.07 per
// row^2) a slope of 40 puts the beamlet's peak over 280 rows away and the
// anchor below e^-5000, so neither touches a term that is not already zero.
template <int ROWS, int WAVES, bool HG = false>
__global__ void __launch_bounds__(64 * WAVES) eval_fp64_rotor_kernel(EvalGeom g, const Rec64 *__restrict__ rec,
                                                                     const RecSq64 *__restrict__ sqt,
                                                                     double2 *__restrict__ partial,
                                                                     double2 *__restrict__ out,
                                                                     const RecHG64 *__restrict__ hg = nullptr) {
    constexpr int CH = 64;  // records per LDS tile (8 KiB + 16 KiB of sigma tables + 12 KiB HG)
    constexpr int H = ROWS / 2;
    static_assert(H <= 16, "FP64 rotor form: at most 32 rows per lane");
    static_assert(!HG || ROWS <= 16, "FP64 rotor form with higher-order factors: at most 16 rows per lane");
    __shared__ Rec64 tile[CH];
    __shared__ RecSq64 stile[CH];
    __shared__ RecHG64 htile[HG ? CH : 1];
    const int w = work_item(blockIdx.x, gridDim.x);
    if (w >= g.work) return;
    const int tiles = g.tiles_x * g.tiles_y;
    const int seg = w / tiles;
    const int t = w - seg * tiles;
    const int ty = t / g.tiles_x, tx = t - ty * g.tiles_x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ix = tx * 64 + lane;
    const int iy0 = (ty * WAVES + wv) * ROWS;
    const double a = g.a0 + ix * g.dx;
    const double dy = g.dy;
    const double bh = g.b0 + (iy0 + H) * g.dy;

    double acc_re[ROWS], acc_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) acc_re[k] = acc_im[k] = 0.0;

    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
    for (int64_t j0 = jb; j0 < je; j0 += CH) {
        const int cnt = (int)min((int64_t)CH, je - j0);
        __syncthreads();
        {
            const double2 *src = reinterpret_cast<const double2 *>(rec + j0);
            double2 *dst = reinterpret_cast<double2 *>(tile);
            for (int i = threadIdx.x; i < cnt * 8; i += 64 * WAVES) dst[i] = src[i];
            const double2 *qs = reinterpret_cast<const double2 *>(sqt + j0);
            double2 *qd = reinterpret_cast<double2 *>(stile);
            for (int i = threadIdx.x; i < cnt * 16; i += 64 * WAVES) qd[i] = qs[i];
            if constexpr (HG) {
                const double2 *hs = reinterpret_cast<const double2 *>(hg + j0);
                double2 *hd = reinterpret_cast<double2 *>(htile);
                for (int i = threadIdx.x; i < cnt * 12; i += 64 * WAVES) hd[i] = hs[i];
            }
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; jj++) {
            const Rec64 &r = tile[jj];
            const RecSq64 &sq = stile[jj];
            const double da = a - r.arho, db = bh - r.brho;
            const double q = r.p[2] + r.p[4] * da;
            const double T0 = r.p[0] + da * (r.p[1] + r.p[3] * da) + db * (q + r.p[5] * db);
            const double T1 = dy * (q + 2.0 * r.p[5] * db);
            const double ql = r.l[2] + r.l[4] * da;
            const double L0 = r.l[0] + da * (r.l[1] + r.l[3] * da) + db * (ql + r.l[5] * db);
            const double U1 = fmin(fmax(dy * (ql + 2.0 * r.l[5] * db), -40.0), 40.0);
            const double m0 = L0 < -700.0 ? 0.0 : exp_cw64(L0);
            const double2 cs0 = cis_turns64(T0 - rint(T0));
            const double zr = m0 * cs0.x, zi = m0 * cs0.y;
            [[maybe_unused]] double hq[5][2];
            if constexpr (HG) {
                hg_row_poly(htile[jj], da, db, dy, hq);
                acc_re[H] += zr * hq[0][0] - zi * hq[0][1];
                acc_im[H] += zr * hq[0][1] + zi * hq[0][0];
            } else {
                acc_re[H] += zr;
                acc_im[H] += zi;
            }
            const double2 cs1 = cis_turns64(T1 - rint(T1));
            const double c1 = cs1.x, s1 = cs1.y;
            if (ROWS - 1 - H > 0) {
                const double mu = exp_cw64(U1);
                const double ur = mu * c1, ui = mu * s1;
                double pr = zr, pi = zi;
#pragma unroll
                for (int k = 1; k < ROWS - H; k++) {
                    const double nr = fma(pr, ur, -(pi * ui));
                    const double ni = fma(pr, ui, pi * ur);
                    pr = nr;
                    pi = ni;
                    const double sr = sq.sq[k - 1][0], si = sq.sq[k - 1][1];
                    if constexpr (HG) {
                        double Px, Py;
                        horner4(hq, (double)k, Px, Py);
                        const double tr = fma(pr, sr, -(pi * si)), ti = fma(pr, si, pi * sr);
                        acc_re[H + k] = fma(tr, Px, fma(-ti, Py, acc_re[H + k]));
                        acc_im[H + k] = fma(tr, Py, fma(ti, Px, acc_im[H + k]));
                    } else {
                        acc_re[H + k] = fma(pr, sr, fma(-pi, si, acc_re[H + k]));
                        acc_im[H + k] = fma(pr, si, fma(pi, sr, acc_im[H + k]));
                    }
                }
            }
            if (H > 0) {
                const double md = exp_cw64(-U1);
                const double vr = md * c1, vi = -(md * s1);
                double pr = zr, pi = zi;
#pragma unroll
                for (int k = 1; k <= H; k++) {
                    const double nr = fma(pr, vr, -(pi * vi));
                    const double ni = fma(pr, vi, pi * vr);
                    pr = nr;
                    pi = ni;
                    const double sr = sq.sq[k - 1][0], si = sq.sq[k - 1][1];
                    if constexpr (HG) {
                        double Px, Py;
                        horner4(hq, -(double)k, Px, Py);
                        const double tr = fma(pr, sr, -(pi * si)), ti = fma(pr, si, pi * sr);
                        acc_re[H - k] = fma(tr, Px, fma(-ti, Py, acc_re[H - k]));
                        acc_im[H - k] = fma(tr, Py, fma(ti, Px, acc_im[H - k]));
                    } else {
                        acc_re[H - k] = fma(pr, sr, fma(-pi, si, acc_re[H - k]));
                        acc_im[H - k] = fma(pr, si, fma(pi, sr, acc_im[H - k]));
                    }
                }
            }
        }
    }
    if (ix >= g.nx) return;
    const int64_t M = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int k = 0; k < ROWS; k++) {
        const int iy = iy0 + k;
        if (iy < g.ny) {
            const int64_t p = (int64_t)iy * g.nx + ix;
            const double2 v = make_double2(acc_re[k], acc_im[k]);
            if (g.nseg == 1)
                out[p] = v;
            else
                partial[(int64_t)seg * M + p] = v;
        }
    }
}

// the guard's condition (EvalGuard), the same for every thread
__device__ inline bool guard_holds(const EvalGuard &gd) {
    if (!gd.status) return true;
    const uint32_t st = gd.status[0], key = gd.status[1];
    return !(st & FLAG_ERRORS) && (st & gd.mask) == gd.flags && (!gd.check_key || key == gd.key);
}

__global__ void __launch_bounds__(256) reduce_mixed_kernel(int64_t M, int32_t nseg2, const float2 *__restrict__ part2,
                                                           int32_t nseg4, const float4 *__restrict__ part4,
                                                           float2 *__restrict__ out, EvalGuard gd) {
    if (!guard_holds(gd)) return;
    // A batch of segments' loads is issued before any of them is added, so a
    // pixel costs one memory round trip per batch (32 float2 or 16 float4
    // partials) instead of one per few segments; the sums still run in
    // segment order.
    constexpr int B2 = 32, B4 = 16;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        int s = 0;
        for (; s + B2 <= nseg2; s += B2) {
            float2 v[B2];
#pragma unroll
            for (int u = 0; u < B2; u++) v[u] = part2[(int64_t)(s + u) * M + p];
#pragma unroll
            for (int u = 0; u < B2; u++) {
                re += (double)v[u].x;
                im += (double)v[u].y;
            }
        }
#pragma unroll 8
        for (; s < nseg2; s++) {
            const float2 v = part2[(int64_t)s * M + p];
            re += (double)v.x;
            im += (double)v.y;
        }
        s = 0;
        for (; s + B4 <= nseg4; s += B4) {
            float4 v[B4];
#pragma unroll
            for (int u = 0; u < B4; u++) v[u] = part4[(int64_t)(s + u) * M + p];
#pragma unroll
            for (int u = 0; u < B4; u++) {
                re += (double)v[u].x - (double)v[u].z;
                im += (double)v[u].y - (double)v[u].w;
            }
        }
#pragma unroll 8
        for (; s < nseg4; s++) {
            const float4 v = part4[(int64_t)s * M + p];
            re += (double)v.x - (double)v.z;
            im += (double)v.y - (double)v.w;
        }
        out[p] = make_float2((float)re, (float)im);
    }
}

__global__ void __launch_bounds__(256) reduce_fp64_kernel(int64_t M, int32_t nseg, const double2 *__restrict__ part,
                                                          double2 *__restrict__ out, EvalGuard gd) {
    if (!guard_holds(gd)) return;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
#pragma unroll 8
        for (int s = 0; s < nseg; s++) {
            const double2 v = part[(int64_t)s * M + p];
            re += v.x;
            im += v.y;
        }
        out[p] = make_double2(re, im);
    }
}

template <int ROWS, int WAVES>
hipError_t launch_eval_t(int precision, int form, const EvalGeom &g, const void *rec, const void *hg,
                         const RecSq64 *q64, void *partial, void *out, hipStream_t s) {
    const int grid = (g.work + 7) / 8 * 8;
    if (precision == 0 && form == 2) {
        if (!q64) return hipErrorInvalidValue;
        if (hg)
            eval_fp64_rotor_kernel<ROWS, WAVES, true><<<grid, 64 * WAVES, 0, s>>>(
                g, static_cast<const Rec64 *>(rec), q64, static_cast<double2 *>(partial), static_cast<double2 *>(out),
                static_cast<const RecHG64 *>(hg));
        else
            eval_fp64_rotor_kernel<ROWS, WAVES><<<grid, 64 * WAVES, 0, s>>>(
                g, static_cast<const Rec64 *>(rec), q64, static_cast<double2 *>(partial), static_cast<double2 *>(out));
        return hipGetLastError();
    }
    if (hg) {
        if (precision == 1 && form == 2)
            eval_mixed_kernel<ROWS, WAVES, 2, true><<<grid, 64 * WAVES, 0, s>>>(
                g, static_cast<const Rec32 *>(rec), static_cast<float4 *>(partial), static_cast<float2 *>(out),
                static_cast<const RecHG32 *>(hg));
        else if (precision == 1 && form == 0)
            eval_mixed_kernel<ROWS, WAVES, 0, true><<<grid, 64 * WAVES, 0, s>>>(
                g, static_cast<const Rec32 *>(rec), static_cast<float4 *>(partial), static_cast<float2 *>(out),
                static_cast<const RecHG32 *>(hg));
        else if constexpr (ROWS <= 8) {
            if (precision != 0) return hipErrorInvalidValue;
            eval_fp64_kernel<ROWS, WAVES, true><<<grid, 64 * WAVES, 0, s>>>(
                g, static_cast<const Rec64 *>(rec), static_cast<double2 *>(partial), static_cast<double2 *>(out),
                static_cast<const RecHG64 *>(hg));
        } else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (precision == 1 && form == 2)
        eval_mixed_kernel<ROWS, WAVES, 2><<<grid, 64 * WAVES, 0, s>>>(g, static_cast<const Rec32 *>(rec),
                                                                      static_cast<float4 *>(partial),
                                                                      static_cast<float2 *>(out));
    else if (precision == 1 && form == 1)
        eval_mixed_kernel<ROWS, WAVES, 1><<<grid, 64 * WAVES, 0, s>>>(g, static_cast<const Rec32 *>(rec),
                                                                      static_cast<float4 *>(partial),
                                                                      static_cast<float2 *>(out));
    else if (precision == 1)
        eval_mixed_kernel<ROWS, WAVES, 0><<<grid, 64 * WAVES, 0, s>>>(g, static_cast<const Rec32 *>(rec),
                                                                      static_cast<float4 *>(partial),
                                                                      static_cast<float2 *>(out));
    else if constexpr (ROWS <= 8)
        eval_fp64_kernel<ROWS, WAVES><<<grid, 64 * WAVES, 0, s>>>(g, static_cast<const Rec64 *>(rec),
                                                                  static_cast<double2 *>(partial),
                                                                  static_cast<double2 *>(out));
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sigma(const EvalGeom &g, const Rec64 *r64, RecSq64 *q64, Rec32 *r32, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    if ((q64 == nullptr) == (r32 == nullptr)) return hipErrorInvalidValue;
    sigma_kernel<<<(unsigned)((g.n + 15) / 16), 256, 0, s>>>(g.n, g.dy, r64, q64, r32);
    return hipGetLastError();
}

hipError_t launch_status_post(const StatusPost &sp, hipStream_t s) {
    if (!sp.status || !sp.post) return hipErrorInvalidValue;
    status_post_kernel<<<1, 64, 0, s>>>(sp);
    return hipGetLastError();
}

hipError_t launch_setup(const BeamletsDev &b, const PlaneGeom &pl, double global_turns, Rec64 *r64, Rec32 *r32,
                        RecHG64 *h64, RecHG32 *h32, RecCut64 *c64, RecCut32 *c32, uint32_t *status,
                        uint32_t *status_next, hipStream_t s) {
    if (b.n == 0) return hipSuccess;
    const int64_t blocks = (b.n + 255) / 256;
    setup_kernel<<<(unsigned)blocks, 256, 0, s>>>(b, pl, global_turns, r64, r32, h64, h32, c64, c32, status,
                                                  status_next);
    return hipGetLastError();
}

hipError_t launch_eval(int precision, int rows, int waves, int form, const EvalGeom &g, const void *rec, const void *hg,
                       const RecSq64 *q64, void *partial, void *out, hipStream_t s) {
#define GBD_CASE(R, W) \
    if (rows == R && waves == W) return launch_eval_t<R, W>(precision, form, g, rec, hg, q64, partial, out, s);
    GBD_CASE(1, 1) GBD_CASE(1, 2) GBD_CASE(1, 4)
    GBD_CASE(2, 1) GBD_CASE(2, 2) GBD_CASE(2, 4)
    GBD_CASE(4, 1) GBD_CASE(4, 2) GBD_CASE(4, 4)
    GBD_CASE(8, 1) GBD_CASE(8, 2) GBD_CASE(8, 4)
#undef GBD_CASE
    if (precision == 1 && rows == 16) {
        if (waves == 1) return launch_eval_t<16, 1>(precision, form, g, rec, hg, q64, partial, out, s);
        if (waves == 2) return launch_eval_t<16, 2>(precision, form, g, rec, hg, q64, partial, out, s);
        if (waves == 4) return launch_eval_t<16, 4>(precision, form, g, rec, hg, q64, partial, out, s);
    }
    if (precision == 0 && form == 2 && !hg && q64 && (rows == 16 || rows == 32)) {
        const int grid = (g.work + 7) / 8 * 8;
        double2 *pt = static_cast<double2 *>(partial), *o = static_cast<double2 *>(out);
        const Rec64 *r = static_cast<const Rec64 *>(rec);
        if (rows == 16 && waves == 1) eval_fp64_rotor_kernel<16, 1><<<grid, 64, 0, s>>>(g, r, q64, pt, o);
        else if (rows == 16 && waves == 2) eval_fp64_rotor_kernel<16, 2><<<grid, 128, 0, s>>>(g, r, q64, pt, o);
        else if (rows == 16 && waves == 4) eval_fp64_rotor_kernel<16, 4><<<grid, 256, 0, s>>>(g, r, q64, pt, o);
        else if (rows == 32 && waves == 1) eval_fp64_rotor_kernel<32, 1><<<grid, 64, 0, s>>>(g, r, q64, pt, o);
        else if (rows == 32 && waves == 2) eval_fp64_rotor_kernel<32, 2><<<grid, 128, 0, s>>>(g, r, q64, pt, o);
        else if (rows == 32 && waves == 4) eval_fp64_rotor_kernel<32, 4><<<grid, 256, 0, s>>>(g, r, q64, pt, o);
        else return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (precision == 0 && form == 2 && hg && q64 && rows == 16) {
        const int grid = (g.work + 7) / 8 * 8;
        double2 *pt = static_cast<double2 *>(partial), *o = static_cast<double2 *>(out);
        const Rec64 *r = static_cast<const Rec64 *>(rec);
        const RecHG64 *h = static_cast<const RecHG64 *>(hg);
        if (waves == 1) eval_fp64_rotor_kernel<16, 1, true><<<grid, 64, 0, s>>>(g, r, q64, pt, o, h);
        else if (waves == 2) eval_fp64_rotor_kernel<16, 2, true><<<grid, 128, 0, s>>>(g, r, q64, pt, o, h);
        else if (waves == 4) eval_fp64_rotor_kernel<16, 4, true><<<grid, 256, 0, s>>>(g, r, q64, pt, o, h);
        else return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (precision == 1 && rows == 32 && form == 2 && hg) {
        const int grid = (g.work + 7) / 8 * 8;
        const Rec32 *r = static_cast<const Rec32 *>(rec);
        const RecHG32 *h = static_cast<const RecHG32 *>(hg);
        float4 *pt = static_cast<float4 *>(partial);
        float2 *o = static_cast<float2 *>(out);
        if (waves == 1)
            eval_mixed_kernel<32, 1, 2, true><<<grid, 64, 0, s>>>(g, r, pt, o, h);
        else if (waves == 2)
            eval_mixed_kernel<32, 2, 2, true><<<grid, 128, 0, s>>>(g, r, pt, o, h);
        else if (waves == 4)
            eval_mixed_kernel<32, 4, 2, true><<<grid, 256, 0, s>>>(g, r, pt, o, h);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (precision == 1 && rows == 32 && form == 2) {
        const int grid = (g.work + 7) / 8 * 8;
        if (waves == 1)
            eval_mixed_kernel<32, 1, 2><<<grid, 64, 0, s>>>(g, static_cast<const Rec32 *>(rec),
                                                            static_cast<float4 *>(partial), static_cast<float2 *>(out));
        else if (waves == 2)
            eval_mixed_kernel<32, 2, 2><<<grid, 128, 0, s>>>(g, static_cast<const Rec32 *>(rec),
                                                             static_cast<float4 *>(partial), static_cast<float2 *>(out));
        else if (waves == 4)
            eval_mixed_kernel<32, 4, 2><<<grid, 256, 0, s>>>(g, static_cast<const Rec32 *>(rec),
                                                             static_cast<float4 *>(partial), static_cast<float2 *>(out));
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

__global__ void __launch_bounds__(256) fill_zero_kernel(uint4 *__restrict__ p, int64_t n16,
                                                        unsigned char *__restrict__ tail, int32_t n_tail) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t; i < n16; i += (int64_t)gridDim.x * blockDim.x) p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (t < n_tail) tail[t] = 0;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (!p || (reinterpret_cast<uintptr_t>(p) & 15) != 0) return hipErrorInvalidValue;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int32_t n_tail = (int32_t)(bytes % 16);
    int64_t blocks = (n16 + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    fill_zero_kernel<<<(unsigned)blocks, 256, 0, s>>>(static_cast<uint4 *>(p), n16,
                                                      static_cast<unsigned char *>(p) + n16 * 16, n_tail);
    return hipGetLastError();
}

hipError_t launch_reduce(int precision, const EvalGeom &g, int32_t nseg2, const void *partial, void *out,
                         hipStream_t s, const EvalGuard &guard) {
    const int64_t M = (int64_t)g.nx * g.ny;
    if (M == 0) return hipSuccess;
    if (nseg2 < 0 || nseg2 > g.nseg || (precision != 1 && nseg2 != 0)) return hipErrorInvalidValue;
    const int64_t blocks = min((M + 255) / 256, (int64_t)4096);
    if (precision == 1)
        reduce_mixed_kernel<<<(unsigned)blocks, 256, 0, s>>>(
            M, nseg2, static_cast<const float2 *>(partial), g.nseg - nseg2,
            reinterpret_cast<const float4 *>(static_cast<const char *>(partial) + reduce_wide_offset(nseg2, M)),
            static_cast<float2 *>(out), guard);
    else
        reduce_fp64_kernel<<<(unsigned)blocks, 256, 0, s>>>(M, g.nseg, static_cast<const double2 *>(partial),
                                                            static_cast<double2 *>(out), guard);
    return hipGetLastError();
}

}  // namespace gbd
