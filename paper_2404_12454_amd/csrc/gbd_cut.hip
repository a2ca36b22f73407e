// Truncated beamlets: a Gaussian beamlet whose input envelope is cut by a
// straight edge (kept where e . r <= t) arrives on a plane normal to the axis
// as its Gaussian field times erfc(zeta) / 2, zeta = z0 + za da + zb db (the
// setup kernel's RecCut record).  Direct form: every pixel of every cut
// beamlet forms the Gaussian phasor as the direct mixed (or FP64) form does
// and the complementary error function through the Faddeeva function
// w(u) = e^(-u^2) erfc(-i u):
//   Re zeta >= 0:  E erfc(zeta) / 2 = e^(log E - zeta^2) w(i zeta) / 2,
//   Re zeta <  0:  E erfc(zeta) / 2 = E - e^(log E - zeta^2) w(-i zeta) / 2,
// so the exponent log E - zeta^2 is formed before any exponential (each of
// e^(log E) and erfc(zeta) alone can under- or overflow where their product
// is finite) and w is only taken in the upper half plane, where |w| <= 1.  w
// by Weideman's rational approximation (FaddeevaCoef).  The cut beamlets are
// few (those near an aperture edge), so the others keep the fast forms and
// this kernel adds its segments to the same partial sums.
#include "gbd_device.h"

namespace gbd {

namespace {

using namespace dev;

// w(u) for Im u >= 0, FP32 (u = (ur, ui))
__device__ inline float2 faddeeva32(const FaddeevaCoef &fc, float ur, float ui) {
    const float L = fc.L32;
    // 1 / (L - i u) = 1 / ((L + ui) - i ur)
    const float dr = L + ui, di = -ur;
    const float inv = __builtin_amdgcn_rcpf(fmaf(dr, dr, di * di));
    const float vr = dr * inv, vi = -di * inv;
    // Z = (L + i u) / (L - i u) = ((L - ui) + i ur) v
    const float nr = L - ui, ni = ur;
    const float Zr = nr * vr - ni * vi, Zi = nr * vi + ni * vr;
    float pr = fc.a32[kFaddeevaN32 - 1], pi = 0.0f;
#pragma unroll
    for (int n = kFaddeevaN32 - 2; n >= 0; n--) {
        const float tr = fmaf(pr, Zr, fmaf(-pi, Zi, fc.a32[n]));
        pi = fmaf(pr, Zi, pi * Zr);
        pr = tr;
    }
    // w = v (2 p v + 1 / sqrt(pi))
    const float sr = fmaf(2.0f * pr, vr, fmaf(-2.0f * pi, vi, 0.56418958354775628f));
    const float si = 2.0f * (pr * vi + pi * vr);
    return make_float2(vr * sr - vi * si, vr * si + vi * sr);
}

__device__ inline cd faddeeva64(const FaddeevaCoef &fc, double ur, double ui) {
    const double L = fc.L64;
    const cd v = cdiv(mk(1.0, 0.0), mk(L + ui, -ur));
    const cd Z = mul(mk(L - ui, ur), v);
    cd p = mk(fc.a64[kFaddeevaN64 - 1], 0.0);
#pragma unroll
    for (int n = kFaddeevaN64 - 2; n >= 0; n--) p = add(mul(p, Z), mk(fc.a64[n], 0.0));
    return mul(v, add(scl(mul(p, v), 2.0), mk(0.56418958354775628695, 0.0)));
}

template <int ROWS, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) eval_cut_mixed_kernel(EvalGeom g, const Rec32 *__restrict__ rec,
                                                                    const RecCut32 *__restrict__ cut,
                                                                    FaddeevaCoef fc, int32_t seg_base,
                                                                    float4 *__restrict__ partial) {
    __shared__ Rec32 tile[kMixedTile];
    __shared__ RecCut32 ctile[kMixedTile];
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
    const float af = (float)a, b0f = (float)b0, dyf = (float)dy;
    constexpr float kLog2e = 1.4426950408889634f, kInv2Pi = 0.15915494309189535f;

    float s_re[ROWS], s_im[ROWS], c_re[ROWS], c_im[ROWS], acc_re[ROWS], acc_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) s_re[k] = s_im[k] = c_re[k] = c_im[k] = acc_re[k] = acc_im[k] = 0.0f;
    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
    for (int64_t j0 = jb; j0 < je; j0 += kMixedTile) {
        const int cnt = (int)min((int64_t)kMixedTile, je - j0);
        __syncthreads();
        {
            const float4 *src = reinterpret_cast<const float4 *>(rec + j0);
            float4 *dst = reinterpret_cast<float4 *>(tile);
            for (int i = threadIdx.x; i < cnt * kRec32Vec4; i += 64 * WAVES) dst[i] = src[i];
            const float4 *cs = reinterpret_cast<const float4 *>(cut + j0);
            float4 *cd4 = reinterpret_cast<float4 *>(ctile);
            for (int i = threadIdx.x; i < cnt * 2; i += 64 * WAVES) cd4[i] = cs[i];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; jj++) {
            const Rec32 &r = tile[jj];
            const RecCut32 &c = ctile[jj];
            const double da = a - r.arho, db = b0 - r.brho;
            const double q = r.p[2] + r.p[4] * da;
            const double T0 = r.p[0] + da * (r.p[1] + r.p[3] * da) + db * (q + r.p[5] * db);
            const double T1 = dy * (q + 2.0 * r.p[5] * db);
            const double T2 = r.p[5] * dy2;
            const float daf = af - r.arho_f, dbf0 = b0f - r.brho_f;
            const float qf = r.m[2] + r.m[4] * daf;
            const float Uc = r.m[0] + daf * (r.m[1] + r.m[3] * daf);
            const float zr0 = fmaf(c.za[0], daf, c.z0[0]), zi0 = fmaf(c.za[1], daf, c.z0[1]);
#pragma unroll
            for (int k = 0; k < ROWS; k++) {
                const double th = T0 + (double)k * (T1 + (double)k * T2);
                const float ph = (float)__builtin_amdgcn_fract(th);
                const float dbf = fmaf((float)k, dyf, dbf0);
                const float L = Uc + dbf * (qf + r.m[5] * dbf);
                // zeta, folded into the right half plane
                float zr = fmaf(c.zb[0], dbf, zr0), zi = fmaf(c.zb[1], dbf, zi0);
                const bool neg = zr < 0.0f;
                zr = neg ? -zr : zr;
                zi = neg ? -zi : zi;
                // e^(log E - zeta^2) / 2: log2-amplitude and phase in turns
                const float L2 = L - 1.0f - (zr * zr - zi * zi) * kLog2e;
                const float ph2 = __builtin_amdgcn_fractf(ph - 2.0f * zr * zi * kInv2Pi);
                const float m2 = __builtin_amdgcn_exp2f(L2);
                const float er = m2 * __builtin_amdgcn_cosf(ph2), ei = m2 * __builtin_amdgcn_sinf(ph2);
                const float2 W = faddeeva32(fc, -zi, zr);  // w(i zeta)
                float tr = er * W.x - ei * W.y, ti = er * W.y + ei * W.x;
                if (neg) {
                    const float m = __builtin_amdgcn_exp2f(L);
                    tr = m * __builtin_amdgcn_cosf(ph) - tr;
                    ti = m * __builtin_amdgcn_sinf(ph) - ti;
                }
                acc_re[k] += tr;
                acc_im[k] += ti;
            }
        }
#pragma unroll
        for (int k = 0; k < ROWS; k++) {
            kahan(s_re[k], c_re[k], acc_re[k]);
            kahan(s_im[k], c_im[k], acc_im[k]);
            acc_re[k] = acc_im[k] = 0.0f;
        }
    }
    if (ix >= g.nx) return;
    const int64_t M = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int k = 0; k < ROWS; k++) {
        const int iy = iy0 + k;
        if (iy < g.ny)
            partial[(int64_t)(seg_base + seg) * M + (int64_t)iy * g.nx + ix] =
                make_float4(s_re[k], s_im[k], c_re[k], c_im[k]);
    }
}

template <int ROWS, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) eval_cut_fp64_kernel(EvalGeom g, const Rec64 *__restrict__ rec,
                                                                   const RecCut64 *__restrict__ cut,
                                                                   FaddeevaCoef fc, int32_t seg_base,
                                                                   double2 *__restrict__ partial) {
    constexpr int CH = 64;
    __shared__ Rec64 tile[CH];
    __shared__ RecCut64 ctile[CH];
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
            const double2 *cs = reinterpret_cast<const double2 *>(cut + j0);
            double2 *cd2 = reinterpret_cast<double2 *>(ctile);
            for (int i = threadIdx.x; i < cnt * 4; i += 64 * WAVES) cd2[i] = cs[i];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; jj++) {
            const Rec64 &r = tile[jj];
            const RecCut64 &c = ctile[jj];
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
                const double dbk = fma((double)k, dy, db);
                const double lnm = Vc + dbk * (ql + r.l[5] * dbk);
                double zr = c.z0[0] + c.za[0] * da + c.zb[0] * dbk;
                double zi = c.z0[1] + c.za[1] * da + c.zb[1] * dbk;
                const bool neg = zr < 0.0;
                zr = neg ? -zr : zr;
                zi = neg ? -zi : zi;
                // e^(log E - zeta^2) / 2 (phase in turns)
                double ph2 = rr - zr * zi / kPi;
                ph2 -= rint(ph2);
                double s2, c2;
                sincospi(2.0 * ph2, &s2, &c2);
                const double m2 = 0.5 * exp(lnm - (zr * zr - zi * zi));
                const cd W = faddeeva64(fc, -zi, zr);
                double tr = m2 * (c2 * W.re - s2 * W.im), ti = m2 * (c2 * W.im + s2 * W.re);
                if (neg) {
                    double s, cc;
                    sincospi(2.0 * rr, &s, &cc);
                    const double m = exp(lnm);
                    tr = m * cc - tr;
                    ti = m * s - ti;
                }
                acc_re[k] += tr;
                acc_im[k] += ti;
            }
        }
    }
    if (ix >= g.nx) return;
    const int64_t M = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int k = 0; k < ROWS; k++) {
        const int iy = iy0 + k;
        if (iy < g.ny)
            partial[(int64_t)(seg_base + seg) * M + (int64_t)iy * g.nx + ix] = make_double2(acc_re[k], acc_im[k]);
    }
}

}  // namespace

hipError_t launch_eval_cut(int precision, const EvalGeom &g, const void *rec, const void *cut,
                           const FaddeevaCoef &fc, int32_t seg_base, void *partial, hipStream_t s) {
    const int grid = (g.work + 7) / 8 * 8;
    if (precision == 1)
        eval_cut_mixed_kernel<kCutRows32, 4><<<grid, 256, 0, s>>>(g, static_cast<const Rec32 *>(rec),
                                                                 static_cast<const RecCut32 *>(cut), fc, seg_base,
                                                                 static_cast<float4 *>(partial));
    else
        eval_cut_fp64_kernel<kCutRows64, 4><<<grid, 256, 0, s>>>(g, static_cast<const Rec64 *>(rec),
                                                                static_cast<const RecCut64 *>(cut), fc, seg_base,
                                                                static_cast<double2 *>(partial));
    return hipGetLastError();
}

}  // namespace gbd
