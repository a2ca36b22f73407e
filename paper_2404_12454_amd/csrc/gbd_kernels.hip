// gfx950 kernels of plane-evaluation Gaussian beamlet decomposition.
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
#include "gbd_internal.h"

#include <math.h>

namespace gbd {

namespace {

constexpr double kPi = 3.14159265358979323846;

struct cd {
    double re, im;
};
__device__ inline cd mk(double r, double i) { return cd{r, i}; }
__device__ inline cd add(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ inline cd sub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ inline cd mul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cd scl(cd a, double s) { return cd{a.re * s, a.im * s}; }
__device__ inline double cabs2(cd a) { return hypot(a.re, a.im); }
__device__ inline cd cdiv(cd a, cd b) {
    // Smith's algorithm: no overflow for widely scaled operands.
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, d = b.re + b.im * r;
        return cd{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    }
    double r = b.re / b.im, d = b.re * r + b.im;
    return cd{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
// principal square root (branch cut on the negative real axis, sign of the
// imaginary part's zero respected)
__device__ inline cd csqrt_p(cd z) {
    double m = hypot(z.re, z.im);
    if (m == 0.0) return cd{0.0, z.im};
    if (z.re >= 0.0) {
        double t = sqrt(0.5 * (m + z.re));
        return cd{t, z.im / (2.0 * t)};
    }
    double t = sqrt(0.5 * (m - z.re));
    return cd{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// Eigenvalues admitted on the principal-root branch: the open lower half
// plane and the positive real axis (reached from 1 without crossing the cut).
__device__ inline bool on_branch(cd mu) {
    double m = hypot(mu.re, mu.im);
    double tol = 1e-12 * m;
    if (!(m > 0.0)) return false;
    if (mu.im > tol) return false;
    if (mu.im >= -tol && mu.re <= 0.0) return false;
    return true;
}

__global__ void __launch_bounds__(256) setup_kernel(BeamletsDev b, PlaneGeom pl, double gturns,
                                                    Rec64 *__restrict__ r64, Rec32 *__restrict__ r32,
                                                    uint32_t *__restrict__ status) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= b.n) return;
    const double *M = b.abcd + (b.n_abcd == 1 ? 0 : 16 * j);
    double A[2][2], B[2][2], C[2][2], D[2][2];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int c = 0; c < 2; c++) {
            A[r][c] = M[4 * r + c];
            B[r][c] = M[4 * r + c + 2];
            C[r][c] = M[4 * (r + 2) + c];
            D[r][c] = M[4 * (r + 2) + c + 2];
        }
    const double r1[2] = {b.r1[2 * j], b.r1[2 * j + 1]};
    const double t1[2] = {b.th1[2 * j], b.th1[2 * j + 1]};
    const double w0 = b.w0[b.n_w0 == 1 ? 0 : j];
    const cd amp = mk(b.amp[2 * j], b.amp[2 * j + 1]);
    const double W = b.path[j];
    const double lam = b.lam;

    // base ray at the ABCD output plane
    double r2M[2], th[2];
#pragma unroll
    for (int r = 0; r < 2; r++) {
        r2M[r] = A[r][0] * r1[0] + A[r][1] * r1[1] + B[r][0] * t1[0] + B[r][1] * t1[1];
        th[r] = C[r][0] * r1[0] + C[r][1] * r1[1] + D[r][0] * t1[0] + D[r][1] * t1[1];
    }
    // where the base ray (r2M + z th, z) meets the plane
    const double nd = pl.n[0] * th[0] + pl.n[1] * th[1] + pl.n[2];
    const double dl = sqrt(th[0] * th[0] + th[1] * th[1] + 1.0);
    Rec64 o64 = {};
    Rec32 o32 = {};
    uint32_t flag = 0;
    if (!(fabs(nd) > 1e-6 * dl)) {
        flag |= FLAG_PARALLEL;
    } else {
        const double z = (pl.n[0] * (pl.O[0] - r2M[0]) + pl.n[1] * (pl.O[1] - r2M[1]) + pl.n[2] * pl.O[2]) / nd;
        const double X[3] = {r2M[0] + z * th[0] - pl.O[0], r2M[1] + z * th[1] - pl.O[1], z - pl.O[2]};
        const double arho = pl.e1[0] * X[0] + pl.e1[1] * X[1] + pl.e1[2] * X[2];
        const double brho = pl.e2[0] * X[0] + pl.e2[1] * X[1] + pl.e2[2] * X[2];

        // system extended by free space z; Q1^-1 = -i kappa I
        const double kappa = lam / (kPi * w0 * w0);
        cd Mm[2][2], Nm[2][2];
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int c = 0; c < 2; c++) {
                Mm[r][c] = mk(A[r][c] + z * C[r][c], -kappa * (B[r][c] + z * D[r][c]));
                Nm[r][c] = mk(C[r][c], -kappa * D[r][c]);
            }
        // Q^-1 = Nm Mm^-1 (2x2 closed-form inverse), symmetrised
        const cd det = sub(mul(Mm[0][0], Mm[1][1]), mul(Mm[0][1], Mm[1][0]));
        cd Mi[2][2];
        Mi[0][0] = cdiv(Mm[1][1], det);
        Mi[1][1] = cdiv(Mm[0][0], det);
        Mi[0][1] = cdiv(scl(Mm[0][1], -1.0), det);
        Mi[1][0] = cdiv(scl(Mm[1][0], -1.0), det);
        cd Q[2][2];
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int c = 0; c < 2; c++) Q[r][c] = add(mul(Nm[r][0], Mi[0][c]), mul(Nm[r][1], Mi[1][c]));
        const cd qo = scl(add(Q[0][1], Q[1][0]), 0.5);
        Q[0][1] = qo;
        Q[1][0] = qo;
        // amplitude det(Mm)^(-1/2) from the eigenvalues' principal roots
        const cd tr = add(Mm[0][0], Mm[1][1]);
        const cd disc = csqrt_p(sub(mul(tr, tr), scl(det, 4.0)));
        const cd mu1 = scl(add(tr, disc), 0.5), mu2 = scl(sub(tr, disc), 0.5);
        if (!on_branch(mu1) || !on_branch(mu2)) flag |= FLAG_BRANCH;
        const cd gamma = cdiv(mk(1.0, 0.0), mul(csqrt_p(mu1), csqrt_p(mu2)));

        // misalignment phase at the hit point, in turns (l0 handled by the host)
        const double r2[2] = {r2M[0] + z * th[0], r2M[1] + z * th[1]};
        const double S = 0.5 * (th[0] * r2[0] + th[1] * r2[1] - t1[0] * r1[0] - t1[1] * r1[1]);
        const double tau = (z + W + S) / lam;

        // plane basis seen from the beamlet: w = Pm d, zeta = ez . d
        const double *e[2] = {pl.e1, pl.e2};
        double Pm[2][2], ez[2];
#pragma unroll
        for (int c = 0; c < 2; c++) {
            ez[c] = e[c][2];
#pragma unroll
            for (int r = 0; r < 2; r++) Pm[r][c] = e[c][r] - e[c][2] * th[r];
        }
        const cd trQ = add(Q[0][0], Q[1][1]);
        const cd trQ2 = add(add(mul(Q[0][0], Q[0][0]), mul(Q[1][1], Q[1][1])), scl(mul(Q[0][1], Q[1][0]), 2.0));
        // G = Pm^T Q Pm
        cd QP[2][2], G[2][2];
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int c = 0; c < 2; c++) QP[r][c] = add(scl(Q[r][0], Pm[0][c]), scl(Q[r][1], Pm[1][c]));
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int c = 0; c < 2; c++) G[r][c] = add(scl(QP[0][c], Pm[0][r]), scl(QP[1][c], Pm[1][r]));
        const double h = 1.0 + 0.5 * (th[0] * th[0] + th[1] * th[1]);
        // (1 + |th|^2/2) ez + Pm^T th
        const double lin[2] = {h * ez[0] + Pm[0][0] * th[0] + Pm[1][0] * th[1],
                               h * ez[1] + Pm[0][1] * th[0] + Pm[1][1] * th[1]};
        const double i4pi = 1.0 / (4.0 * kPi), i8pi = 1.0 / (8.0 * kPi), kh = kPi / lam;
        // phase polynomial (turns)
        double p[6], l[6];
        const cd ag = mul(amp, gamma);
        double tred = tau - rint(tau);
        double p0 = atan2(ag.im, ag.re) / (2.0 * kPi) - tred - gturns;
        p[0] = p0 - rint(p0);
        p[1] = -lin[0] / lam - trQ.im * ez[0] * i4pi;
        p[2] = -lin[1] / lam - trQ.im * ez[1] * i4pi;
        p[3] = -G[0][0].re / (2.0 * lam) + trQ2.im * ez[0] * ez[0] * i8pi;
        p[4] = 2.0 * (-G[0][1].re / (2.0 * lam) + trQ2.im * ez[0] * ez[1] * i8pi);
        p[5] = -G[1][1].re / (2.0 * lam) + trQ2.im * ez[1] * ez[1] * i8pi;
        // log-amplitude polynomial (natural log)
        l[0] = log(cabs2(ag));
        l[1] = -0.5 * trQ.re * ez[0];
        l[2] = -0.5 * trQ.re * ez[1];
        l[3] = kh * G[0][0].im + 0.25 * trQ2.re * ez[0] * ez[0];
        l[4] = 2.0 * (kh * G[0][1].im + 0.25 * trQ2.re * ez[0] * ez[1]);
        l[5] = kh * G[1][1].im + 0.25 * trQ2.re * ez[1] * ez[1];
        bool fin = isfinite(arho) && isfinite(brho) && isfinite(ag.re) && isfinite(ag.im);
#pragma unroll
        for (int i = 0; i < 6; i++) fin = fin && isfinite(p[i]) && (i == 0 || isfinite(l[i]));
        if (!fin) flag |= FLAG_NONFINITE;
        o64.arho = arho;
        o64.brho = brho;
        o32.arho = arho;
        o32.brho = brho;
        o32.arho_f = (float)arho;
        o32.brho_f = (float)brho;
        const double il2 = 1.4426950408889634074;  // 1 / ln 2
#pragma unroll
        for (int i = 0; i < 6; i++) {
            o64.p[i] = p[i];
            o64.l[i] = l[i];
            o32.p[i] = p[i];
            o32.m[i] = (float)(l[i] * il2);
        }
    }
    if (flag) {
        atomicOr(status, flag);
        // a refused beamlet contributes nothing
        o64.l[0] = -INFINITY;
        o32.m[0] = -INFINITY;
    }
    r64[j] = o64;
    r32[j] = o32;
}

// XCD-aware work mapping: workgroup b runs on XCD (b mod 8); give each XCD a
// contiguous range of (segment, tile) work items so that the beamlet records
// of a segment stay in one L2.  The grid is padded to a multiple of 8.
__device__ inline int work_item(int b, int G) { return (b & 7) * (G >> 3) + (b >> 3); }

__device__ inline void kahan(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Mixed form: FP64 phase polynomial reduced to turns, FP32 hardware exp2 /
// sin / cos (v_sin_f32 and v_cos_f32 take revolutions), FP32 per-tile sums
// folded into compensated (Kahan) FP32 accumulators.
// Each lane owns ROWS pixels of one detector column; a wavefront spans 64
// consecutive columns (coalesced stores); WAVES wavefronts stack in y.
template <int ROWS, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) eval_mixed_kernel(EvalGeom g, const Rec32 *__restrict__ rec,
                                                                float4 *__restrict__ partial,
                                                                float2 *__restrict__ out) {
    constexpr int CH = 128;  // records per LDS tile (12 KiB)
    __shared__ Rec32 tile[CH];
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
    const float af = (float)a, b0f = (float)b0, dyf = (float)g.dy;

    float acc_re[ROWS], acc_im[ROWS], s_re[ROWS], s_im[ROWS], c_re[ROWS], c_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) acc_re[k] = acc_im[k] = s_re[k] = s_im[k] = c_re[k] = c_im[k] = 0.0f;

    const int64_t jb = (int64_t)seg * g.seg_len;
    const int64_t je = min(g.n, jb + g.seg_len);
    for (int64_t j0 = jb; j0 < je; j0 += CH) {
        const int cnt = (int)min((int64_t)CH, je - j0);
        __syncthreads();
        {
            const float4 *src = reinterpret_cast<const float4 *>(rec + j0);
            float4 *dst = reinterpret_cast<float4 *>(tile);
            for (int i = threadIdx.x; i < cnt * 6; i += 64 * WAVES) dst[i] = src[i];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; jj++) {
            const Rec32 &r = tile[jj];
            // phase, restricted to this lane's column, as a quadratic in the row step k
            const double da = a - r.arho, db = b0 - r.brho;
            const double q = r.p[2] + r.p[4] * da;
            const double T0 = r.p[0] + da * (r.p[1] + r.p[3] * da) + db * (q + r.p[5] * db);
            const double T1 = dy * (q + 2.0 * r.p[5] * db);
            const double T2 = r.p[5] * dy2;
            // log2-amplitude in FP32, evaluated from each pixel's own row offset
            // (an expansion in k would cancel catastrophically far from the spot)
            const float daf = af - r.arho_f, dbf0 = b0f - r.brho_f;
            const float qf = r.m[2] + r.m[4] * daf;
            const float Uc = r.m[0] + daf * (r.m[1] + r.m[3] * daf);
#pragma unroll
            for (int k = 0; k < ROWS; k++) {
                const double th = T0 + (double)k * (T1 + (double)k * T2);
                const float ph = (float)__builtin_amdgcn_fract(th);
                const float dbf = fmaf((float)k, dyf, dbf0);
                const float L = Uc + dbf * (qf + r.m[5] * dbf);
                const float m = __builtin_amdgcn_exp2f(L);
                acc_re[k] = fmaf(m, __builtin_amdgcn_cosf(ph), acc_re[k]);
                acc_im[k] = fmaf(m, __builtin_amdgcn_sinf(ph), acc_im[k]);
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
// device math library), plain FP64 accumulation.
template <int ROWS, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) eval_fp64_kernel(EvalGeom g, const Rec64 *__restrict__ rec,
                                                               double2 *__restrict__ partial,
                                                               double2 *__restrict__ out) {
    constexpr int CH = 64;  // records per LDS tile (8 KiB)
    __shared__ Rec64 tile[CH];
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
            const double V0 = r.l[0] + da * (r.l[1] + r.l[3] * da) + db * (ql + r.l[5] * db);
            const double V1 = dy * (ql + 2.0 * r.l[5] * db);
            const double V2 = r.l[5] * dy2;
#pragma unroll
            for (int k = 0; k < ROWS; k++) {
                const double th = T0 + (double)k * (T1 + (double)k * T2);
                const double rr = th - rint(th);
                double s, c;
                sincospi(2.0 * rr, &s, &c);
                const double m = exp(V0 + (double)k * (V1 + (double)k * V2));
                acc_re[k] = fma(m, c, acc_re[k]);
                acc_im[k] = fma(m, s, acc_im[k]);
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

__global__ void __launch_bounds__(256) reduce_mixed_kernel(int64_t M, int32_t nseg, const float4 *__restrict__ part,
                                                           float2 *__restrict__ out) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int s = 0; s < nseg; s++) {
            const float4 v = part[(int64_t)s * M + p];
            re += (double)v.x - (double)v.z;
            im += (double)v.y - (double)v.w;
        }
        out[p] = make_float2((float)re, (float)im);
    }
}

__global__ void __launch_bounds__(256) reduce_fp64_kernel(int64_t M, int32_t nseg, const double2 *__restrict__ part,
                                                          double2 *__restrict__ out) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int s = 0; s < nseg; s++) {
            const double2 v = part[(int64_t)s * M + p];
            re += v.x;
            im += v.y;
        }
        out[p] = make_double2(re, im);
    }
}

template <int ROWS, int WAVES>
hipError_t launch_eval_t(int precision, const EvalGeom &g, const void *rec, void *partial, void *out, hipStream_t s) {
    const int grid = (g.work + 7) / 8 * 8;
    if (precision == 1)
        eval_mixed_kernel<ROWS, WAVES><<<grid, 64 * WAVES, 0, s>>>(g, static_cast<const Rec32 *>(rec),
                                                                   static_cast<float4 *>(partial),
                                                                   static_cast<float2 *>(out));
    else
        eval_fp64_kernel<ROWS, WAVES><<<grid, 64 * WAVES, 0, s>>>(g, static_cast<const Rec64 *>(rec),
                                                                  static_cast<double2 *>(partial),
                                                                  static_cast<double2 *>(out));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_setup(const BeamletsDev &b, const PlaneGeom &pl, double global_turns, Rec64 *r64, Rec32 *r32,
                        uint32_t *status, hipStream_t s) {
    if (b.n == 0) return hipSuccess;
    const int64_t blocks = (b.n + 255) / 256;
    setup_kernel<<<(unsigned)blocks, 256, 0, s>>>(b, pl, global_turns, r64, r32, status);
    return hipGetLastError();
}

hipError_t launch_eval(int precision, int rows, int waves, const EvalGeom &g, const void *rec, void *partial,
                       void *out, hipStream_t s) {
#define GBD_CASE(R, W) \
    if (rows == R && waves == W) return launch_eval_t<R, W>(precision, g, rec, partial, out, s);
    GBD_CASE(1, 1) GBD_CASE(1, 2) GBD_CASE(1, 4)
    GBD_CASE(2, 1) GBD_CASE(2, 2) GBD_CASE(2, 4)
    GBD_CASE(4, 1) GBD_CASE(4, 2) GBD_CASE(4, 4)
    GBD_CASE(8, 1) GBD_CASE(8, 2) GBD_CASE(8, 4)
#undef GBD_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(int precision, const EvalGeom &g, const void *partial, void *out, hipStream_t s) {
    const int64_t M = (int64_t)g.nx * g.ny;
    if (M == 0) return hipSuccess;
    const int64_t blocks = min((M + 255) / 256, (int64_t)4096);
    if (precision == 1)
        reduce_mixed_kernel<<<(unsigned)blocks, 256, 0, s>>>(M, g.nseg, static_cast<const float4 *>(partial),
                                                             static_cast<float2 *>(out));
    else
        reduce_fp64_kernel<<<(unsigned)blocks, 256, 0, s>>>(M, g.nseg, static_cast<const double2 *>(partial),
                                                            static_cast<double2 *>(out));
    return hipGetLastError();
}

}  // namespace gbd
