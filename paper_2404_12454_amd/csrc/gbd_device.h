// Device-side building blocks shared by the single-instance and batched
// kernels: complex FP64 helpers, the per-beamlet FP64 setup, and the mixed
// precision tile accumulation of the N x M evaluation.
#pragma once

#include "gbd_internal.h"

#include <math.h>

namespace gbd {
namespace dev {

constexpr double kPi = 3.14159265358979323846;

struct cd {
    double re, im;
};
__device__ inline cd mk(double r, double i) { return cd{r, i}; }
__device__ inline cd add(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ inline cd sub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ inline cd mul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cd scl(cd a, double s) { return cd{a.re * s, a.im * s}; }
__device__ inline cd cdiv(cd a, cd b) {
    // Smith's algorithm: no overflow for widely scaled operands.
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, d = b.re + b.im * r;
        return cd{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    }
    const double r = b.re / b.im, d = b.re * r + b.im;
    return cd{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
// principal square root (cut on the negative real axis; the sign of a zero
// imaginary part picks the side)
__device__ inline cd csqrt_p(cd z) {
    const double m = hypot(z.re, z.im);
    if (m == 0.0) return cd{0.0, z.im};
    if (z.re >= 0.0) {
        const double t = sqrt(0.5 * (m + z.re));
        return cd{t, z.im / (2.0 * t)};
    }
    const double t = sqrt(0.5 * (m - z.re));
    return cd{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// Eigenvalues admitted on the principal-root branch: the open lower half
// plane and the positive real axis (reached from 1 without crossing the cut).
__device__ inline bool on_branch(cd mu) {
    const double m = hypot(mu.re, mu.im);
    const double tol = 1e-12 * m;
    if (!(m > 0.0)) return false;
    if (mu.im > tol) return false;
    if (mu.im >= -tol && mu.re <= 0.0) return false;
    return true;
}

__device__ inline double il2_dev() { return 1.4426950408889634074; }  // 1 / ln 2

// sigma^(k^2) of the rotor recurrence in FP64 for a beamlet whose row
// quadratic coefficients are p5 (turns / m^2) and l5 (ln amplitude / m^2), on
// rows dy apart: the phase k^2 p5 dy^2 is reduced mod 1 before the
// trigonometry (k^2 integer), the exponent capped so a refused steep grid
// still gives finite values.  Rounded, it is the mixed rotor form's FP32
// table; both tables are computed from the FP64 records when a rotor form
// runs (the batched setup fills the FP32 one itself).
__device__ inline double2 rotor_sigma(double p5, double l5, double dy, int k) {
    const double t2 = p5 * dy * dy;
    const double u2 = l5 * il2_dev() * dy * dy;
    const double kk = (double)(k * k);
    double ph = kk * t2;
    ph -= rint(ph);
    double sn, cs;
    sincospi(2.0 * ph, &sn, &cs);
    const double g = exp2(fmin(kk * u2, 64.0));
    return make_double2(g * cs, g * sn);
}

// One beamlet propagated onto the plane; writes its phasor records (either
// pointer may be null) and returns FLAG_* bits (0 = fine).
// Higher-order beamlets: h64 / h32 (either may be null) receive the
// Hermite-Gaussian factor's coefficients of every beamlet (orders (0, 0)
// give the factor 1).  Truncated beamlets (j >= n - n_cut): c64 / c32
// receive the truncation factor's coefficients at j - (n - n_cut); their
// FLAG_STEEP / FLAG_CROSS are not reported (they are evaluated by the
// direct form of their own kernel).
// log2 of the largest modulus of a separable factor's envelope 2^(c1 d + c2 d^2)
// over the pixel offsets d_k = d0 + k step, k = 0 .. n-1, of one grid axis:
// the lattice points at both ends and, for a decaying envelope, the two next
// to its vertex (a grid that misses the spot must not be bounded by the spot)
__device__ inline double log2_envelope_max(double c1, double c2, double d0, double step, int n) {
    if (n <= 0) return 0.0;
    auto f = [&](int k) {
        const double d = d0 + k * step;
        return c1 * d + c2 * d * d;
    };
    double m = fmax(f(0), f(n - 1));
    if (c2 < 0.0 && n > 2) {
        const double kv = fmin(fmax((-c1 / (2.0 * c2) - d0) / step, 0.0), (double)(n - 1));
        const int k = (int)floor(kv);
        m = fmax(m, fmax(f(k), f(k + 1 < n ? k + 1 : k)));
    }
    return m;
}

// The same bound for an envelope times a higher-order axis polynomial
// |c0 + c1 g + c2 g^2|, g = G d (|G| = ga, |c0| = a0c, |c1| = a1, |c2| = a2):
// |P| <= Pm(|d|) = a0c + a1 ga |d| + a2 ga^2 d^2, increasing in |d|.  Where
// the envelope decays, beyond 8 / sqrt(-c2) of its vertex it lies 64 bits
// below its largest value on the lattice (env), so the bound is the larger of
// env + log2 Pm(|vertex| + 8 / sqrt(-c2)) and env - 64 + log2 Pm(T), T the
// largest |d| on the lattice; otherwise env + log2 Pm(T).
__device__ inline double log2_hg_envelope_max(double c1, double c2, double d0, double step, int n, double a0c,
                                              double a1, double a2, double ga) {
    const double env = log2_envelope_max(c1, c2, d0, step, n);
    if (n <= 0) return env;
    auto pm = [&](double r) { return log2(a0c + a1 * ga * r + a2 * ga * ga * r * r); };
    const double T = fmax(fabs(d0), fabs(d0 + (n - 1) * step));
    if (!(c2 < 0.0)) return env + pm(T);
    const double R = fmin(T, fabs(-c1 / (2.0 * c2)) + 8.0 / sqrt(-c2));
    return fmax(env + pm(R), env - 64.0 + pm(T));
}

// sep_peak (optional): log2 of the largest modulus of the beamlet's term over
// the grid, U's part of it stored in the Rec32 record (pad) for the FP16
// separable form's range balancing; -inf for a beamlet that contributes nothing.
// l5_out and r32_copy (optional): the FP64 ln-amplitude curvature l5 (with
// p5 of the record, the source of the rotor tables when a later pass fills
// them) and a copy of the finished Rec32 record.
__device__ inline uint32_t setup_one(const BeamletsDev &b, const PlaneGeom &pl, double gturns, int64_t j,
                                     Rec64 *r64, Rec32 *r32, RecHG64 *h64 = nullptr, RecHG32 *h32 = nullptr,
                                     RecCut64 *c64 = nullptr, RecCut32 *c32 = nullptr, bool sigma32 = true,
                                     float *sep_peak = nullptr, double *l5_out = nullptr,
                                     Rec32 *r32_copy = nullptr) {
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

    // base ray at the ABCD output plane (Appendix A, ab/cd laws), or the
    // traced one of ray-traced inputs
    double r2M[2], th[2];
    const double *tb = b.base ? b.base + 5 * j : nullptr;
#pragma unroll
    for (int r = 0; r < 2; r++) {
        if (tb) {
            r2M[r] = tb[r];
            th[r] = tb[2 + r];
        } else {
            r2M[r] = A[r][0] * r1[0] + A[r][1] * r1[1] + B[r][0] * t1[0] + B[r][1] * t1[1];
            th[r] = C[r][0] * r1[0] + C[r][1] * r1[1] + D[r][0] * t1[0] + D[r][1] * t1[1];
        }
    }
    // where the base ray (r2M + z th, z) meets the plane
    const double nd = pl.n[0] * th[0] + pl.n[1] * th[1] + pl.n[2];
    const double dl = sqrt(th[0] * th[0] + th[1] * th[1] + 1.0);
    Rec64 o64 = {};
    Rec32 o32 = {};
    RecHG64 oh = {};
    RecCut64 oc = {};
    const int64_t cut0 = b.n - b.n_cut;
    const bool is_cut = b.edge && j >= cut0;
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
        // complex-curvature law Q^-1 = Nm Mm^-1 (closed-form 2x2 inverse), symmetrised
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

        // misalignment phase at the hit point, in turns (l0 handled by the
        // host): Euler's relation for the eikonal, or the traced optical path
        // plus the free-space extension
        const double r2[2] = {r2M[0] + z * th[0], r2M[1] + z * th[1]};
        const double S = tb ? tb[4] + 0.5 * z * (th[0] * th[0] + th[1] * th[1])
                            : 0.5 * (th[0] * r2[0] + th[1] * r2[1] - t1[0] * r1[0] - t1[1] * r1[1]);
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
        double p[6], l[6];
        const cd ag = mul(amp, gamma);
        const double tred = tau - rint(tau);
        const double p0 = atan2(ag.im, ag.re) / (2.0 * kPi) - tred - gturns;
        // phase polynomial (turns)
        p[0] = p0 - rint(p0);
        p[1] = -lin[0] / lam - trQ.im * ez[0] * i4pi;
        p[2] = -lin[1] / lam - trQ.im * ez[1] * i4pi;
        p[3] = -G[0][0].re / (2.0 * lam) + trQ2.im * ez[0] * ez[0] * i8pi;
        p[4] = 2.0 * (-G[0][1].re / (2.0 * lam) + trQ2.im * ez[0] * ez[1] * i8pi);
        p[5] = -G[1][1].re / (2.0 * lam) + trQ2.im * ez[1] * ez[1] * i8pi;
        // log-amplitude polynomial (natural log)
        l[0] = log(hypot(ag.re, ag.im));
        l[1] = -0.5 * trQ.re * ez[0];
        l[2] = -0.5 * trQ.re * ez[1];
        l[3] = kh * G[0][0].im + 0.25 * trQ2.re * ez[0] * ez[0];
        l[4] = 2.0 * (kh * G[0][1].im + 0.25 * trQ2.re * ez[0] * ez[1]);
        l[5] = kh * G[1][1].im + 0.25 * trQ2.re * ez[1] * ez[1];
        bool fin = isfinite(arho) && isfinite(brho) && isfinite(ag.re) && isfinite(ag.im);
        // higher-order factors' coefficient moduli (x: |cx0|, |cx1|, |cx2|, |g_xx|; y likewise)
        double hgb[8] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0};
        bool has_hgb = false;
#pragma unroll
        for (int i = 0; i < 6; i++) fin = fin && isfinite(p[i]) && (i == 0 || isfinite(l[i]));
        if (h64 || h32) {
            // elegant Hermite-Gaussian factor: with A' = A + z C, the
            // derivatives of the envelope's log E with respect to the input
            // centre are L w (L = -i k (C^T - A'^T Q)) and the constant
            // H = i k (C^T A' - A'^T Q A'); on the plane w = Pm d, so
            // g = w0 L Pm d and h = w0^2 H
            const int hm = b.order ? b.order[2 * j] : 0, hn = b.order ? b.order[2 * j + 1] : 0;
            const double k = 2.0 * kPi / lam, w2 = w0 * w0;
            double Ap[2][2];
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int c = 0; c < 2; c++) Ap[r][c] = A[r][c] + z * C[r][c];
            cd AQ[2][2], Lm[2][2], Hm[2][2];  // A'^T Q, L, H
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int c = 0; c < 2; c++) AQ[r][c] = add(scl(Q[0][c], Ap[0][r]), scl(Q[1][c], Ap[1][r]));
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    const cd v = sub(mk(C[c][r], 0.0), AQ[r][c]);
                    Lm[r][c] = mk(k * v.im, -k * v.re);
                    const cd u = sub(mk(C[0][r] * Ap[0][c] + C[1][r] * Ap[1][c], 0.0),
                                     add(scl(AQ[r][0], Ap[0][c]), scl(AQ[r][1], Ap[1][c])));
                    Hm[r][c] = mk(-k * u.im, k * u.re);
                }
            cd Gh[2][2];
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    Gh[r][c] = scl(add(scl(Lm[r][0], Pm[0][c]), scl(Lm[r][1], Pm[1][c])), w0);
                    oh.g[r][c][0] = Gh[r][c].re;
                    oh.g[r][c][1] = Gh[r][c].im;
                }
            const cd hxx = scl(Hm[0][0], w2), hyy = scl(Hm[1][1], w2);
            const cd hxy = scl(add(Hm[0][1], Hm[1][0]), 0.5 * w2);
            oh.cx0[0] = hm == 0 ? 1.0 : hm == 2 ? hxx.re : 0.0;
            oh.cx0[1] = hm == 2 ? hxx.im : 0.0;
            oh.cy0[0] = hn == 0 ? 1.0 : hn == 2 ? hyy.re : 0.0;
            oh.cy0[1] = hn == 2 ? hyy.im : 0.0;
            oh.cx1 = hm == 1 ? 1.0 : 0.0;
            oh.cx2 = hm == 2 ? 1.0 : 0.0;
            oh.cy1 = hn == 1 ? 1.0 : 0.0;
            oh.cy2 = hn == 2 ? 1.0 : 0.0;
            oh.ex0 = hm == 2 ? 0.0 : 1.0;
            oh.ex1 = hm == 2 ? 1.0 : 0.0;
            oh.ey0 = hn == 2 ? 0.0 : 1.0;
            oh.ey1 = hn == 2 ? 1.0 : 0.0;
            hgb[0] = hypot(oh.cx0[0], oh.cx0[1]);
            hgb[1] = fabs(oh.cx1);
            hgb[2] = fabs(oh.cx2);
            hgb[3] = hypot(Gh[0][0].re, Gh[0][0].im);
            hgb[4] = hypot(oh.cy0[0], oh.cy0[1]);
            hgb[5] = fabs(oh.cy1);
            hgb[6] = fabs(oh.cy2);
            hgb[7] = hypot(Gh[1][1].re, Gh[1][1].im);
            has_hgb = true;
            const cd k1 = scl(hxy, (double)(hm * hn));
            const cd k0 = (hm == 2 && hn == 2) ? scl(mul(hxy, hxy), 2.0) : mk(0.0, 0.0);
            oh.k1[0] = k1.re;
            oh.k1[1] = k1.im;
            oh.k0[0] = k0.re;
            oh.k0[1] = k0.im;
            if (hm | hn) {
                flag |= FLAG_HG;
                if (ez[0] != 0.0 || ez[1] != 0.0) flag |= FLAG_HG_TILT;
                const bool off = (hm && (Gh[0][1].re != 0.0 || Gh[0][1].im != 0.0)) ||
                                 (hn && (Gh[1][0].re != 0.0 || Gh[1][0].im != 0.0));
                if (off || k1.re != 0.0 || k1.im != 0.0) flag |= FLAG_CROSS;
            }
            const double *hv = &oh.g[0][0][0];
            for (int i = 0; i < (int)(sizeof(RecHG64) / sizeof(double)); i++) fin = fin && isfinite(hv[i]);
        }
        if (is_cut) {
            // truncation by the edge e . r <= t: with B' = B + z D the envelope's
            // slope derivatives are lt = D^T - B'^T Q and ht = D^T B' - B'^T Q B';
            // zeta = (e . c - t + e^T lt w) / sqrt(-2 i e^T ht e / k), w = Pm d
            const double *ed = b.edge + 3 * j;
            const double e[2] = {ed[0], ed[1]};
            const double k = 2.0 * kPi / lam;
            double Bp[2][2];
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int c = 0; c < 2; c++) Bp[r][c] = B[r][c] + z * D[r][c];
            cd lt[2][2], ht[2][2];
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    // (B'^T Q)_rc and (B'^T Q B')_rc
                    const cd bq = add(scl(Q[0][c], Bp[0][r]), scl(Q[1][c], Bp[1][r]));
                    lt[r][c] = sub(mk(D[c][r], 0.0), bq);
                    cd bqb = mk(0.0, 0.0);
#pragma unroll
                    for (int t = 0; t < 2; t++)
                        bqb = add(bqb, scl(add(scl(Q[0][t], Bp[0][r]), scl(Q[1][t], Bp[1][r])), Bp[t][c]));
                    ht[r][c] = sub(mk(D[0][r] * Bp[0][c] + D[1][r] * Bp[1][c], 0.0), bqb);
                }
            cd q = mk(0.0, 0.0);
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int c = 0; c < 2; c++) q = add(q, scl(ht[r][c], e[r] * e[c]));
            const cd sq = csqrt_p(mk(2.0 * q.im / k, -2.0 * q.re / k));
            const cd n0 = mk(e[0] * r1[0] + e[1] * r1[1] - ed[2], 0.0);
            cd na = mk(0.0, 0.0), nb = mk(0.0, 0.0);
#pragma unroll
            for (int r = 0; r < 2; r++)
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    na = add(na, scl(lt[r][c], e[r] * Pm[c][0]));
                    nb = add(nb, scl(lt[r][c], e[r] * Pm[c][1]));
                }
            const cd z0 = cdiv(n0, sq), za = cdiv(na, sq), zb = cdiv(nb, sq);
            oc.z0[0] = z0.re;
            oc.z0[1] = z0.im;
            oc.za[0] = za.re;
            oc.za[1] = za.im;
            oc.zb[0] = zb.re;
            oc.zb[1] = zb.im;
            for (int i = 0; i < 6; i++) fin = fin && isfinite((&oc.z0[0])[i]);
            if (ez[0] != 0.0 || ez[1] != 0.0) flag |= FLAG_HG_TILT;
        }
        if (!fin) flag |= FLAG_NONFINITE;
        if (!is_cut && fabs(l[5]) * il2_dev() * pl.dy * pl.dy > kStepCurvature) flag |= FLAG_STEEP;
        if (!is_cut && (p[4] != 0.0 || l[4] != 0.0)) flag |= FLAG_CROSS;
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
        // row-step terms of the stepped kernel (k^2 t2 with k integer: reduce mod 1)
        const double t2 = p[5] * pl.dy * pl.dy;
        o32.t2 = (float)(t2 - rint(t2));
        const float dyf = (float)pl.dy;
        o32.u2 = o32.m[5] * (dyf * dyf);
        o32.s2 = exp2f(fminf(2.0f * o32.u2, 1.0f));
        {
            // separable factors' moduli over the grid: |U| <= 2^umax, |V| <= 2^vmax
            const double a0 = -0.5 * (pl.nx - 1) * pl.dx, b0 = -0.5 * (pl.ny - 1) * pl.dy;
            // (with a higher-order factor, times its axis polynomial's bound)
            const double umax =
                (double)o32.m[0] +
                (has_hgb ? log2_hg_envelope_max(o32.m[1], o32.m[3], a0 - arho, pl.dx, pl.nx, hgb[0], hgb[1], hgb[2],
                                                hgb[3])
                         : log2_envelope_max(o32.m[1], o32.m[3], a0 - arho, pl.dx, pl.nx));
            const double vmax = has_hgb ? log2_hg_envelope_max(o32.m[2], o32.m[5], b0 - brho, pl.dy, pl.ny, hgb[4],
                                                               hgb[5], hgb[6], hgb[7])
                                        : log2_envelope_max(o32.m[2], o32.m[5], b0 - brho, pl.dy, pl.ny);
            const bool ok = isfinite(umax) && isfinite(vmax);
            o32.pad = ok ? (float)umax : 0.0f;
            if (sep_peak) *sep_peak = ok ? (float)(umax + vmax) : -INFINITY;
        }
        // rotor form: sigma^(k^2), rounded from FP64 (else left to
        // sigma32_kernel, run only before a rotor-form evaluation)
        if (sigma32) {
#pragma unroll
            for (int k = 1; k <= kRotorRows; k++) {
                const double2 sq = rotor_sigma(p[5], l[5], pl.dy, k);
                o32.sq[k - 1][0] = (float)sq.x;
                o32.sq[k - 1][1] = (float)sq.y;
            }
        }
    }
    if (flag & FLAG_ERRORS) {
        // a refused beamlet contributes nothing (the host refuses the call anyway)
        o64.l[0] = -INFINITY;
        o32.m[0] = -INFINITY;
    }
    if (l5_out) *l5_out = o64.l[5];
    if (r32_copy) *r32_copy = o32;
    if (r64) r64[j] = o64;
    if (r32) {
        if (sigma32) {
            r32[j] = o32;
        } else {
            // the rotor tables are left to launch_sigma, run before every
            // rotor-form evaluation: the record's first 112 bytes only
            static_assert(offsetof(Rec32, sq) == 112, "Rec32 layout");
            const uint4 *src = reinterpret_cast<const uint4 *>(&o32);
            uint4 *dst = reinterpret_cast<uint4 *>(r32 + j);
#pragma unroll
            for (int k = 0; k < 7; k++) dst[k] = src[k];
        }
    }
    if (is_cut && c64) c64[j - cut0] = oc;
    if (is_cut && c32) {
        RecCut32 o;
#pragma unroll
        for (int i = 0; i < 2; i++) {
            o.z0[i] = (float)oc.z0[i];
            o.za[i] = (float)oc.za[i];
            o.zb[i] = (float)oc.zb[i];
            o.pad[i] = 0.0f;
        }
        c32[j - cut0] = o;
    }
    if (h64) h64[j] = oh;
    if (h32) {
        RecHG32 o;
        const double *src = &oh.g[0][0][0];
        float *dst = &o.g[0][0][0];
#pragma unroll
        for (int i = 0; i < (int)(sizeof(RecHG32) / sizeof(float)); i++) dst[i] = (float)src[i];
        h32[j] = o;
    }
    return flag;
}

// Hermite-Gaussian factor P (the polynomial of RecHG64) at the pixel offset
// (da, db), FP64.
__device__ inline cd hg_factor(const RecHG64 &h, double da, double db) {
    const cd gx = mk(h.g[0][0][0] * da + h.g[0][1][0] * db, h.g[0][0][1] * da + h.g[0][1][1] * db);
    const cd gy = mk(h.g[1][0][0] * da + h.g[1][1][0] * db, h.g[1][0][1] * da + h.g[1][1][1] * db);
    const cd px = add(mk(h.cx0[0], h.cx0[1]), mul(gx, mk(h.cx1 + h.cx2 * gx.re, h.cx2 * gx.im)));
    const cd py = add(mk(h.cy0[0], h.cy0[1]), mul(gy, mk(h.cy1 + h.cy2 * gy.re, h.cy2 * gy.im)));
    const cd ax = mk(h.ex0 + h.ex1 * gx.re, h.ex1 * gx.im);
    const cd ay = mk(h.ey0 + h.ey1 * gy.re, h.ey1 * gy.im);
    return add(add(mul(px, py), mul(mk(h.k1[0], h.k1[1]), mul(ax, ay))), mk(h.k0[0], h.k0[1]));
}

// The same factor in FP32 with the x part of g = G d already formed for the
// lane's column (gxa = G[.][0] da): only the row offset db varies.
__device__ inline float2 hg_factor32(const RecHG32 &h, float gxa_r, float gxa_i, float gya_r, float gya_i, float db) {
    const float gxr = fmaf(h.g[0][1][0], db, gxa_r), gxi = fmaf(h.g[0][1][1], db, gxa_i);
    const float gyr = fmaf(h.g[1][1][0], db, gya_r), gyi = fmaf(h.g[1][1][1], db, gya_i);
    // Px = cx0 + gx (cx1 + cx2 gx), likewise Py
    const float txr = fmaf(h.cx2, gxr, h.cx1), txi = h.cx2 * gxi;
    const float pxr = h.cx0[0] + (gxr * txr - gxi * txi), pxi = h.cx0[1] + (gxr * txi + gxi * txr);
    const float tyr = fmaf(h.cy2, gyr, h.cy1), tyi = h.cy2 * gyi;
    const float pyr = h.cy0[0] + (gyr * tyr - gyi * tyi), pyi = h.cy0[1] + (gyr * tyi + gyi * tyr);
    const float axr = fmaf(h.ex1, gxr, h.ex0), axi = h.ex1 * gxi;
    const float ayr = fmaf(h.ey1, gyr, h.ey0), ayi = h.ey1 * gyi;
    const float cr = axr * ayr - axi * ayi, ci = axr * ayi + axi * ayr;
    const float re = (pxr * pyr - pxi * pyi) + (h.k1[0] * cr - h.k1[1] * ci) + h.k0[0];
    const float im = (pxr * pyi + pxi * pyr) + (h.k1[0] * ci + h.k1[1] * cr) + h.k0[1];
    return make_float2(re, im);
}

// FP64 exponentials without the special-case paths a general library exp and
// sincospi carry (their arguments here are bounded), each within a few units
// in the last place:
// exp_cw64(g) = e^g by Cody and Waite's reduction g = n ln 2 + r, ln 2 split
// into a head of 32 significant bits (n ln2_hi exact for |n| < 2^21) and a
// tail, |r| <= ln 2 / 2, e^r by its Taylor series to r^12 (truncation below
// 2e-16 relative), scaled by 2^n; g is clamped at -1100, where the result is
// zero anyway, so that g = -inf (a masked term) gives 0, not NaN.
__device__ inline double exp_cw64(double g) {
    g = fmax(g, -1100.0);
    const double n = rint(g * 1.4426950408889634);                  // 1 / ln 2
    double r = fma(-n, 0.6931471806019545, g);                      // ln 2, head
    r = fma(-n, -4.2009150726810846e-11, r);                         // ln 2, tail
    double e = 1.0 / 479001600.0;                                    // 1 / 12!
    e = fma(e, r, 1.0 / 39916800.0);
    e = fma(e, r, 1.0 / 3628800.0);
    e = fma(e, r, 1.0 / 362880.0);
    e = fma(e, r, 1.0 / 40320.0);
    e = fma(e, r, 1.0 / 5040.0);
    e = fma(e, r, 1.0 / 720.0);
    e = fma(e, r, 1.0 / 120.0);
    e = fma(e, r, 1.0 / 24.0);
    e = fma(e, r, 1.0 / 6.0);
    e = fma(e, r, 0.5);
    e = fma(e, r, 1.0);
    e = fma(e, r, 1.0);
    return ldexp(e, (int)n);
}

// (cos 2 pi T, sin 2 pi T) for T in [-1/2, 1/2] turns: q = round(4 T) quarter
// turns, r = T - q / 4 in [-1/8, 1/8], theta = 2 pi r in [-pi/4, pi/4], sin and
// cos of theta by their Taylor series to theta^15 and theta^16 (truncation
// below 1e-16 relative), then turned by q quarter turns.
__device__ inline double2 cis_turns64(double T) {
    const double q = rint(4.0 * T);
    const double th = (T - 0.25 * q) * 6.283185307179586;           // 2 pi
    const double z = th * th;
    double sp = -1.0 / 1307674368000.0;                              // -1 / 15!
    sp = fma(sp, z, 1.0 / 6227020800.0);
    sp = fma(sp, z, -1.0 / 39916800.0);
    sp = fma(sp, z, 1.0 / 362880.0);
    sp = fma(sp, z, -1.0 / 5040.0);
    sp = fma(sp, z, 1.0 / 120.0);
    sp = fma(sp, z, -1.0 / 6.0);
    const double sn = fma(th * z, sp, th);
    double cp = 1.0 / 20922789888000.0;                              // 1 / 16!
    cp = fma(cp, z, -1.0 / 87178291200.0);
    cp = fma(cp, z, 1.0 / 479001600.0);
    cp = fma(cp, z, -1.0 / 3628800.0);
    cp = fma(cp, z, 1.0 / 40320.0);
    cp = fma(cp, z, -1.0 / 720.0);
    cp = fma(cp, z, 1.0 / 24.0);
    cp = fma(cp, z, -0.5);
    const double cs = fma(z, cp, 1.0);
    // turn (cs, sn) by q quarter turns: i^q
    const int qi = (int)q & 3;
    double c = (qi & 1) ? sn : cs, s = (qi & 1) ? cs : sn;
    c = (qi == 1 || qi == 2) ? -c : c;
    s = (qi & 2) ? -s : s;
    return make_double2(c, s);
}

// e^g (cos 2 pi T, sin 2 pi T), T in [-1/2, 1/2]
__device__ inline double2 cexp_turns64(double g, double T) {
    const double m = exp_cw64(g);
    const double2 cs = cis_turns64(T);
    return make_double2(m * cs.x, m * cs.y);
}

// fused multiply-add in the precision of its arguments
__device__ inline float fm(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fm(double a, double b, double c) { return fma(a, b, c); }

// The Hermite-Gaussian factor along a lane's column as a polynomial in the
// row step k from the anchor row (plane offsets da, db there, row pitch dy):
// gx = ax + k sx, gy = ay + k sy with ax = G[0][0] da + G[0][1] db,
// sx = G[0][1] dy (likewise y); Px, Py are quadratics and ax, ay linear in
// k, so P = Px Py + k1 ax ay + k0 has degree <= 4.  q[i] = (re, im) of the
// coefficient of k^i (T float with RecHG32 records, double with RecHG64).
template <typename T, typename RecHG>
__device__ inline void hg_row_poly(const RecHG &h, T da, T db, T dy, T (&q)[5][2]) {
    const T axr = fm(h.g[0][1][0], db, h.g[0][0][0] * da), axi = fm(h.g[0][1][1], db, h.g[0][0][1] * da);
    const T ayr = fm(h.g[1][1][0], db, h.g[1][0][0] * da), ayi = fm(h.g[1][1][1], db, h.g[1][0][1] * da);
    const T sxr = h.g[0][1][0] * dy, sxi = h.g[0][1][1] * dy;
    const T syr = h.g[1][1][0] * dy, syi = h.g[1][1][1] * dy;
    // Px = cx0 + cx1 g + cx2 g^2 at g = a + s k:
    //   px0 = cx0 + a (cx1 + cx2 a), px1 = s (cx1 + 2 cx2 a), px2 = cx2 s^2
    auto quad = [](T c0r, T c0i, T c1, T c2, T ar, T ai, T sr, T si, T (&p)[3][2]) {
        const T tr = fm(c2, ar, c1), ti = c2 * ai;
        p[0][0] = c0r + (ar * tr - ai * ti);
        p[0][1] = c0i + (ar * ti + ai * tr);
        const T ur = fm(T(2) * c2, ar, c1), ui = T(2) * c2 * ai;
        p[1][0] = sr * ur - si * ui;
        p[1][1] = sr * ui + si * ur;
        p[2][0] = c2 * (sr * sr - si * si);
        p[2][1] = c2 * (T(2) * sr * si);
    };
    T px[3][2], py[3][2];
    quad(h.cx0[0], h.cx0[1], h.cx1, h.cx2, axr, axi, sxr, sxi, px);
    quad(h.cy0[0], h.cy0[1], h.cy1, h.cy2, ayr, ayi, syr, syi, py);
    // Px Py (product of quadratics)
#pragma unroll
    for (int i = 0; i < 5; i++) q[i][0] = q[i][1] = T(0);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            q[i + j][0] += px[i][0] * py[j][0] - px[i][1] * py[j][1];
            q[i + j][1] += px[i][0] * py[j][1] + px[i][1] * py[j][0];
        }
    // k1 ax ay + k0, ax = (ex0 + ex1 a) + ex1 s k
    const T x0r = fm(h.ex1, axr, h.ex0), x0i = h.ex1 * axi, x1r = h.ex1 * sxr, x1i = h.ex1 * sxi;
    const T y0r = fm(h.ey1, ayr, h.ey0), y0i = h.ey1 * ayi, y1r = h.ey1 * syr, y1i = h.ey1 * syi;
    const T m0r = x0r * y0r - x0i * y0i, m0i = x0r * y0i + x0i * y0r;
    const T m1r = (x0r * y1r - x0i * y1i) + (x1r * y0r - x1i * y0i);
    const T m1i = (x0r * y1i + x0i * y1r) + (x1r * y0i + x1i * y0r);
    const T m2r = x1r * y1r - x1i * y1i, m2i = x1r * y1i + x1i * y1r;
    const T kr = h.k1[0], ki = h.k1[1];
    q[0][0] += (kr * m0r - ki * m0i) + h.k0[0];
    q[0][1] += (kr * m0i + ki * m0r) + h.k0[1];
    q[1][0] += kr * m1r - ki * m1i;
    q[1][1] += kr * m1i + ki * m1r;
    q[2][0] += kr * m2r - ki * m2i;
    q[2][1] += kr * m2i + ki * m2r;
}

// q0 + k (q1 + k (q2 + k (q3 + k q4))) for real k, as (re, im).
template <typename T>
__device__ inline void horner4(const T (&q)[5][2], T k, T &re_out, T &im_out) {
    T re = fm(q[4][0], k, q[3][0]), im = fm(q[4][1], k, q[3][1]);
    re = fm(re, k, q[2][0]);
    im = fm(im, k, q[2][1]);
    re = fm(re, k, q[1][0]);
    im = fm(im, k, q[1][1]);
    re_out = fm(re, k, q[0][0]);
    im_out = fm(im, k, q[0][1]);
}

__device__ inline void kahan(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

constexpr int kMixedTile = 128;  // Rec32 records staged per LDS tile (30 KiB)

// Mixed-precision sum over beamlets [jb, je) of the ROWS pixels a lane owns:
// pixel k of the lane sits at plane coordinates (a, b0 + k dy).  The FP64
// phase along the lane's column is a quadratic in k, reduced to turns with
// fract and converted to FP32; the log2-amplitude is an FP32 quadratic in the
// pixel's own row offset; v_exp_f32 computes 2^x and v_sin_f32 / v_cos_f32
// take revolutions.  Per-tile FP32 sums are folded into Kahan-compensated
// (s, c) accumulators, value = s - c.  All threads of the workgroup must call
// this together (it synchronises on the LDS tile).
// With HG, each beamlet's phasor is multiplied by its Hermite-Gaussian
// factor (records hg, staged in htile beside the phasor records).
template <int ROWS, int NT, bool HG = false>
__device__ inline void mixed_accumulate(Rec32 *tile, const Rec32 *__restrict__ rec, int64_t jb, int64_t je,
                                        double a, double b0, double dy, float (&s_re)[ROWS], float (&s_im)[ROWS],
                                        float (&c_re)[ROWS], float (&c_im)[ROWS], RecHG32 *htile = nullptr,
                                        const RecHG32 *__restrict__ hg = nullptr) {
    const double dy2 = dy * dy;
    const float af = (float)a, b0f = (float)b0, dyf = (float)dy;
    float acc_re[ROWS], acc_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) acc_re[k] = acc_im[k] = 0.0f;
    for (int64_t j0 = jb; j0 < je; j0 += kMixedTile) {
        const int cnt = (int)min((int64_t)kMixedTile, je - j0);
        __syncthreads();
        {
            const float4 *src = reinterpret_cast<const float4 *>(rec + j0);
            float4 *dst = reinterpret_cast<float4 *>(tile);
            for (int i = threadIdx.x; i < cnt * kRec32Vec4; i += NT) dst[i] = src[i];
            if constexpr (HG) {
                const float4 *hs = reinterpret_cast<const float4 *>(hg + j0);
                float4 *hd = reinterpret_cast<float4 *>(htile);
                for (int i = threadIdx.x; i < cnt * (int)(sizeof(RecHG32) / 16); i += NT) hd[i] = hs[i];
            }
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; jj++) {
            const Rec32 &r = tile[jj];
            const double da = a - r.arho, db = b0 - r.brho;
            const double q = r.p[2] + r.p[4] * da;
            const double T0 = r.p[0] + da * (r.p[1] + r.p[3] * da) + db * (q + r.p[5] * db);
            const double T1 = dy * (q + 2.0 * r.p[5] * db);
            const double T2 = r.p[5] * dy2;
            // log2-amplitude from each pixel's own row offset (an expansion
            // in k would cancel catastrophically far from the spot)
            const float daf = af - r.arho_f, dbf0 = b0f - r.brho_f;
            const float qf = r.m[2] + r.m[4] * daf;
            const float Uc = r.m[0] + daf * (r.m[1] + r.m[3] * daf);
            float gxa_r = 0.0f, gxa_i = 0.0f, gya_r = 0.0f, gya_i = 0.0f;
            if constexpr (HG) {
                const RecHG32 &h = htile[jj];
                gxa_r = h.g[0][0][0] * daf;
                gxa_i = h.g[0][0][1] * daf;
                gya_r = h.g[1][0][0] * daf;
                gya_i = h.g[1][0][1] * daf;
            }
#pragma unroll
            for (int k = 0; k < ROWS; k++) {
                const double th = T0 + (double)k * (T1 + (double)k * T2);
                const float ph = (float)__builtin_amdgcn_fract(th);
                const float dbf = fmaf((float)k, dyf, dbf0);
                const float L = Uc + dbf * (qf + r.m[5] * dbf);
                const float m = __builtin_amdgcn_exp2f(L);
                if constexpr (HG) {
                    const float cr = m * __builtin_amdgcn_cosf(ph), ci = m * __builtin_amdgcn_sinf(ph);
                    const float2 P = hg_factor32(htile[jj], gxa_r, gxa_i, gya_r, gya_i, dbf);
                    acc_re[k] += cr * P.x - ci * P.y;
                    acc_im[k] += cr * P.y + ci * P.x;
                } else {
                    acc_re[k] = fmaf(m, __builtin_amdgcn_cosf(ph), acc_re[k]);
                    acc_im[k] = fmaf(m, __builtin_amdgcn_sinf(ph), acc_im[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ROWS; k++) {
            kahan(s_re[k], c_re[k], acc_re[k]);
            kahan(s_im[k], c_im[k], acc_im[k]);
            acc_re[k] = acc_im[k] = 0.0f;
        }
    }
}

// Faster mixed form for well-sampled grids.  Per (lane, beamlet) the FP64
// phase at the lane's first row is reduced to turns; the row-step terms T1,
// T2 enter as k T1 + k^2 T2 with k integer, so they are reduced modulo 1 in
// FP64 without changing the phase mod 1, and the in-column phase is formed
// in FP32 (v_sin / v_cos take revolutions, no further reduction needed).  The
// amplitude 2^(L0 + k U1 + k^2 U2) is stepped by two multiplications per row;
// the setup kernel flags (FLAG_STEEP) grids where |U2| > kStepCurvature and
// the host then uses mixed_accumulate instead.
template <int ROWS, int NT>
__device__ inline void mixed_accumulate_step(Rec32 *tile, const Rec32 *__restrict__ rec, int64_t jb, int64_t je,
                                             double a, double b0, double dy, float (&s_re)[ROWS],
                                             float (&s_im)[ROWS], float (&c_re)[ROWS], float (&c_im)[ROWS]) {
    const float af = (float)a, b0f = (float)b0, dyf = (float)dy;
    float acc_re[ROWS], acc_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) acc_re[k] = acc_im[k] = 0.0f;
    for (int64_t j0 = jb; j0 < je; j0 += kMixedTile) {
        const int cnt = (int)min((int64_t)kMixedTile, je - j0);
        __syncthreads();
        {
            const float4 *src = reinterpret_cast<const float4 *>(rec + j0);
            float4 *dst = reinterpret_cast<float4 *>(tile);
            for (int i = threadIdx.x; i < cnt * kRec32Vec4; i += NT) dst[i] = src[i];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; jj++) {
            const Rec32 &r = tile[jj];
            const double da = a - r.arho, db = b0 - r.brho;
            const double q = r.p[2] + r.p[4] * da;
            const double T0 = r.p[0] + da * (r.p[1] + r.p[3] * da) + db * (q + r.p[5] * db);
            const double T1 = dy * (q + 2.0 * r.p[5] * db);
            const float base = (float)__builtin_amdgcn_fract(T0);
            const float t1 = (float)(T1 - rint(T1));
            const float t2 = r.t2;
            const float daf = af - r.arho_f, dbf = b0f - r.brho_f;
            const float qf = r.m[2] + r.m[4] * daf;
            const float L0 = r.m[0] + daf * (r.m[1] + r.m[3] * daf) + dbf * (qf + r.m[5] * dbf);
            const float U1 = dyf * (qf + 2.0f * r.m[5] * dbf);
            // clamps only act where the amplitude is already below 2^-126
            float m = __builtin_amdgcn_exp2f(L0);
            float rat = __builtin_amdgcn_exp2f(fminf(U1 + r.u2, 64.0f));
            const float s2 = r.s2;
#pragma unroll
            for (int k = 0; k < ROWS; k++) {
                const float ph = (k == 0) ? base : fmaf((float)k, fmaf((float)k, t2, t1), base);
                acc_re[k] = fmaf(m, __builtin_amdgcn_cosf(ph), acc_re[k]);
                acc_im[k] = fmaf(m, __builtin_amdgcn_sinf(ph), acc_im[k]);
                if (k + 1 < ROWS) {
                    m *= rat;
                    rat *= s2;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ROWS; k++) {
            kahan(s_re[k], c_re[k], acc_re[k]);
            kahan(s_im[k], c_im[k], acc_im[k]);
            acc_re[k] = acc_im[k] = 0.0f;
        }
    }
}

// Rotor form for well-sampled grids.  Along a lane's column one beamlet's
// phasor is the exponential of a quadratic in the row index; about the
// lane's middle row h it factors as
//   E(h + k) = E(h) rho^k sigma^(k^2),
// rho = 2^U1 e^(2 pi i t1) per (lane, beamlet) and sigma = 2^u2 e^(2 pi i t2)
// per beamlet and plane, whose powers sigma^(k^2) the record carries.  E(h)
// takes the FP64 anchor phase reduced to turns and three transcendentals,
// rho and 1/rho four more; every other row costs one complex multiplication
// (rho^k, stepped outward in both directions from h, so at most ROWS/2 steps)
// and one complex multiply-add, no transcendental.  An anchor amplitude below
// 2^-126 is flushed to zero and |U1| is capped at 64: with |u2| at most
// kStepCurvature a term the flush removes lies 2^42 or more below its
// beamlet's peak (peaks up to 1; the margin grows with the peak), and the cap
// only acts on flushed anchors.  Per-tile FP32 sums are folded into the
// Kahan-compensated (s, c) accumulators up to 16 rows; at 32 rows by plain
// FP32 addition (c stays zero), one rounding per 128-beamlet tile: measured
// 20 % faster than the compensated fold there (204 against 249 registers) at
// an unchanged error against FP64.
//
// With HG each beamlet's Hermite-Gaussian factor multiplies its phasor.
// Along the column g = G d is linear in the row step k from the anchor, so
// the factor is a polynomial of degree <= 4 in k; its coefficients are formed
// once per (lane, beamlet) and evaluated by Horner's rule per row (8 FP32
// instructions), centred on the anchor so |k| <= ROWS / 2.
template <int ROWS, int NT, bool HG = false>
__device__ inline void mixed_accumulate_rotor(Rec32 *tile, const Rec32 *__restrict__ rec, int64_t jb, int64_t je,
                                              double a, double b0, double dy, float (&s_re)[ROWS],
                                              float (&s_im)[ROWS], float (&c_re)[ROWS], float (&c_im)[ROWS],
                                              RecHG32 *htile = nullptr, const RecHG32 *__restrict__ hg = nullptr) {
    constexpr int H = ROWS / 2;
    static_assert(H <= kRotorRows, "rotor form: at most 2 * kRotorRows rows per lane");
    const double bh = b0 + H * dy;
    const float af = (float)a, bhf = (float)bh, dyf = (float)dy;
    float acc_re[ROWS], acc_im[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; k++) acc_re[k] = acc_im[k] = 0.0f;
    for (int64_t j0 = jb; j0 < je; j0 += kMixedTile) {
        const int cnt = (int)min((int64_t)kMixedTile, je - j0);
        __syncthreads();
        {
            const float4 *src = reinterpret_cast<const float4 *>(rec + j0);
            float4 *dst = reinterpret_cast<float4 *>(tile);
            for (int i = threadIdx.x; i < cnt * kRec32Vec4; i += NT) dst[i] = src[i];
            if constexpr (HG) {
                const float4 *hs = reinterpret_cast<const float4 *>(hg + j0);
                float4 *hd = reinterpret_cast<float4 *>(htile);
                for (int i = threadIdx.x; i < cnt * (int)(sizeof(RecHG32) / 16); i += NT) hd[i] = hs[i];
            }
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; jj++) {
            const Rec32 &r = tile[jj];
            const double da = a - r.arho, db = bh - r.brho;
            const double q = r.p[2] + r.p[4] * da;
            const double T0 = r.p[0] + da * (r.p[1] + r.p[3] * da) + db * (q + r.p[5] * db);
            const double T1 = dy * (q + 2.0 * r.p[5] * db);
            const float base = (float)__builtin_amdgcn_fract(T0);
            const float t1 = (float)(T1 - rint(T1));
            const float daf = af - r.arho_f, dbf = bhf - r.brho_f;
            const float qf = r.m[2] + r.m[4] * daf;
            const float L0 = r.m[0] + daf * (r.m[1] + r.m[3] * daf) + dbf * (qf + r.m[5] * dbf);
            const float U1 = fminf(fmaxf(dyf * (qf + 2.0f * r.m[5] * dbf), -64.0f), 64.0f);
            const float m0 = L0 < -126.0f ? 0.0f : __builtin_amdgcn_exp2f(L0);
            const float zr = m0 * __builtin_amdgcn_cosf(base), zi = m0 * __builtin_amdgcn_sinf(base);
            const float c1 = __builtin_amdgcn_cosf(t1), s1 = __builtin_amdgcn_sinf(t1);
            // Hermite-Gaussian factor P(k) = hq0 + k (hq1 + k (hq2 + k (hq3 + k hq4)))
            [[maybe_unused]] float hq[5][2];
            if constexpr (HG) hg_row_poly(htile[jj], daf, dbf, dyf, hq);
            if constexpr (HG) {
                acc_re[H] += zr * hq[0][0] - zi * hq[0][1];
                acc_im[H] += zr * hq[0][1] + zi * hq[0][0];
            } else {
                acc_re[H] += zr;
                acc_im[H] += zi;
            }
            if (ROWS - 1 - H > 0) {
                const float mu = __builtin_amdgcn_exp2f(U1);
                const float ur = mu * c1, ui = mu * s1;
                float pr = zr, pi = zi;
#pragma unroll
                for (int k = 1; k < ROWS - H; k++) {
                    const float nr = fmaf(pr, ur, -(pi * ui));
                    const float ni = fmaf(pr, ui, pi * ur);
                    pr = nr;
                    pi = ni;
                    const float sr = r.sq[k - 1][0], si = r.sq[k - 1][1];
                    if constexpr (HG) {
                        float Px, Py;
                        horner4(hq, (float)k, Px, Py);
                        const float tr = fmaf(pr, sr, -(pi * si)), ti = fmaf(pr, si, pi * sr);
                        acc_re[H + k] = fmaf(tr, Px, fmaf(-ti, Py, acc_re[H + k]));
                        acc_im[H + k] = fmaf(tr, Py, fmaf(ti, Px, acc_im[H + k]));
                    } else {
                        acc_re[H + k] = fmaf(pr, sr, fmaf(-pi, si, acc_re[H + k]));
                        acc_im[H + k] = fmaf(pr, si, fmaf(pi, sr, acc_im[H + k]));
                    }
                }
            }
            if (H > 0) {
                const float md = __builtin_amdgcn_exp2f(-U1);
                const float vr = md * c1, vi = -(md * s1);
                float pr = zr, pi = zi;
#pragma unroll
                for (int k = 1; k <= H; k++) {
                    const float nr = fmaf(pr, vr, -(pi * vi));
                    const float ni = fmaf(pr, vi, pi * vr);
                    pr = nr;
                    pi = ni;
                    const float sr = r.sq[k - 1][0], si = r.sq[k - 1][1];
                    if constexpr (HG) {
                        float Px, Py;
                        horner4(hq, -(float)k, Px, Py);
                        const float tr = fmaf(pr, sr, -(pi * si)), ti = fmaf(pr, si, pi * sr);
                        acc_re[H - k] = fmaf(tr, Px, fmaf(-ti, Py, acc_re[H - k]));
                        acc_im[H - k] = fmaf(tr, Py, fmaf(ti, Px, acc_im[H - k]));
                    } else {
                        acc_re[H - k] = fmaf(pr, sr, fmaf(-pi, si, acc_re[H - k]));
                        acc_im[H - k] = fmaf(pr, si, fmaf(pi, sr, acc_im[H - k]));
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ROWS; k++) {
            if constexpr (ROWS <= 16) {
                kahan(s_re[k], c_re[k], acc_re[k]);
                kahan(s_im[k], c_im[k], acc_im[k]);
            } else {
                s_re[k] += acc_re[k];
                s_im[k] += acc_im[k];
            }
            acc_re[k] = acc_im[k] = 0.0f;
        }
    }
}

// XCD-aware work mapping: workgroup b runs on XCD (b mod 8); give each XCD a
// contiguous range of work items.  The grid is padded to a multiple of 8.
__device__ inline int work_item(int b, int G) { return (b & 7) * (G >> 3) + (b >> 3); }

}  // namespace dev
}  // namespace gbd
