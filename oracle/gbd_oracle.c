/*
 * gbd_oracle.c -- plain FP64 reference of plane-evaluation Gaussian beamlet
 * decomposition (arXiv:2404.12454).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  The product path
 * (the HIP library) never calls it, and the two share no code.
 *
 * Conventions.  Time dependence exp(+i w t), so a field picks up exp(-i k L)
 * over an optical path L; a Gaussian beam is exp(-(i k / 2) r^T Q^-1 r) with
 * Q^-1 = 1/R - i lambda / (pi w^2) (the complex-beam-parameter equation of
 * Sec. 1 with the sign of its imaginary part matched to the exp(-i k l)
 * Collins kernels of Sec. 2).  Metres; paraxial slopes; ray vectors ordered
 * (x, y, theta_x, theta_y); 4x4 matrices row-major with 2x2 blocks
 * [[A, B], [C, D]].  Phases are carried in turns (path / lambda).
 *
 * What is computed, per beamlet j (each step cites the paper):
 *  1. Q1^-1 = -i lambda / (pi w0^2) I                    (complex-q equation)
 *  2. base ray  r2M = A r1M + B th1M,  th2M = C r1M + D th1M
 *                                                      (Appendix A, ab/cd laws)
 *     or, for ray-traced inputs (Sec. 2.2: base and parabasal rays give the
 *     differential ABCD), the traced base ray at the output plane, whose
 *     optical path beyond l0 replaces the eikonal term of step 5
 *  3. the base ray (r2M + z th2M, z) meets the detector plane at plane
 *     coordinates (a_rho, b_rho) and axial offset z_rho; the system is
 *     extended by free space z_rho: A' = A + z C, B' = B + z D
 *  4. Q^-1 = (C' + D' Q1^-1)(A' + B' Q1^-1)^-1          (Gaussian solution of
 *     the Collins integral, Sec. 4.1); amplitude det(A' + B' Q1^-1)^(-1/2)
 *     taken as the product of the principal square roots of the two
 *     eigenvalues (Appendix C: Gouy phase from the eigenvalues)
 *  5. misalignment phase: the completed-square form of Appendix A
 *     (tilt-phase equation) rewritten through the ab/cd laws,
 *     exp(-i k [l0 + z + W + (th2M . r2M' - th1M . r1M) / 2]),
 *     with r2M' = r2M + z th2M measured at the hit point
 *  6. field on the plane (plane-evaluation, Sec. 3): with d = (a - a_rho,
 *     b - b_rho), zeta = e_z . d and w = Pm d (Pm's columns are
 *     e_i,perp - e_iz th2M):
 *       log E_j = log(a_j gamma) - 2 pi i tau
 *                 - i k [(1 + |th|^2/2) zeta + th . w]
 *                 - tr(Q^-1) zeta / 2 + tr(Q^-2) zeta^2 / 4
 *                 - (i k / 2) w^T Q^-1 w
 *     which is exact for a plane normal to the axis (e_z = 0, the paper's
 *     setting) and the second-order expansion about the hit point of the
 *     exact paraxial beamlet field for a tilted plane.
 *  7. E = sum_j E_j, in beamlet index order.
 * Higher-order beamlets (the Hermite solutions of the reduced Collins
 * integral that Sec. 2.1 lists as usable in beamlet decomposition): the
 * elegant Hermite-Gaussian input H_m(u_x) H_n(u_y) e^(-|u|^2)
 * e^(-i k th1 . (r - c)), u = (r - c) / w0, is w0^(m+n) times the
 * derivative d^(m+n) / dc_x^m dc_y^n of the Gaussian envelope with the tilt
 * phase held fixed, and propagation commutes with that derivative; so the
 * output is the Gaussian beamlet's field times a polynomial in
 * g = L w (L = -i k (C^T - A'^T Q), linear in the offset w from the base
 * ray) and the constant H = i k (C^T A' - A'^T Q A'), exact on planes normal
 * to the axis.
 * The point-evaluation form (model 1) instead extends the system to every
 * pixel's own axial position and evaluates steps 4-6 there exactly.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOTSYMPLECTIC (-2)
#define OR_EBRANCH (-3)
#define OR_EPARALLEL (-4)

typedef double complex cplx;

/* ---- small 2x2 helpers (closed forms, Appendix C) ---- */
typedef struct { cplx m[2][2]; } cm2;
typedef struct { double m[2][2]; } rm2;

static cm2 cm2_mul(cm2 x, cm2 y) {
    cm2 r;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            r.m[i][j] = x.m[i][0] * y.m[0][j] + x.m[i][1] * y.m[1][j];
    return r;
}
static cplx cm2_det(cm2 x) { return x.m[0][0] * x.m[1][1] - x.m[0][1] * x.m[1][0]; }
static cm2 cm2_inv(cm2 x) {
    cplx d = cm2_det(x);
    cm2 r;
    r.m[0][0] = x.m[1][1] / d;
    r.m[1][1] = x.m[0][0] / d;
    r.m[0][1] = -x.m[0][1] / d;
    r.m[1][0] = -x.m[1][0] / d;
    return r;
}
/* eigenvalues of a 2x2 complex matrix from its characteristic polynomial */
static void cm2_eig(cm2 x, cplx *mu1, cplx *mu2) {
    cplx tr = x.m[0][0] + x.m[1][1];
    cplx disc = csqrt(tr * tr - 4.0 * cm2_det(x));
    *mu1 = 0.5 * (tr + disc);
    *mu2 = 0.5 * (tr - disc);
}

/* Accepted eigenvalue domain for the principal-root branch: the open lower
 * half plane plus the positive real axis.  An eigenvalue reached from 1 by a
 * physical path (B' >= 0) never leaves it; anything else is refused. */
static int branch_ok(cplx mu) {
    double tol = 1e-12 * cabs(mu);
    if (!(cabs(mu) > 0.0)) return 0;
    if (cimag(mu) > tol) return 0;
    if (cimag(mu) >= -tol && creal(mu) <= 0.0) return 0;
    return 1;
}

/* Symplectic relations of the ABCD blocks (Sec. 2.1, symplectic equations),
 * to relative tolerance tol. */
static int symplectic_ok(const double *M, double tol) {
    double A[2][2], B[2][2], C[2][2], D[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            A[i][j] = M[4 * i + j];
            B[i][j] = M[4 * i + j + 2];
            C[i][j] = M[4 * (i + 2) + j];
            D[i][j] = M[4 * (i + 2) + j + 2];
        }
    double worst = 0.0;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            /* B A^T = A B^T */
            double x1 = 0, y1 = 0, s1 = 0;
            /* B^T D = D^T B */
            double x2 = 0, y2 = 0, s2 = 0;
            /* D C^T = C D^T */
            double x3 = 0, y3 = 0, s3 = 0;
            /* A^T C = C^T A */
            double x4 = 0, y4 = 0, s4 = 0;
            /* A D^T - B C^T = I */
            double x5 = 0, s5 = 0;
            for (int k = 0; k < 2; k++) {
                x1 += B[i][k] * A[j][k]; y1 += A[i][k] * B[j][k];
                s1 += fabs(B[i][k] * A[j][k]) + fabs(A[i][k] * B[j][k]);
                x2 += B[k][i] * D[k][j]; y2 += D[k][i] * B[k][j];
                s2 += fabs(B[k][i] * D[k][j]) + fabs(D[k][i] * B[k][j]);
                x3 += D[i][k] * C[j][k]; y3 += C[i][k] * D[j][k];
                s3 += fabs(D[i][k] * C[j][k]) + fabs(C[i][k] * D[j][k]);
                x4 += A[k][i] * C[k][j]; y4 += C[k][i] * A[k][j];
                s4 += fabs(A[k][i] * C[k][j]) + fabs(C[k][i] * A[k][j]);
                x5 += A[i][k] * D[j][k] - B[i][k] * C[j][k];
                s5 += fabs(A[i][k] * D[j][k]) + fabs(B[i][k] * C[j][k]);
            }
            double e;
            e = fabs(x1 - y1) / (s1 + 1e-300); if (e > worst && s1 > 0) worst = e;
            e = fabs(x2 - y2) / (s2 + 1e-300); if (e > worst && s2 > 0) worst = e;
            e = fabs(x3 - y3) / (s3 + 1e-300); if (e > worst && s3 > 0) worst = e;
            e = fabs(x4 - y4) / (s4 + 1e-300); if (e > worst && s4 > 0) worst = e;
            e = fabs(x5 - (i == j ? 1.0 : 0.0)) / (s5 + 1.0);
            if (e > worst) worst = e;
        }
    return worst <= tol;
}

/* Differential matrices from ray tracing can have a vanishing block (A at a
 * focus), where entry-wise relative residuals mean nothing.  Scale positions
 * by s and angles by 1/s with s^2 = sqrt(|B|_F / |C|_F), a symplectic change of
 * variables that leaves A and D and gives B and C equal norms, and require
 * every entry of M'^T J M' - J within tol * max(1, max|M'|)^2. */
static int symplectic_scaled_ok(const double *M, double tol) {
    double nb = 0.0, nc = 0.0;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            nb += M[4 * i + j + 2] * M[4 * i + j + 2];
            nc += M[4 * (i + 2) + j] * M[4 * (i + 2) + j];
        }
    double s2 = 1.0;
    if (nb > 0.0 && nc > 0.0) s2 = sqrt(sqrt(nb / nc));
    double P[4][4], top = 1.0;
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            double v = M[4 * i + j];
            if (i < 2 && j >= 2) v = v / s2;
            else if (i >= 2 && j < 2) v = v * s2;
            P[i][j] = v;
            if (fabs(v) > top) top = fabs(v);
        }
    /* M'^T J M' with J = [[0, I], [-I, 0]]: entry (r, c) = sum_k P[k][r] P[k+2][c] - P[k+2][r] P[k][c] */
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            double v = 0.0;
            for (int k = 0; k < 2; k++) v += P[k][r] * P[k + 2][c] - P[k + 2][r] * P[k][c];
            double want = (r < 2 && c == r + 2) ? 1.0 : (r >= 2 && c == r - 2) ? -1.0 : 0.0;
            if (!(fabs(v - want) <= tol * top * top)) return 0;
        }
    return 1;
}

/* ---- detector plane ---- */
typedef struct {
    double O[3], n[3], e1[3], e2[3];
    int32_t nx, ny;
    double dx, dy;
} or_plane;

static int make_plane(const double *origin, const double *normal, const double *xhint,
                      int32_t nx, int32_t ny, double dx, double dy, or_plane *p) {
    double nn = sqrt(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2]);
    if (!(nn > 0.0) || nx < 0 || ny < 0 || !(dx > 0.0) || !(dy > 0.0)) return OR_EINVAL;
    for (int i = 0; i < 3; i++) { p->O[i] = origin[i]; p->n[i] = normal[i] / nn; }
    double hn = xhint[0] * p->n[0] + xhint[1] * p->n[1] + xhint[2] * p->n[2];
    double e[3];
    for (int i = 0; i < 3; i++) e[i] = xhint[i] - hn * p->n[i];
    double en = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    double hl = sqrt(xhint[0] * xhint[0] + xhint[1] * xhint[1] + xhint[2] * xhint[2]);
    if (!(en > 1e-9 * hl)) return OR_EINVAL;
    for (int i = 0; i < 3; i++) p->e1[i] = e[i] / en;
    p->e2[0] = p->n[1] * p->e1[2] - p->n[2] * p->e1[1];
    p->e2[1] = p->n[2] * p->e1[0] - p->n[0] * p->e1[2];
    p->e2[2] = p->n[0] * p->e1[1] - p->n[1] * p->e1[0];
    p->nx = nx; p->ny = ny; p->dx = dx; p->dy = dy;
    return OR_OK;
}

/* ---- one beamlet propagated by an ABCD extended with free space z ---- */
typedef struct {
    cm2 Qinv;        /* complex curvature at the output */
    cplx gamma;      /* det(A' + B' Q1^-1)^(-1/2), eigenvalue branch */
    double r2[2];    /* base-ray position at the output (r2M + z th2M) */
    double th2[2];   /* base-ray slope */
    double tau;      /* (z + W + S') / lambda in turns, l0 excluded */
    /* higher-order (elegant Hermite-Gaussian) beamlets: the envelope's
     * d log E / dc = L w and d^2 log E / dc dc^T = H, c the input centre,
     * w = r - r2 */
    cplx L[2][2], H[2][2];
    /* truncated beamlets: the envelope's derivatives with respect to the
     * input slope th1 (centre fixed), d log E / d th1 = -i k lt w and
     * d^2 log E / d th1^2 = i k ht */
    cplx lt[2][2], ht[2][2];
} or_prop;

typedef struct {
    double lam, l0;
    double r1[2], th1[2], w0, W;
    cplx a;
    const double *M;
    const double *base; /* NULL, or a traced base ray at the ABCD output plane:
                           (x, y, l, m, optical path - l0) */
    int hm, hn;         /* elegant Hermite-Gaussian orders (0, 0 = Gaussian) */
} or_in;

static int propagate(const or_in *b, double z, or_prop *out) {
    double A[2][2], B[2][2], C[2][2], D[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            A[i][j] = b->M[4 * i + j];
            B[i][j] = b->M[4 * i + j + 2];
            C[i][j] = b->M[4 * (i + 2) + j];
            D[i][j] = b->M[4 * (i + 2) + j + 2];
        }
    /* base ray at the ABCD output plane: the ab/cd laws, or a traced ray */
    double r2M[2], th2M[2];
    for (int i = 0; i < 2; i++) {
        if (b->base) {
            r2M[i] = b->base[i];
            th2M[i] = b->base[2 + i];
        } else {
            r2M[i] = A[i][0] * b->r1[0] + A[i][1] * b->r1[1] + B[i][0] * b->th1[0] + B[i][1] * b->th1[1];
            th2M[i] = C[i][0] * b->r1[0] + C[i][1] * b->r1[1] + D[i][0] * b->th1[0] + D[i][1] * b->th1[1];
        }
    }
    /* free-space extension by z */
    double Ap[2][2], Bp[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            Ap[i][j] = A[i][j] + z * C[i][j];
            Bp[i][j] = B[i][j] + z * D[i][j];
        }
    const cplx q1 = -I * b->lam / (M_PI * b->w0 * b->w0); /* Q1^-1 = q1 * I */
    cm2 Mm, Nm;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            Mm.m[i][j] = Ap[i][j] + Bp[i][j] * q1;
            Nm.m[i][j] = C[i][j] + D[i][j] * q1;
        }
    cm2 Q = cm2_mul(Nm, cm2_inv(Mm));
    cplx off = 0.5 * (Q.m[0][1] + Q.m[1][0]);
    Q.m[0][1] = off;
    Q.m[1][0] = off;
    cplx mu1, mu2;
    cm2_eig(Mm, &mu1, &mu2);
    if (!branch_ok(mu1) || !branch_ok(mu2)) return OR_EBRANCH;
    out->Qinv = Q;
    out->gamma = 1.0 / (csqrt(mu1) * csqrt(mu2));
    for (int i = 0; i < 2; i++) {
        out->r2[i] = r2M[i] + z * th2M[i];
        out->th2[i] = th2M[i];
    }
    /* eikonal along the base ray beyond l0: Euler's relation for the point
     * eikonal, or the traced optical path; then the free-space extension */
    double S;
    if (b->base)
        S = b->base[4] + 0.5 * z * (th2M[0] * th2M[0] + th2M[1] * th2M[1]);
    else
        S = 0.5 * (th2M[0] * out->r2[0] + th2M[1] * out->r2[1] - b->th1[0] * b->r1[0] - b->th1[1] * b->r1[1]);
    out->tau = (z + b->W + S) / b->lam;
    /* Derivatives with respect to the input centre c of the envelope (th1
     * and the tilt phase's reference fixed).  With log E = -i k [S + th2 . w
     * + w^T Q w / 2] + const, r2 = A' c + B' th1, th2 = C c + D th1,
     * w = r - r2, and dS/dc = A'^T th2 - th1 (the eikonal's end-point
     * derivatives), d log E / dc = -i k [(C^T - A'^T Q) w - th1]; the -th1
     * is the tilt phase's own dependence on c, removed by holding its
     * reference fixed:
     *   g = L w, L = -i k (C^T - A'^T Q),
     *   H = d g / dc = i k (C^T A' - A'^T Q A')  (C^T A' symmetric) */
    const double k = 2.0 * M_PI / b->lam;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            cplx AQ = 0.0; /* (A'^T Q)_ij */
            for (int r = 0; r < 2; r++) AQ += Ap[r][i] * Q.m[r][j];
            out->L[i][j] = -I * k * (C[j][i] - AQ);
        }
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            cplx v = 0.0;
            for (int r = 0; r < 2; r++) {
                v += C[r][i] * Ap[r][j];
                for (int t = 0; t < 2; t++) v -= Ap[r][i] * Q.m[r][t] * Ap[t][j];
            }
            out->H[i][j] = I * k * v;
        }
    /* Derivatives with respect to the input slope th1 (centre fixed): with
     * dr2/dth1 = B', dth2/dth1 = D and dS/dth1 = B'^T th2 (the eikonal's
     * end-point derivative), d log E / dth1 = -i k (D^T - B'^T Q) w, with no
     * constant term, and its derivative -i k (D^T - B'^T Q)(-B'):
     *   lt = D^T - B'^T Q,  ht = D^T B' - B'^T Q B' */
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            cplx BQ = 0.0, v = 0.0; /* (B'^T Q)_ij, (D^T B' - B'^T Q B')_ij */
            for (int r = 0; r < 2; r++) {
                BQ += Bp[r][i] * Q.m[r][j];
                v += D[r][i] * Bp[r][j];
                for (int t = 0; t < 2; t++) v -= Bp[r][i] * Q.m[r][t] * Bp[t][j];
            }
            out->lt[i][j] = D[j][i] - BQ;
            out->ht[i][j] = v;
        }
    return OR_OK;
}

/* Elegant Hermite-Gaussian factor of orders (m, n) <= 2: the derivative
 * d^(m+n) E / dc_x^m dc_y^n divided by E, from g = d log E / dc and the
 * constant H = d^2 log E / dc^2 (Faa di Bruno for the exponential of a
 * quadratic in c). */
static cplx hermite_factor(int m, int n, const cplx g[2], cplx H[2][2]) {
    const cplx gx = g[0], gy = g[1], hxx = H[0][0], hyy = H[1][1], hxy = 0.5 * (H[0][1] + H[1][0]);
    switch (3 * m + n) {
    case 0: return 1.0;
    case 1: return gy;
    case 2: return gy * gy + hyy;
    case 3: return gx;
    case 4: return gx * gy + hxy;
    case 5: return gx * gy * gy + 2.0 * hxy * gy + hyy * gx;
    case 6: return gx * gx + hxx;
    case 7: return gx * gx * gy + 2.0 * hxy * gx + hxx * gy;
    case 8: return gx * gx * gy * gy + 4.0 * hxy * gx * gy + hyy * gx * gx + hxx * gy * gy + hxx * hyy + 2.0 * hxy * hxy;
    }
    return NAN;
}

static cplx higher_order(const or_in *b, const or_prop *P, const double w[2]) {
    if (b->hm == 0 && b->hn == 0) return 1.0;
    cplx g[2];
    for (int i = 0; i < 2; i++) g[i] = P->L[i][0] * w[0] + P->L[i][1] * w[1];
    cplx H[2][2] = {{P->H[0][0], P->H[0][1]}, {P->H[1][0], P->H[1][1]}};
    return pow(b->w0, b->hm + b->hn) * hermite_factor(b->hm, b->hn, g, H);
}

/* the base-ray hit point on the plane: a_rho, b_rho, z_rho */
static int hit_point(const or_in *b, const or_plane *p, double *arho, double *brho, double *zrho) {
    or_prop p0;
    int rc = propagate(b, 0.0, &p0);
    if (rc) return rc;
    double d[3] = {p0.th2[0], p0.th2[1], 1.0};
    double X0[3] = {p0.r2[0], p0.r2[1], 0.0};
    double nd = p->n[0] * d[0] + p->n[1] * d[1] + p->n[2] * d[2];
    double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(fabs(nd) > 1e-6 * dl)) return OR_EPARALLEL;
    double z = (p->n[0] * (p->O[0] - X0[0]) + p->n[1] * (p->O[1] - X0[1]) + p->n[2] * (p->O[2] - X0[2])) / nd;
    double X[3];
    for (int i = 0; i < 3; i++) X[i] = X0[i] + z * d[i] - p->O[i];
    *arho = p->e1[0] * X[0] + p->e1[1] * X[1] + p->e1[2] * X[2];
    *brho = p->e2[0] * X[0] + p->e2[1] * X[1] + p->e2[2] * X[2];
    *zrho = z;
    return OR_OK;
}

static double reduce_turns(double t) { return t - nearbyint(t); }

/* field of one beamlet at plane coordinates (a, b): plane-evaluation model */
typedef struct {
    or_prop P;
    double arho, brho;
    double Pm[2][2]; /* columns i: e_i,perp - e_iz th2M */
    double ez[2];
    cplx pref;       /* a_j gamma exp(-2 pi i (tau - rint tau)) */
    or_in in;        /* the beamlet's inputs (orders, waist) */
} or_beam_on_plane;

static int beam_on_plane(const or_in *b, const or_plane *p, or_beam_on_plane *o) {
    double zr;
    int rc = hit_point(b, p, &o->arho, &o->brho, &zr);
    if (rc) return rc;
    rc = propagate(b, zr, &o->P);
    if (rc) return rc;
    const double *e[2] = {p->e1, p->e2};
    for (int c = 0; c < 2; c++) {
        o->ez[c] = e[c][2];
        for (int r = 0; r < 2; r++) o->Pm[r][c] = e[c][r] - e[c][2] * o->P.th2[r];
    }
    o->pref = b->a * o->P.gamma * cexp(-2.0 * M_PI * I * reduce_turns(o->P.tau));
    o->in = *b;
    return OR_OK;
}

static cplx field_plane_model(const or_beam_on_plane *o, double lam, double a, double b) {
    const double k = 2.0 * M_PI / lam;
    double d[2] = {a - o->arho, b - o->brho};
    double zeta = o->ez[0] * d[0] + o->ez[1] * d[1];
    double w[2] = {o->Pm[0][0] * d[0] + o->Pm[0][1] * d[1], o->Pm[1][0] * d[0] + o->Pm[1][1] * d[1]};
    const double *th = o->P.th2;
    double th2 = th[0] * th[0] + th[1] * th[1];
    const cm2 *Q = &o->P.Qinv;
    cplx trQ = Q->m[0][0] + Q->m[1][1];
    cm2 Q2 = cm2_mul(*Q, *Q);
    cplx trQ2 = Q2.m[0][0] + Q2.m[1][1];
    cplx wQw = w[0] * (Q->m[0][0] * w[0] + Q->m[0][1] * w[1]) + w[1] * (Q->m[1][0] * w[0] + Q->m[1][1] * w[1]);
    cplx logE = -I * k * ((1.0 + 0.5 * th2) * zeta + th[0] * w[0] + th[1] * w[1])
                - 0.5 * trQ * zeta + 0.25 * trQ2 * zeta * zeta
                - 0.5 * I * k * wQw;
    return o->pref * cexp(logE) * higher_order(&o->in, &o->P, w);
}

/* exact paraxial field of one beamlet at the 3-D point X (point evaluation) */
static int field_point_exact(const or_in *b, const double X[3], cplx *E) {
    or_prop P;
    int rc = propagate(b, X[2], &P);
    if (rc) return rc;
    const double k = 2.0 * M_PI / b->lam;
    double w[2] = {X[0] - P.r2[0], X[1] - P.r2[1]};
    const cm2 *Q = &P.Qinv;
    cplx wQw = w[0] * (Q->m[0][0] * w[0] + Q->m[0][1] * w[1]) + w[1] * (Q->m[1][0] * w[0] + Q->m[1][1] * w[1]);
    cplx logE = -I * k * (P.th2[0] * w[0] + P.th2[1] * w[1]) - 0.5 * I * k * wQw;
    *E = b->a * P.gamma * cexp(-2.0 * M_PI * I * reduce_turns(P.tau)) * cexp(logE) * higher_order(b, &P, w);
    return OR_OK;
}

static or_in load_in(int64_t j, double lam, double l0, const double *r1, const double *th1,
                     const double *w0, int64_t nw0, const double *amp, const double *path,
                     const double *abcd, int shared, const double *base, const int32_t *order) {
    or_in b;
    b.lam = lam;
    b.l0 = l0;
    b.r1[0] = r1[2 * j];
    b.r1[1] = r1[2 * j + 1];
    b.th1[0] = th1 ? th1[2 * j] : 0.0;
    b.th1[1] = th1 ? th1[2 * j + 1] : 0.0;
    b.w0 = (nw0 == 1) ? w0[0] : w0[j];
    b.W = path ? path[j] : 0.0;
    b.a = amp ? (amp[2 * j] + I * amp[2 * j + 1]) : 1.0;
    b.M = shared ? abcd : abcd + 16 * j;
    b.base = base ? base + 5 * j : NULL;
    b.hm = order ? order[2 * j] : 0;
    b.hn = order ? order[2 * j + 1] : 0;
    return b;
}

static int valid_inputs(int64_t n, double lam, double l0, const double *r1, const double *th1,
                        const double *w0, int64_t nw0, const double *amp, const double *path,
                        const double *abcd, int shared, const double *base, double tol) {
    if (n < 0 || !(lam > 0.0) || !isfinite(lam) || !isfinite(l0)) return OR_EINVAL;
    if (n == 0) return OR_OK;
    if (!r1 || !w0 || !abcd || !(nw0 == 1 || nw0 == n)) return OR_EINVAL;
    for (int64_t j = 0; j < n; j++) {
        if (!isfinite(r1[2 * j]) || !isfinite(r1[2 * j + 1])) return OR_EINVAL;
        if (th1 && (!isfinite(th1[2 * j]) || !isfinite(th1[2 * j + 1]))) return OR_EINVAL;
        if (amp && (!isfinite(amp[2 * j]) || !isfinite(amp[2 * j + 1]))) return OR_EINVAL;
        if (path && !isfinite(path[j])) return OR_EINVAL;
        if (base)
            for (int e = 0; e < 5; e++)
                if (!isfinite(base[5 * j + e])) return OR_EINVAL;
    }
    for (int64_t j = 0; j < nw0; j++)
        if (!(w0[j] > 0.0) || !isfinite(w0[j])) return OR_EINVAL;
    int64_t nm = shared ? 1 : n;
    for (int64_t j = 0; j < nm; j++) {
        for (int e = 0; e < 16; e++)
            if (!isfinite(abcd[16 * j + e])) return OR_EINVAL;
        if (!(base ? symplectic_scaled_ok(abcd + 16 * j, tol) : symplectic_ok(abcd + 16 * j, tol)))
            return OR_ENOTSYMPLECTIC;
    }
    return OR_OK;
}

/*
 * oracle_eval: coherent sum of n beamlets on the detector plane.
 *   model 0: plane-evaluation (steps 1-7 above); model 1: exact paraxial
 *   point evaluation per pixel.
 *   pix_ix/pix_iy: NULL for the full [ny][nx] grid (npix ignored), else the
 *   npix listed pixels.  out: interleaved complex128.
 *   extra_point: if non-NULL, a 2-element (a, b) plane coordinate evaluated
 *   into out_extra (used for the on-axis normalisation of the Airy metric).
 * Returns 0 or a negative OR_E* code; on error out is left untouched.
 */
int oracle_eval_base(int64_t n, double lam, double l0, const double *r1, const double *th1,
                     const double *w0, int64_t nw0, const double *amp, const double *path,
                     const double *abcd, int shared_abcd, const double *base, double sympl_tol,
                     const int32_t *order,
                     const double *origin, const double *normal, const double *xhint,
                     int32_t nx, int32_t ny, double dx, double dy,
                     int64_t npix, const int32_t *pix_ix, const int32_t *pix_iy,
                     int model, double *out, const double *extra_point, double *out_extra) {
    if (!(sympl_tol > 0.0)) return OR_EINVAL;
    if (order)
        for (int64_t j = 0; j < 2 * n; j++)
            if (order[j] < 0 || order[j] > 2) return OR_EINVAL;
    int rc = valid_inputs(n, lam, l0, r1, th1, w0, nw0, amp, path, abcd, shared_abcd, base, sympl_tol);
    if (rc) return rc;
    or_plane pl;
    rc = make_plane(origin, normal, xhint, nx, ny, dx, dy, &pl);
    if (rc) return rc;
    if (model != 0 && model != 1) return OR_EINVAL;
    int64_t m = pix_ix ? npix : (int64_t)nx * ny;
    if (pix_ix) {
        if (!pix_iy || npix < 0) return OR_EINVAL;
        for (int64_t p = 0; p < npix; p++)
            if (pix_ix[p] < 0 || pix_ix[p] >= nx || pix_iy[p] < 0 || pix_iy[p] >= ny) return OR_EINVAL;
    }
    /* per-beamlet propagation onto the plane (plane-evaluation setup) */
    or_beam_on_plane *bp = (or_beam_on_plane *)malloc(sizeof(or_beam_on_plane) * (size_t)(n > 0 ? n : 1));
    if (!bp) return OR_EINVAL;
    for (int64_t j = 0; j < n; j++) {
        or_in b = load_in(j, lam, l0, r1, th1, w0, nw0, amp, path, abcd, shared_abcd, base, order);
        rc = beam_on_plane(&b, &pl, &bp[j]);
        /* a higher-order beamlet's plane-evaluation field is the exact
         * paraxial one only on planes normal to the axis */
        if (!rc && (b.hm || b.hn) && (model == 0 || extra_point) && (bp[j].ez[0] != 0.0 || bp[j].ez[1] != 0.0))
            rc = OR_EINVAL;
        if (rc) { free(bp); return rc; }
    }
    /* the exact model must also be valid at every pixel's own axial position */
    const cplx global = cexp(-2.0 * M_PI * I * reduce_turns(l0 / lam));
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < m; p++) {
        int32_t ix = pix_ix ? pix_ix[p] : (int32_t)(p % nx);
        int32_t iy = pix_ix ? pix_iy[p] : (int32_t)(p / nx);
        double a = (ix - 0.5 * (nx - 1)) * dx;
        double bb = (iy - 0.5 * (ny - 1)) * dy;
        cplx E = 0.0;
        if (model == 0) {
            for (int64_t j = 0; j < n; j++) E += field_plane_model(&bp[j], lam, a, bb);
        } else {
            double X[3];
            for (int i = 0; i < 3; i++) X[i] = pl.O[i] + a * pl.e1[i] + bb * pl.e2[i];
            for (int64_t j = 0; j < n; j++) {
                or_in b = load_in(j, lam, l0, r1, th1, w0, nw0, amp, path, abcd, shared_abcd, base, order);
                cplx Ej;
                if (field_point_exact(&b, X, &Ej)) {
#pragma omp atomic write
                    err = 1;
                    Ej = 0.0;
                }
                E += Ej;
            }
        }
        E *= global;
        out[2 * p] = creal(E);
        out[2 * p + 1] = cimag(E);
    }
    if (extra_point && out_extra) {
        cplx E = 0.0;
        for (int64_t j = 0; j < n; j++) E += field_plane_model(&bp[j], lam, extra_point[0], extra_point[1]);
        E *= global;
        out_extra[0] = creal(E);
        out_extra[1] = cimag(E);
    }
    free(bp);
    return err ? OR_EBRANCH : OR_OK;
}

/* oracle_eval: the same without traced base rays, symplectic tolerance 1e-10 */
/*
 * Truncated beamlets (Sec. 2.1 names truncated-beam solutions of the reduced
 * Collins integral as usable in beamlet decomposition): the input envelope is
 * cut by a straight edge, kept where e . r <= t (e a unit vector in the input
 * plane).  The step function is a superposition of plane-wave tilts,
 * H(t - e.r) = (1/2 pi) int ds int dkappa e^(i kappa (s - e.r)) over s <= t,
 * and each tilted copy of the Gaussian propagates as a Gaussian whose log is
 * quadratic in the tilt (derivatives lt, ht above); the two Gaussian
 * integrals leave the factor
 *     Phi = erfc(zeta) / 2,
 *     zeta = (e . c - t + e^T lt w) / sqrt(-2 i e^T ht e / k)   (principal root),
 * c the beamlet centre, w the offset from the base ray, so the truncated
 * beamlet is its Gaussian field times Phi.
 *
 * oracle_trunc_terms writes, for every listed pixel p and beamlet j of the
 * inputs (all taken as truncated, edge[j] = (e_x, e_y, t)), the complex log of
 * the Gaussian term log E_jp (global phase l0 / lambda included) and zeta_jp,
 * [npix][n][2] each, on a plane normal to the axis (plane evaluation is exact
 * there; other planes: OR_EINVAL).  The caller forms E_jp Phi_jp with a
 * complex error function.
 */
int oracle_trunc_terms(int64_t n, double lam, double l0, const double *r1, const double *th1,
                       const double *w0, int64_t nw0, const double *amp, const double *path,
                       const double *abcd, int shared_abcd, const double *edge,
                       const double *origin, const double *normal, const double *xhint,
                       int32_t nx, int32_t ny, double dx, double dy,
                       int64_t npix, const int32_t *pix_ix, const int32_t *pix_iy,
                       double *log_out, double *zeta_out) {
    int rc = valid_inputs(n, lam, l0, r1, th1, w0, nw0, amp, path, abcd, shared_abcd, NULL, 1e-10);
    if (rc) return rc;
    if (n > 0 && !edge) return OR_EINVAL;
    for (int64_t j = 0; j < n; j++) {
        const double ex = edge[3 * j], ey = edge[3 * j + 1];
        if (!isfinite(edge[3 * j + 2]) || fabs(ex * ex + ey * ey - 1.0) > 1e-12) return OR_EINVAL;
    }
    or_plane pl;
    rc = make_plane(origin, normal, xhint, nx, ny, dx, dy, &pl);
    if (rc) return rc;
    int64_t m = pix_ix ? npix : (int64_t)nx * ny;
    if (pix_ix) {
        if (!pix_iy || npix < 0) return OR_EINVAL;
        for (int64_t p = 0; p < npix; p++)
            if (pix_ix[p] < 0 || pix_ix[p] >= nx || pix_iy[p] < 0 || pix_iy[p] >= ny) return OR_EINVAL;
    }
    or_beam_on_plane *bp = (or_beam_on_plane *)malloc(sizeof(or_beam_on_plane) * (size_t)(n > 0 ? n : 1));
    cplx *zs = (cplx *)malloc(sizeof(cplx) * (size_t)(n > 0 ? n : 1));
    if (!bp || !zs) { free(bp); free(zs); return OR_EINVAL; }
    const double k = 2.0 * M_PI / lam;
    for (int64_t j = 0; j < n; j++) {
        or_in b = load_in(j, lam, l0, r1, th1, w0, nw0, amp, path, abcd, shared_abcd, NULL, NULL);
        rc = beam_on_plane(&b, &pl, &bp[j]);
        if (!rc && (bp[j].ez[0] != 0.0 || bp[j].ez[1] != 0.0)) rc = OR_EINVAL;
        if (rc) { free(bp); free(zs); return rc; }
        const double e[2] = {edge[3 * j], edge[3 * j + 1]};
        cplx q = 0.0;
        for (int r = 0; r < 2; r++)
            for (int c = 0; c < 2; c++) q += e[r] * bp[j].P.ht[r][c] * e[c];
        zs[j] = csqrt(-2.0 * I * q / k);
    }
    const cplx global = -2.0 * M_PI * I * reduce_turns(l0 / lam);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < m; p++) {
        int32_t ix = pix_ix ? pix_ix[p] : (int32_t)(p % nx);
        int32_t iy = pix_ix ? pix_iy[p] : (int32_t)(p / nx);
        double a = (ix - 0.5 * (nx - 1)) * dx;
        double bb = (iy - 0.5 * (ny - 1)) * dy;
        for (int64_t j = 0; j < n; j++) {
            const or_beam_on_plane *o = &bp[j];
            double d[2] = {a - o->arho, bb - o->brho};
            double w[2] = {o->Pm[0][0] * d[0] + o->Pm[0][1] * d[1], o->Pm[1][0] * d[0] + o->Pm[1][1] * d[1]};
            const double *th = o->P.th2;
            const cm2 *Q = &o->P.Qinv;
            cplx wQw = w[0] * (Q->m[0][0] * w[0] + Q->m[0][1] * w[1]) + w[1] * (Q->m[1][0] * w[0] + Q->m[1][1] * w[1]);
            /* normal plane: zeta-free form of the plane-evaluation exponent */
            cplx logE = clog(o->pref) - I * k * (th[0] * w[0] + th[1] * w[1]) - 0.5 * I * k * wQw + global;
            const double e[2] = {edge[3 * j], edge[3 * j + 1]};
            const double c[2] = {r1[2 * j], r1[2 * j + 1]};
            cplx num = e[0] * c[0] + e[1] * c[1] - edge[3 * j + 2];
            for (int r = 0; r < 2; r++)
                for (int cc = 0; cc < 2; cc++) num += e[r] * o->P.lt[r][cc] * w[cc];
            const cplx zeta = num / zs[j];
            const int64_t at = 2 * (p * n + j);
            log_out[at] = creal(logE);
            log_out[at + 1] = cimag(logE);
            zeta_out[at] = creal(zeta);
            zeta_out[at + 1] = cimag(zeta);
        }
    }
    free(bp);
    free(zs);
    return OR_OK;
}

int oracle_eval(int64_t n, double lam, double l0, const double *r1, const double *th1,
                const double *w0, int64_t nw0, const double *amp, const double *path,
                const double *abcd, int shared_abcd,
                const double *origin, const double *normal, const double *xhint,
                int32_t nx, int32_t ny, double dx, double dy,
                int64_t npix, const int32_t *pix_ix, const int32_t *pix_iy,
                int model, double *out, const double *extra_point, double *out_extra) {
    return oracle_eval_base(n, lam, l0, r1, th1, w0, nw0, amp, path, abcd, shared_abcd, NULL, 1e-10, NULL, origin,
                            normal, xhint, nx, ny, dx, dy, npix, pix_ix, pix_iy, model, out, extra_point,
                            out_extra);
}

/*
 * oracle_beamlet: one beamlet propagated by its ABCD extended with free space
 * z (no plane).  out[0..7] = Q^-1 (row-major, re/im interleaved), out[8..9] =
 * gamma, out[10..11] = base-ray position, out[12..13] = slope, out[14] = tau
 * (turns, l0 excluded).
 */
int oracle_beamlet(double lam, const double *r1, const double *th1, double w0, double W,
                   const double *abcd, double z, double *out) {
    int rc = valid_inputs(1, lam, 0.0, r1, th1, &w0, 1, NULL, &W, abcd, 1, NULL, 1e-10);
    if (rc) return rc;
    or_in b = load_in(0, lam, 0.0, r1, th1, &w0, 1, NULL, &W, abcd, 1, NULL, NULL);
    or_prop P;
    rc = propagate(&b, z, &P);
    if (rc) return rc;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            out[2 * (2 * i + j)] = creal(P.Qinv.m[i][j]);
            out[2 * (2 * i + j) + 1] = cimag(P.Qinv.m[i][j]);
        }
    out[8] = creal(P.gamma);
    out[9] = cimag(P.gamma);
    out[10] = P.r2[0];
    out[11] = P.r2[1];
    out[12] = P.th2[0];
    out[13] = P.th2[1];
    out[14] = P.tau;
    return OR_OK;
}

/* thread count of the OpenMP pixel loop (0 = leave the runtime default) */
#ifdef _OPENMP
#include <omp.h>
#endif
int oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* symplectic check exposed for the input-validation tests */
int oracle_symplectic_ok(const double *abcd) { return symplectic_ok(abcd, 1e-10); }
