// Point evaluation (the per-point algorithm that plane evaluation replaces,
// Sec. 2.2), paraxial form, FP64: every pixel evaluates every beamlet's exact
// paraxial field at the pixel's own 3-D position, i.e. the beamlet's system
// extended by free space to that pixel's axial distance z.  With
// Mm(z) = (A + zC) - i kappa (B + zD) = Mm0 + z Nm, Nm = C - i kappa D:
//   Q(z)^-1 det Mm(z) = Nm adj(Mm0) + z det(Nm) I        (complex-curvature law)
//   det Mm(z) = d0 + d1 z + d2 z^2,  tr Mm(z) = t0 + t1 z
// and the amplitude is the product of the principal roots of Mm(z)'s
// eigenvalues (Appendix C), recomputed per pixel.  On a plane normal to the
// axis this equals plane evaluation; on a tilted plane it is the exact
// paraxial reference the plane expansion approximates.
#include "gbd_device.h"

namespace gbd {

namespace {

using namespace dev;

__global__ void __launch_bounds__(256) point_setup_kernel(BeamletsDev b, double gturns, RecPt *__restrict__ out) {
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
    const double kappa = b.lam / (kPi * w0 * w0);
    RecPt o;
    const double *tb = b.base ? b.base + 5 * j : nullptr;  // traced base ray, if any
#pragma unroll
    for (int r = 0; r < 2; r++) {
        o.r2[r] = tb ? tb[r] : A[r][0] * r1[0] + A[r][1] * r1[1] + B[r][0] * t1[0] + B[r][1] * t1[1];
        o.th[r] = tb ? tb[2 + r] : C[r][0] * r1[0] + C[r][1] * r1[1] + D[r][0] * t1[0] + D[r][1] * t1[1];
    }
    cd M0[2][2], N[2][2];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int c = 0; c < 2; c++) {
            M0[r][c] = mk(A[r][c], -kappa * B[r][c]);
            N[r][c] = mk(C[r][c], -kappa * D[r][c]);
        }
    // P0 = N adj(M0), adj([[a, b], [c, d]]) = [[d, -b], [-c, a]]; symmetrised
    cd adj[2][2];
    adj[0][0] = M0[1][1];
    adj[1][1] = M0[0][0];
    adj[0][1] = scl(M0[0][1], -1.0);
    adj[1][0] = scl(M0[1][0], -1.0);
    cd P[2][2];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int c = 0; c < 2; c++) P[r][c] = add(mul(N[r][0], adj[0][c]), mul(N[r][1], adj[1][c]));
    const cd poff = scl(add(P[0][1], P[1][0]), 0.5);
    o.p00[0] = P[0][0].re; o.p00[1] = P[0][0].im;
    o.p01[0] = poff.re; o.p01[1] = poff.im;
    o.p11[0] = P[1][1].re; o.p11[1] = P[1][1].im;
    const cd d0 = sub(mul(M0[0][0], M0[1][1]), mul(M0[0][1], M0[1][0]));
    const cd d2 = sub(mul(N[0][0], N[1][1]), mul(N[0][1], N[1][0]));
    const cd d1 = sub(add(mul(M0[0][0], N[1][1]), mul(N[0][0], M0[1][1])),
                      add(mul(M0[0][1], N[1][0]), mul(N[0][1], M0[1][0])));
    o.d0[0] = d0.re; o.d0[1] = d0.im;
    o.d1[0] = d1.re; o.d1[1] = d1.im;
    o.d2[0] = d2.re; o.d2[1] = d2.im;
    const cd t0 = add(M0[0][0], M0[1][1]), tt = add(N[0][0], N[1][1]);
    o.t0[0] = t0.re; o.t0[1] = t0.im;
    o.t1[0] = tt.re; o.t1[1] = tt.im;
    o.amp[0] = b.amp[2 * j];
    o.amp[1] = b.amp[2 * j + 1];
    // turns: l0/lambda (reduced on the host) + (W + S0)/lambda, and per unit z
    const double S0 = tb ? tb[4] : 0.5 * (o.th[0] * o.r2[0] + o.th[1] * o.r2[1] - t1[0] * r1[0] - t1[1] * r1[1]);
    const double c0 = (b.path[j] + S0) / b.lam;
    const double c0r = (c0 - rint(c0)) + gturns;
    o.c0 = c0r - rint(c0r);
    o.c1 = (1.0 + 0.5 * (o.th[0] * o.th[0] + o.th[1] * o.th[1])) / b.lam;
    o.pad[0] = o.pad[1] = 0.0;
    out[j] = o;
}

// One pixel per lane; beamlet records staged through LDS.
__global__ void __launch_bounds__(256) point_eval_kernel(PlaneGeom pl, double lam, const RecPt *__restrict__ rec,
                                                         int64_t n, double2 *__restrict__ out,
                                                         uint32_t *__restrict__ status) {
    constexpr int CH = 32;
    __shared__ RecPt tile[CH];
    const int64_t M = (int64_t)pl.nx * pl.ny;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < M;
    const int iy = live ? (int)(p / pl.nx) : 0, ix = live ? (int)(p - (int64_t)iy * pl.nx) : 0;
    const double a = (ix - 0.5 * (pl.nx - 1)) * pl.dx, bb = (iy - 0.5 * (pl.ny - 1)) * pl.dy;
    const double X = pl.O[0] + a * pl.e1[0] + bb * pl.e2[0];
    const double Y = pl.O[1] + a * pl.e1[1] + bb * pl.e2[1];
    const double z = pl.O[2] + a * pl.e1[2] + bb * pl.e2[2];
    const double il = 1.0 / lam, pil = kPi / lam;
    double er = 0.0, ei = 0.0;
    bool bad = false;
    for (int64_t j0 = 0; j0 < n; j0 += CH) {
        const int cnt = (int)min((int64_t)CH, n - j0);
        __syncthreads();
        {
            const double2 *src = reinterpret_cast<const double2 *>(rec + j0);
            double2 *dst = reinterpret_cast<double2 *>(tile);
            constexpr int V = sizeof(RecPt) / 16;
            for (int i = threadIdx.x; i < cnt * V; i += 256) dst[i] = src[i];
        }
        __syncthreads();
        for (int jj = 0; jj < cnt; jj++) {
            const RecPt &r = tile[jj];
            const double w0 = X - r.r2[0] - z * r.th[0], w1 = Y - r.r2[1] - z * r.th[1];
            const cd det = add(mk(r.d0[0], r.d0[1]), scl(add(mk(r.d1[0], r.d1[1]), scl(mk(r.d2[0], r.d2[1]), z)), z));
            // w^T (Q det) w = w^T P0 w + z det(Nm) |w|^2
            const cd num = add(add(scl(mk(r.p00[0], r.p00[1]), w0 * w0), scl(mk(r.p01[0], r.p01[1]), 2.0 * w0 * w1)),
                               add(scl(mk(r.p11[0], r.p11[1]), w1 * w1), scl(mk(r.d2[0], r.d2[1]), z * (w0 * w0 + w1 * w1))));
            const cd wqw = cdiv(num, det);
            const cd tr = add(mk(r.t0[0], r.t0[1]), scl(mk(r.t1[0], r.t1[1]), z));
            const cd disc = csqrt_p(sub(mul(tr, tr), scl(det, 4.0)));
            const cd mu1 = scl(add(tr, disc), 0.5), mu2 = scl(sub(tr, disc), 0.5);
            bad = bad || !on_branch(mu1) || !on_branch(mu2);
            const cd g = mul(mk(r.amp[0], r.amp[1]), cdiv(mk(1.0, 0.0), mul(csqrt_p(mu1), csqrt_p(mu2))));
            // phase in turns: -(c0 + c1 z + th.w / lambda + Re(wQw) / (2 lambda)); amplitude e^{(pi/lambda) Im wQw}
            double T = r.c0 + r.c1 * z + (r.th[0] * w0 + r.th[1] * w1) * il + 0.5 * wqw.re * il;
            T -= rint(T);
            double s, c;
            sincospi(-2.0 * T, &s, &c);
            const double m = exp(pil * wqw.im);
            er += m * (g.re * c - g.im * s);
            ei += m * (g.re * s + g.im * c);
        }
    }
    if (bad && live) atomicOr(status, FLAG_BRANCH);
    if (live) out[p] = make_double2(er, ei);
}

}  // namespace

hipError_t launch_point(const BeamletsDev &b, const PlaneGeom &pl, double gturns, RecPt *rec, double2 *out,
                        uint32_t *status, hipStream_t s) {
    const int64_t M = (int64_t)pl.nx * pl.ny;
    if (b.n > 0) {
        point_setup_kernel<<<(unsigned)((b.n + 255) / 256), 256, 0, s>>>(b, gturns, rec);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (M == 0) return hipSuccess;
    point_eval_kernel<<<(unsigned)((M + 255) / 256), 256, 0, s>>>(pl, b.lam, rec, b.n, out, status);
    return hipGetLastError();
}

}  // namespace gbd
