// Real-ray trace through a sequence of conic mirrors, FP64, one beamlet per
// lane: the base ray and eight parabasal rays (each input coordinate -/+ h)
// give the beamlet's traced base ray at the output plane and its
// differential ray-transfer matrix by central differences (the base and
// parabasal rays of the point-evaluation algorithm, Sec. 2.2; the system of
// Appendix B is two conic mirrors).
//
// A mirror: vertex z_v, vertex curvature c = 1/R, conic k; with u = z - z_v
// its surface is G = c (x^2 + y^2) + (1 + k) c u^2 - 2 u = 0 and the part
// used is the sheet through the vertex, 1 - (1 + k) c u >= 0.  Along a ray
// (unit direction e) G is a quadratic in the path s; the nearest root s > 0
// on that sheet is the hit, and e turns into e - 2 (e . m) m with m the unit
// gradient of G.  Coordinates: position on the planes z_in / z_out and the x,
// y direction cosines (canonical, so the exact ray map is symplectic); after
// an odd number of reflections the output frame is the global one turned by
// pi about x.
#include "gbd_device.h"

namespace gbd {

namespace {

struct TraceRay {
    double x, y, l, m, path;
    uint32_t flags;
};

__device__ inline TraceRay trace_ray(const TraceSystem &S, double x, double y, double l, double m) {
    TraceRay out{0.0, 0.0, 0.0, 0.0, 0.0, 0u};
    const double n2 = 1.0 - (l * l + m * m);
    if (!(n2 > 0.0)) {
        out.flags = TRACE_MISSED;
        return out;
    }
    double P[3] = {x, y, S.z_in};
    double e[3] = {l, m, sqrt(n2)};
    double s_tot = 0.0;
    for (int i = 0; i < S.n; i++) {
        const TraceMirror &M = S.m[i];
        const double ck = (1.0 + M.k) * M.c;
        const double u = P[2] - M.zv;
        // G(P + s e) = A2 s^2 + 2 A1 s + A0
        const double A2 = M.c * (e[0] * e[0] + e[1] * e[1]) + ck * e[2] * e[2];
        const double A1 = M.c * (P[0] * e[0] + P[1] * e[1]) + ck * u * e[2] - e[2];
        const double A0 = M.c * (P[0] * P[0] + P[1] * P[1]) + ck * u * u - 2.0 * u;
        double root[2];
        int nroot = 0;
        if (A2 != 0.0) {
            const double D = A1 * A1 - A2 * A0;
            if (D >= 0.0) {
                const double w = -A1 - copysign(sqrt(D), A1);
                root[nroot++] = w / A2;
                if (w != 0.0) root[nroot++] = A0 / w;
            }
        } else if (A1 != 0.0) {
            root[nroot++] = -0.5 * A0 / A1;
        }
        double s = -1.0;
        for (int r = 0; r < nroot; r++)
            if (root[r] > 0.0 && 1.0 - ck * (u + root[r] * e[2]) >= 0.0 && (s < 0.0 || root[r] < s)) s = root[r];
        if (!(s > 0.0)) {
            out.flags |= TRACE_MISSED;
            return out;
        }
        P[0] += s * e[0];
        P[1] += s * e[1];
        P[2] += s * e[2];
        s_tot += s;
        const double rho = sqrt(P[0] * P[0] + P[1] * P[1]);
        if (rho < M.r_min || rho > M.r_max) out.flags |= TRACE_VIGNETTED;
        // unit gradient of G and the mirror reflection
        const double g0 = M.c * P[0], g1 = M.c * P[1], g2 = ck * (P[2] - M.zv) - 1.0;
        const double gi = 1.0 / sqrt(g0 * g0 + g1 * g1 + g2 * g2);
        const double proj = 2.0 * (e[0] * g0 + e[1] * g1 + e[2] * g2) * gi * gi;
        e[0] -= proj * g0;
        e[1] -= proj * g1;
        e[2] -= proj * g2;
    }
    if (e[2] == 0.0) {
        out.flags |= TRACE_MISSED;
        return out;
    }
    const double s = (S.z_out - P[2]) / e[2];
    if (s < 0.0) out.flags |= TRACE_BACKWARD;
    const double flip = e[2] > 0.0 ? 1.0 : -1.0;
    out.x = P[0] + s * e[0];
    out.y = flip * (P[1] + s * e[1]);
    out.l = e[0];
    out.m = flip * e[1];
    out.path = s_tot + s;
    return out;
}

__global__ void __launch_bounds__(128) trace_kernel(TraceSystem S, int64_t n, const double *__restrict__ r1,
                                                    const double *__restrict__ th1, double h_r, double h_t,
                                                    double *__restrict__ base, double *__restrict__ abcd,
                                                    int32_t *__restrict__ flags) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double v[4] = {r1[2 * j], r1[2 * j + 1], th1 ? th1[2 * j] : 0.0, th1 ? th1[2 * j + 1] : 0.0};
    const TraceRay b = trace_ray(S, v[0], v[1], v[2], v[3]);
    uint32_t fl = b.flags;
    base[5 * j + 0] = b.x;
    base[5 * j + 1] = b.y;
    base[5 * j + 2] = b.l;
    base[5 * j + 3] = b.m;
    base[5 * j + 4] = b.path - S.l0;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const double h = c < 2 ? h_r : h_t;
        double up[4] = {v[0], v[1], v[2], v[3]}, dn[4] = {v[0], v[1], v[2], v[3]};
        up[c] += h;
        dn[c] -= h;
        const TraceRay p = trace_ray(S, up[0], up[1], up[2], up[3]);
        const TraceRay q = trace_ray(S, dn[0], dn[1], dn[2], dn[3]);
        fl |= p.flags | q.flags;
        const double inv = 0.5 / h;
        abcd[16 * j + 0 + c] = (p.x - q.x) * inv;
        abcd[16 * j + 4 + c] = (p.y - q.y) * inv;
        abcd[16 * j + 8 + c] = (p.l - q.l) * inv;
        abcd[16 * j + 12 + c] = (p.m - q.m) * inv;
    }
    flags[j] = (int32_t)fl;
}

}  // namespace

hipError_t launch_trace(const TraceSystem &S, int64_t n, const double *r1, const double *th1, double h_r,
                        double h_t, double *base, double *abcd, int32_t *flags, hipStream_t s) {
    if (n == 0) return hipSuccess;
    trace_kernel<<<(unsigned)((n + 127) / 128), 128, 0, s>>>(S, n, r1, th1, h_r, h_t, base, abcd, flags);
    return hipGetLastError();
}

}  // namespace gbd
