/*
 * raytrace.c -- plain FP64 sequential real-ray trace through conic mirrors,
 * giving every beamlet's base ray and its differential ray-transfer matrix
 * from parabasal rays (the inputs the point-evaluation algorithm of Sec. 2.2
 * obtains from ray tracing; the system is the Ritchey-Chretien telescope of
 * Appendix B).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  The product path
 * (the HIP library) never calls it, and the two share no code.
 *
 * Geometry.  Global frame, z the optical axis, metres, refractive index 1.
 * A mirror is a conic of revolution with vertex at z = zv, vertex curvature
 * c = 1/R (R signed in the global frame: the surface's centre of curvature is
 * at zv + R) and conic constant k:
 *     F(x, y, z) = c (x^2 + y^2) - 2 (z - zv) + (1 + k) c (z - zv)^2 = 0,
 * equivalently the sag z - zv = c r^2 / (1 + sqrt(1 - (1 + k) c^2 r^2)).
 * A ray p + t d (unit d, t the geometric and optical path) meets it at the
 * nearest forward root of the quadratic F(p + t d) = 0 that lies on the
 * sheet through the vertex; it is reflected as
 * d' = d - 2 (d . n) n with n = grad F / |grad F|.  A ray whose hit lies
 * outside the clear annulus [r_min, r_max] is vignetted.
 *
 * Ray coordinates are (x, y, l, m): position on a plane z = const and the x,
 * y direction cosines (canonical coordinates, so the differential matrix is
 * symplectic).  After an odd number of reflections the output travels -z;
 * the output frame is then turned by pi about the x axis (y -> -y, m -> -m)
 * so that it looks along its own direction of travel.
 *
 * Differential matrix.  Each of the four input coordinates is perturbed by
 * +-h (h = dr for positions, dth for direction cosines) and the parabasal
 * rays traced; the central differences form the 4 x 4 matrix
 * d(x2, y2, l2, m2) / d(x1, y1, l1, m1) = [[A, B], [C, D]].
 */
#include <math.h>
#include <stdint.h>

#define RT_OK 0
#define RT_EINVAL (-1)

enum { RT_VIGNETTED = 1, RT_MISSED = 2, RT_BACKWARD = 4 };

typedef struct {
    double zv, c, k, rmin, rmax;
} rt_mirror;

typedef struct {
    double x, y, l, m, opl;
    int flags;
} rt_out;

/* The nearest forward intersection t > 0 of the ray with the conic's vertex
 * sheet.  F(q + t d) = a t^2 + 2 b t + c0; its roots, in the cancellation-free
 * pair of forms, are kept if they lie on the sheet through the vertex, where
 * 1 - (1 + k) c (z - zv) >= 0 (the sag formula's branch). */
static int surface_hit(double a, double b, double c0, double ak, double qz, double dz, double *t) {
    double r[2];
    int nr = 0;
    if (a == 0.0) {
        if (b == 0.0) return 0;
        r[nr++] = -c0 / (2.0 * b);
    } else {
        const double disc = b * b - a * c0;
        if (disc < 0.0) return 0;
        const double s = sqrt(disc);
        const double qq = -(b + (b >= 0.0 ? s : -s));
        r[nr++] = qq / a;
        if (qq != 0.0) r[nr++] = c0 / qq;
    }
    int found = 0;
    for (int i = 0; i < nr; i++) {
        if (!(r[i] > 0.0)) continue;
        if (1.0 - ak * (qz + r[i] * dz) < 0.0) continue;
        if (!found || r[i] < *t) *t = r[i];
        found = 1;
    }
    return found;
}

static rt_out trace_one(int nm, const rt_mirror *mir, double z_in, double z_out, double x, double y,
                        double l, double m) {
    rt_out o = {0, 0, 0, 0, 0, 0};
    const double nz2 = 1.0 - l * l - m * m;
    if (!(nz2 > 0.0)) {
        o.flags = RT_MISSED;
        return o;
    }
    double p[3] = {x, y, z_in}, d[3] = {l, m, sqrt(nz2)};
    double path = 0.0;
    for (int s = 0; s < nm; s++) {
        const rt_mirror *M = &mir[s];
        const double q[3] = {p[0], p[1], p[2] - M->zv};
        const double ak = (1.0 + M->k) * M->c;
        const double a = M->c * (d[0] * d[0] + d[1] * d[1]) + ak * d[2] * d[2];
        const double b = M->c * (q[0] * d[0] + q[1] * d[1]) - d[2] + ak * q[2] * d[2];
        const double c0 = M->c * (q[0] * q[0] + q[1] * q[1]) - 2.0 * q[2] + ak * q[2] * q[2];
        double t = 0.0;
        if (!surface_hit(a, b, c0, ak, q[2], d[2], &t)) {
            o.flags |= RT_MISSED;
            return o;
        }
        for (int i = 0; i < 3; i++) p[i] += t * d[i];
        path += t;
        const double r = hypot(p[0], p[1]);
        if (r < M->rmin || r > M->rmax) o.flags |= RT_VIGNETTED;
        /* unit normal and reflection */
        double g[3] = {2.0 * M->c * p[0], 2.0 * M->c * p[1], -2.0 + 2.0 * ak * (p[2] - M->zv)};
        const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        for (int i = 0; i < 3; i++) g[i] /= gn;
        const double dn = d[0] * g[0] + d[1] * g[1] + d[2] * g[2];
        for (int i = 0; i < 3; i++) d[i] -= 2.0 * dn * g[i];
    }
    if (d[2] == 0.0) {
        o.flags |= RT_MISSED;
        return o;
    }
    const double t = (z_out - p[2]) / d[2];
    if (t < 0.0) o.flags |= RT_BACKWARD;
    for (int i = 0; i < 3; i++) p[i] += t * d[i];
    path += t;
    const double sgn = d[2] > 0.0 ? 1.0 : -1.0;
    o.x = p[0];
    o.y = sgn * p[1];
    o.l = d[0];
    o.m = sgn * d[1];
    o.opl = path;
    return o;
}

/*
 * oracle_trace: n base rays (x1, y1) on the plane z = z_in with direction
 * cosines (l1, m1) (th1 may be NULL: along +z) through nm mirrors given as
 * [nm][5] = (zv, R, k, r_min, r_max) (R = 0: plane mirror), to the plane
 * z = z_out.  Writes base[n][5] = (x2, y2, l2, m2, opl - l0),
 * abcd[n][16] (row-major [[A, B], [C, D]]) and flags[n] (RT_* bits of the
 * base ray and its eight parabasal rays; 0 = clean).  Returns 0 or RT_EINVAL.
 */
int oracle_trace(int32_t nm, const double *mirrors, double z_in, double z_out, double l0, int64_t n,
                 const double *r1, const double *th1, double dr, double dth, double *base, double *abcd,
                 int32_t *flags) {
    if (nm < 0 || nm > 64 || n < 0 || !(dr > 0.0) || !(dth > 0.0)) return RT_EINVAL;
    if (n > 0 && (!r1 || !base || !abcd || !flags)) return RT_EINVAL;
    if (nm > 0 && !mirrors) return RT_EINVAL;
    rt_mirror mir[64];
    for (int s = 0; s < nm; s++) {
        const double *e = mirrors + 5 * s;
        for (int i = 0; i < 5; i++)
            if (!isfinite(e[i])) return RT_EINVAL;
        mir[s].zv = e[0];
        mir[s].c = e[1] == 0.0 ? 0.0 : 1.0 / e[1];
        mir[s].k = e[2];
        mir[s].rmin = e[3];
        mir[s].rmax = e[4];
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; j++) {
        const double in[4] = {r1[2 * j], r1[2 * j + 1], th1 ? th1[2 * j] : 0.0, th1 ? th1[2 * j + 1] : 0.0};
        const rt_out o = trace_one(nm, mir, z_in, z_out, in[0], in[1], in[2], in[3]);
        int fl = o.flags;
        base[5 * j + 0] = o.x;
        base[5 * j + 1] = o.y;
        base[5 * j + 2] = o.l;
        base[5 * j + 3] = o.m;
        base[5 * j + 4] = o.opl - l0;
        for (int col = 0; col < 4; col++) {
            const double h = col < 2 ? dr : dth;
            double a[4], b[4];
            for (int i = 0; i < 4; i++) a[i] = b[i] = in[i];
            a[col] += h;
            b[col] -= h;
            const rt_out p = trace_one(nm, mir, z_in, z_out, a[0], a[1], a[2], a[3]);
            const rt_out q = trace_one(nm, mir, z_in, z_out, b[0], b[1], b[2], b[3]);
            fl |= p.flags | q.flags;
            const double dp[4] = {p.x - q.x, p.y - q.y, p.l - q.l, p.m - q.m};
            for (int row = 0; row < 4; row++) abcd[16 * j + 4 * row + col] = dp[row] / (2.0 * h);
        }
        flags[j] = fl;
    }
    return RT_OK;
}
