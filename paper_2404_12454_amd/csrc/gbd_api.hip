// Host side of the C ABI declared in include/gbd.h.
#include "../../include/gbd.h"
#include "gbd_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

using namespace gbd;

struct gbd_ctx_s {
    int device;
    hipStream_t stream;
    int cus;
    gbd_plan_s *own_plan;  // plan used by gbd_eval
};

struct gbd_beamlets_s {
    gbd_ctx_s *ctx;
    BeamletsDev dev;
    void *mem;
};

struct gbd_plane_s {
    PlaneGeom g;
};

struct gbd_plan_s {
    gbd_ctx_s *ctx;
    int64_t capacity;
    int64_t n;
    PlaneGeom pl;
    bool ready;
    Rec64 *r64;
    Rec32 *r32;
    uint32_t *status_dev;
    uint32_t *status_host;  // pinned
    void *scratch;
    size_t scratch_bytes;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? GBD_ENOMEM : GBD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                    \
    do {                                       \
        hipError_t e_ = (call);                \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Ray-transfer matrices must be symplectic: M^T J M = J with
// J = [[0, I], [-I, 0]] (equivalent to the block relations of Sec. 2.1).
bool symplectic(const double *m) {
    static const double J[4][4] = {{0, 0, 1, 0}, {0, 0, 0, 1}, {-1, 0, 0, 0}, {0, -1, 0, 0}};
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            double v = 0.0, mag = 0.0;
            for (int i = 0; i < 4; i++)
                for (int k = 0; k < 4; k++) {
                    const double t = m[4 * i + r] * J[i][k] * m[4 * k + c];
                    v += t;
                    mag += fabs(t);
                }
            if (fabs(v - J[r][c]) > 1e-10 * (mag + fabs(J[r][c]))) return false;
        }
    return true;
}

bool finite_all(const double *p, int64_t count) {
    for (int64_t i = 0; i < count; i++)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int ensure_device(gbd_ctx_s *ctx) {
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    return GBD_OK;
}

struct Shape {
    int rows, waves, nseg;
};

Shape choose_shape(const gbd_ctx_s *ctx, int precision, int64_t n, const PlaneGeom &pl, const gbd_eval_opts *o) {
    Shape s;
    s.rows = (precision == GBD_MIXED) ? 8 : 4;
    s.waves = 4;
    s.nseg = 0;
    if (o) {
        if (o->rows_per_lane) s.rows = o->rows_per_lane;
        if (o->waves) s.waves = o->waves;
        if (o->segments) s.nseg = o->segments;
    }
    if (s.nseg <= 0) {
        // enough workgroups to keep every SIMD of every CU busy ~6 waves deep,
        // while each segment keeps at least two LDS tiles of beamlets
        const int64_t tx = (pl.nx + 63) / 64;
        const int64_t ty = (pl.ny + s.waves * s.rows - 1) / (s.waves * s.rows);
        const int64_t tiles = std::max<int64_t>(1, tx * ty);
        const int64_t target_blocks = (int64_t)ctx->cus * 4 * 6 / s.waves;
        int64_t seg = (target_blocks + tiles - 1) / tiles;
        seg = std::min<int64_t>(seg, std::max<int64_t>(1, n / 256));
        s.nseg = (int)std::max<int64_t>(1, std::min<int64_t>(seg, 1024));
    }
    return s;
}

bool valid_shape(int rows, int waves) {
    return (rows == 1 || rows == 2 || rows == 4 || rows == 8) && (waves == 1 || waves == 2 || waves == 4);
}

EvalGeom make_geom(const PlaneGeom &pl, int64_t n, const Shape &s) {
    EvalGeom g;
    g.nx = pl.nx;
    g.ny = pl.ny;
    g.dx = pl.dx;
    g.dy = pl.dy;
    g.a0 = -0.5 * (pl.nx - 1) * pl.dx;
    g.b0 = -0.5 * (pl.ny - 1) * pl.dy;
    g.tiles_x = (pl.nx + 63) / 64;
    g.tiles_y = (pl.ny + s.waves * s.rows - 1) / (s.waves * s.rows);
    g.n = n;
    int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(s.nseg, std::max<int64_t>(1, n)));
    g.seg_len = (n + nseg - 1) / nseg;
    if (g.seg_len == 0) g.seg_len = 1;
    g.nseg = (int32_t)((n + g.seg_len - 1) / g.seg_len);
    if (g.nseg < 1) g.nseg = 1;
    g.work = g.tiles_x * g.tiles_y * g.nseg;
    return g;
}

int plan_eval_impl(gbd_ctx_s *ctx, gbd_plan_s *plan, int precision, void *out, int64_t out_bytes,
                   const gbd_eval_opts *opts) {
    if (!plan->ready) return fail(GBD_EINVAL, "gbd_plan_eval: plan has no valid setup");
    if (precision != GBD_FP64 && precision != GBD_MIXED) return fail(GBD_EINVAL, "precision must be GBD_FP64 or GBD_MIXED");
    const int64_t M = (int64_t)plan->pl.nx * plan->pl.ny;
    const int64_t elem = precision == GBD_FP64 ? 16 : 8;
    if (M == 0) return GBD_OK;
    if (!out) return fail(GBD_EINVAL, "field_out is NULL");
    if (out_bytes < M * elem)
        return fail(GBD_ERANGE, "field_out holds %lld bytes, %lld needed", (long long)out_bytes, (long long)(M * elem));
    Shape s = choose_shape(ctx, precision, plan->n, plan->pl, opts);
    if (!valid_shape(s.rows, s.waves)) return fail(GBD_EINVAL, "unsupported rows_per_lane %d / waves %d", s.rows, s.waves);
    int rc = ensure_device(ctx);
    if (rc) return rc;
    if (plan->n == 0) {
        HIP_TRY(hipMemsetAsync(out, 0, (size_t)(M * elem), ctx->stream), "hipMemsetAsync");
        return GBD_OK;
    }
    EvalGeom g = make_geom(plan->pl, plan->n, s);
    if ((int64_t)g.tiles_x * g.tiles_y * g.nseg > (int64_t)0x7fffffff - 8)
        return fail(GBD_ERANGE, "grid too large");
    if (g.nseg > 1) {
        const size_t need = (size_t)g.nseg * (size_t)M * 16;
        if (need > plan->scratch_bytes) {
            if (plan->scratch) (void)hipFree(plan->scratch);
            plan->scratch = nullptr;
            plan->scratch_bytes = 0;
            HIP_TRY(hipMalloc(&plan->scratch, need), "hipMalloc(segment partials)");
            plan->scratch_bytes = need;
        }
    }
    const void *rec = precision == GBD_FP64 ? (const void *)plan->r64 : (const void *)plan->r32;
    HIP_TRY(launch_eval(precision, s.rows, s.waves, g, rec, plan->scratch, out, ctx->stream), "eval kernel launch");
    if (g.nseg > 1) HIP_TRY(launch_reduce(precision, g, plan->scratch, out, ctx->stream), "reduce kernel launch");
    return GBD_OK;
}

int plan_setup_impl(gbd_ctx_s *ctx, gbd_plan_s *plan, gbd_beamlets_s *b, gbd_plane_s *p) {
    if (b->dev.n > plan->capacity)
        return fail(GBD_ERANGE, "plan capacity %lld < %lld beamlets", (long long)plan->capacity, (long long)b->dev.n);
    int rc = ensure_device(ctx);
    if (rc) return rc;
    plan->ready = false;
    plan->n = b->dev.n;
    plan->pl = p->g;
    if (b->dev.n > 0) {
        // the axial term l0 / lambda is common to every beamlet: reduce it once
        const double g0 = b->dev.l0 / b->dev.lam;
        const double gturns = g0 - nearbyint(g0);
        HIP_TRY(hipMemsetAsync(plan->status_dev, 0, sizeof(uint32_t), ctx->stream), "hipMemsetAsync(status)");
        HIP_TRY(launch_setup(b->dev, p->g, gturns, plan->r64, plan->r32, plan->status_dev, ctx->stream),
                "setup kernel launch");
        HIP_TRY(hipMemcpyAsync(plan->status_host, plan->status_dev, sizeof(uint32_t), hipMemcpyDeviceToHost,
                               ctx->stream),
                "status copy");
        HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        const uint32_t st = *plan->status_host;
        if (st & FLAG_PARALLEL) return fail(GBD_EPARALLEL, "a base ray is parallel to the detector plane");
        if (st & FLAG_BRANCH)
            return fail(GBD_EBRANCH, "an eigenvalue of A + B Q1^-1 lies off the principal branch (inverting system)");
        if (st & FLAG_NONFINITE) return fail(GBD_EINVAL, "non-finite beamlet parameters after propagation");
    }
    plan->ready = true;
    return GBD_OK;
}

void plan_destroy(gbd_plan_s *plan) {
    if (!plan) return;
    if (plan->r64) (void)hipFree(plan->r64);
    if (plan->r32) (void)hipFree(plan->r32);
    if (plan->status_dev) (void)hipFree(plan->status_dev);
    if (plan->status_host) (void)hipHostFree(plan->status_host);
    if (plan->scratch) (void)hipFree(plan->scratch);
    delete plan;
}

int plan_new(gbd_ctx_s *ctx, int64_t capacity, gbd_plan_s **out) {
    gbd_plan_s *p = new (std::nothrow) gbd_plan_s();
    if (!p) return fail(GBD_ENOMEM, "host allocation failed");
    p->ctx = ctx;
    p->capacity = capacity;
    const size_t cap = (size_t)std::max<int64_t>(1, capacity);
    hipError_t e = hipMalloc(&p->r64, cap * sizeof(Rec64));
    if (e == hipSuccess) e = hipMalloc(&p->r32, cap * sizeof(Rec32));
    if (e == hipSuccess) e = hipMalloc(&p->status_dev, sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc(&p->status_host, sizeof(uint32_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        plan_destroy(p);
        return hip_fail(e, "plan allocation");
    }
    *out = p;
    return GBD_OK;
}

}  // namespace

extern "C" {

const char *gbd_last_error(void) { return g_err.c_str(); }

int gbd_ctx_create(gbd_ctx_t *out, int device, void *hip_stream) {
    if (!out) return fail(GBD_EINVAL, "out is NULL");
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count), "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(GBD_EINVAL, "device %d out of range (%d devices)", device, count);
    HIP_TRY(hipSetDevice(device), "hipSetDevice");
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
    gbd_ctx_s *c = new (std::nothrow) gbd_ctx_s();
    if (!c) return fail(GBD_ENOMEM, "host allocation failed");
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->cus = cus > 0 ? cus : 256;
    c->own_plan = nullptr;
    *out = c;
    return GBD_OK;
}

int gbd_ctx_set_stream(gbd_ctx_t ctx, void *hip_stream) {
    if (!ctx) return fail(GBD_EINVAL, "ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return GBD_OK;
}

void gbd_ctx_destroy(gbd_ctx_t ctx) {
    if (!ctx) return;
    plan_destroy(ctx->own_plan);
    delete ctx;
}

int gbd_beamlets(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0, const double *r1,
                 const double *th1, const double *w0, int64_t n_w0, const double *amp, const double *path,
                 const double *abcd, int64_t n_abcd) {
    if (!ctx || !out) return fail(GBD_EINVAL, "ctx/out is NULL");
    if (n < 0) return fail(GBD_EINVAL, "n < 0");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(GBD_EINVAL, "lambda must be finite and > 0");
    if (!std::isfinite(l0)) return fail(GBD_EINVAL, "l0 must be finite");
    if (n > 0) {
        if (!r1 || !w0 || !abcd) return fail(GBD_EINVAL, "r1, w0 and abcd are required");
        if (!(n_w0 == 1 || n_w0 == n)) return fail(GBD_EINVAL, "n_w0 must be 1 or n");
        if (!(n_abcd == 1 || n_abcd == n)) return fail(GBD_EINVAL, "n_abcd must be 1 or n");
        if (!finite_all(r1, 2 * n) || (th1 && !finite_all(th1, 2 * n)) || (amp && !finite_all(amp, 2 * n)) ||
            (path && !finite_all(path, n)) || !finite_all(abcd, 16 * n_abcd))
            return fail(GBD_EINVAL, "non-finite input");
        for (int64_t i = 0; i < n_w0; i++)
            if (!(w0[i] > 0.0) || !std::isfinite(w0[i])) return fail(GBD_EINVAL, "w0[%lld] must be finite and > 0", (long long)i);
        for (int64_t i = 0; i < n_abcd; i++)
            if (!symplectic(abcd + 16 * i))
                return fail(GBD_ENOTSYMPLECTIC, "abcd[%lld] is not symplectic", (long long)i);
    } else {
        n_w0 = 1;
        n_abcd = 1;
    }
    int rc = ensure_device(ctx);
    if (rc) return rc;
    // one device block: r1, th1, amp [n][2]; w0 [n_w0]; path [n]; abcd [n_abcd][16]
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    const size_t off_r1 = 0, off_th1 = off_r1 + 2 * nn, off_amp = off_th1 + 2 * nn, off_w0 = off_amp + 2 * nn,
                 off_path = off_w0 + (size_t)n_w0, off_abcd = off_path + nn, total = off_abcd + 16 * (size_t)n_abcd;
    std::vector<double> host(total, 0.0);
    if (n > 0) {
        memcpy(&host[off_r1], r1, 2 * n * sizeof(double));
        if (th1) memcpy(&host[off_th1], th1, 2 * n * sizeof(double));
        if (amp)
            memcpy(&host[off_amp], amp, 2 * n * sizeof(double));
        else
            for (int64_t j = 0; j < n; j++) host[off_amp + 2 * j] = 1.0;
        memcpy(&host[off_w0], w0, n_w0 * sizeof(double));
        if (path) memcpy(&host[off_path], path, n * sizeof(double));
        memcpy(&host[off_abcd], abcd, 16 * n_abcd * sizeof(double));
    } else {
        host[off_w0] = 1.0;
        for (int i = 0; i < 4; i++) host[off_abcd + 5 * i] = 1.0;
    }
    void *mem = nullptr;
    HIP_TRY(hipMalloc(&mem, total * sizeof(double)), "hipMalloc(beamlets)");
    hipError_t e = hipMemcpyAsync(mem, host.data(), total * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(e, "beamlet upload");
    }
    gbd_beamlets_s *b = new (std::nothrow) gbd_beamlets_s();
    if (!b) {
        (void)hipFree(mem);
        return fail(GBD_ENOMEM, "host allocation failed");
    }
    double *d = static_cast<double *>(mem);
    b->ctx = ctx;
    b->mem = mem;
    b->dev.n = n;
    b->dev.n_w0 = n_w0;
    b->dev.n_abcd = n_abcd;
    b->dev.lam = lambda;
    b->dev.l0 = l0;
    b->dev.r1 = d + off_r1;
    b->dev.th1 = d + off_th1;
    b->dev.amp = d + off_amp;
    b->dev.w0 = d + off_w0;
    b->dev.path = d + off_path;
    b->dev.abcd = d + off_abcd;
    *out = b;
    return GBD_OK;
}

void gbd_beamlets_free(gbd_beamlets_t b) {
    if (!b) return;
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

int gbd_plane(gbd_ctx_t ctx, gbd_plane_t *out, const double origin[3], const double normal[3], const double xhint[3],
              int32_t nx, int32_t ny, double dx, double dy) {
    if (!ctx || !out || !origin || !normal || !xhint) return fail(GBD_EINVAL, "NULL argument");
    if (nx < 0 || ny < 0) return fail(GBD_EINVAL, "nx, ny must be >= 0");
    if (!(dx > 0.0) || !(dy > 0.0) || !std::isfinite(dx) || !std::isfinite(dy)) return fail(GBD_EINVAL, "dx, dy must be finite and > 0");
    if (!finite_all(origin, 3) || !finite_all(normal, 3) || !finite_all(xhint, 3)) return fail(GBD_EINVAL, "non-finite plane");
    PlaneGeom g;
    const double nn = sqrt(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2]);
    if (!(nn > 0.0)) return fail(GBD_EINVAL, "normal has zero length");
    for (int i = 0; i < 3; i++) {
        g.O[i] = origin[i];
        g.n[i] = normal[i] / nn;
    }
    // e1: xhint with its normal component removed (Gram-Schmidt); e2 = n x e1
    const double hn = xhint[0] * g.n[0] + xhint[1] * g.n[1] + xhint[2] * g.n[2];
    double e1[3];
    for (int i = 0; i < 3; i++) e1[i] = xhint[i] - hn * g.n[i];
    const double el = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    const double hl = sqrt(xhint[0] * xhint[0] + xhint[1] * xhint[1] + xhint[2] * xhint[2]);
    if (!(el > 1e-9 * hl)) return fail(GBD_EINVAL, "xhint is parallel to the normal");
    for (int i = 0; i < 3; i++) g.e1[i] = e1[i] / el;
    g.e2[0] = g.n[1] * g.e1[2] - g.n[2] * g.e1[1];
    g.e2[1] = g.n[2] * g.e1[0] - g.n[0] * g.e1[2];
    g.e2[2] = g.n[0] * g.e1[1] - g.n[1] * g.e1[0];
    g.nx = nx;
    g.ny = ny;
    g.dx = dx;
    g.dy = dy;
    gbd_plane_s *p = new (std::nothrow) gbd_plane_s();
    if (!p) return fail(GBD_ENOMEM, "host allocation failed");
    p->g = g;
    *out = p;
    return GBD_OK;
}

void gbd_plane_free(gbd_plane_t p) { delete p; }

int gbd_plan_create(gbd_ctx_t ctx, gbd_plan_t *out, int64_t capacity) {
    if (!ctx || !out) return fail(GBD_EINVAL, "ctx/out is NULL");
    if (capacity < 0) return fail(GBD_EINVAL, "capacity < 0");
    int rc = ensure_device(ctx);
    if (rc) return rc;
    return plan_new(ctx, capacity, out);
}

int gbd_plan_setup(gbd_ctx_t ctx, gbd_plan_t plan, gbd_beamlets_t b, gbd_plane_t p) {
    if (!ctx || !plan || !b || !p) return fail(GBD_EINVAL, "NULL argument");
    return plan_setup_impl(ctx, plan, b, p);
}

int gbd_plan_eval(gbd_ctx_t ctx, gbd_plan_t plan, int precision, void *field_out, int64_t out_bytes,
                  const gbd_eval_opts *opts) {
    if (!ctx || !plan) return fail(GBD_EINVAL, "NULL argument");
    return plan_eval_impl(ctx, plan, precision, field_out, out_bytes, opts);
}

void gbd_plan_free(gbd_plan_t plan) { plan_destroy(plan); }

int gbd_plan_shape(gbd_ctx_t ctx, gbd_plan_t plan, int precision, const gbd_eval_opts *opts, gbd_eval_opts *resolved) {
    if (!ctx || !plan || !resolved) return fail(GBD_EINVAL, "NULL argument");
    Shape s = choose_shape(ctx, precision, plan->n, plan->pl, opts);
    EvalGeom g = make_geom(plan->pl, plan->n, s);
    resolved->rows_per_lane = s.rows;
    resolved->waves = s.waves;
    resolved->segments = g.nseg;
    resolved->reserved = 0;
    return GBD_OK;
}

int gbd_eval(gbd_ctx_t ctx, gbd_beamlets_t b, gbd_plane_t p, int precision, void *field_out, int64_t out_bytes,
             const gbd_eval_opts *opts) {
    if (!ctx || !b || !p) return fail(GBD_EINVAL, "NULL argument");
    if (precision != GBD_FP64 && precision != GBD_MIXED) return fail(GBD_EINVAL, "precision must be GBD_FP64 or GBD_MIXED");
    const int64_t M = (int64_t)p->g.nx * p->g.ny;
    const int64_t elem = precision == GBD_FP64 ? 16 : 8;
    if (M > 0 && !field_out) return fail(GBD_EINVAL, "field_out is NULL");
    if (M > 0 && out_bytes < M * elem)
        return fail(GBD_ERANGE, "field_out holds %lld bytes, %lld needed", (long long)out_bytes, (long long)(M * elem));
    if (!ctx->own_plan || ctx->own_plan->capacity < b->dev.n) {
        plan_destroy(ctx->own_plan);
        ctx->own_plan = nullptr;
        int rc = ensure_device(ctx);
        if (rc) return rc;
        rc = plan_new(ctx, std::max<int64_t>(b->dev.n, 1024), &ctx->own_plan);
        if (rc) return rc;
    }
    int rc = plan_setup_impl(ctx, ctx->own_plan, b, p);
    if (rc) return rc;
    return plan_eval_impl(ctx, ctx->own_plan, precision, field_out, out_bytes, opts);
}

}  // extern "C"
