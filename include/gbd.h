/*
 * gbd.h -- C ABI of the MI355X plane-evaluation Gaussian beamlet
 * decomposition library (arXiv:2404.12454, "A Generalized Expression for
 * Accelerating Beamlet Decomposition Simulations").
 *
 * The library evaluates, at every pixel of a (possibly tilted) detector
 * plane, the coherent sum of N complex Gaussian beamlets (Sec. 1, sum-of-
 * Gaussians equation).  Each beamlet is propagated once through its 4x4
 * ray-transfer matrix with the Gaussian solution of the Collins integral
 * (Sec. 4.1, complex-curvature law) and aligned to the common plane with the
 * misalignment phase of Sec. 3 (plane-evaluation) / Appendix A; the field
 * over the plane is then a per-beamlet phasor evaluated at every pixel.
 *
 * Conventions
 *  - Metres; paraxial slopes; ray vectors ordered (x, y, theta_x, theta_y);
 *    4x4 matrices row-major with 2x2 blocks [[A, B], [C, D]].
 *  - Time dependence exp(+i w t): a path L contributes exp(-i k L); a beamlet
 *    is exp(-(i k/2) r^T Q^-1 r) with Q^-1 = 1/R - i lambda/(pi w^2).
 *  - World frame: z is the optical axis measured from the ABCD output plane.
 *  - Pixel (ix, iy) of a plane sits at origin + a e1 + b e2 with
 *    a = (ix - (nx-1)/2) dx, b = (iy - (ny-1)/2) dy; e1 is xhint projected
 *    onto the plane (normalised), e2 = normal x e1.  Fields are [ny][nx].
 *  - Host input arrays are borrowed: copied during the call, never retained.
 *    Handles are owned by the caller and released with the *_free calls.
 *  - Device output buffers are caller-owned and written asynchronously on the
 *    context's HIP stream; the caller synchronises that stream.
 *  - Every entry point returns GBD_OK (0) or a negative GBD_E* code and sets
 *    a thread-local message readable with gbd_last_error().  Arguments are
 *    validated before any launch, so a failing call writes no output.
 *  - Not thread-safe per handle; distinct contexts may be used concurrently.
 */
#ifndef GBD_H
#define GBD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GBD_OK = 0,
    GBD_EINVAL = -1,          /* bad argument, non-finite input, w0 <= 0, bad plane */
    GBD_ENOTSYMPLECTIC = -2,  /* an ABCD violates the symplectic relations (Sec. 2.1) */
    GBD_EBRANCH = -3,         /* an eigenvalue of A + B Q1^-1 leaves the principal branch */
    GBD_EPARALLEL = -4,       /* a base ray is parallel to the detector plane */
    GBD_ENOMEM = -5,          /* device allocation failed */
    GBD_EHIP = -6,            /* HIP runtime error (message has the HIP error string) */
    GBD_ERANGE = -7           /* output buffer too small / size beyond a stated maximum */
};

enum { GBD_FP64 = 0, GBD_MIXED = 1 };

typedef struct gbd_ctx_s *gbd_ctx_t;
typedef struct gbd_beamlets_s *gbd_beamlets_t;
typedef struct gbd_plane_s *gbd_plane_t;
typedef struct gbd_plan_s *gbd_plan_t;

/* Launch shape of the N x M evaluation kernels.  All-zero = library choice
 * (autotuner cache if filled, else built-in defaults). */
typedef struct {
    int32_t rows_per_lane;  /* pixels per lane along a detector column: 1, 2, 4 or 8 */
    int32_t waves;          /* wavefronts per workgroup: 1, 2 or 4 */
    int32_t segments;       /* beamlet segments evaluated by separate workgroups, 0 = auto */
    int32_t reserved;
} gbd_eval_opts;

/* --- context ------------------------------------------------------------ */

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
int gbd_ctx_create(gbd_ctx_t *out, int device, void *hip_stream);
/* Rebind the context to another stream of the same device. */
int gbd_ctx_set_stream(gbd_ctx_t ctx, void *hip_stream);
void gbd_ctx_destroy(gbd_ctx_t ctx);
/* Thread-local description of the last failure in this thread. */
const char *gbd_last_error(void);

/* --- a1: pupil decomposition (Sec. 2.2 beamlet decomposition, Sec. 6 OF) --
 * n beamlets; lambda > 0 (m); l0 = axial length of the ABCD system (m),
 * the axial propagation distance of the Collins integral (Sec. 2.1).
 *   r1   [n][2]        beamlet centres in the input plane (required)
 *   th1  [n][2]        base-ray slopes in the input plane (NULL = 0)
 *   w0   [n_w0]        1/e field waist, n_w0 == 1 (shared) or n, all > 0
 *   amp  [n][2]        complex amplitude re, im (NULL = 1)
 *   path [n]           input optical path W_j of the beamlet centre (NULL = 0)
 *   abcd [n_abcd][16]  row-major 4x4 ray-transfer matrices, n_abcd == 1 or n;
 *                      each must satisfy the symplectic relations (Sec. 2.1)
 *                      to 1e-10 relative, else GBD_ENOTSYMPLECTIC.
 * n == 0 is allowed (the field is then zero).  The inputs are validated,
 * copied and uploaded to device memory owned by the handle. */
int gbd_beamlets(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0,
                 const double *r1, const double *th1, const double *w0, int64_t n_w0,
                 const double *amp, const double *path, const double *abcd, int64_t n_abcd);
void gbd_beamlets_free(gbd_beamlets_t b);

/* --- detector plane (Sec. 3: the common evaluation plane) ----------------
 * origin[3], normal[3] (any length > 0), xhint[3] (not parallel to normal);
 * nx, ny >= 0 pixels of pitch dx, dy > 0.  Planes need not be normal to the
 * optical axis (tilted-detector extension; exact when normal is along z). */
int gbd_plane(gbd_ctx_t ctx, gbd_plane_t *out, const double origin[3], const double normal[3],
              const double xhint[3], int32_t nx, int32_t ny, double dx, double dy);
void gbd_plane_free(gbd_plane_t p);

/* --- a4/a5: field evaluation ----------------------------------------------
 * field_out: device pointer to [ny][nx] interleaved complex: complex128 for
 * GBD_FP64 (all-FP64 arithmetic), complex64 for GBD_MIXED (FP64 phase and
 * coordinates, FP32 exp2/sin/cos, FP32 compensated accumulation).
 * out_bytes: size of field_out in bytes (GBD_ERANGE if too small).
 * Runs the per-beamlet setup (a2/a3) and the N x M evaluation on the
 * context stream.  Plane-dependent checks (GBD_EPARALLEL, GBD_EBRANCH) are
 * made by the setup kernel; this call synchronises on them before launching
 * the evaluation, so a failing call leaves field_out untouched. */
int gbd_eval(gbd_ctx_t ctx, gbd_beamlets_t b, gbd_plane_t p, int precision, void *field_out,
             int64_t out_bytes, const gbd_eval_opts *opts);

/* Split form of gbd_eval for callers that re-use the per-beamlet records:
 * gbd_plan_create allocates device records for up to `capacity` beamlets;
 * gbd_plan_setup runs the FP64 per-beamlet kernel (Q-law, eigenvalue-branch
 * amplitude, base ray, hit point on the plane, phasor coefficients) and
 * synchronises on its status; gbd_plan_eval runs only the N x M kernels and
 * does not synchronise. */
int gbd_plan_create(gbd_ctx_t ctx, gbd_plan_t *out, int64_t capacity);
int gbd_plan_setup(gbd_ctx_t ctx, gbd_plan_t plan, gbd_beamlets_t b, gbd_plane_t p);
int gbd_plan_eval(gbd_ctx_t ctx, gbd_plan_t plan, int precision, void *field_out, int64_t out_bytes,
                  const gbd_eval_opts *opts);
void gbd_plan_free(gbd_plan_t plan);

/* Number of beamlet segments (and launch shape) gbd_plan_eval would use. */
int gbd_plan_shape(gbd_ctx_t ctx, gbd_plan_t plan, int precision, const gbd_eval_opts *opts,
                   gbd_eval_opts *resolved);

#ifdef __cplusplus
}
#endif
#endif /* GBD_H */
