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
    int32_t rows_per_lane;  /* pixels per lane along a detector column: 1, 2, 4, 8, 16, 32
                               (32: rotor form only, runs 16 where the form resolves to
                               direct or stepped; the FP64 direct form runs at most 8) */
    int32_t waves;          /* wavefronts per workgroup: 1, 2 or 4 */
    int32_t segments;       /* beamlet segments evaluated by separate workgroups, 0 = auto.
                               The mixed separable form sums a segment in plain FP32, so
                               it raises any count (automatic, tuned or explicit) to at
                               least ceil(N / 16384): at most 16,384 beamlets per FP32 sum */
    int32_t variant;        /* 0 = auto.  FP64: 1 = direct (exp and sincospi per pixel), 3 =
                               rotor (the recurrence below in FP64; well-sampled grids; at
                               most 16 rows with higher-order beamlets), 4 = separable (below, on FP64
                               MFMA; no cross terms, higher-order factors included); auto:
                               separable, else rotor, else direct; a request that does not
                               apply resolves as auto among the others.
                               Mixed: 1 = direct: FP64 phase and exp2
                               per pixel; 2 = stepped: FP64 phase per lane and beamlet
                               with FP32 row steps, amplitude stepped by multiplication;
                               3 = rotor: per lane and beamlet an FP64 anchor phasor at
                               the lane's middle row, the other rows by complex
                               recurrence (anchor x rho^k x sigma^(k^2)); 4 = separable:
                               E = sum_j U_j(x) V_j(y) as a complex matrix product on
                               FP16 MFMA with every factor (of a higher-order beamlet:
                               times its axis polynomial) split into FP16 hi and lo
                               halves (the hi x hi, hi x lo and lo x hi products, FP32
                               accumulation; each beamlet's factors scaled by powers of
                               two into FP16's range from the setup's bounds over the
                               grid, so a term's error stays below 2^-20 of itself or
                               2^-38 of the largest term over the grid, whichever is
                               larger; a higher-order factor's bound takes its
                               polynomial's largest modulus near the spot, which can
                               exceed the term's, loosening the second figure by that
                               ratio); 5 = separable
                               on FP32 MFMA in three real products per pair (Gauss's
                               form).  Workgroup tiles: 4 x 2 wavefronts of 64 x 64
                               pixels in FP16 halves (gbd_plan_shape reports 64 rows, 8
                               waves), 2 x 4 of 64 x 32 on FP32 (32 and 8); rows_per_lane
                               and waves do not apply.
                               Separable is used (auto) or honoured (4, 5) when no beamlet's
                               phasor has a cross term (rotationally symmetric systems on
                               a plane normal to the axis); stepped and rotor when the
                               setup finds every beamlet's log2-amplitude curvature below
                               0.1 per row^2 (well-sampled spots).  Auto: separable, else
                               rotor, else direct; a request that does not apply falls
                               back to auto's choice among the others. */
} gbd_eval_opts;

/* --- context ------------------------------------------------------------ */

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
int gbd_ctx_create(gbd_ctx_t *out, int device, void *hip_stream);
/* Rebind the context to another stream of the same device (waits for the
 * work already enqueued on the old one). */
int gbd_ctx_set_stream(gbd_ctx_t ctx, void *hip_stream);
void gbd_ctx_destroy(gbd_ctx_t ctx);
/* Kernel timing, for measurement: while enabled, every plan evaluation
 * (gbd_plan_eval, gbd_eval; not the allocation-free gbd_plan_eval_noalloc)
 * times its N x M evaluation kernel of the whole beamlets (after the rotor
 * form's table kernel, before any truncated-beamlet kernel and the segment
 * reduction) with a pair of HIP events on the context stream: stamped with
 * the kernel's own start and end for the separable forms, recorded around
 * the launch for the others.  gbd_ctx_kernel_times waits for
 * the recorded pairs, writes up to `cap` of their durations in milliseconds,
 * oldest first, to ms_out (host), sets *n to how many there were and
 * forgets them all.  Disabling keeps pending pairs until they are taken. */
int gbd_ctx_set_kernel_timing(gbd_ctx_t ctx, int enable);
int gbd_ctx_kernel_times(gbd_ctx_t ctx, float *ms_out, int32_t cap, int32_t *n);
/* Thread-local description of the last failure in this thread. */
const char *gbd_last_error(void);

/* --- pupil decomposition (Sec. 2.2 beamlet decomposition, Sec. 6 OF) ------
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
 * copied and uploaded to device memory held by the handle: a block of the
 * context's pool, which gbd_beamlets_free returns there for the context's
 * next handle (at most 4 GiB wait; the pool's blocks go back to the driver
 * once the context and all its handles are destroyed).  A handle is used
 * with the context that created it: the calls that take one refuse a handle
 * of another context (GBD_EINVAL), whose upload may still be in flight on
 * that context's stream. */
int gbd_beamlets(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0,
                 const double *r1, const double *th1, const double *w0, int64_t n_w0,
                 const double *amp, const double *path, const double *abcd, int64_t n_abcd);

/* --- ray-traced inputs (Sec. 2.2: beamlets carried by a base ray and
 * parabasal rays through the system; Appendix B's telescope is two conic
 * mirrors) -------------------------------------------------------------------
 * gbd_trace: real-ray trace, FP64 on the device, of n base rays through
 * n_mirrors (<= 8) conic mirrors, each a row (z_vertex, R, k, r_min, r_max)
 * of `mirrors`: vertex on the axis, vertex radius of curvature signed in the
 * global frame (the centre of curvature at z_vertex + R; 0 = plane mirror),
 * conic constant, clear annulus (m).  Rays start on the plane z = z_in at
 * r1 [n][2] with x, y direction cosines th1 [n][2] (NULL = along +z) and end
 * on the plane z = z_out; after an odd number of reflections the output frame
 * is the global one turned by pi about x.  Every input coordinate is also
 * perturbed by -/+ dr (positions) or dth (direction cosines) and the central
 * differences give the differential matrix.  Writes (host arrays, caller-
 * owned): base_out [n][5] = (x, y, l, m, optical path - l0) at z_out,
 * abcd_out [n][16] row-major [[A, B], [C, D]] = d(x, y, l, m)_out /
 * d(x, y, l, m)_in, flags_out [n] = bits 1 vignetted (a hit outside a
 * mirror's annulus), 2 missed, 4 the output plane behind the ray, over the
 * base ray and its eight parabasal rays.  Synchronises the context stream.
 * gbd_beamlets_traced: as gbd_beamlets with per-beamlet traced inputs: abcd
 * [n][16] the differential matrices, base [n][5] the traced base rays, which
 * replace the ab/cd-law base ray and whose path (beyond l0) replaces the
 * eikonal term of the misalignment phase.  Finite-difference matrices carry
 * truncation and rounding error and can have a vanishing block (A at a
 * focus), so the symplectic relations are checked scale-free: with the
 * symplectic balancing M' = diag(1/s, 1/s, s, s) M diag(s, s, 1/s, 1/s),
 * s^2 = sqrt(|B|_F / |C|_F), every entry of M'^T J M' - J must lie within
 * sympl_tol * max(1, max|M'|)^2, sympl_tol in (0, 1e-3] (1e-7 suits
 * gbd_trace's output at dr = 1e-5 m, dth = 1e-7), else GBD_ENOTSYMPLECTIC. */
int gbd_trace(gbd_ctx_t ctx, int32_t n_mirrors, const double *mirrors, double z_in, double z_out, double l0,
              int64_t n, const double *r1, const double *th1, double dr, double dth, double *base_out,
              double *abcd_out, int32_t *flags_out);
int gbd_beamlets_traced(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0, const double *r1,
                        const double *th1, const double *w0, int64_t n_w0, const double *amp, const double *path,
                        const double *abcd, const double *base, double sympl_tol);
/* --- higher-order beamlets (Sec. 2.1: the Hermite-Gaussian solutions of the
 * reduced Collins integral serve in beamlet decomposition like the
 * fundamental one; Sec. 7.1: higher-order beams through a system) ---------
 * As gbd_beamlets, plus order [n][2] (int32, host, required for n > 0): the
 * orders (m, n), each in 0 ... 2 (else GBD_EINVAL), of elegant
 * Hermite-Gaussian beamlets launched as
 *   H_m(u_x) H_n(u_y) exp(-|u|^2) exp(-i k th1 . (r - r1)),  u = (r - r1) / w0,
 * H the physicists' Hermite polynomials: the Gaussian beamlet's envelope
 * differentiated m times along x and n times along y with respect to its
 * centre (times w0^(m+n)), its tilt phase held.  Propagation commutes with
 * that derivative, so on the detector the beamlet is its Gaussian field
 * times a polynomial in the offset from the base ray.  Evaluation
 * (gbd_eval, gbd_plan_eval) takes such beamlets on planes normal to the axis
 * only (else GBD_EINVAL from the setup), in FP64 or in the mixed direct,
 * rotor or separable form (a request for the stepped form resolves to the
 * direct one; the separable form applies where no beamlet's factor has
 * cross terms).  gbd_eval_point and gbd_eval_batch
 * refuse beamlets with a nonzero order (GBD_EINVAL).  Orders all (0, 0)
 * give the fundamental beamlets. */
int gbd_beamlets_hg(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0, const double *r1,
                    const double *th1, const double *w0, int64_t n_w0, const double *amp, const double *path,
                    const double *abcd, int64_t n_abcd, const int32_t *order);
/* --- truncated beamlets (Sec. 2.1: truncated-beam solutions of the reduced
 * Collins integral serve in beamlet decomposition; Sec. 7.1: truncated
 * beamlets for the hard edges of apertures) ------------------------------
 * As gbd_beamlets, plus edge [n][3] (host, required for n > 0): beamlet j's
 * input envelope is kept where e . r <= t, edge[j] = (e_x, e_y, t), e a unit
 * vector (|e|^2 within 1e-12 of 1, else GBD_EINVAL) and t in metres in the
 * input plane; e = (0, 0) leaves the beamlet whole.  On the detector a cut
 * beamlet is its Gaussian field times erfc(zeta) / 2, zeta complex and
 * linear in the offset from the base ray (the step function written as a
 * superposition of tilts, each propagated as a Gaussian).  The library keeps
 * the cut beamlets after the whole ones: the whole ones are evaluated in the
 * chosen form (FP64, direct, stepped, rotor or separable), the cut ones by a
 * direct-form kernel with the complex error function (Weideman's rational
 * approximation of the Faddeeva function, N = 40 in FP64 and 16 in the mixed
 * form), both into the same ordered segment sums.  Planes normal to the axis
 * only (else GBD_EINVAL from the setup); a plane through an exact image of
 * the input plane (B' = 0, an infinitely sharp edge) gives GBD_EINVAL
 * (non-finite factor).  gbd_eval_point and gbd_eval_batch refuse cut
 * beamlets (GBD_EINVAL). */
int gbd_beamlets_truncated(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0,
                           const double *r1, const double *th1, const double *w0, int64_t n_w0, const double *amp,
                           const double *path, const double *abcd, int64_t n_abcd, const double *edge);
void gbd_beamlets_free(gbd_beamlets_t b);

/* --- detector plane (Sec. 3: the common evaluation plane) ----------------
 * origin[3], normal[3] (any length > 0), xhint[3] (not parallel to normal);
 * nx, ny >= 0 pixels of pitch dx, dy > 0.  Planes need not be normal to the
 * optical axis (tilted-detector extension; exact when normal is along z). */
int gbd_plane(gbd_ctx_t ctx, gbd_plane_t *out, const double origin[3], const double normal[3],
              const double xhint[3], int32_t nx, int32_t ny, double dx, double dy);
void gbd_plane_free(gbd_plane_t p);

/* --- field evaluation (Sec. 3 plane evaluation, Sec. 1 coherent sum) -----
 * field_out: device pointer to [ny][nx] interleaved complex: complex128 for
 * GBD_FP64 (all-FP64 arithmetic), complex64 for GBD_MIXED (FP64 phase and
 * coordinates, FP32 exp2/sin/cos; FP32 sums per beamlet segment, added in
 * FP64 across segments: Kahan-compensated in the direct and stepped forms
 * and in the rotor form up to 16 rows per lane, 128-beamlet tile sums added
 * plainly in the rotor form at 32 rows, a plain FP32 MFMA sum of at most
 * 16,384 beamlets in the separable form).
 * out_bytes: size of field_out in bytes (GBD_ERANGE if too small).
 * Runs the per-beamlet setup (propagation, plane transfer) and the N x M
 * evaluation on the context stream.  Plane-dependent checks (GBD_EPARALLEL,
 * GBD_EBRANCH) are made by the setup kernel; this call waits for them
 * before it returns, and a failing call leaves field_out untouched.  After a
 * successful call the next one launches its evaluation right behind its
 * setup, with the previous call's form and FP16 scale, before it reads the
 * new status (no host round trip between the kernels): the final reduction
 * writes field_out only if that status has no error and selects the same
 * form and scale; otherwise nothing is written, and on a change of form or
 * scale the evaluation runs again.  Evaluations that write field_out
 * without a reduction (a single segment, no beamlets) are launched after
 * the status is read. */
int gbd_eval(gbd_ctx_t ctx, gbd_beamlets_t b, gbd_plane_t p, int precision, void *field_out,
             int64_t out_bytes, const gbd_eval_opts *opts);

/* Split form of gbd_eval for callers that re-use the per-beamlet records:
 * gbd_plan_create allocates device records for up to `capacity` beamlets;
 * gbd_plan_setup runs the FP64 per-beamlet kernel (Q-law, eigenvalue-branch
 * amplitude, base ray, hit point on the plane, phasor coefficients) and
 * synchronises on its status; gbd_plan_eval runs the N x M kernels (before a
 * rotor form also a small kernel that fills the form's sigma^(k^2) tables in
 * the plan's records) and does not synchronise.  A plan's calls are ordered
 * on the context stream; calls on one plan must not overlap from two streams. */
int gbd_plan_create(gbd_ctx_t ctx, gbd_plan_t *out, int64_t capacity);
int gbd_plan_setup(gbd_ctx_t ctx, gbd_plan_t plan, gbd_beamlets_t b, gbd_plane_t p);
int gbd_plan_eval(gbd_ctx_t ctx, gbd_plan_t plan, int precision, void *field_out, int64_t out_bytes,
                  const gbd_eval_opts *opts);
void gbd_plan_free(gbd_plan_t plan);

/* --- allocation-free evaluation ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * gbd_plan_eval_noalloc is gbd_plan_eval (same arguments, same kernels)
 * with its segment partial sums in a static device buffer of
 * GBD_NOALLOC_SCRATCH_BYTES (64 MiB) instead of a buffer the plan grows; it
 * calls no hipMalloc, hipFree or other allocating routine (an empty plan's
 * output is cleared by a kernel, not a memset).  Every GPU the library runs
 * on holds its own buffer from the first gbd_ctx_create on that device until
 * the process ends.  Launch shape: gbd_plan_eval's, except that an automatic
 * segment count (built-in or tuned) is lowered to the largest whose partial
 * sums fit the buffer (truncated beamlets' segments within half of it; the
 * mixed separable form's floor of ceil(N / 16384) kept); with the same
 * resolved shape the field equals gbd_plan_eval's bit for bit.  GBD_ERANGE,
 * before any launch: an explicit opts->segments whose partials do not fit,
 * or a workload whose fewest allowed segments do not (partials take
 * 8 bytes per pixel and segment in the mixed separable form, 16 otherwise;
 * one segment without truncated beamlets takes none).  All calls on one GPU
 * share its buffer, which keeps the last call's contents (every partial is
 * written before it is read): calls that overlap in time on one GPU, from two
 * streams, threads or contexts, race; calls ordered on one stream do not. */
#define GBD_NOALLOC_SCRATCH_BYTES (64ll << 20)
int gbd_plan_eval_noalloc(gbd_ctx_t ctx, gbd_plan_t plan, int precision, void *field_out, int64_t out_bytes,
                          const gbd_eval_opts *opts);

/* Number of beamlet segments (and launch shape) gbd_plan_eval would use. */
int gbd_plan_shape(gbd_ctx_t ctx, gbd_plan_t plan, int precision, const gbd_eval_opts *opts,
                   gbd_eval_opts *resolved);

/* --- autotuner ---------------------------------------------------------------
 * gbd_autotune: times every launch shape of gbd_plan_eval for this plan and
 * precision (rows_per_lane in {2,4,8} (and 16, 32 where a rotor form applies) x waves in
 * {1,2,4} x segment counts of
 * 1/2, 1, 2 and 4 times the automatic choice; where the separable form
 * applies, whose tile is fixed, the segment counts only; `reps` timed
 * launches each, HIP events on the context stream), stores the fastest in
 * the context's cache keyed by (form family, precision, log2 N, log2 M) and
 * returns it in *best (resolved segment count) and its time in *best_ms.
 * Later calls with all-zero opts (segments 0 for the separable form) on the
 * same bucket use it.  Synchronises; overwrites no caller buffer.
 * gbd_autotune_batch: the same over rows_per_lane x waves for gbd_eval_batch
 * on these instances (host wall time per call), cached by (log2 pairs,
 * log2 instances).
 * gbd_autotune_save / _load: the cache as a text file (load returns the
 * number of entries read, or a negative code). */
int gbd_autotune(gbd_ctx_t ctx, gbd_plan_t plan, int precision, int32_t reps, gbd_eval_opts *best, double *best_ms);
int gbd_autotune_batch(gbd_ctx_t ctx, int32_t n_inst, const gbd_beamlets_t *beamlets, const gbd_plane_t *planes,
                       const float *airy, int64_t airy_bytes, int32_t reps, gbd_eval_opts *best, double *best_ms);
int gbd_autotune_save(gbd_ctx_t ctx, const char *path);
int gbd_autotune_load(gbd_ctx_t ctx, const char *path);

/* --- measurement: issue rates of the instruction classes the evaluation
 * kernels use (for pricing their rooflines) ---------------------------------
 * gbd_issue_probe runs a kernel of 8 workgroups x 256 threads per CU whose
 * threads issue `iters` (>= 1) rounds of independent chains of one class:
 * 0 v_fma_f32, 1 v_fma_f64, 2 v_sin_f32, 3 v_exp_f32, 7 v_fmac_f32,
 * 8 v_mul_f32 (16 chains per thread), 4 v_mfma_f32_16x16x4_f32,
 * 5 v_mfma_f32_16x16x32_f16, 6 v_mfma_f64_16x16x4_f64 (4 chains per
 * wavefront), 9 classes 5 and 0 together (per round 4 MFMA and 16 v_fma_f32
 * chains, all independent; counted as its MFMA instructions); after one untimed
 * launch it times one launch with HIP events on the context stream
 * (synchronises) and returns the time in *ms_out and the wavefront-
 * instructions of that class the launch issued in *wave_instructions_out.
 * Owns its scratch (allocated and freed in the call). */
int gbd_issue_probe(gbd_ctx_t ctx, int32_t cls, int32_t iters, double *ms_out, double *wave_instructions_out);

/* --- point evaluation (paraxial, FP64) --------------------------------------
 * The per-point algorithm that plane evaluation replaces (Sec. 2.2, in its
 * paraxial form): every pixel evaluates every beamlet's exact paraxial field
 * at the pixel's own 3-D position (the beamlet's ABCD extended by free space
 * to that axial distance; complex-curvature law and eigenvalue-branch
 * amplitude recomputed per pixel).  Equal to gbd_eval (GBD_FP64) on planes
 * normal to the axis; the exact reference of the tilted-plane expansion
 * otherwise.  field_out: device complex128 [ny][nx].  Synchronises; returns
 * GBD_EBRANCH (field_out then invalid) if a pixel's eigenvalues leave the
 * principal branch. */
int gbd_eval_point(gbd_ctx_t ctx, gbd_beamlets_t b, gbd_plane_t p, void *field_out, int64_t out_bytes);

/* --- analytic reference irradiance ----------------------------------------
 * out[iy][ix] = (2 J1(v)/v)^2 with v = pi D r / (lambda f), r the distance of
 * the pixel from the plane origin: the Airy pattern of an unobscured circular
 * pupil of diameter D focused at focal length f, normalised to 1 on axis (the
 * analytic reference of Sec. 4.2 and of the search in Sec. 6).  FP64
 * evaluation, FP32 device output; out_bytes >= 4 nx ny. */
int gbd_airy(gbd_ctx_t ctx, gbd_plane_t p, double D, double f, double lambda, float *out, int64_t out_bytes);

/* --- batched parameter sweep (Sec. 6) --------------------------------------
 * Evaluates n_inst independent instances (beamlets[i] on planes[i], mixed
 * precision) in one persistent launch whose workgroups pull (instance, pixel
 * tile) items, largest instances first, from an atomic queue.
 *   airy        device float [ny][nx] reference irradiance shared by all
 *               instances (all planes then need the same nx, ny), or NULL
 *   zone_edges  n_zones + 1 non-decreasing radii (m, in plane coordinates)
 *               bounding annular zones, n_zones in [0, 4] (Sec. 6's zone
 *               study); NULL when n_zones == 0
 *   metrics_out host double [n_inst][2 + n_zones]: RMS and peak over all
 *               pixels of |E/E(0)|^2 - airy, E(0) the field at the plane
 *               origin, then the RMS of each zone; required iff airy != NULL
 *   fields_out  optional device complex64 fields, instance after instance
 *               ([n_inst][ny_i][nx_i]); fields_bytes its size
 * opts: variant as for gbd_eval's mixed form (auto: separable where no
 * beamlet of any instance has a cross term, each item then a 256 x 128
 * pixel tile in FP16 halves with each instance's own scale (4) or a 128 x 128
 * one on FP32 MFMA (5); else rotor, else direct); rows_per_lane and waves as for
 * gbd_eval for the other forms (segments is ignored; default 32 x 4 for the
 * rotor form, else 16 x 4, or the autotuner's choice).  Every item sums all
 * of its instance's beamlets, so a field equals gbd_eval's with the same
 * form and shape and one segment, bit for bit.  In the separable form that
 * is one plain FP32 sum per pixel, whose error grows with the instance's
 * beamlet count, so the separable form applies (auto or requested) only when
 * no instance has more than 16,384 beamlets, the longest FP32 sum gbd_eval
 * allows; otherwise the batch resolves as auto among the other forms.
 * Synchronises the context stream (setup status, then metrics). */
int gbd_eval_batch(gbd_ctx_t ctx, int32_t n_inst, const gbd_beamlets_t *beamlets, const gbd_plane_t *planes,
                   const float *airy, int64_t airy_bytes, const double *zone_edges, int32_t n_zones,
                   double *metrics_out, void *fields_out, int64_t fields_bytes, const gbd_eval_opts *opts);

/* --- surrogate network ------------------------------------------------------
 * A multilayer perceptron n_in -> width (SiLU) x depth -> 1 trained with AdamW
 * on the mean squared error (the figure of merit of Sec. 6 as a function of
 * the decomposition's free parameters).  Parameters are one flat FP32 vector:
 * for each layer W [out][in] row-major then b [out]; the handle owns the
 * parameters, gradients and AdamW moments on the device.
 * mode GBD_MLP_BF16: hidden-layer products on BF16 MFMA (operands rounded to
 * BF16, FP32 accumulate); GBD_MLP_FP32: the same products in FP32.  The head,
 * loss, bias gradients and optimiser are FP32 in both modes.
 *   x      device float [*][n_in] inputs; rows: optional device int32 [batch]
 *          row indices into x (NULL = rows 0..batch-1); target likewise [*]
 *   y      device float [batch] predictions
 *   backward runs the forward pass, then leaves the gradients of
 *          mean((y - target)^2) in the handle; loss_dev (optional, device) gets
 *          the loss
 *   adamw  one decoupled-weight-decay Adam step with bias correction
 *   train  `steps` minibatch steps in one call, each exactly backward on rows
 *          [s][0..batch) (device int32 [steps][batch], required) then adamw
 *          with learning rate lr_host[s] (host float [steps]); loss_sum_dev
 *          (optional, device float) has each step's loss added to it in step
 *          order.  The same kernels as the separate calls, without a host
 *          round trip per step.
 *   set_params uploads parameters and zeroes the optimiser state. */
enum { GBD_MLP_FP32 = 0, GBD_MLP_BF16 = 1 };
typedef struct gbd_mlp_s *gbd_mlp_t;
int gbd_mlp_create(gbd_ctx_t ctx, gbd_mlp_t *out, int32_t n_in, int32_t width, int32_t depth, int32_t max_batch,
                   int mode);
void gbd_mlp_free(gbd_mlp_t m);
int64_t gbd_mlp_num_params(gbd_mlp_t m);
int gbd_mlp_set_params(gbd_mlp_t m, const float *params_host, int64_t n);
int gbd_mlp_get_params(gbd_mlp_t m, float *params_host, int64_t n);
int gbd_mlp_get_grads(gbd_mlp_t m, float *grads_host, int64_t n);
int gbd_mlp_forward(gbd_mlp_t m, const float *x, const int32_t *rows, int32_t batch, float *y);
int gbd_mlp_backward(gbd_mlp_t m, const float *x, const float *target, const int32_t *rows, int32_t batch,
                     float *loss_dev);
int gbd_mlp_adamw(gbd_mlp_t m, float lr, float beta1, float beta2, float eps, float weight_decay);
int gbd_mlp_train(gbd_mlp_t m, const float *x, const float *target, const int32_t *rows, int32_t steps, int32_t batch,
                  const float *lr_host, float beta1, float beta2, float eps, float weight_decay, float *loss_sum_dev);

#ifdef __cplusplus
}
#endif
#endif /* GBD_H */
