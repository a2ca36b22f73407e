// Internal types shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <tuple>
#include <utility>

namespace gbd {

// Detector plane in the world frame (normal, e1, e2 orthonormal).
struct PlaneGeom {
    double O[3], n[3], e1[3], e2[3];
    int32_t nx, ny;
    double dx, dy;
};

// Beamlet inputs resident in HBM (structure of arrays).
struct BeamletsDev {
    int64_t n;
    int64_t n_w0;
    int64_t n_abcd;
    double lam;
    double l0;
    const double *r1;    // [n][2]
    const double *th1;   // [n][2]
    const double *w0;    // [n_w0]
    const double *amp;   // [n][2]
    const double *path;  // [n]
    const double *abcd;  // [n_abcd][16]
    const double *base;  // [n][5] traced base ray at the output plane (x, y, l, m,
                         // optical path - l0), or null: the ab/cd laws
    const int32_t *order;  // [n][2] elegant Hermite-Gaussian orders (m, n) in 0..2, or null
    const double *edge;    // [n][3] truncating edges (e_x, e_y, t): keep e . r <= t, or null
    int64_t n_cut;         // truncated beamlets; they are stored last, [n - n_cut, n)
};

// Per-beamlet phasor on the plane, about the base-ray hit point (a_rho, b_rho):
//   log E_j(d) = ln|.| + 2 pi i Theta(d),  d = (a - a_rho, b - b_rho)
//   Theta(d) = p0 + p1 da + p2 db + p3 da^2 + p4 da db + p5 db^2   (turns)
//   ln|E_j|  = l0 + l1 da + l2 db + l3 da^2 + l4 da db + l5 db^2
struct alignas(16) Rec64 {
    double arho, brho;
    double p[6];
    double l[6];
    double pad[2];
};
static_assert(sizeof(Rec64) == 128, "Rec64 layout");

// Mixed-precision record: FP64 phase in turns, FP32 log2-amplitude, and the
// lane-independent row-step terms for this plane's dy:
//   stepped form: t2 = p5 dy^2 reduced mod 1, u2 = m5 dy^2, s2 = 2^(2 u2);
//   rotor form:   sq[k-1] = sigma^(k^2), sigma = 2^(u2) e^(2 pi i t2), k = 1..16
//                 (filled by launch_sigma before a rotor-form evaluation; the
//                 setups leave it unset; the batch fills it with launch_batch_sigma).
struct alignas(16) Rec32 {
    double arho, brho;
    double p[6];
    float m[6];   // l / ln 2
    float arho_f, brho_f;
    float t2, u2, s2, pad;
    float sq[16][2];
};
static_assert(sizeof(Rec32) == 240, "Rec32 layout");
constexpr int kRec32Vec4 = sizeof(Rec32) / 16;

// FP64 rotor form: sigma^(k^2), k = 1..16, of each beamlet in FP64 (the Rec32
// table's source values), computed from the Rec64 records when that form runs.
struct alignas(16) RecSq64 {
    double sq[16][2];
};
static_assert(sizeof(RecSq64) == 256, "RecSq64 layout");

// Elegant Hermite-Gaussian factor of a higher-order beamlet on a plane
// normal to the axis, as a polynomial in the pixel offset d = (da, db) from
// the base-ray hit point:
//   g = G d  (complex 2 x 2; w0 times the derivative of log E with respect
//            to the input centre, linear in the offset),
//   P = Px(gx) Py(gy) + k1 ax ay + k0,
//   Px = cx0 + gx (cx1 + cx2 gx),  ax = ex0 + ex1 gx  (likewise y),
// with the coefficients chosen by the orders (m, n): for m = 0, 1, 2,
// (cx0, cx1, cx2) = (1, 0, 0), (0, 1, 0), (hxx, 0, 1) and (ex0, ex1) = (1, 0)
// or (0, 1) for m = 2; k1 = m n hxy and k0 = 2 hxy^2 for m = n = 2, else 0;
// h = w0^2 times the constant second derivative.  The beamlet's field is its
// Gaussian phasor times P.
struct alignas(16) RecHG64 {
    double g[2][2][2];  // G[r][c] (re, im)
    double cx0[2], cy0[2];
    double cx1, cx2, cy1, cy2;
    double k1[2], k0[2];
    double ex0, ex1, ey0, ey1;
};
static_assert(sizeof(RecHG64) == 192, "RecHG64 layout");
struct alignas(16) RecHG32 {
    float g[2][2][2];
    float cx0[2], cy0[2];
    float cx1, cx2, cy1, cy2;
    float k1[2], k0[2];
    float ex0, ex1, ey0, ey1;
};
static_assert(sizeof(RecHG32) == 96, "RecHG32 layout");

// Truncation factor of a cut beamlet (Gaussian envelope kept on one side of
// a straight edge) on a plane normal to the axis: erfc(zeta) / 2 with
//   zeta = z0 + za da + zb db,  d = (da, db) the offset from the hit point.
struct alignas(16) RecCut64 {
    double z0[2], za[2], zb[2];
    double pad[2];
};
static_assert(sizeof(RecCut64) == 64, "RecCut64 layout");
struct alignas(16) RecCut32 {
    float z0[2], za[2], zb[2];
    float pad[2];
};
static_assert(sizeof(RecCut32) == 32, "RecCut32 layout");

// Weideman's rational approximation of the Faddeeva function
// w(u) = e^(-u^2) erfc(-i u), Im u >= 0:
//   w(u) = 2 p(Z) / (L - i u)^2 + 1 / (sqrt(pi) (L - i u)),  Z = (L + i u) / (L - i u),
//   p(Z) = sum_{n < N} a_{n+1} Z^n,  L = sqrt(N / sqrt 2),
// a_n the Fourier coefficients of e^(-s^2) (L^2 + s^2), s = L tan(theta / 2).
// N = 40 for FP64 (relative error 2e-14 over the upper half plane), 16 for
// the mixed form (4e-7 in exact arithmetic, 5e-7 with FP32 rounding).
constexpr int kFaddeevaN64 = 40, kFaddeevaN32 = 16;
constexpr int kCutRows32 = 2, kCutRows64 = 4;  // rows per lane of the truncated-beamlet kernels (4 wavefronts)
struct FaddeevaCoef {
    double L64, a64[kFaddeevaN64];
    float L32, a32[kFaddeevaN32];
};

enum : uint32_t {
    FLAG_PARALLEL = 1u,
    FLAG_BRANCH = 2u,
    FLAG_NONFINITE = 4u,
    // a higher-order or truncated beamlet on a plane tilted against the axis,
    // where its plane-evaluation field is not the exact paraxial one
    FLAG_HG_TILT = 8u,
    FLAG_ERRORS = 15u,
    // not an error: the log2-amplitude curvature along a column exceeds
    // kStepCurvature per row^2, so the amplitude recurrence is not used
    FLAG_STEEP = 16u,
    // not an error: the phasor has a cross term (p4 or l4 nonzero), so the
    // plane's two axes do not separate
    FLAG_CROSS = 32u,
    // not an error: some beamlet is of higher order, so the evaluation
    // multiplies its Hermite-Gaussian factor in (direct and separable forms)
    FLAG_HG = 64u,
};

// largest |d^2 log2(amplitude) / d row^2| / 2 for which the mixed kernel may
// step the amplitude along a column by multiplication: over 16 rows no term
// above 2^-80 of its beamlet's peak can then underflow; the rotor form (up
// to 32 rows, at most 16 steps from its anchor) keeps sigma^(k^2) within
// 2^(+-25.6)
constexpr double kStepCurvature = 0.1;
constexpr int kRotorRows = 16;  // sigma^(k^2) entries: rows per lane up to 2 * 16

// Pixel grid handed to the evaluation kernels.
struct EvalGeom {
    int32_t nx, ny;
    double dx, dy;
    double a0, b0;       // plane coordinates of pixel (0, 0)
    int32_t tiles_x, tiles_y;
    int32_t nseg;        // beamlet segments
    int64_t seg_len;     // beamlets per segment (last one may be shorter)
    int64_t n;           // beamlets
    int32_t work;        // tiles_x * tiles_y * nseg work items
};

// --- batched sweep ------------------------------------------------------
constexpr int kMaxZones = 4;

// per instance, for the batched setup kernel
struct BatchInst {
    BeamletsDev b;
    PlaneGeom pl;
    int64_t rec_off;
    double gturns;
};

// per instance, for the batched evaluation
struct BatchEval {
    int64_t rec_off, n;
    int32_t nx, ny, tiles_x, tiles_y;
    double dx, dy, a0, b0;
    int64_t item_off;   // first work item; an instance's items are contiguous, in tile order
    int64_t field_off;  // element offset of this instance in the optional field output
    int32_t scale;      // FP16 halves form: its accumulators hold the field times 2^scale
    int32_t e0_off, e0_chunks;  // its normalisation chunks (kE0Chunk beamlets each), contiguous
};

// beamlets per workgroup of the normalisation sum
constexpr int kE0Chunk = 2048;

struct BatchArgs {
    const BatchEval *inst;
    int32_t n_inst;
    const int32_t *items;  // [n_items][2] = (instance, tile), largest instances first
    int32_t n_items;
    const Rec32 *rec;
    const double2 *e0;     // field at the plane origin, per instance
    const float *airy;     // reference irradiance [ny][nx] shared by all instances, or null
    float2 *fields;        // optional complex64 fields
    double *part;          // [n_items][2 + 2 n_zones] partial metrics
    uint32_t *counter;     // work-queue head, zeroed before the launch
    int32_t n_zones;
    double zone_r2[kMaxZones + 1];  // squared radii bounding the annular zones
};

// peak: per instance, the largest beamlet term modulus over the grid as
// ceil(log2) + 2048 (0: none), the setup kernel's atomic maximum; zero on entry.
// flags[0 .. 3] and the n_inst peaks after them set for a batch setup (the
// first bad instance to 0x7f7f7f7f, the rest to 0)
hipError_t launch_batch_clear(uint32_t *flags, int32_t n_inst, hipStream_t s);
// The records' first 112 bytes; l5[j] receives beamlet j's FP64 l5 (the rotor
// tables' source) and, unless e0t is null, e0t[j] its term at the plane origin.
hipError_t launch_batch_setup(const BatchInst *inst, const int64_t *offs, int32_t n_inst, int64_t total,
                              Rec32 *rec, double *l5, double2 *e0t, uint32_t *status, int32_t *bad, uint32_t *peak,
                              hipStream_t s);
// the rotor tables of every record (before a rotor-form evaluation)
hipError_t launch_batch_sigma(const BatchInst *inst, const int64_t *offs, int32_t n_inst, int64_t total,
                              const double *l5, Rec32 *rec, hipStream_t s);
// E(0) per instance from the setup's terms: e0map[c] is the instance of chunk
// c (n_chunks of them, each instance's in order from BatchEval::e0_off); part
// holds n_chunks sums
hipError_t launch_batch_e0(const BatchEval *inst, int32_t n_inst, const int32_t *e0map, int32_t n_chunks,
                           const double2 *e0t, double2 *part, double2 *e0, hipStream_t s);
// form 3: the separable form (rows and waves do not apply), in FP16 halves
// when half (scales from BatchEval::scale), else on FP32 MFMA
hipError_t launch_batch_eval(int rows, int waves, int form, bool half, int cus, const BatchArgs &a, hipStream_t s);
hipError_t launch_batch_finalize(const BatchEval *inst, int32_t n_inst, const double *part, int32_t n_zones,
                                 double *metrics, hipStream_t s);
hipError_t launch_airy(int32_t nx, int32_t ny, double dx, double dy, double vscale, float *out, hipStream_t s);

// --- real-ray trace through conic mirrors ----------------------------------
constexpr int kMaxMirrors = 8;
struct TraceMirror {
    double zv, c, k, r_min, r_max;  // vertex, curvature 1/R (0: plane), conic, clear annulus
};
struct TraceSystem {
    int32_t n;
    double z_in, z_out, l0;
    TraceMirror m[kMaxMirrors];
};
enum : uint32_t { TRACE_VIGNETTED = 1u, TRACE_MISSED = 2u, TRACE_BACKWARD = 4u };
hipError_t launch_trace(const TraceSystem &S, int64_t n, const double *r1, const double *th1, double h_r,
                        double h_t, double *base, double *abcd, int32_t *flags, hipStream_t s);

// --- point evaluation (paraxial, FP64) -----------------------------------
// Per beamlet: base ray at the ABCD output plane, P0 = Nm adj(Mm0) (complex
// symmetric), det Mm(z) = d0 + d1 z + d2 z^2, tr Mm(z) = t0 + t1 z,
// amplitude, phase constant c0 (turns, reduced) and c1 = d(turns)/dz.
struct alignas(16) RecPt {
    double r2[2], th[2];
    double p00[2], p01[2], p11[2];
    double d0[2], d1[2], d2[2];
    double t0[2], t1[2];
    double amp[2];
    double c0, c1;
    double pad[2];
};
static_assert(sizeof(RecPt) % 16 == 0, "RecPt layout");

hipError_t launch_point(const BeamletsDev &b, const PlaneGeom &pl, double gturns, RecPt *rec, double2 *out,
                        uint32_t *status, hipStream_t s);

// --- surrogate network ----------------------------------------------------
// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak] and
// B(k, n) = B[k sbk + n sbn]; epilogue 0: C = acc + bias, H = SiLU(C);
// 1: C = acc * SiLU'(zmul[m][n]); 2: C = acc.
struct MlpGemm {
    int M, N, K;
    const float *A;
    int64_t sam, sak;
    const float *B;
    int64_t sbk, sbn;
    const float *bias;
    const float *zmul;
    float *C;
    float *H;
    int epi;
};

hipError_t launch_mlp_gemm(int bf16, const MlpGemm &g, hipStream_t s);
hipError_t launch_mlp_accum(float *acc, const float *v, hipStream_t s);
hipError_t launch_mlp_gather(const float *X, const float *y, const int32_t *idx, int B, int n_in, float *Xb, float *yb,
                             hipStream_t s);
hipError_t launch_mlp_head_forward(const float *H, const float *w, const float *w0, int B, int W, float *yhat,
                                   hipStream_t s);
hipError_t launch_mlp_head_backward(const float *yhat, const float *y, const float *H, const float *w, const float *Z,
                                    int B, int W, float *g, float *loss, float *dw, float *dZ, hipStream_t s);
hipError_t launch_mlp_colsum(const float *dZ, int B, int W, float *db, hipStream_t s);
hipError_t launch_mlp_adamw(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                            float eps, float wd, float c1, float c2, hipStream_t s);

// status: two device words, zero on entry: [0] receives the OR of the
// beamlets' FLAG_* bits, [1] the largest beamlet term modulus over the grid
// as ceil(log2) + 2048 (0: none; the FP16 separable form's range); and
// status_next: the next setup's two words, set to zero (the host alternates
// the pairs, so no separate clear is needed).
// A finished setup's status[0] (flags, < 256) and status[1] (key, < 4096)
// posted to the host: (seq << 32) | flags | key << 8 in one system-scope
// store into *post (coherent host memory), which the host polls for seq (an
// event after a copy would end with a system-scope release that stalls the
// stream for the cache writeback).  Any kernel that runs after the setup in
// stream order can make it: status_post_kernel, or the first thread of
// workgroup 0 of a separable-form evaluation kernel handed a StatusPost whose
// post is set (post null: nothing to post).
struct StatusPost {
    const uint32_t *status = nullptr;
    uint64_t *post = nullptr;
    uint32_t seq = 0;
};
__device__ inline void post_status(const StatusPost &sp) {
    const uint32_t f = sp.status[0], k = sp.status[1];
    const uint64_t w = ((uint64_t)sp.seq << 32) | (uint64_t)(f & 0xffu) | ((uint64_t)(k & 0xfffu) << 8);
    __hip_atomic_store(sp.post, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
hipError_t launch_status_post(const StatusPost &sp, hipStream_t s);
hipError_t launch_setup(const BeamletsDev &b, const PlaneGeom &pl, double global_turns, Rec64 *r64,
                        Rec32 *r32, RecHG64 *h64, RecHG32 *h32, RecCut64 *c64, RecCut32 *c32,
                        uint32_t *status, uint32_t *status_next, hipStream_t s);

// The rotor forms' sigma^(k^2) tables (k = 1..16) of the g.n beamlets, from
// their FP64 records on rows g.dy apart: into q64 (FP64 rotor form) or the
// Rec32 records r32 (mixed rotor forms), exactly one of the two non-null.
// launch_setup leaves them unset; run before a rotor-form evaluation.
hipError_t launch_sigma(const EvalGeom &g, const Rec64 *r64, RecSq64 *q64, Rec32 *r32, hipStream_t s);

// Truncated beamlets (direct form with the complex error function): the n
// beamlets of g (records rec / cut, both starting at the first truncated
// beamlet) summed per segment into partial segments seg_base + s; precision
// 0 FP64 (double2 partials), 1 mixed (float4 (sum, compensation)).
hipError_t launch_eval_cut(int precision, const EvalGeom &g, const void *rec, const void *cut,
                           const FaddeevaCoef &fc, int32_t seg_base, void *partial, hipStream_t s);

// Mixed precision only, form = 0 direct: per-pixel FP64 phase and exp2;
// 1 stepped: phase stepped in FP32 from an FP64 anchor and amplitude stepped
// by multiplication along each lane's column; 2 rotor: each lane's column
// factored as anchor x rho^k x sigma^(k^2), no per-pixel transcendental.
// hg: RecHG64 / RecHG32 records of higher-order beamlets (direct and FP64
// forms only), or null.  precision 0 with form 2: the FP64 rotor form, q64
// its sigma^(k^2) tables; form 2 reads the tables launch_sigma fills.
hipError_t launch_eval(int precision, int rows, int waves, int form, const EvalGeom &g, const void *rec,
                       const void *hg, const RecSq64 *q64, void *partial, void *out, hipStream_t s);

// A condition on the setup status words (flags, key) that the output write
// waits for: an evaluation launched before the host has read the setup's
// status writes its output only if no error flag is set, the flags under
// `mask` equal `flags` and, when check_key, the key equals `key` (the form
// and the FP16 scale it was launched with).  status null: no condition.
struct EvalGuard {
    const uint32_t *status = nullptr;
    uint32_t mask = 0, flags = 0, key = 0;
    int32_t check_key = 0;
};

// Sums the g.nseg segment partials of every pixel in segment order, in FP64.
// Mixed precision: the first nseg2 segments are compact (float2 sums), the
// others float4 (sum, compensation) starting at reduce_wide_offset(nseg2, M)
// bytes into partial; FP64: double2 (nseg2 must be 0).  Writes nothing unless
// the guard's condition holds.
hipError_t launch_reduce(int precision, const EvalGeom &g, int32_t nseg2, const void *partial, void *out,
                         hipStream_t s, const EvalGuard &guard = EvalGuard());
inline size_t reduce_wide_offset(int32_t nseg2, int64_t M) { return ((size_t)nseg2 * (size_t)M * 8 + 15) & ~(size_t)15; }

// Issue-rate probe (gbd_probe.hip): `blocks` workgroups of 256 threads,
// `iters` rounds of one instruction class (gbd_issue_probe's classes);
// sink is never written (its store is guarded by a condition false at run time).
hipError_t launch_issue_probe(int cls, int blocks, int iters, float *sink, hipStream_t s);

// Zeroes `bytes` bytes at p (16-byte aligned) with a kernel, not a memset
// node (for callers that capture the stream into a graph).
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);

// Separable (matrix) form on FP32 MFMA (single evaluations and the batched
// sweep): wavefront tiles of kSepTileX x kSepTileY pixels, kSepWavesX x
// kSepWavesY wavefronts per workgroup (128 x 128 pixels, one workgroup per
// CU at the register and LDS budget).
constexpr int kSepWavesX = 2, kSepWavesY = 4;
constexpr int kSepTileX = 64, kSepTileY = 32;
// The FP16 halves form (single evaluations and the batched sweep): wavefront
// tiles of kSepHTile x kSepHTile pixels, kSepHWavesX x kSepHWavesY wavefronts
// per workgroup (256 x 128 pixels, one workgroup per CU).
constexpr int kSepHWavesX = 4, kSepHWavesY = 2, kSepHTile = 64;
constexpr int64_t kSepMaxSegLen = 16384;  // beamlets per FP32 segment at most (automatic segment count)
// The FP64 separable form on FP64 MFMA: wavefront tiles of 64 x 32 pixels
// (kSepRows64 rows), kSep64WavesX x kSep64WavesY wavefronts per workgroup
// (128 x 128 pixels, one workgroup per CU); double2 partials.
constexpr int kSepRows64 = 32;
constexpr int kSep64WavesX = 2, kSep64WavesY = 4;
static_assert(kSep64WavesX == kSepWavesX && kSepRows64 == kSepTileY,
              "separable tiles: the host derives the y count of wavefronts from the workgroup size");
// A kernel launch whose start and stop events (either may be null) take the
// kernel's own start and end times from its dispatch (hipExtLaunchKernel),
// with no marker packets of their own on the stream between the kernels.
template <typename... P, size_t... I>
hipError_t launch_timed_args(void (*k)(P...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t t0, hipEvent_t t1,
                             std::tuple<std::decay_t<P>...> &a, std::index_sequence<I...>) {
    void *p[sizeof...(P) > 0 ? sizeof...(P) : 1] = {static_cast<void *>(&std::get<I>(a))...};
    return hipExtLaunchKernel(reinterpret_cast<const void *>(k), grid, block, p, 0, s, t0, t1, 0);
}
template <typename... P, typename... A>
hipError_t launch_timed(void (*k)(P...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t t0, hipEvent_t t1,
                        A... a) {
    static_assert(sizeof...(P) == sizeof...(A), "kernel arguments");
    if (!t0 && !t1) {
        k<<<grid, block, 0, s>>>(a...);
        return hipGetLastError();
    }
    std::tuple<std::decay_t<P>...> args{a...};  // each converted to its parameter's type
    return launch_timed_args(k, grid, block, s, t0, t1, args, std::index_sequence_for<P...>());
}

// hg: higher-order factors without cross terms (G diagonal), or null.
// t0, t1 (optional): events that take the kernel's start and end times;
// sp (optional): a setup status the kernel posts at its start.
hipError_t launch_eval_sep64(const EvalGeom &g, const Rec64 *rec, const RecHG64 *hg, double2 *partial, double2 *out,
                             hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr,
                             const StatusPost &sp = StatusPost());

// hg: higher-order factors without cross terms (k1 = k0 = 0, G diagonal), or null.
// Partials as float2 (no compensation term): the compact segments of
// launch_reduce.
hipError_t launch_eval_sep(const EvalGeom &g, const Rec32 *rec, const RecHG32 *hg, float2 *partial, float2 *out,
                           hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr,
                           const StatusPost &sp = StatusPost());

// The same form for fundamental beamlets on FP16 MFMA (v_mfma_f32_16x16x32_f16)
// with every factor split into FP16 hi and lo halves (products hi hi, hi lo,
// lo hi): beamlet j's U factor is
// scaled by 2^(kSepHalfExp - u_j) (u_j = log2 of its largest modulus over the
// grid, Rec32::pad) and its V factor by 2^(scale - kSepHalfExp + u_j), so both
// stay below 2^kSepHalfExp and the accumulators hold the field times
// 2^scale (scale = 2 kSepHalfExp - P, 2^P the largest term over the grid,
// from the setup); partials and output are written descaled.
constexpr int kSepHalfExp = 14;
hipError_t launch_eval_seph(const EvalGeom &g, const Rec32 *rec, const RecHG32 *hg, int scale, float2 *partial,
                            float2 *out, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr,
                            const StatusPost &sp = StatusPost());

}  // namespace gbd
