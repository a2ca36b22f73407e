// Internal types shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Mixed-precision record: FP64 phase in turns, FP32 log2-amplitude.
struct alignas(16) Rec32 {
    double arho, brho;
    double p[6];
    float m[6];   // l / ln 2
    float arho_f, brho_f;
};
static_assert(sizeof(Rec32) == 96, "Rec32 layout");

enum : uint32_t {
    FLAG_PARALLEL = 1u,
    FLAG_BRANCH = 2u,
    FLAG_NONFINITE = 4u,
};

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

hipError_t launch_setup(const BeamletsDev &b, const PlaneGeom &pl, double global_turns, Rec64 *r64,
                        Rec32 *r32, uint32_t *status, hipStream_t s);

hipError_t launch_eval(int precision, int rows, int waves, const EvalGeom &g, const void *rec,
                       void *partial, void *out, hipStream_t s);

hipError_t launch_reduce(int precision, const EvalGeom &g, const void *partial, void *out, hipStream_t s);

}  // namespace gbd
