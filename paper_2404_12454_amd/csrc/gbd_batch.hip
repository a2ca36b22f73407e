// Batched parameter sweep (Sec. 6): many independent GBD instances of uneven
// size in one persistent launch, with the Airy figure of merit (Sec. 4.2 and
// Sec. 6: RMS difference of the peak-normalised irradiance to the analytic
// Airy pattern, plus annular zones) reduced in the same kernel.
//
//  batch_setup_kernel  per-beamlet FP64 setup over the concatenated beamlets,
//                      with each beamlet's term at its plane's origin
//  batch_sigma_kernel  the rotor tables, before a rotor-form evaluation only
//  batch_e0_kernel     field at each plane's origin (the normalisation point)
//  batch_eval_kernel   persistent workgroups pull (instance, pixel tile) items,
//                      largest instances first, from an atomic queue head;
//                      each item sums all of its instance's beamlets (mixed
//                      precision) and reduces its metric contribution with
//                      wavefront shuffles
//  batch_sep_kernel    the same with the separable (matrix) form where no
//                      beamlet's phasor has a cross term: items are
//                      (instance, workgroup tile: 256 x 128 pixels in FP16
//                      halves, 128 x 128 on FP32 MFMA when requested), each
//                      an MFMA accumulation over all of the instance's
//                      beamlets
//  batch_finalize      per instance, fixed-order sum of its items' partials
//  airy_kernel         reference irradiance (2 J1(v)/v)^2 in FP64
#include "gbd_device.h"
#include "gbd_sep_core.h"

namespace gbd {

namespace {

using namespace dev;

// The batch's flag words before its setup: [0] status 0, [1] first bad
// instance 0x7f7f7f7f, [2] queue head 0, [3] 0, [4 ...] the n_inst peaks 0.
__global__ void __launch_bounds__(256) batch_clear_kernel(uint32_t *__restrict__ flags, int32_t n_inst) {
    const int64_t n = 4 + (int64_t)n_inst;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flags[i] = i == 1 ? 0x7f7f7f7fu : 0u;
}

// the instance holding beamlet j: the last i with offs[i] <= j (empty
// instances skipped)
__device__ inline int instance_of(const int64_t *__restrict__ offs, int32_t n_inst, int64_t j) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= j)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// E(0) term of one beamlet: the mixed-precision phasor of its record at plane
// coordinates (0, 0), each part widened to FP64 for the sum
__device__ inline double2 e0_term(const Rec32 &r) {
    const double da = -r.arho, db = -r.brho;
    const double th = r.p[0] + da * (r.p[1] + r.p[3] * da) + db * (r.p[2] + r.p[4] * da + r.p[5] * db);
    const float ph = (float)__builtin_amdgcn_fract(th);
    const float daf = -r.arho_f, dbf = -r.brho_f;
    const float L = r.m[0] + daf * (r.m[1] + r.m[3] * daf) + dbf * (r.m[2] + r.m[4] * daf + r.m[5] * dbf);
    const float m = __builtin_amdgcn_exp2f(L);
    return make_double2((double)(m * __builtin_amdgcn_cosf(ph)), (double)(m * __builtin_amdgcn_sinf(ph)));
}

// The records' first 112 bytes (the rotor tables are left to
// batch_sigma_kernel, run only before a rotor-form evaluation), with each
// beamlet's FP64 l5 for that pass and, when e0t is given, its E(0) term.
__global__ void __launch_bounds__(256) batch_setup_kernel(const BatchInst *__restrict__ inst,
                                                          const int64_t *__restrict__ offs, int32_t n_inst,
                                                          int64_t total, Rec32 *__restrict__ rec,
                                                          double *__restrict__ l5, double2 *__restrict__ e0t,
                                                          uint32_t *__restrict__ status, int32_t *__restrict__ bad,
                                                          uint32_t *__restrict__ peak) {
    const int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = j0 < total;
    const int64_t j = live ? j0 : total - 1;  // a lane past the end repeats the last beamlet, writing nothing
    const int lo = instance_of(offs, n_inst, j);
    const BatchInst &I = inst[lo];
    float pk = -INFINITY;
    uint32_t flag = 0;
    if (live) {
        double l5v;
        Rec32 o;
        flag = setup_one(I.b, I.pl, I.gturns, j - offs[lo], nullptr, rec + I.rec_off, nullptr, nullptr, nullptr,
                         nullptr, false, &pk, &l5v, &o);
        l5[j] = l5v;
        if (e0t) e0t[j] = e0_term(o);
    }
    if (flag) atomicOr(status, flag);
    if (flag & FLAG_ERRORS) atomicMin(bad, lo);
    // the instance's largest term over its grid (the FP16 halves form's
    // range): one atomic per wavefront when all its lanes hold one instance
    // (instances are hundreds of beamlets long), else one per lane
    uint32_t key = (live && isfinite(pk)) ? (uint32_t)fminf(fmaxf(ceilf(pk) + 2048.0f, 1.0f), 4095.0f) : 0u;
    const int lo0 = __shfl(lo, 0);
    if (__all(lo == lo0)) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) key = max(key, (uint32_t)__shfl_xor((int)key, o));
        if ((threadIdx.x & 63) == 0 && key) atomicMax(peak + lo0, key);
    } else if (key) {
        atomicMax(peak + lo, key);
    }
}

// Rotor tables sigma^(k^2), k = 1..16, rows dy apart (each instance's dy),
// rounded into the records: thread t of a block computes entry t % 16 of
// beamlet 16 (block) + t / 16, from the record's p5 and the setup's l5 (the
// values the single evaluation's tables come from).
__global__ void __launch_bounds__(256) batch_sigma_kernel(const BatchInst *__restrict__ inst,
                                                          const int64_t *__restrict__ offs, int32_t n_inst,
                                                          int64_t total, const double *__restrict__ l5,
                                                          Rec32 *__restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const int k = (threadIdx.x & 15) + 1;
    if (j >= total) return;
    const double dy = inst[instance_of(offs, n_inst, j)].pl.dy;
    const double2 v = rotor_sigma(rec[j].p[5], l5[j], dy, k);
    rec[j].sq[k - 1][0] = (float)v.x;
    rec[j].sq[k - 1][1] = (float)v.y;
}

// E(0): the instance's E(0) terms summed in FP64, each workgroup one chunk
// of kE0Chunk beamlets of one instance (a fixed-order tree in LDS), then
// batch_e0_sum_kernel adds an instance's chunk sums in chunk order.
__global__ void __launch_bounds__(256) batch_e0_kernel(const BatchEval *__restrict__ inst,
                                                       const int32_t *__restrict__ e0map,
                                                       const double2 *__restrict__ e0t, double2 *__restrict__ part) {
    __shared__ double sre[256], sim[256];
    const int32_t c = blockIdx.x;
    const BatchEval &I = inst[e0map[c]];
    const int64_t j0 = (int64_t)(c - I.e0_off) * kE0Chunk, j1 = min(I.n, j0 + kE0Chunk);
    double re = 0.0, im = 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
        const double2 t = e0t[I.rec_off + j];
        re += t.x;
        im += t.y;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sre[threadIdx.x] += sre[threadIdx.x + h];
            sim[threadIdx.x] += sim[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[c] = make_double2(sre[0], sim[0]);
}

__global__ void __launch_bounds__(64) batch_e0_sum_kernel(const BatchEval *__restrict__ inst, int32_t n_inst,
                                                          const double2 *__restrict__ part,
                                                          double2 *__restrict__ e0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    const BatchEval &I = inst[i];
    double re = 0.0, im = 0.0;
    for (int k = 0; k < I.e0_chunks; k++) {
        const double2 q = part[I.e0_off + k];
        re += q.x;
        im += q.y;
    }
    e0[i] = make_double2(re, im);
}

template <int WIDTH>
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = WIDTH / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WIDTH);
    return v;
}
template <int WIDTH>
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = WIDTH / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WIDTH));
    return v;
}

template <int ROWS, int WAVES, int FORM>
__global__ void __launch_bounds__(64 * WAVES) batch_eval_kernel(BatchArgs A) {
    constexpr int NQ = 2 + 2 * kMaxZones;
    __shared__ Rec32 tile[kMixedTile];
    __shared__ int s_item;
    __shared__ double red[WAVES][NQ];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int PS = 2 + 2 * A.n_zones;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(A.counter, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);  // uniform: the instance fields load as scalars
        __syncthreads();
        if (item >= A.n_items) break;  // uniform across the workgroup
        const int i = A.items[2 * item], t = A.items[2 * item + 1];
        const BatchEval I = A.inst[i];
        const int ty = t / I.tiles_x, tx = t - ty * I.tiles_x;
        const int ix = tx * 64 + lane;
        const int iy0 = (ty * WAVES + wv) * ROWS;
        const double a = I.a0 + ix * I.dx;
        const double b0 = I.b0 + iy0 * I.dy;
        float s_re[ROWS], s_im[ROWS], c_re[ROWS], c_im[ROWS];
#pragma unroll
        for (int k = 0; k < ROWS; k++) s_re[k] = s_im[k] = c_re[k] = c_im[k] = 0.0f;
        if constexpr (FORM == 2)
            mixed_accumulate_rotor<ROWS, 64 * WAVES>(tile, A.rec + I.rec_off, 0, I.n, a, b0, I.dy, s_re, s_im, c_re,
                                                     c_im);
        else if constexpr (FORM == 1)
            mixed_accumulate_step<ROWS, 64 * WAVES>(tile, A.rec + I.rec_off, 0, I.n, a, b0, I.dy, s_re, s_im, c_re,
                                                    c_im);
        else
            mixed_accumulate<ROWS, 64 * WAVES>(tile, A.rec + I.rec_off, 0, I.n, a, b0, I.dy, s_re, s_im, c_re, c_im);

        // epilogue: optional field store, irradiance error against the reference
        double q[NQ];
#pragma unroll
        for (int z = 0; z < NQ; z++) q[z] = 0.0;
        const double2 e0 = A.e0[i];
        const double n0 = e0.x * e0.x + e0.y * e0.y;
        const double inv0 = n0 > 0.0 ? 1.0 / n0 : 0.0;  // an empty instance compares a zero field
#pragma unroll
        for (int k = 0; k < ROWS; k++) {
            const int iy = iy0 + k;
            if (ix < I.nx && iy < I.ny) {
                const int64_t p = (int64_t)iy * I.nx + ix;
                const float er = s_re[k] - c_re[k], ei = s_im[k] - c_im[k];
                if (A.fields) A.fields[I.field_off + p] = make_float2(er, ei);
                if (A.airy) {
                    const double d = ((double)er * er + (double)ei * ei) * inv0 - (double)A.airy[p];
                    q[0] += d * d;
                    q[1] = fmax(q[1], fabs(d));
                    const double bk = b0 + k * I.dy;
                    const double r2 = a * a + bk * bk;
#pragma unroll
                    for (int z = 0; z < kMaxZones; z++)
                        if (z < A.n_zones && r2 >= A.zone_r2[z] && r2 < A.zone_r2[z + 1]) {
                            q[2 + 2 * z] += d * d;
                            q[3 + 2 * z] += 1.0;
                        }
                }
            }
        }
        if (A.airy) {
#pragma unroll
            for (int z = 0; z < NQ; z++) q[z] = (z == 1) ? wave_max<64>(q[z]) : wave_sum<64>(q[z]);
            if (lane == 0)
#pragma unroll
                for (int z = 0; z < NQ; z++) red[wv][z] = q[z];
            __syncthreads();
            if (threadIdx.x == 0) {
                double *dst = A.part + (int64_t)item * PS;
                for (int z = 0; z < PS; z++) {
                    double v = red[0][z];
                    for (int w = 1; w < WAVES; w++) v = (z == 1) ? fmax(v, red[w][z]) : v + red[w][z];
                    dst[z] = v;
                }
            }
        }
        __syncthreads();
    }
}

// Separable form: the single-instance kernel's accumulation with one beamlet
// segment (so a field equals gbd_eval's with the same variant, 4 in FP16
// halves (HALF) or 5 on FP32 MFMA, and one segment bit for bit), then the
// same epilogue from the MFMA accumulators (lane l holds rows 4 (l / 16) + e,
// column l % 16 of each 16 x 16 block).
// The FP16 halves form takes the single evaluation's 256 x 128 workgroup
// tiles (HTileLarge), the FP32 one its 128 x 128 (the k3 layout).
template <bool HALF>
using BatchTile = typename std::conditional<HALF, sep::HTileLarge, sep::Sep3Tile>::type;

template <bool HALF>
__global__ void __launch_bounds__(64 * BatchTile<HALF>::WX * BatchTile<HALF>::WY) batch_sep_kernel(BatchArgs A) {
    using T = BatchTile<HALF>;
    constexpr int WX = T::WX, WY = T::WY, BX = T::BX, BY = T::BY;
    constexpr int WAVES = WX * WY, NQ = 2 + 2 * kMaxZones;
    __shared__ typename std::conditional<HALF, sep::SepHLdsT<T>, sep::Sep3Lds<false>>::type L;
    __shared__ int s_item;
    __shared__ double red[WAVES][NQ];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int wx = wv % WX, wy = wv / WX;
    const int li = lane & 15, lk = lane >> 4;
    const int PS = 2 + 2 * A.n_zones;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(A.counter, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);  // uniform: the instance fields load as scalars
        __syncthreads();
        if (item >= A.n_items) break;  // uniform across the workgroup
        const int i = A.items[2 * item], t = A.items[2 * item + 1];
        const BatchEval I = A.inst[i];
        const int ty = t / I.tiles_x, tx = t - ty * I.tiles_x;
        const int x0 = (tx * WX + wx) * 16 * BX, y0 = (ty * WY + wy) * 16 * BY;
        sep::f4 accR[BY][BX], accI[BY][BX];
        if (I.n > 0) {
            const sep::SepGeom sg{I.nx, I.ny, I.a0, I.b0, I.dx, I.dy};
            if constexpr (HALF) {
                sep::sep_accumulate_h<T>(sg, A.rec + I.rec_off, nullptr, 0, I.n, tx, ty, I.scale, L, accR, accI);
#pragma unroll
                for (int p = 0; p < BY; p++)
#pragma unroll
                    for (int q = 0; q < BX; q++)
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            accR[p][q][e] = ldexpf(accR[p][q][e], -I.scale);
                            accI[p][q][e] = ldexpf(accI[p][q][e], -I.scale);
                        }
            } else {
                sep::sep_accumulate_3m<false>(sg, A.rec + I.rec_off, nullptr, 0, I.n, tx, ty, L, accR, accI);
            }
        } else {
#pragma unroll
            for (int p = 0; p < BY; p++)
#pragma unroll
                for (int q = 0; q < BX; q++) accR[p][q] = accI[p][q] = sep::f4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        double qm[NQ];
#pragma unroll
        for (int z = 0; z < NQ; z++) qm[z] = 0.0;
        const double2 e0 = A.e0[i];
        const double n0 = e0.x * e0.x + e0.y * e0.y;
        const double inv0 = n0 > 0.0 ? 1.0 / n0 : 0.0;  // an empty instance compares a zero field
#pragma unroll
        for (int p = 0; p < BY; p++)
#pragma unroll
            for (int q = 0; q < BX; q++) {
                const int ix = x0 + 16 * q + li;
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int iy = y0 + 16 * p + 4 * lk + e;
                    if (ix < I.nx && iy < I.ny) {
                        const int64_t px = (int64_t)iy * I.nx + ix;
                        const float er = accR[p][q][e], ei = accI[p][q][e];
                        if (A.fields) A.fields[I.field_off + px] = make_float2(er, ei);
                        if (A.airy) {
                            const double d = ((double)er * er + (double)ei * ei) * inv0 - (double)A.airy[px];
                            qm[0] += d * d;
                            qm[1] = fmax(qm[1], fabs(d));
                            const double a = I.a0 + ix * I.dx, bk = I.b0 + iy * I.dy;
                            const double r2 = a * a + bk * bk;
#pragma unroll
                            for (int z = 0; z < kMaxZones; z++)
                                if (z < A.n_zones && r2 >= A.zone_r2[z] && r2 < A.zone_r2[z + 1]) {
                                    qm[2 + 2 * z] += d * d;
                                    qm[3 + 2 * z] += 1.0;
                                }
                        }
                    }
                }
            }
        if (A.airy) {
#pragma unroll
            for (int z = 0; z < NQ; z++) qm[z] = (z == 1) ? wave_max<64>(qm[z]) : wave_sum<64>(qm[z]);
            if (lane == 0)
#pragma unroll
                for (int z = 0; z < NQ; z++) red[wv][z] = qm[z];
            __syncthreads();
            if (threadIdx.x == 0) {
                double *dst = A.part + (int64_t)item * PS;
                for (int z = 0; z < PS; z++) {
                    double v = red[0][z];
                    for (int w = 1; w < WAVES; w++) v = (z == 1) ? fmax(v, red[w][z]) : v + red[w][z];
                    dst[z] = v;
                }
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(64) batch_finalize_kernel(const BatchEval *__restrict__ inst, int32_t n_inst,
                                                            const double *__restrict__ part, int32_t n_zones,
                                                            double *__restrict__ metrics) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst) return;
    const BatchEval I = inst[i];
    const int PS = 2 + 2 * n_zones;
    const int tiles = I.tiles_x * I.tiles_y;
    double s = 0.0, mx = 0.0, zs[kMaxZones], zc[kMaxZones];
    for (int z = 0; z < kMaxZones; z++) zs[z] = zc[z] = 0.0;
    for (int t = 0; t < tiles; t++) {
        const double *q = part + (I.item_off + t) * PS;
        s += q[0];
        mx = fmax(mx, q[1]);
        for (int z = 0; z < n_zones; z++) {
            zs[z] += q[2 + 2 * z];
            zc[z] += q[3 + 2 * z];
        }
    }
    double *o = metrics + (int64_t)i * (2 + n_zones);
    const double M = (double)I.nx * I.ny;
    o[0] = M > 0 ? sqrt(s / M) : 0.0;
    o[1] = mx;
    for (int z = 0; z < n_zones; z++) o[2 + z] = zc[z] > 0 ? sqrt(zs[z] / zc[z]) : 0.0;
}

// (2 J1(v)/v)^2 with v = vscale * r, r the distance from the plane origin.
__global__ void __launch_bounds__(256) airy_kernel(int32_t nx, int32_t ny, double dx, double dy, double vscale,
                                                   float *__restrict__ out) {
    const int64_t M = (int64_t)nx * ny;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        const int iy = (int)(p / nx), ix = (int)(p - (int64_t)iy * nx);
        const double a = (ix - 0.5 * (nx - 1)) * dx, b = (iy - 0.5 * (ny - 1)) * dy;
        const double v = vscale * hypot(a, b);
        const double f = v > 0.0 ? 2.0 * j1(v) / v : 1.0;
        out[p] = (float)(f * f);
    }
}

template <int ROWS, int WAVES, int FORM>
hipError_t launch_batch_eval_t(int cus, const BatchArgs &a, hipStream_t s) {
    int per_cu = 0;
    hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_eval_kernel<ROWS, WAVES, FORM>, 64 * WAVES, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const int grid = (int)min((int64_t)a.n_items, (int64_t)cus * per_cu);
    if (grid <= 0) return hipSuccess;
    batch_eval_kernel<ROWS, WAVES, FORM><<<grid, 64 * WAVES, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_batch_clear(uint32_t *flags, int32_t n_inst, hipStream_t s) {
    const int64_t blocks = min((4 + (int64_t)n_inst + 255) / 256, (int64_t)1024);
    batch_clear_kernel<<<(unsigned)blocks, 256, 0, s>>>(flags, n_inst);
    return hipGetLastError();
}

hipError_t launch_batch_setup(const BatchInst *inst, const int64_t *offs, int32_t n_inst, int64_t total, Rec32 *rec,
                              double *l5, double2 *e0t, uint32_t *status, int32_t *bad, uint32_t *peak,
                              hipStream_t s) {
    if (total == 0) return hipSuccess;
    batch_setup_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(inst, offs, n_inst, total, rec, l5, e0t,
                                                                       status, bad, peak);
    return hipGetLastError();
}

hipError_t launch_batch_sigma(const BatchInst *inst, const int64_t *offs, int32_t n_inst, int64_t total,
                              const double *l5, Rec32 *rec, hipStream_t s) {
    if (total == 0) return hipSuccess;
    batch_sigma_kernel<<<(unsigned)((total + 15) / 16), 256, 0, s>>>(inst, offs, n_inst, total, l5, rec);
    return hipGetLastError();
}

hipError_t launch_batch_e0(const BatchEval *inst, int32_t n_inst, const int32_t *e0map, int32_t n_chunks,
                           const double2 *e0t, double2 *part, double2 *e0, hipStream_t s) {
    if (n_inst == 0) return hipSuccess;
    if (n_chunks > 0) batch_e0_kernel<<<n_chunks, 256, 0, s>>>(inst, e0map, e0t, part);
    batch_e0_sum_kernel<<<(n_inst + 63) / 64, 64, 0, s>>>(inst, n_inst, part, e0);
    return hipGetLastError();
}

hipError_t launch_batch_eval(int rows, int waves, int form, bool half, int cus, const BatchArgs &a, hipStream_t s) {
    if (form == 3) {
        int per_cu = 0;
        const int th = half ? 64 * BatchTile<true>::WX * BatchTile<true>::WY
                            : 64 * BatchTile<false>::WX * BatchTile<false>::WY;
        static_assert(BatchTile<false>::WX == kSepWavesX && BatchTile<false>::WY == kSepWavesY &&
                          BatchTile<true>::WX == kSepHWavesX && BatchTile<true>::WY == kSepHWavesY,
                      "batched separable tiles: host and kernel disagree");
        hipError_t e = half ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_sep_kernel<true>, th, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_sep_kernel<false>, th, 0);
        if (e != hipSuccess) return e;
        if (per_cu < 1) per_cu = 1;
        const int grid = (int)min((int64_t)a.n_items, (int64_t)cus * per_cu);
        if (grid <= 0) return hipSuccess;
        if (half)
            batch_sep_kernel<true><<<grid, th, 0, s>>>(a);
        else
            batch_sep_kernel<false><<<grid, th, 0, s>>>(a);
        return hipGetLastError();
    }
#define GBD_CASE(R, W)                                                                         \
    if (rows == R && waves == W)                                                               \
        return form == 2   ? launch_batch_eval_t<R, W, 2>(cus, a, s)                           \
               : form == 1 ? launch_batch_eval_t<R, W, 1>(cus, a, s)                           \
                           : launch_batch_eval_t<R, W, 0>(cus, a, s);
    GBD_CASE(1, 1) GBD_CASE(1, 2) GBD_CASE(1, 4)
    GBD_CASE(2, 1) GBD_CASE(2, 2) GBD_CASE(2, 4)
    GBD_CASE(4, 1) GBD_CASE(4, 2) GBD_CASE(4, 4)
    GBD_CASE(8, 1) GBD_CASE(8, 2) GBD_CASE(8, 4)
    GBD_CASE(16, 1) GBD_CASE(16, 2) GBD_CASE(16, 4)
#undef GBD_CASE
    if (rows == 32 && form == 2) {  // rotor form only
        if (waves == 1) return launch_batch_eval_t<32, 1, 2>(cus, a, s);
        if (waves == 2) return launch_batch_eval_t<32, 2, 2>(cus, a, s);
        if (waves == 4) return launch_batch_eval_t<32, 4, 2>(cus, a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batch_finalize(const BatchEval *inst, int32_t n_inst, const double *part, int32_t n_zones,
                                 double *metrics, hipStream_t s) {
    if (n_inst == 0) return hipSuccess;
    batch_finalize_kernel<<<(n_inst + 63) / 64, 64, 0, s>>>(inst, n_inst, part, n_zones, metrics);
    return hipGetLastError();
}

hipError_t launch_airy(int32_t nx, int32_t ny, double dx, double dy, double vscale, float *out, hipStream_t s) {
    const int64_t M = (int64_t)nx * ny;
    if (M == 0) return hipSuccess;
    const int64_t blocks = min((M + 255) / 256, (int64_t)4096);
    airy_kernel<<<(unsigned)blocks, 256, 0, s>>>(nx, ny, dx, dy, vscale, out);
    return hipGetLastError();
}

}  // namespace gbd
