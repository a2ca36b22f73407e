// Host side of the C ABI declared in include/gbd.h.
#include "../../include/gbd.h"
#include "gbd_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

using namespace gbd;

// Segment partials of gbd_plan_eval_noalloc: a static device array, so that
// entry point allocates nothing.  Each GPU the library runs on holds its own
// copy until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host it names a stand-in, not device memory): gbd_ctx_create
// takes each device's address with hipGetSymbolAddress once, with that
// device current, and every use goes through that address.
static __device__ __align__(256) unsigned char scratch[GBD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];  // per device: the address of its `scratch`
}  // namespace

// grow-only device buffer
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct BatchWork {
    DevBuf rec, l5, e0t, tab1, tab2, e0, e0part, part, metrics, flags, point;
    uint32_t *host_flags = nullptr;  // pinned: the point evaluation's status
    void *stage = nullptr;           // pinned staging of the batch tables
    size_t stage_bytes = 0;
    hipEvent_t stage_ev = nullptr;   // after the last copy from stage
    bool stage_pending = false;      // stage_ev recorded and not yet waited for
};

// autotuner cache key: (kind, precision, log2 N bucket, log2 M bucket)
struct TuneKey {
    int kind, precision, ln, lm;
    bool operator<(const TuneKey &o) const {
        if (kind != o.kind) return kind < o.kind;
        if (precision != o.precision) return precision < o.precision;
        if (ln != o.ln) return ln < o.ln;
        return lm < o.lm;
    }
};
struct TuneVal {
    int rows, waves, seg_scale_pct;  // segments = auto count * pct / 100
    double ms;
};

// Device blocks of beamlet handles, by power-of-two size class (4 KiB and
// up): a freed handle's block waits in its class for the next handle of the
// same context instead of going back to the driver (hipMalloc and hipFree
// take tens of microseconds each, and a parameter sweep creates and frees
// thousands of handles).  A reused block is written by an upload on the
// context stream, after every kernel that read its previous contents there
// (gbd_ctx_set_stream waits for the old stream first).  At most
// kPoolCacheBytes wait; the pool frees them once the context and every handle
// drawn from it are gone.
constexpr size_t kPoolCacheBytes = (size_t)4 << 30;
struct DevPool {
    std::mutex mu;
    std::map<size_t, std::vector<void *>> cached;
    size_t cached_bytes = 0;
    ~DevPool() {
        for (auto &kv : cached)
            for (void *p : kv.second) (void)hipFree(p);
    }
    static size_t size_class(size_t bytes) {
        size_t c = 4096;
        while (c < bytes) c <<= 1;
        return c;
    }
    // a block of size class cls on the current device
    hipError_t get(size_t cls, void **p) {
        {
            std::lock_guard<std::mutex> lock(mu);
            auto it = cached.find(cls);
            if (it != cached.end() && !it->second.empty()) {
                *p = it->second.back();
                it->second.pop_back();
                cached_bytes -= cls;
                return hipSuccess;
            }
        }
        return hipMalloc(p, cls);
    }
    void put(void *p, size_t cls) {
        {
            std::lock_guard<std::mutex> lock(mu);
            if (cached_bytes + cls <= kPoolCacheBytes) {
                cached[cls].push_back(p);
                cached_bytes += cls;
                return;
            }
        }
        (void)hipFree(p);
    }
};

struct gbd_ctx_s {
    int device;
    std::shared_ptr<DevPool> pool;  // beamlet handles' device blocks
    // pinned staging of beamlet uploads: rewritten once the previous upload's
    // copy has run (up_ev), so a handle's creation does not wait for its own
    void *up_stage = nullptr;
    size_t up_bytes = 0;
    hipEvent_t up_ev = nullptr;
    bool up_pending = false;
    hipStream_t stream;
    int cus;
    gbd_plan_s *own_plan;  // plan used by gbd_eval
    BatchWork batch;
    std::map<TuneKey, TuneVal> tuned;
    // kernel timing (gbd_ctx_set_kernel_timing): recorded event pairs, and
    // spare pairs for reuse
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed, spare_events;
};

struct gbd_beamlets_s {
    gbd_ctx_s *ctx;
    BeamletsDev dev;
    void *mem;
    size_t mem_class;               // mem's size class in pool
    std::shared_ptr<DevPool> pool;  // where mem returns (kept alive past the context)
    bool higher_order;  // some beamlet has a nonzero Hermite-Gaussian order
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
    uint32_t flags;  // FLAG_STEEP / FLAG_CROSS / FLAG_HG of the last setup (which mixed forms apply)
    Rec64 *r64;
    Rec32 *r32;
    RecSq64 *q64;  // FP64 sigma^(k^2) tables of the FP64 rotor form
    RecHG64 *h64;  // Hermite-Gaussian factors, allocated at the first setup of higher-order beamlets
    RecHG32 *h32;
    RecCut64 *c64;  // truncation factors, allocated at the first setup of truncated beamlets
    RecCut32 *c32;
    int64_t n_cut;  // truncated beamlets of the last setup (the last n_cut records)
    uint32_t *status_dev;   // two (flags, peak) word pairs used by alternate setups; each setup clears the other
    int status_parity;      // the pair the next setup uses
    bool status_zeroed;     // both words cleared (once, before the first setup)
    uint64_t *status_post;  // coherent host memory: the last setup's status words and sequence number
    uint32_t status_seq;    // the last launched setup's sequence number
    int sep_scale;          // FP16 separable form: accumulators hold the field times 2^sep_scale
    uint32_t sep_key;       // the status key sep_scale came from
    void *scratch;
    size_t scratch_bytes;
    uint32_t *status_cur;  // the last launched setup's status pair (null: none launched)
    bool spec_ok;  // the last setup succeeded: gbd_eval may launch the next evaluation before reading the status
};

// plan_eval_impl under a guard: the configuration writes the output without
// the guarded reduction (no partials), so it cannot run before the status
constexpr int kNoSpeculation = 1;

struct gbd_mlp_s {
    gbd_ctx_s *ctx;
    int n_in, width, depth, max_batch, mode;
    int64_t P;
    std::vector<int64_t> woff, boff;  // per layer (depth hidden + head): W and b offsets in the flat vector
    float *mem;                       // one allocation holding everything below
    float *params, *grads, *m, *v;
    float *Z, *H;                     // [depth][max_batch][width]
    float *dz0, *dz1;                 // [max_batch][width]
    float *xb, *yb, *yhat, *g, *loss;
    int64_t step;
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
bool symplectic(const double *m, double tol = 1e-10) {
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
            if (fabs(v - J[r][c]) > tol * (mag + fabs(J[r][c]))) return false;
        }
    return true;
}

// Traced (finite-difference) matrices: a block can vanish (A at a focus), so
// entry-wise relative residuals are ill-posed.  Balance with the symplectic
// similarity diag(1/s, 1/s, s, s) M diag(s, s, 1/s, 1/s), s^2 = sqrt(|B| / |C|)
// (Frobenius norms), which leaves A and D and scales B, C to equal norms, and
// bound max |M'^T J M' - J| by tol * max(1, max |M'|)^2.
bool symplectic_balanced(const double *m, double tol) {
    double nb = 0.0, nc = 0.0;
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) {
            nb += m[4 * r + c + 2] * m[4 * r + c + 2];
            nc += m[4 * (r + 2) + c] * m[4 * (r + 2) + c];
        }
    const double s2 = (nb > 0.0 && nc > 0.0) ? sqrt(sqrt(nb) / sqrt(nc)) : 1.0;
    double b[16], big = 1.0;
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            double v = m[4 * r + c];
            if (r < 2 && c >= 2) v /= s2;
            if (r >= 2 && c < 2) v *= s2;
            b[4 * r + c] = v;
            big = fmax(big, fabs(v));
        }
    static const double J[4][4] = {{0, 0, 1, 0}, {0, 0, 0, 1}, {-1, 0, 0, 0}, {0, -1, 0, 0}};
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            double v = 0.0;
            for (int i = 0; i < 4; i++)
                for (int k = 0; k < 4; k++) v += b[4 * i + r] * J[i][k] * b[4 * k + c];
            if (!(fabs(v - J[r][c]) <= tol * big * big)) return false;
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
    int rows, waves, nseg, form;
    bool half;  // mixed separable form in FP16 hi/lo halves (else FP32 MFMA)
};

// mixed kernel form (0 direct, 1 stepped, 2 rotor, 3 separable): requested
// or automatic.  The stepped and rotor forms need a well-sampled grid (no
// FLAG_STEEP), the separable form phasors without cross terms (no
// FLAG_CROSS); a request that does not apply falls back to the automatic
// choice among the others.
int pick_form(int precision, uint32_t flags, const gbd_eval_opts *o, bool allow_sep = true) {
    const bool steep = (flags & FLAG_STEEP) != 0;
    if (precision != GBD_MIXED) {
        // FP64: direct, rotor (needs a well-sampled grid) or separable (needs
        // phasors and higher-order factors without cross terms).  A request
        // that does not apply falls back to the automatic choice among the
        // others.
        const bool sep64 = allow_sep && !(flags & FLAG_CROSS);
        const bool rot64 = !steep;
        const int v = o ? (o->variant == 5 ? 4 : o->variant) : 0;
        if (v == 1) return 0;
        if (v == 3 && rot64) return 2;
        if (v == 4 && sep64) return 3;
        return sep64 ? 3 : rot64 ? 2 : 0;
    }
    const bool sep = allow_sep && !(flags & FLAG_CROSS);
    const int v = o ? (o->variant == 5 ? 4 : o->variant) : 0;  // 5: the separable form on FP32 MFMA
    if (v == 1) return 0;
    // higher-order beamlets: the stepped form does not carry their factor
    if (v == 2) return (steep || (flags & FLAG_HG)) ? 0 : 1;
    if (v == 3) return steep ? 0 : 2;
    return sep ? 3 : steep ? 0 : 2;
}

// the variant a resolved form reports (gbd_eval_opts.variant)
int form_variant(int precision, int form, bool half = false) {
    return (precision == GBD_MIXED && form == 3 && !half) ? 5 : form + 1;
}

int ilog2(int64_t v) {
    int r = 0;
    while (v > 1) {
        v >>= 1;
        r++;
    }
    return r;
}

// cache kinds: single evaluations in a VALU form, batched sweeps, single
// evaluations in the separable form (only the segment count applies)
constexpr int kTuneEval = 0, kTuneBatch = 1, kTuneSep = 2;
TuneKey tune_key(int kind, int precision, int64_t n, int64_t m) { return TuneKey{kind, precision, ilog2(n), ilog2(m)}; }

// Fewest segments a form allows: the mixed separable form sums a segment in
// plain FP32 on the matrix cores, at most kSepMaxSegLen beamlets per sum.
int64_t min_segments(int precision, int form, int64_t n) {
    return (form == 3 && precision == GBD_MIXED) ? (n + kSepMaxSegLen - 1) / kSepMaxSegLen : 1;
}

// Workgroup tile of a separable shape in pixels.
void sep_wg_tile(const Shape &s, int &px, int &py) {
    if (s.half) {
        px = kSepHWavesX * kSepHTile;
        py = kSepHWavesY * kSepHTile;
    } else {
        px = kSepTileX * kSepWavesX;
        py = s.rows * (s.waves / kSepWavesX);
    }
}

// Launch shape and mixed form.  32 rows per lane is a rotor-form shape: where
// the form resolves to direct or stepped it runs 16.
Shape choose_shape(const gbd_ctx_s *ctx, int precision, int64_t n, const PlaneGeom &pl, uint32_t flags,
                   const gbd_eval_opts *o) {
    Shape s;
    s.form = pick_form(precision, flags, o);
    // the mixed separable form runs on FP16 MFMA in hi/lo halves unless the
    // FP32 one is requested (variant 5); the setup bounds higher-order
    // factors with their axis polynomials for the FP16 scaling
    s.half = s.form == 3 && precision == GBD_MIXED && !(o && o->variant == 5);
    if (s.form == 3) {
        // separable form: fixed 64 x 32 pixel tile per wavefront (s.rows is
        // the tile height), 2 x 4 wavefronts per workgroup (s.waves), or in
        // FP16 halves 64 x 64 per wavefront, 4 x 2 wavefronts; the row and
        // wavefront options of the other forms do not apply
        const bool mixed = precision == GBD_MIXED;
        s.rows = s.half ? kSepHTile : mixed ? kSepTileY : kSepRows64;
        s.waves = s.half ? kSepHWavesX * kSepHWavesY : kSepWavesX * (mixed ? kSepWavesY : kSep64WavesY);
        int wgx, wgy;
        sep_wg_tile(s, wgx, wgy);
        s.nseg = (o && o->segments > 0) ? o->segments : 0;
        // the MFMA accumulators sum a segment in plain FP32: its error grows
        // with the segment's length (823,592 beamlets on 64^2 pixels: 1.6e-7
        // at 3,217 per segment, 6.1e-7 at 12,868, 3.4e-6 at 51,474, 1.4e-5
        // at 205,898), so mixed-precision segments hold at most 16,384
        // beamlets, whatever the count's source (automatic, tuned or explicit)
        const int64_t min_seg = min_segments(precision, s.form, n);
        if (s.nseg <= 0) {
            // one round of workgroups, 8 wavefronts per CU (the register
            // budget allows two wavefronts per SIMD; a partial second round
            // leaves CUs idle: on 512^2 pixels, 16 tiles, 16 segments ran
            // 0.78 ms, 32 0.79 ms; with the earlier four-product form's
            // 256 x 128 workgroup tiles 16 segments ran 1.78 ms, 32 0.91 ms,
            // 48 1.22 ms)
            const int64_t tiles =
                std::max<int64_t>(1, (int64_t)((pl.nx + wgx - 1) / wgx) * ((pl.ny + wgy - 1) / wgy));
            const int64_t per_cu = 8 / s.waves;
            int64_t seg = ((int64_t)ctx->cus * per_cu + tiles - 1) / tiles;
            auto it = ctx->tuned.find(tune_key(kTuneSep, precision, n, (int64_t)pl.nx * pl.ny));
            if (it != ctx->tuned.end()) seg = std::max<int64_t>(1, seg * it->second.seg_scale_pct / 100);
            seg = std::min<int64_t>(seg, std::max<int64_t>(1, n / 256));
            s.nseg = (int)std::max<int64_t>(1, std::min<int64_t>(seg, 1024));
        }
        // the cap wins over the 1024-segment limit (above 16.7 M beamlets)
        if (s.nseg < min_seg) s.nseg = (int)std::min<int64_t>(min_seg, 0x7fffffff);
        return s;
    }
    // rotor form: 32 rows per lane where the grid fills a 4-wave tile
    s.rows = (s.form == 2 && pl.ny >= 128) ? 32 : (precision != GBD_MIXED && s.form == 0) ? 4 : 16;
    s.waves = 4;
    s.nseg = 0;
    int seg_pct = 100;
    const bool user = o && (o->rows_per_lane || o->waves || o->segments);
    if (!user) {
        auto it = ctx->tuned.find(tune_key(kTuneEval, precision, n, (int64_t)pl.nx * pl.ny));
        if (it != ctx->tuned.end()) {
            s.rows = it->second.rows;
            s.waves = it->second.waves;
            seg_pct = it->second.seg_scale_pct;
        }
    }
    if (o) {
        if (o->rows_per_lane) s.rows = o->rows_per_lane;
        if (o->waves) s.waves = o->waves;
        if (o->segments) s.nseg = o->segments;
    }
    if (s.rows == 32 && s.form != 2) s.rows = 16;
    if (precision != GBD_MIXED && s.form == 0 && s.rows > 8) s.rows = 8;  // FP64 direct form: up to 8 rows
    // FP64 rotor form with higher-order factors: up to 16 rows (registers)
    if (precision != GBD_MIXED && s.form == 2 && (flags & FLAG_HG) && s.rows > 16) s.rows = 16;
    if (s.nseg <= 0) {
        // enough workgroups to keep every SIMD of every CU busy ~6 waves deep,
        // while each segment keeps at least two LDS tiles of beamlets
        const int64_t tx = (pl.nx + 63) / 64;
        const int64_t ty = (pl.ny + s.waves * s.rows - 1) / (s.waves * s.rows);
        const int64_t tiles = std::max<int64_t>(1, tx * ty);
        const int64_t target_blocks = (int64_t)ctx->cus * 4 * 6 / s.waves;
        int64_t seg = (target_blocks + tiles - 1) / tiles;
        seg = std::max<int64_t>(1, seg * seg_pct / 100);
        seg = std::min<int64_t>(seg, std::max<int64_t>(1, n / 256));
        s.nseg = (int)std::max<int64_t>(1, std::min<int64_t>(seg, 1024));
    }
    return s;
}

bool valid_shape(int rows, int waves, int precision = GBD_MIXED) {
    const bool r = rows == 1 || rows == 2 || rows == 4 || rows == 8 || rows == 16 || rows == 32;
    (void)precision;
    return r && (waves == 1 || waves == 2 || waves == 4);
}

EvalGeom make_geom(const PlaneGeom &pl, int64_t n, const Shape &s) {
    EvalGeom g;
    g.nx = pl.nx;
    g.ny = pl.ny;
    g.dx = pl.dx;
    g.dy = pl.dy;
    g.a0 = -0.5 * (pl.nx - 1) * pl.dx;
    g.b0 = -0.5 * (pl.ny - 1) * pl.dy;
    if (s.form == 3) {
        int wgx, wgy;
        sep_wg_tile(s, wgx, wgy);
        g.tiles_x = (pl.nx + wgx - 1) / wgx;
        g.tiles_y = (pl.ny + wgy - 1) / wgy;
    } else {
        g.tiles_x = (pl.nx + 63) / 64;
        g.tiles_y = (pl.ny + s.waves * s.rows - 1) / (s.waves * s.rows);
    }
    g.n = n;
    int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(s.nseg, std::max<int64_t>(1, n)));
    g.seg_len = (n + nseg - 1) / nseg;
    if (g.seg_len == 0) g.seg_len = 1;
    g.nseg = (int32_t)((n + g.seg_len - 1) / g.seg_len);
    if (g.nseg < 1) g.nseg = 1;
    g.work = g.tiles_x * g.tiles_y * g.nseg;
    return g;
}

// Weideman's coefficients for the Faddeeva function (FaddeevaCoef): a_n,
// n = 1..N, are the Fourier coefficients of the even, 2 pi-periodic
// F(theta) = e^(-s^2) (L^2 + s^2), s = L tan(theta / 2), taken by the
// midpoint rule (spectrally accurate for a smooth periodic integrand).
void weideman(int N, double *L, double *a) {
    *L = std::sqrt(N / std::sqrt(2.0));
    const int K = 4096;
    const double pi = 3.14159265358979323846;
    for (int n = 1; n <= N; n++) {
        double acc = 0.0;
        for (int i = 0; i < K; i++) {
            const double th = -pi + (i + 0.5) * 2.0 * pi / K;
            const double t = *L * std::tan(0.5 * th);
            acc += std::exp(-t * t) * (*L * *L + t * t) * std::cos(n * th);
        }
        a[n - 1] = acc / K;
    }
}

const FaddeevaCoef &faddeeva_coef() {
    static const FaddeevaCoef fc = [] {
        FaddeevaCoef f{};
        weideman(kFaddeevaN64, &f.L64, f.a64);
        double L32, a32[kFaddeevaN32];
        weideman(kFaddeevaN32, &L32, a32);
        f.L32 = (float)L32;
        for (int i = 0; i < kFaddeevaN32; i++) f.a32[i] = (float)a32[i];
        return f;
    }();
    return fc;
}

// Launch geometry of the truncated-beamlet kernel: 64-column tiles of
// 4 wavefronts x kCutRows rows, segments for ~6 wavefronts per SIMD, each
// segment at least 32 beamlets.
EvalGeom cut_geom(const gbd_ctx_s *ctx, int precision, const PlaneGeom &pl, int64_t n_cut, int64_t max_seg = 1024) {
    Shape s;
    s.form = 0;
    s.half = false;
    s.waves = 4;
    s.rows = precision == GBD_MIXED ? kCutRows32 : kCutRows64;
    const int64_t tx = (pl.nx + 63) / 64;
    const int64_t ty = (pl.ny + s.waves * s.rows - 1) / (s.waves * s.rows);
    const int64_t tiles = std::max<int64_t>(1, tx * ty);
    int64_t seg = ((int64_t)ctx->cus * 6 + tiles - 1) / tiles;
    seg = std::min<int64_t>(seg, std::max<int64_t>(1, n_cut / 32));
    s.nseg = (int)std::max<int64_t>(1, std::min<int64_t>(seg, max_seg));
    return make_geom(pl, n_cut, s);
}

// fixed: a caller-provided partial-sum buffer of fixed_bytes (the static
// buffer of gbd_plan_eval_noalloc), used instead of the plan's grow-only one;
// then nothing is allocated and an automatic segment count is lowered to fit.
// guard (gbd_eval's launch ahead of the setup status): the output is
// written only by the guarded reduction, or nothing is launched and the call
// returns kNoSpeculation; guard->check_key is set when the form's FP16 scale
// depends on the key.
// post_req (with post set): a setup status still to be posted, by the
// separable form's evaluation kernel at its start, else by status_post_kernel
// ahead of this evaluation's first kernel; post is cleared once a launch has
// taken it (a call that launches nothing leaves it set).
int plan_eval_impl(gbd_ctx_s *ctx, gbd_plan_s *plan, int precision, void *out, int64_t out_bytes,
                   const gbd_eval_opts *opts, void *fixed = nullptr, size_t fixed_bytes = 0,
                   EvalGuard *guard = nullptr, StatusPost *post_req = nullptr) {
    if (!plan->ready && !guard) return fail(GBD_EINVAL, "gbd_plan_eval: plan has no valid setup");
    if (precision != GBD_FP64 && precision != GBD_MIXED) return fail(GBD_EINVAL, "precision must be GBD_FP64 or GBD_MIXED");
    const int64_t M = (int64_t)plan->pl.nx * plan->pl.ny;
    const int64_t elem = precision == GBD_FP64 ? 16 : 8;
    if (M == 0) return GBD_OK;
    if (!out) return fail(GBD_EINVAL, "field_out is NULL");
    if (out_bytes < M * elem)
        return fail(GBD_ERANGE, "field_out holds %lld bytes, %lld needed", (long long)out_bytes, (long long)(M * elem));
    if (opts && (opts->variant < 0 || opts->variant > 5)) return fail(GBD_EINVAL, "variant must be 0 ... 5");
    // rows_per_lane and waves do not apply to the separable form (its tile is
    // fixed; gbd_plan_shape reports it, and handing that shape back is fine)
    const bool sep_form = pick_form(precision, plan->flags, opts) == 3;
    if (opts && opts->rows_per_lane && !sep_form &&
        !valid_shape(opts->rows_per_lane, opts->waves ? opts->waves : 4, precision))
        return fail(GBD_EINVAL, "unsupported rows_per_lane %d / waves %d", opts->rows_per_lane, opts->waves);
    Shape s = choose_shape(ctx, precision, plan->n - plan->n_cut, plan->pl, plan->flags, opts);
    if (s.form != 3 && !valid_shape(s.rows, s.waves, precision))
        return fail(GBD_EINVAL, "unsupported rows_per_lane %d / waves %d", s.rows, s.waves);
    int rc = ensure_device(ctx);
    if (rc) return rc;
    if (guard && plan->n == 0) return kNoSpeculation;
    if (plan->n == 0) {
        if (fixed)
            HIP_TRY(launch_fill_zero(out, (size_t)(M * elem), ctx->stream), "zero fill launch");
        else
            HIP_TRY(hipMemsetAsync(out, 0, (size_t)(M * elem), ctx->stream), "hipMemsetAsync");
        return GBD_OK;
    }
    // the whole beamlets [0, n_main) in the chosen form; truncated ones
    // [n_main, n) by their own kernel into the following segments
    const int64_t n_main = plan->n - plan->n_cut;
    // the mixed separable form's partials are compact (float2) and come first
    const bool compact = n_main > 0 && s.form == 3 && precision == GBD_MIXED;
    EvalGeom g{}, gc{};
    int32_t nseg_main = 0, nseg_cut = 0;
    if (n_main > 0) {
        g = make_geom(plan->pl, n_main, s);
        nseg_main = g.nseg;
    }
    if (plan->n_cut > 0) {
        gc = cut_geom(ctx, precision, plan->pl, plan->n_cut);
        nseg_cut = gc.nseg;
    }
    if (fixed) {
        // partial bytes of nm main and nc truncated segments (none when one
        // segment writes the output directly)
        const size_t per_main = (size_t)M * (compact ? 8 : 16), per_cut = (size_t)M * 16;
        auto need_of = [&](int64_t nm, int64_t nc) -> size_t {
            if (nm + nc <= 1 && nc == 0) return 0;
            return compact ? reduce_wide_offset((int32_t)nm, M) + (size_t)nc * per_cut : (size_t)(nm + nc) * per_cut;
        };
        if (need_of(nseg_main, nseg_cut) > fixed_bytes) {
            if (opts && opts->segments > 0)
                return fail(GBD_ERANGE, "%d segments of %lld pixels need %zu bytes of partial sums; the static buffer "
                            "holds %zu", (int)(nseg_main + nseg_cut), (long long)M, need_of(nseg_main, nseg_cut),
                            fixed_bytes);
            if (nseg_cut > 0) {  // truncated beamlets: at most half the buffer
                const int64_t max_cut = (int64_t)((fixed_bytes / 2) / per_cut);
                if (max_cut < 1)
                    return fail(GBD_ERANGE, "%lld pixels: one segment of partial sums (%zu bytes) exceeds half the "
                                "static buffer (%zu bytes)", (long long)M, per_cut, fixed_bytes);
                if (nseg_cut > max_cut) {
                    gc = cut_geom(ctx, precision, plan->pl, plan->n_cut, max_cut);
                    nseg_cut = gc.nseg;
                }
            }
            if (n_main > 0) {
                const size_t used = (size_t)nseg_cut * per_cut + (compact ? 16 : 0);
                int64_t max_main = used < fixed_bytes ? (int64_t)((fixed_bytes - used) / per_main) : 0;
                if (nseg_cut == 0 && max_main < 2) max_main = 1;  // one segment: no partials
                const int64_t floor_seg = min_segments(precision, s.form, n_main);
                if (max_main < std::max<int64_t>(floor_seg, 1))
                    return fail(GBD_ERANGE, "%lld beamlets on %lld pixels need at least %lld segments of partial sums; "
                                "the static buffer (%zu bytes) holds %lld", (long long)n_main, (long long)M,
                                (long long)std::max<int64_t>(floor_seg, 1), fixed_bytes, (long long)max_main);
                if (nseg_main > max_main) {
                    s.nseg = (int)max_main;
                    g = make_geom(plan->pl, n_main, s);
                    nseg_main = g.nseg;
                }
            }
            if (need_of(nseg_main, nseg_cut) > fixed_bytes)
                return fail(GBD_ERANGE, "partial sums need %zu bytes; the static buffer holds %zu",
                            need_of(nseg_main, nseg_cut), fixed_bytes);
        }
    }
    if (n_main > 0 && (int64_t)g.tiles_x * g.tiles_y * g.nseg > (int64_t)0x7fffffff - 8)
        return fail(GBD_ERANGE, "grid too large");
    if (nseg_cut > 0 && (int64_t)gc.tiles_x * gc.tiles_y * gc.nseg > (int64_t)0x7fffffff - 8)
        return fail(GBD_ERANGE, "grid too large");
    const int32_t total = nseg_main + nseg_cut;
    const bool reduce = total > 1 || nseg_cut > 0;
    if (guard && !reduce) return kNoSpeculation;
    StatusPost sp;  // the post handed to the separable form's kernel
    if (post_req && post_req->post) {
        if (n_main > 0 && s.form == 3) {
            sp = *post_req;
        } else {
            HIP_TRY(launch_status_post(*post_req, ctx->stream), "status post launch");
            post_req->post = nullptr;
        }
    }
    const int32_t nseg2 = compact ? nseg_main : 0;
    void *partial = fixed ? fixed : plan->scratch;
    if (reduce && !fixed) {
        const size_t need = (size_t)total * (size_t)M * 16;  // bounds the compact layout too
        if (need > plan->scratch_bytes) {
            if (plan->scratch) (void)hipFree(plan->scratch);
            plan->scratch = nullptr;
            plan->scratch_bytes = 0;
            HIP_TRY(hipMalloc(&plan->scratch, need), "hipMalloc(segment partials)");
            plan->scratch_bytes = need;
        }
        partial = plan->scratch;
    }
    if (n_main > 0) {
        const void *rec = precision == GBD_FP64 ? (const void *)plan->r64 : (const void *)plan->r32;
        const bool hg = (plan->flags & FLAG_HG) != 0;
        const void *hrec = !hg ? nullptr : precision == GBD_FP64 ? (const void *)plan->h64 : (const void *)plan->h32;
        EvalGeom gl = g;
        if (reduce) gl.nseg = std::max<int32_t>(total, 2);  // segment partials, never the output
        if (s.form == 2)
            HIP_TRY(launch_sigma(gl, plan->r64, precision == GBD_FP64 ? plan->q64 : nullptr,
                                 precision == GBD_FP64 ? nullptr : plan->r32, ctx->stream),
                    "sigma table kernel launch");
        std::pair<hipEvent_t, hipEvent_t> tev{nullptr, nullptr};
        if (ctx->timing && !fixed) {  // the allocation-free path records none
            if (!ctx->spare_events.empty()) {
                tev = ctx->spare_events.back();
                ctx->spare_events.pop_back();
            } else {
                // timing only (read after a later synchronisation): no
                // system-scope fence, whose cache writeback would stall the
                // stream between the kernels
                HIP_TRY(hipEventCreateWithFlags(&tev.first, hipEventDisableSystemFence), "hipEventCreate");
                const hipError_t e = hipEventCreateWithFlags(&tev.second, hipEventDisableSystemFence);
                if (e != hipSuccess) {
                    (void)hipEventDestroy(tev.first);
                    return hip_fail(e, "hipEventCreate");
                }
            }
            ctx->timed.push_back(tev);
            // the separable forms' launches take the kernel's own times; the
            // others are bracketed by event records
            if (s.form != 3) HIP_TRY(hipEventRecord(tev.first, ctx->stream), "hipEventRecord");
        }
        if (s.form == 3 && precision == GBD_FP64)
            HIP_TRY(launch_eval_sep64(gl, plan->r64, static_cast<const RecHG64 *>(hrec),
                                      static_cast<double2 *>(partial), static_cast<double2 *>(out), ctx->stream,
                                      tev.first, tev.second, sp),
                    "eval kernel launch");
        else if (s.form == 3 && s.half)
            HIP_TRY(launch_eval_seph(gl, plan->r32, static_cast<const RecHG32 *>(hrec), plan->sep_scale,
                                     static_cast<float2 *>(partial), static_cast<float2 *>(out), ctx->stream,
                                     tev.first, tev.second, sp),
                    "eval kernel launch");
        else if (s.form == 3)
            HIP_TRY(launch_eval_sep(gl, plan->r32, static_cast<const RecHG32 *>(hrec),
                                    static_cast<float2 *>(partial), static_cast<float2 *>(out), ctx->stream,
                                    tev.first, tev.second, sp),
                    "eval kernel launch");
        else
            HIP_TRY(launch_eval(precision, s.rows, s.waves, s.form, gl, rec, hrec, plan->q64, partial, out,
                                ctx->stream),
                    "eval kernel launch");
        if (tev.second && s.form != 3) HIP_TRY(hipEventRecord(tev.second, ctx->stream), "hipEventRecord");
        if (post_req) post_req->post = nullptr;  // posted by the kernel just launched (form 3), or above
    }
    if (nseg_cut > 0) {
        const void *rec = precision == GBD_FP64 ? (const void *)(plan->r64 + n_main) : (const void *)(plan->r32 + n_main);
        const void *crec = precision == GBD_FP64 ? (const void *)plan->c64 : (const void *)plan->c32;
        void *wide = static_cast<char *>(partial) + reduce_wide_offset(nseg2, M);
        HIP_TRY(launch_eval_cut(precision, gc, rec, crec, faddeeva_coef(), nseg_main - nseg2, wide, ctx->stream),
                "truncated-beamlet kernel launch");
    }
    if (reduce) {
        EvalGeom gr = n_main > 0 ? g : gc;
        gr.nseg = total;
        EvalGuard gd;
        if (guard) {
            guard->check_key = s.form == 3 && s.half;  // the FP16 form's scale came from the key
            gd = *guard;
        }
        HIP_TRY(launch_reduce(precision, gr, nseg2, partial, out, ctx->stream, gd), "reduce kernel launch");
    }
    return GBD_OK;
}

// The post of the last launched setup's status.
StatusPost pending_post(const gbd_plan_s *plan) {
    StatusPost sp;
    sp.status = plan->status_cur;
    sp.post = plan->status_post;
    sp.seq = plan->status_seq;
    return sp;
}

// The setup in two halves: plan_setup_launch enqueues the setup kernel and
// the post of its status pair (status_post_kernel; with post false the
// caller has the post made, as gbd_eval does by its evaluation kernel), and
// plan_setup_finish waits for the post and takes the status.
int plan_setup_launch(gbd_ctx_s *ctx, gbd_plan_s *plan, gbd_beamlets_s *b, gbd_plane_s *p, bool post = true) {
    if (b->dev.n > plan->capacity)
        return fail(GBD_ERANGE, "plan capacity %lld < %lld beamlets", (long long)plan->capacity, (long long)b->dev.n);
    int rc = ensure_device(ctx);
    if (rc) return rc;
    plan->ready = false;
    plan->spec_ok = false;
    plan->status_cur = nullptr;
    plan->n = b->dev.n;
    plan->pl = p->g;
    plan->n_cut = b->dev.n_cut;
    if (b->dev.n_cut > 0 && (!plan->c64 || !plan->c32)) {
        const size_t cap = (size_t)std::max<int64_t>(1, plan->capacity);
        if (!plan->c64) HIP_TRY(hipMalloc(&plan->c64, cap * sizeof(RecCut64)), "hipMalloc(truncation records)");
        if (!plan->c32) HIP_TRY(hipMalloc(&plan->c32, cap * sizeof(RecCut32)), "hipMalloc(truncation records)");
    }
    if (b->dev.order && (!plan->h64 || !plan->h32)) {
        const size_t cap = (size_t)std::max<int64_t>(1, plan->capacity);
        if (!plan->h64) HIP_TRY(hipMalloc(&plan->h64, cap * sizeof(RecHG64)), "hipMalloc(Hermite-Gaussian records)");
        if (!plan->h32) HIP_TRY(hipMalloc(&plan->h32, cap * sizeof(RecHG32)), "hipMalloc(Hermite-Gaussian records)");
    }
    if (b->dev.n > 0) {
        // the axial term l0 / lambda is common to every beamlet: reduce it once
        const double g0 = b->dev.l0 / b->dev.lam;
        const double gturns = g0 - nearbyint(g0);
        if (!plan->status_zeroed) {
            HIP_TRY(hipMemsetAsync(plan->status_dev, 0, 4 * sizeof(uint32_t), ctx->stream), "hipMemsetAsync(status)");
            plan->status_zeroed = true;
        }
        const bool hg = b->dev.order != nullptr;
        const bool cut = b->dev.n_cut > 0;
        uint32_t *status = plan->status_dev + 2 * plan->status_parity;
        uint32_t *status_next = plan->status_dev + 2 * (plan->status_parity ^ 1);
        HIP_TRY(launch_setup(b->dev, p->g, gturns, plan->r64, plan->r32, hg ? plan->h64 : nullptr,
                             hg ? plan->h32 : nullptr, cut ? plan->c64 : nullptr, cut ? plan->c32 : nullptr,
                             status, status_next, ctx->stream),
                "setup kernel launch");
        plan->status_parity ^= 1;
        plan->status_seq++;
        plan->status_cur = status;
        if (post) HIP_TRY(launch_status_post(pending_post(plan), ctx->stream), "status post launch");
    }
    return GBD_OK;
}

int plan_setup_finish(gbd_ctx_s *ctx, gbd_plan_s *plan) {
    plan->flags = 0;
    if (plan->status_cur) {
        // poll the posted word for this setup's sequence number: busy at
        // first, then yielding; after a second (a stream with long work queued
        // ahead) wait for the stream, after which the post is visible
        const uint32_t seq = plan->status_seq;
        const volatile uint64_t *post = plan->status_post;
        uint64_t w = *post;
        const auto t0 = std::chrono::steady_clock::now();
        for (uint32_t spins = 0; (uint32_t)(w >> 32) != seq; w = *post) {
            if (++spins < 4096) continue;
            const auto dt = std::chrono::steady_clock::now() - t0;
            if (dt > std::chrono::seconds(1)) {
                HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
                w = *post;
                if ((uint32_t)(w >> 32) != seq) return fail(GBD_EHIP, "the setup status was not posted");
                break;
            }
            if (dt > std::chrono::microseconds(200)) std::this_thread::yield();
        }
        const uint32_t st = (uint32_t)w & 0xffu;
        // FP16 separable form: largest term 2^P over the grid -> scale 2^(2 kSepHalfExp - P)
        const uint32_t key = ((uint32_t)w >> 8) & 0xfffu;
        plan->sep_key = key;
        plan->sep_scale = key ? 2 * kSepHalfExp - ((int)key - 2048) : 0;
        if (st & FLAG_PARALLEL) return fail(GBD_EPARALLEL, "a base ray is parallel to the detector plane");
        if (st & FLAG_BRANCH)
            return fail(GBD_EBRANCH, "an eigenvalue of A + B Q1^-1 lies off the principal branch (inverting system)");
        if (st & FLAG_NONFINITE) return fail(GBD_EINVAL, "non-finite beamlet parameters after propagation");
        if (st & FLAG_HG_TILT)
            return fail(GBD_EINVAL, "higher-order and truncated beamlets need a detector plane normal to the axis");
        plan->flags = st & (FLAG_STEEP | FLAG_CROSS | FLAG_HG);
    }
    plan->ready = true;
    plan->spec_ok = plan->status_cur != nullptr;
    return GBD_OK;
}

int plan_setup_impl(gbd_ctx_s *ctx, gbd_plan_s *plan, gbd_beamlets_s *b, gbd_plane_s *p) {
    const int rc = plan_setup_launch(ctx, plan, b, p);
    return rc ? rc : plan_setup_finish(ctx, plan);
}

void plan_destroy(gbd_plan_s *plan) {
    if (!plan) return;
    if (plan->r64) (void)hipFree(plan->r64);
    if (plan->r32) (void)hipFree(plan->r32);
    if (plan->q64) (void)hipFree(plan->q64);
    if (plan->h64) (void)hipFree(plan->h64);
    if (plan->h32) (void)hipFree(plan->h32);
    if (plan->c64) (void)hipFree(plan->c64);
    if (plan->c32) (void)hipFree(plan->c32);
    if (plan->status_dev) (void)hipFree(plan->status_dev);
    if (plan->scratch) (void)hipFree(plan->scratch);
    if (plan->status_post) {
        // a post still in flight writes this memory: let the device finish first
        (void)hipDeviceSynchronize();
        (void)hipHostFree(plan->status_post);
    }
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
    if (e == hipSuccess) e = hipMalloc(&p->q64, cap * sizeof(RecSq64));
    if (e == hipSuccess) e = hipMalloc(&p->status_dev, 4 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc(&p->status_post, sizeof(uint64_t), hipHostMallocCoherent);
    if (e == hipSuccess) *p->status_post = 0;
    if (e != hipSuccess) {
        plan_destroy(p);
        return hip_fail(e, "plan allocation");
    }
    *out = p;
    return GBD_OK;
}

int grow(DevBuf &b, size_t bytes, const char *what) {
    if (bytes <= b.bytes) return GBD_OK;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    bytes = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) return hip_fail(e, what);
    b.bytes = bytes;
    return GBD_OK;
}

void batch_free(BatchWork &w) {
    DevBuf *all[] = {&w.rec,    &w.l5,   &w.e0t,     &w.tab1,  &w.tab2, &w.e0,
                     &w.e0part, &w.part, &w.metrics, &w.flags, &w.point};
    if (w.stage_ev) {
        (void)hipEventSynchronize(w.stage_ev);
        (void)hipEventDestroy(w.stage_ev);
    }
    for (DevBuf *b : all)
        if (b->p) (void)hipFree(b->p);
    if (w.host_flags) (void)hipHostFree(w.host_flags);
    if (w.stage) (void)hipHostFree(w.stage);
    w = BatchWork();
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
    if (device >= kMaxDevices) return fail(GBD_EINVAL, "device %d: at most %d devices", device, kMaxDevices);
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[device]) {
            void *ptr = nullptr;
            HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(static partial buffer)");
            if (!ptr) return fail(GBD_EHIP, "hipGetSymbolAddress(static partial buffer) returned NULL");
            g_scratch_dev[device] = ptr;
        }
    }
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
    gbd_ctx_s *c = new (std::nothrow) gbd_ctx_s();
    if (!c) return fail(GBD_ENOMEM, "host allocation failed");
    c->pool = std::make_shared<DevPool>();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->cus = cus > 0 ? cus : 256;
    c->own_plan = nullptr;
    *out = c;
    return GBD_OK;
}

int gbd_ctx_set_stream(gbd_ctx_t ctx, void *hip_stream) {
    if (!ctx) return fail(GBD_EINVAL, "ctx is NULL");
    hipStream_t next = static_cast<hipStream_t>(hip_stream);
    if (next != ctx->stream) {
        // pooled blocks are reused in stream order: drain the old stream first
        HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
        HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    }
    ctx->stream = next;
    return GBD_OK;
}

void gbd_ctx_destroy(gbd_ctx_t ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->up_ev) {
        (void)hipEventSynchronize(ctx->up_ev);
        (void)hipEventDestroy(ctx->up_ev);
    }
    if (ctx->up_stage) (void)hipHostFree(ctx->up_stage);
    plan_destroy(ctx->own_plan);
    batch_free(ctx->batch);
    for (auto *v : {&ctx->timed, &ctx->spare_events})
        for (auto &ev : *v) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    delete ctx;
}

int gbd_ctx_set_kernel_timing(gbd_ctx_t ctx, int enable) {
    if (!ctx) return fail(GBD_EINVAL, "ctx is NULL");
    ctx->timing = enable != 0;
    return GBD_OK;
}

int gbd_ctx_kernel_times(gbd_ctx_t ctx, float *ms_out, int32_t cap, int32_t *n) {
    if (!ctx || !n || (cap > 0 && !ms_out)) return fail(GBD_EINVAL, "NULL argument");
    if (cap < 0) return fail(GBD_EINVAL, "negative capacity");
    int rc = ensure_device(ctx);
    if (rc) return rc;
    int32_t k = 0;
    hipError_t first_err = hipSuccess;
    for (auto &ev : ctx->timed) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(ev.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.first, ev.second);
        if (e != hipSuccess && first_err == hipSuccess) first_err = e;
        if (k < cap) ms_out[k] = ms;
        k++;
        ctx->spare_events.push_back(ev);
    }
    ctx->timed.clear();
    *n = k;
    if (first_err != hipSuccess) return hip_fail(first_err, "kernel timing events");
    return GBD_OK;
}

static int beamlets_impl(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0, const double *r1,
                  const double *th1, const double *w0, int64_t n_w0, const double *amp, const double *path,
                  const double *abcd, int64_t n_abcd, const double *base, double sympl_tol,
                  const int32_t *order = nullptr, const double *edge = nullptr) {
    if (!ctx || !out) return fail(GBD_EINVAL, "ctx/out is NULL");
    if (!(sympl_tol > 0.0 && sympl_tol <= 1e-3)) return fail(GBD_EINVAL, "sympl_tol must be in (0, 1e-3]");
    if (n < 0) return fail(GBD_EINVAL, "n < 0");
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(GBD_EINVAL, "lambda must be finite and > 0");
    if (!std::isfinite(l0)) return fail(GBD_EINVAL, "l0 must be finite");
    if (n > 0) {
        if (!r1 || !w0 || !abcd) return fail(GBD_EINVAL, "r1, w0 and abcd are required");
        if (!(n_w0 == 1 || n_w0 == n)) return fail(GBD_EINVAL, "n_w0 must be 1 or n");
        if (!(n_abcd == 1 || n_abcd == n)) return fail(GBD_EINVAL, "n_abcd must be 1 or n");
        if (!finite_all(r1, 2 * n) || (th1 && !finite_all(th1, 2 * n)) || (amp && !finite_all(amp, 2 * n)) ||
            (path && !finite_all(path, n)) || !finite_all(abcd, 16 * n_abcd) || (base && !finite_all(base, 5 * n)))
            return fail(GBD_EINVAL, "non-finite input");
        for (int64_t i = 0; i < n_w0; i++)
            if (!(w0[i] > 0.0) || !std::isfinite(w0[i])) return fail(GBD_EINVAL, "w0[%lld] must be finite and > 0", (long long)i);
        for (int64_t i = 0; i < n_abcd; i++)
            if (!(base ? symplectic_balanced(abcd + 16 * i, sympl_tol) : symplectic(abcd + 16 * i, sympl_tol)))
                return fail(GBD_ENOTSYMPLECTIC, "abcd[%lld] is not symplectic", (long long)i);
        if (order)
            for (int64_t i = 0; i < 2 * n; i++)
                if (order[i] < 0 || order[i] > 2)
                    return fail(GBD_EINVAL, "order[%lld][%lld] = %d is outside 0 ... 2", (long long)(i / 2),
                                (long long)(i % 2), order[i]);
        if (edge) {
            if (!finite_all(edge, 3 * n)) return fail(GBD_EINVAL, "non-finite edge");
            for (int64_t i = 0; i < n; i++) {
                const double ex = edge[3 * i], ey = edge[3 * i + 1];
                if ((ex != 0.0 || ey != 0.0) && !(std::fabs(ex * ex + ey * ey - 1.0) <= 1e-12))
                    return fail(GBD_EINVAL, "edge[%lld]: the normal (e_x, e_y) must have unit length", (long long)i);
            }
        }
    } else {
        n_w0 = 1;
        n_abcd = 1;
        base = nullptr;
        order = nullptr;
        edge = nullptr;
    }
    // truncated beamlets are stored last (stable order otherwise): the
    // evaluation gives them a kernel of their own
    std::vector<int64_t> perm((size_t)std::max<int64_t>(n, 0));
    int64_t n_cut = 0;
    {
        size_t at = 0;
        for (int64_t i = 0; i < n; i++)
            if (!edge || (edge[3 * i] == 0.0 && edge[3 * i + 1] == 0.0)) perm[at++] = i;
        for (int64_t i = 0; i < n; i++)
            if (edge && (edge[3 * i] != 0.0 || edge[3 * i + 1] != 0.0)) {
                perm[at++] = i;
                n_cut++;
            }
    }
    bool higher = false;
    if (order)
        for (int64_t i = 0; i < 2 * n && !higher; i++) higher = order[i] != 0;
    int rc = ensure_device(ctx);
    if (rc) return rc;
    // one device block: r1, th1, amp [n][2]; w0 [n_w0]; path [n]; abcd [n_abcd][16]; base [n][5];
    // edge [n][3]; orders [n][2] int32 packed into the trailing n doubles
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    const size_t off_r1 = 0, off_th1 = off_r1 + 2 * nn, off_amp = off_th1 + 2 * nn, off_w0 = off_amp + 2 * nn,
                 off_path = off_w0 + (size_t)n_w0, off_abcd = off_path + nn, off_base = off_abcd + 16 * (size_t)n_abcd,
                 off_edge = off_base + (base ? 5 * nn : 0), off_order = off_edge + (edge ? 3 * nn : 0),
                 total = off_order + (order ? nn : 0);
    const size_t bytes = total * sizeof(double);
    if (!ctx->up_ev) HIP_TRY(hipEventCreateWithFlags(&ctx->up_ev, hipEventDisableTiming), "hipEventCreate");
    if (ctx->up_pending) HIP_TRY(hipEventSynchronize(ctx->up_ev), "hipEventSynchronize");
    ctx->up_pending = false;
    if (bytes > ctx->up_bytes) {
        if (ctx->up_stage) (void)hipHostFree(ctx->up_stage);
        ctx->up_stage = nullptr;
        ctx->up_bytes = 0;
        const size_t want = std::max<size_t>(bytes, (size_t)1 << 20);
        HIP_TRY(hipHostMalloc(&ctx->up_stage, want, hipHostMallocDefault), "hipHostMalloc(beamlet staging)");
        ctx->up_bytes = want;
    }
    double *host = static_cast<double *>(ctx->up_stage);
    memset(host, 0, bytes);
    if (n > 0) {
        int32_t *ord = reinterpret_cast<int32_t *>(&host[off_order]);
        if (n_w0 == 1) host[off_w0] = w0[0];
        if (n_abcd == 1) memcpy(&host[off_abcd], abcd, 16 * sizeof(double));
        for (int64_t i = 0; i < n; i++) {
            const int64_t j = perm[i];
            host[off_r1 + 2 * i] = r1[2 * j];
            host[off_r1 + 2 * i + 1] = r1[2 * j + 1];
            if (th1) {
                host[off_th1 + 2 * i] = th1[2 * j];
                host[off_th1 + 2 * i + 1] = th1[2 * j + 1];
            }
            host[off_amp + 2 * i] = amp ? amp[2 * j] : 1.0;
            host[off_amp + 2 * i + 1] = amp ? amp[2 * j + 1] : 0.0;
            if (n_w0 == n) host[off_w0 + i] = w0[j];
            if (path) host[off_path + i] = path[j];
            if (n_abcd == n) memcpy(&host[off_abcd + 16 * i], abcd + 16 * j, 16 * sizeof(double));
            if (base) memcpy(&host[off_base + 5 * i], base + 5 * j, 5 * sizeof(double));
            if (edge) memcpy(&host[off_edge + 3 * i], edge + 3 * j, 3 * sizeof(double));
            if (order) {
                ord[2 * i] = order[2 * j];
                ord[2 * i + 1] = order[2 * j + 1];
            }
        }
    } else {
        host[off_w0] = 1.0;
        for (int i = 0; i < 4; i++) host[off_abcd + 5 * i] = 1.0;
    }
    void *mem = nullptr;
    const size_t cls = DevPool::size_class(total * sizeof(double));
    HIP_TRY(ctx->pool->get(cls, &mem), "hipMalloc(beamlets)");
    hipError_t e = hipMemcpyAsync(mem, host, bytes, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(ctx->up_ev, ctx->stream);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(ctx->stream);
        ctx->pool->put(mem, cls);
        return hip_fail(e, "beamlet upload");
    }
    ctx->up_pending = true;
    gbd_beamlets_s *b = new (std::nothrow) gbd_beamlets_s();
    if (!b) {
        ctx->pool->put(mem, cls);
        return fail(GBD_ENOMEM, "host allocation failed");
    }
    double *d = static_cast<double *>(mem);
    b->ctx = ctx;
    b->mem = mem;
    b->mem_class = cls;
    b->pool = ctx->pool;
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
    b->dev.base = base ? d + off_base : nullptr;
    b->dev.order = order ? reinterpret_cast<const int32_t *>(d + off_order) : nullptr;
    b->dev.edge = edge ? d + off_edge : nullptr;
    b->dev.n_cut = n_cut;
    b->higher_order = higher;
    *out = b;
    return GBD_OK;
}

int gbd_beamlets(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0, const double *r1,
                 const double *th1, const double *w0, int64_t n_w0, const double *amp, const double *path,
                 const double *abcd, int64_t n_abcd) {
    return beamlets_impl(ctx, out, n, lambda, l0, r1, th1, w0, n_w0, amp, path, abcd, n_abcd, nullptr, 1e-10);
}

int gbd_beamlets_traced(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0, const double *r1,
                        const double *th1, const double *w0, int64_t n_w0, const double *amp, const double *path,
                        const double *abcd, const double *base, double sympl_tol) {
    if (n > 0 && !base) return fail(GBD_EINVAL, "base is NULL");
    return beamlets_impl(ctx, out, n, lambda, l0, r1, th1, w0, n_w0, amp, path, abcd, n, base, sympl_tol);
}

int gbd_beamlets_hg(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0, const double *r1,
                    const double *th1, const double *w0, int64_t n_w0, const double *amp, const double *path,
                    const double *abcd, int64_t n_abcd, const int32_t *order) {
    if (n > 0 && !order) return fail(GBD_EINVAL, "order is NULL");
    return beamlets_impl(ctx, out, n, lambda, l0, r1, th1, w0, n_w0, amp, path, abcd, n_abcd, nullptr, 1e-10, order);
}

int gbd_beamlets_truncated(gbd_ctx_t ctx, gbd_beamlets_t *out, int64_t n, double lambda, double l0,
                           const double *r1, const double *th1, const double *w0, int64_t n_w0, const double *amp,
                           const double *path, const double *abcd, int64_t n_abcd, const double *edge) {
    if (n > 0 && !edge) return fail(GBD_EINVAL, "edge is NULL");
    return beamlets_impl(ctx, out, n, lambda, l0, r1, th1, w0, n_w0, amp, path, abcd, n_abcd, nullptr, 1e-10,
                         nullptr, edge);
}

int gbd_trace(gbd_ctx_t ctx, int32_t n_mirrors, const double *mirrors, double z_in, double z_out, double l0,
              int64_t n, const double *r1, const double *th1, double dr, double dth, double *base_out,
              double *abcd_out, int32_t *flags_out) {
    if (!ctx) return fail(GBD_EINVAL, "ctx is NULL");
    if (n_mirrors < 0 || n_mirrors > kMaxMirrors) return fail(GBD_EINVAL, "n_mirrors must be in [0, %d]", kMaxMirrors);
    if (n < 0) return fail(GBD_EINVAL, "n < 0");
    if (!(dr > 0.0) || !(dth > 0.0) || !std::isfinite(dr) || !std::isfinite(dth))
        return fail(GBD_EINVAL, "dr and dth must be finite and > 0");
    if (!std::isfinite(z_in) || !std::isfinite(z_out) || !std::isfinite(l0)) return fail(GBD_EINVAL, "non-finite plane");
    if (n_mirrors > 0 && !mirrors) return fail(GBD_EINVAL, "mirrors is NULL");
    if (n > 0 && (!r1 || !base_out || !abcd_out || !flags_out)) return fail(GBD_EINVAL, "NULL array");
    TraceSystem S;
    S.n = n_mirrors;
    S.z_in = z_in;
    S.z_out = z_out;
    S.l0 = l0;
    for (int i = 0; i < n_mirrors; i++) {
        const double *e = mirrors + 5 * i;
        if (!finite_all(e, 5)) return fail(GBD_EINVAL, "non-finite mirror %d", i);
        S.m[i] = TraceMirror{e[0], e[1] == 0.0 ? 0.0 : 1.0 / e[1], e[2], e[3], e[4]};
    }
    if (n > 0 && (!finite_all(r1, 2 * n) || (th1 && !finite_all(th1, 2 * n))))
        return fail(GBD_EINVAL, "non-finite ray");
    if (n == 0) return GBD_OK;
    int rc = ensure_device(ctx);
    if (rc) return rc;
    // device block: r1 [n][2], th1 [n][2], base [n][5], abcd [n][16], flags [n] (int32)
    const size_t nd = (size_t)n;
    const size_t off_th = 2 * nd, off_base = 4 * nd, off_abcd = 9 * nd, off_flags = 25 * nd;
    void *mem = nullptr;
    HIP_TRY(hipMalloc(&mem, off_flags * sizeof(double) + nd * sizeof(int32_t)), "hipMalloc(trace)");
    double *d = static_cast<double *>(mem);
    int32_t *dflags = reinterpret_cast<int32_t *>(d + off_flags);
    hipError_t e = hipMemcpyAsync(d, r1, 2 * nd * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess && th1) e = hipMemcpyAsync(d + off_th, th1, 2 * nd * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_trace(S, n, d, th1 ? d + off_th : nullptr, dr, dth, d + off_base, d + off_abcd, dflags, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(base_out, d + off_base, 5 * nd * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(abcd_out, d + off_abcd, 16 * nd * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(flags_out, dflags, nd * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(mem);
    if (e != hipSuccess) return hip_fail(e, "trace");
    return GBD_OK;
}

void gbd_beamlets_free(gbd_beamlets_t b) {
    if (!b) return;
    if (b->mem) b->pool->put(b->mem, b->mem_class);
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
    if (b->ctx != ctx) return fail(GBD_EINVAL, "the beamlets belong to another context");
    return plan_setup_impl(ctx, plan, b, p);
}

int gbd_plan_eval(gbd_ctx_t ctx, gbd_plan_t plan, int precision, void *field_out, int64_t out_bytes,
                  const gbd_eval_opts *opts) {
    if (!ctx || !plan) return fail(GBD_EINVAL, "NULL argument");
    return plan_eval_impl(ctx, plan, precision, field_out, out_bytes, opts);
}

int gbd_plan_eval_noalloc(gbd_ctx_t ctx, gbd_plan_t plan, int precision, void *field_out, int64_t out_bytes,
                          const gbd_eval_opts *opts) {
    if (!ctx || !plan) return fail(GBD_EINVAL, "NULL argument");
    void *buf = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        buf = g_scratch_dev[ctx->device];
    }
    if (!buf) return fail(GBD_EHIP, "device %d has no static partial buffer address", ctx->device);
    return plan_eval_impl(ctx, plan, precision, field_out, out_bytes, opts, buf, (size_t)GBD_NOALLOC_SCRATCH_BYTES);
}

void gbd_plan_free(gbd_plan_t plan) { plan_destroy(plan); }

int gbd_issue_probe(gbd_ctx_t ctx, int32_t cls, int32_t iters, double *ms_out, double *wave_instructions_out) {
    if (!ctx || !ms_out || !wave_instructions_out) return fail(GBD_EINVAL, "NULL argument");
    if (cls < 0 || cls > 9) return fail(GBD_EINVAL, "class must be 0 ... 9");
    if (iters < 1) return fail(GBD_EINVAL, "iters must be >= 1");
    int rc = ensure_device(ctx);
    if (rc) return rc;
    const int blocks = ctx->cus * 8;
    float *sink = nullptr;
    HIP_TRY(hipMalloc(&sink, (size_t)blocks * 256 * sizeof(float)), "hipMalloc(probe)");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_issue_probe(cls, blocks, iters, sink, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
    if (e == hipSuccess) e = launch_issue_probe(cls, blocks, iters, sink, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess) return hip_fail(e, "issue probe");
    const double waves = (double)blocks * 4.0;
    *ms_out = ms;
    // class 9 counts its MFMA instructions
    *wave_instructions_out = waves * (double)iters * ((cls <= 3 || cls == 7 || cls == 8) ? 16.0 : 4.0);
    return GBD_OK;
}

int gbd_plan_shape(gbd_ctx_t ctx, gbd_plan_t plan, int precision, const gbd_eval_opts *opts, gbd_eval_opts *resolved) {
    if (!ctx || !plan || !resolved) return fail(GBD_EINVAL, "NULL argument");
    Shape s = choose_shape(ctx, precision, plan->n - plan->n_cut, plan->pl, plan->flags, opts);
    EvalGeom g = make_geom(plan->pl, plan->n - plan->n_cut, s);
    resolved->rows_per_lane = s.rows;
    resolved->waves = s.waves;
    resolved->segments = g.nseg;
    resolved->variant = form_variant(precision, s.form, s.half);
    return GBD_OK;
}

int gbd_eval(gbd_ctx_t ctx, gbd_beamlets_t b, gbd_plane_t p, int precision, void *field_out, int64_t out_bytes,
             const gbd_eval_opts *opts) {
    if (!ctx || !b || !p) return fail(GBD_EINVAL, "NULL argument");
    if (b->ctx != ctx) return fail(GBD_EINVAL, "the beamlets belong to another context");
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
    gbd_plan_s *plan = ctx->own_plan;
    if (!plan->spec_ok) {
        int rc = plan_setup_impl(ctx, plan, b, p);
        if (rc) return rc;
        return plan_eval_impl(ctx, plan, precision, field_out, out_bytes, opts);
    }
    // The last setup of this plan succeeded: launch the evaluation right
    // behind this setup with its flags and FP16 scale, before the host has
    // read the new status, so no host round trip separates the two kernels.
    // The reduction writes the output only if the status has no error and
    // the same flags and key (EvalGuard); otherwise it writes nothing and,
    // for a mere change of form or scale, the evaluation runs again below.
    const uint32_t kFormFlags = FLAG_STEEP | FLAG_CROSS | FLAG_HG;
    const uint32_t pflags = plan->flags;
    const uint32_t pkey = plan->sep_key;
    const int pscale = plan->sep_scale;
    int rc = plan_setup_launch(ctx, plan, b, p, false);
    if (rc) return rc;
    if (!plan->status_cur)  // no beamlets: nothing was launched
        return (rc = plan_setup_finish(ctx, plan)) ? rc : plan_eval_impl(ctx, plan, precision, field_out, out_bytes, opts);
    plan->flags = pflags;
    plan->sep_key = pkey;
    plan->sep_scale = pscale;
    EvalGuard guard;
    guard.status = plan->status_cur;
    guard.mask = kFormFlags;
    guard.flags = pflags & kFormFlags;
    guard.key = pkey;
    const size_t timed_before = ctx->timed.size();
    // the setup status is posted by the separable form's kernel at its start
    // (one kernel launch fewer), else by its own kernel
    StatusPost post_req = pending_post(plan);
    const int ahead = plan_eval_impl(ctx, plan, precision, field_out, out_bytes, opts, nullptr, 0, &guard, &post_req);
    if (post_req.post) HIP_TRY(launch_status_post(post_req, ctx->stream), "status post launch");
    rc = plan_setup_finish(ctx, plan);
    if (!rc && ahead == GBD_OK && (plan->flags & kFormFlags) == guard.flags &&
        (!guard.check_key || plan->sep_key == pkey))
        return GBD_OK;
    // the launch ahead wrote nothing: drop its timing pair, if any
    while (ctx->timed.size() > timed_before) {
        ctx->spare_events.push_back(ctx->timed.back());
        ctx->timed.pop_back();
    }
    if (rc) return rc;  // a setup error (the guard kept the output untouched)
    if (ahead != GBD_OK && ahead != kNoSpeculation) return ahead;
    // evaluate with the status just read
    return plan_eval_impl(ctx, plan, precision, field_out, out_bytes, opts);
}

int gbd_autotune(gbd_ctx_t ctx, gbd_plan_t plan, int precision, int32_t reps, gbd_eval_opts *best, double *best_ms) {
    if (!ctx || !plan) return fail(GBD_EINVAL, "NULL argument");
    if (!plan->ready) return fail(GBD_EINVAL, "gbd_autotune: plan has no valid setup");
    if (precision != GBD_FP64 && precision != GBD_MIXED) return fail(GBD_EINVAL, "precision must be GBD_FP64 or GBD_MIXED");
    if (reps < 1) reps = 1;
    const int64_t M = (int64_t)plan->pl.nx * plan->pl.ny;
    if (M == 0 || plan->n == 0) return fail(GBD_EINVAL, "nothing to tune (empty plan)");
    int rc = ensure_device(ctx);
    if (rc) return rc;
    void *out = nullptr;
    const int64_t out_bytes = M * (precision == GBD_FP64 ? 16 : 8);
    HIP_TRY(hipMalloc(&out, (size_t)out_bytes), "hipMalloc(autotune output)");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    TuneVal bestv{0, 0, 100, 1e300};
    static const int rows_c[] = {2, 4, 8, 16, 32}, waves_c[] = {1, 2, 4}, pct_c[] = {50, 100, 200, 400};
    const int64_t n_main = plan->n - plan->n_cut;  // the beamlets choose_shape sizes the form for
    // the separable form has a fixed tile: only its segment count is tuned
    const bool sep = pick_form(precision, plan->flags, nullptr) == 3;
    const int kind = sep ? kTuneSep : kTuneEval;
    const int n_rows = sep ? 1
                           : precision == GBD_MIXED ? ((plan->flags & FLAG_STEEP) ? 4 : 5)
                           : (plan->flags & FLAG_STEEP) ? 3
                           : (plan->flags & FLAG_HG)    ? 4
                                                        : 5;
    const int n_waves = sep ? 1 : 3;
    for (int ri = 0; ri < n_rows && he == hipSuccess && rc == GBD_OK; ri++)
        for (int wi = 0; wi < n_waves && he == hipSuccess && rc == GBD_OK; wi++)
            for (int pi = 0; pi < 4 && he == hipSuccess && rc == GBD_OK; pi++) {
                // a candidate is addressed through the cache so that choose_shape
                // resolves its segment count exactly as a tuned call would
                const TuneKey key = tune_key(kind, precision, n_main, M);
                const auto saved = ctx->tuned.find(key) != ctx->tuned.end() ? ctx->tuned[key] : TuneVal{0, 0, 0, -1};
                ctx->tuned[key] = TuneVal{sep ? 0 : rows_c[ri], sep ? 0 : waves_c[wi], pct_c[pi], 0.0};
                rc = plan_eval_impl(ctx, plan, precision, out, out_bytes, nullptr);  // warm-up / scratch growth
                double ms = 0.0;
                if (rc == GBD_OK) {
                    he = hipEventRecord(e0, ctx->stream);
                    for (int r = 0; r < reps && rc == GBD_OK && he == hipSuccess; r++)
                        rc = plan_eval_impl(ctx, plan, precision, out, out_bytes, nullptr);
                    if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
                    if (he == hipSuccess) he = hipEventSynchronize(e1);
                    float f = 0.f;
                    if (he == hipSuccess) he = hipEventElapsedTime(&f, e0, e1);
                    ms = f / reps;
                }
                if (saved.ms < 0)
                    ctx->tuned.erase(key);
                else
                    ctx->tuned[key] = saved;
                if (rc == GBD_OK && he == hipSuccess && ms < bestv.ms)
                    bestv = TuneVal{sep ? 0 : rows_c[ri], sep ? 0 : waves_c[wi], pct_c[pi], ms};
            }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (rc) return rc;
    if (he != hipSuccess) return hip_fail(he, "autotune timing");
    ctx->tuned[tune_key(kind, precision, n_main, M)] = bestv;
    if (best) {
        const Shape s = choose_shape(ctx, precision, n_main, plan->pl, plan->flags, nullptr);
        const EvalGeom g = make_geom(plan->pl, n_main, s);
        *best = gbd_eval_opts{s.rows, s.waves, g.nseg, form_variant(precision, s.form, s.half)};
    }
    if (best_ms) *best_ms = bestv.ms;
    return GBD_OK;
}

int gbd_autotune_save(gbd_ctx_t ctx, const char *path) {
    if (!ctx || !path) return fail(GBD_EINVAL, "NULL argument");
    FILE *f = fopen(path, "w");
    if (!f) return fail(GBD_EINVAL, "cannot write %s", path);
    fprintf(f, "# kind precision log2N log2M rows waves seg_pct ms\n");
    for (const auto &kv : ctx->tuned)
        fprintf(f, "%d %d %d %d %d %d %d %.6f\n", kv.first.kind, kv.first.precision, kv.first.ln, kv.first.lm,
                kv.second.rows, kv.second.waves, kv.second.seg_scale_pct, kv.second.ms);
    fclose(f);
    return GBD_OK;
}

int gbd_autotune_load(gbd_ctx_t ctx, const char *path) {
    if (!ctx || !path) return fail(GBD_EINVAL, "NULL argument");
    FILE *f = fopen(path, "r");
    if (!f) return fail(GBD_EINVAL, "cannot read %s", path);
    char line[256];
    int loaded = 0;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        TuneKey k;
        TuneVal v;
        if (sscanf(line, "%d %d %d %d %d %d %d %lf", &k.kind, &k.precision, &k.ln, &k.lm, &v.rows, &v.waves,
                   &v.seg_scale_pct, &v.ms) == 8 &&
            (k.kind == kTuneSep ? v.rows == 0 && v.waves == 0
                                : (k.kind == kTuneEval || k.kind == kTuneBatch) && valid_shape(v.rows, v.waves, k.precision)) &&
            v.seg_scale_pct > 0 && v.seg_scale_pct <= 10000) {
            ctx->tuned[k] = v;
            loaded++;
        }
    }
    fclose(f);
    return loaded;
}

int gbd_eval_point(gbd_ctx_t ctx, gbd_beamlets_t b, gbd_plane_t p, void *field_out, int64_t out_bytes) {
    if (!ctx || !b || !p) return fail(GBD_EINVAL, "NULL argument");
    if (b->ctx != ctx) return fail(GBD_EINVAL, "the beamlets belong to another context");
    if (b->higher_order || b->dev.n_cut > 0)
        return fail(GBD_EINVAL, "point evaluation takes whole fundamental Gaussian beamlets only");
    const int64_t M = (int64_t)p->g.nx * p->g.ny;
    if (M == 0) return GBD_OK;
    if (!field_out) return fail(GBD_EINVAL, "field_out is NULL");
    if (out_bytes < M * 16)
        return fail(GBD_ERANGE, "field_out holds %lld bytes, %lld needed", (long long)out_bytes, (long long)(M * 16));
    int rc = ensure_device(ctx);
    if (rc) return rc;
    BatchWork &w = ctx->batch;
    if ((rc = grow(w.point, (size_t)std::max<int64_t>(b->dev.n, 1) * sizeof(RecPt), "point records")) ||
        (rc = grow(w.flags, 4 * sizeof(uint32_t), "flags")))
        return rc;
    if (!w.host_flags) HIP_TRY(hipHostMalloc(&w.host_flags, 4 * sizeof(uint32_t), hipHostMallocDefault), "hipHostMalloc");
    const double g0 = b->dev.l0 / b->dev.lam;
    uint32_t *flags = static_cast<uint32_t *>(w.flags.p);
    HIP_TRY(hipMemsetAsync(flags + 3, 0, sizeof(uint32_t), ctx->stream), "hipMemsetAsync");
    HIP_TRY(launch_point(b->dev, p->g, g0 - nearbyint(g0), static_cast<RecPt *>(w.point.p),
                         static_cast<double2 *>(field_out), flags + 3, ctx->stream),
            "point evaluation launch");
    HIP_TRY(hipMemcpyAsync(w.host_flags + 3, flags + 3, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream),
            "status copy");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (w.host_flags[3] & FLAG_BRANCH)
        return fail(GBD_EBRANCH, "an eigenvalue left the principal branch at some pixel (field_out is not valid)");
    return GBD_OK;
}

int gbd_airy(gbd_ctx_t ctx, gbd_plane_t p, double D, double f, double lambda, float *out, int64_t out_bytes) {
    if (!ctx || !p) return fail(GBD_EINVAL, "NULL argument");
    if (!(D > 0.0) || !(f > 0.0) || !(lambda > 0.0) || !std::isfinite(D) || !std::isfinite(f) || !std::isfinite(lambda))
        return fail(GBD_EINVAL, "D, f and lambda must be finite and > 0");
    const int64_t M = (int64_t)p->g.nx * p->g.ny;
    if (M == 0) return GBD_OK;
    if (!out) return fail(GBD_EINVAL, "out is NULL");
    if (out_bytes < M * 4) return fail(GBD_ERANGE, "out holds %lld bytes, %lld needed", (long long)out_bytes, (long long)(M * 4));
    int rc = ensure_device(ctx);
    if (rc) return rc;
    const double vscale = M_PI * D / (lambda * f);
    HIP_TRY(launch_airy(p->g.nx, p->g.ny, p->g.dx, p->g.dy, vscale, out, ctx->stream), "airy kernel launch");
    return GBD_OK;
}

int gbd_eval_batch(gbd_ctx_t ctx, int32_t n_inst, const gbd_beamlets_t *bs, const gbd_plane_t *ps, const float *airy,
                   int64_t airy_bytes, const double *zone_edges, int32_t n_zones, double *metrics_out,
                   void *fields_out, int64_t fields_bytes, const gbd_eval_opts *opts) {
    if (!ctx) return fail(GBD_EINVAL, "ctx is NULL");
    if (n_inst < 0) return fail(GBD_EINVAL, "n_inst < 0");
    if (n_inst == 0) return GBD_OK;
    if (!bs || !ps) return fail(GBD_EINVAL, "beamlets/planes arrays are NULL");
    if (n_zones < 0 || n_zones > kMaxZones) return fail(GBD_EINVAL, "n_zones must be in [0, %d]", kMaxZones);
    if (n_zones > 0) {
        if (!zone_edges) return fail(GBD_EINVAL, "zone_edges is NULL");
        for (int z = 0; z <= n_zones; z++)
            if (!(zone_edges[z] >= 0.0) || !std::isfinite(zone_edges[z]) || (z > 0 && zone_edges[z] < zone_edges[z - 1]))
                return fail(GBD_EINVAL, "zone_edges must be finite, >= 0 and non-decreasing");
    }
    if (metrics_out && !airy) return fail(GBD_EINVAL, "metrics need the reference irradiance");
    if (airy && !metrics_out) return fail(GBD_EINVAL, "metrics_out is NULL");
    if (opts && (opts->variant < 0 || opts->variant > 5)) return fail(GBD_EINVAL, "variant must be 0 ... 5");
    int rows = 32, waves = 4;  // 32 rows: rotor form; 16 where the form resolves otherwise
    int64_t pairs = 0, n_max = 0;
    for (int32_t i = 0; i < n_inst; i++) {
        if (!bs[i] || !ps[i]) return fail(GBD_EINVAL, "instance %d has a NULL handle", i);
        if (bs[i]->ctx != ctx) return fail(GBD_EINVAL, "instance %d: the beamlets belong to another context", i);
        if (bs[i]->higher_order || bs[i]->dev.n_cut > 0)
            return fail(GBD_EINVAL, "instance %d: the batched sweep takes whole fundamental Gaussian beamlets only", i);
        pairs += bs[i]->dev.n * ((int64_t)ps[i]->g.nx * ps[i]->g.ny);
        n_max = std::max<int64_t>(n_max, bs[i]->dev.n);
    }
    if (!(opts && (opts->rows_per_lane || opts->waves))) {
        auto it = ctx->tuned.find(tune_key(kTuneBatch, GBD_MIXED, pairs, n_inst));
        if (it != ctx->tuned.end()) {
            rows = it->second.rows;
            waves = it->second.waves;
        }
    }
    if (opts) {
        if (opts->rows_per_lane) rows = opts->rows_per_lane;
        if (opts->waves) waves = opts->waves;
    }
    if (!valid_shape(rows, waves)) return fail(GBD_EINVAL, "unsupported batch rows_per_lane %d / waves %d", rows, waves);
    // work items per instance for a given tile height; the count at 16 rows
    // bounds the one at 32 (the row count is final once the form is known)
    auto tiles_of = [&](const PlaneGeom &g, int r) -> int64_t {
        return (int64_t)((g.nx + 63) / 64) * ((g.ny + waves * r - 1) / (waves * r));
    };
    int64_t total = 0, field_elems = 0, n_items = 0;
    for (int32_t i = 0; i < n_inst; i++) {
        const PlaneGeom &g = ps[i]->g;
        if (airy) {
            if (g.nx != ps[0]->g.nx || g.ny != ps[0]->g.ny)
                return fail(GBD_EINVAL, "instances sharing a reference irradiance need equal grids (instance %d)", i);
            if (airy_bytes < (int64_t)g.nx * g.ny * 4) return fail(GBD_ERANGE, "reference irradiance too small");
        }
        total += bs[i]->dev.n;
        field_elems += (int64_t)g.nx * g.ny;
        n_items += tiles_of(g, std::min(rows, 16));
    }
    if (fields_out && fields_bytes < field_elems * 8)
        return fail(GBD_ERANGE, "fields_out holds %lld bytes, %lld needed", (long long)fields_bytes,
                    (long long)(field_elems * 8));
    if (n_items > 0x3fffffff) return fail(GBD_ERANGE, "too many work items");
    if (total / kE0Chunk + n_inst > 0x3fffffff) return fail(GBD_ERANGE, "too many beamlets in the batch");
    int rc = ensure_device(ctx);
    if (rc) return rc;

    // per-beamlet setup of every instance; the status decides the mixed form.
    // The host tables pass through one pinned staging buffer:
    //   [BatchInst x n | offs x (n + 1)]   uploaded before the setup (tab1)
    //   [status x 4 | peaks x n]           read back after it
    //   [BatchEval x n | items | e0map]    uploaded before the evaluation (tab2)
    // each table part in one copy to a device buffer of the same layout.  The
    // host rewrites the buffer only once the stream has passed the previous
    // call's copies from it (stage_ev).
    const int PS = 2 + 2 * n_zones;
    BatchWork &w = ctx->batch;
    const int64_t max_chunks = total / kE0Chunk + n_inst;  // normalisation chunks, at most
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t t1_offs = al(n_inst * sizeof(BatchInst));
    const size_t t1_bytes = t1_offs + al((n_inst + 1) * sizeof(int64_t));
    const size_t rb_bytes = al((4 + (size_t)n_inst) * sizeof(uint32_t));
    const size_t t2_items = al(n_inst * sizeof(BatchEval));
    const size_t t2_e0map = t2_items + al((size_t)std::max<int64_t>(2 * n_items, 2) * sizeof(int32_t));
    const size_t t2_bytes = t2_e0map + al((size_t)max_chunks * sizeof(int32_t));
    if ((rc = grow(w.rec, (size_t)std::max<int64_t>(total, 1) * sizeof(Rec32), "batch records")) ||
        (rc = grow(w.l5, (size_t)std::max<int64_t>(total, 1) * sizeof(double), "batch records")) ||
        (airy && (rc = grow(w.e0t, (size_t)std::max<int64_t>(total, 1) * sizeof(double2), "batch normalisation"))) ||
        (airy && (rc = grow(w.e0part, (size_t)max_chunks * sizeof(double2), "batch normalisation"))) ||
        (rc = grow(w.tab1, t1_bytes, "batch table")) || (rc = grow(w.tab2, t2_bytes, "batch table")) ||
        (rc = grow(w.e0, n_inst * sizeof(double2), "batch normalisation")) ||
        (rc = grow(w.part, (size_t)std::max<int64_t>(n_items, 1) * PS * sizeof(double), "batch partials")) ||
        (rc = grow(w.metrics, (size_t)n_inst * (2 + n_zones) * sizeof(double), "batch metrics")) ||
        (rc = grow(w.flags, rb_bytes, "batch flags")))
        return rc;
    hipStream_t st = ctx->stream;
    if (!w.stage_ev) HIP_TRY(hipEventCreateWithFlags(&w.stage_ev, hipEventDisableTiming), "hipEventCreate");
    if (w.stage_pending) HIP_TRY(hipEventSynchronize(w.stage_ev), "hipEventSynchronize");
    w.stage_pending = false;
    const size_t stage_bytes = t1_bytes + rb_bytes + t2_bytes;
    if (stage_bytes > w.stage_bytes) {
        if (w.stage) (void)hipHostFree(w.stage);
        w.stage = nullptr;
        w.stage_bytes = 0;
        HIP_TRY(hipHostMalloc(&w.stage, stage_bytes, hipHostMallocDefault), "hipHostMalloc(batch staging)");
        w.stage_bytes = stage_bytes;
    }
    char *h1 = static_cast<char *>(w.stage), *hrb = h1 + t1_bytes, *h2 = hrb + rb_bytes;
    char *d1 = static_cast<char *>(w.tab1.p), *d2 = static_cast<char *>(w.tab2.p);
    BatchInst *inst = reinterpret_cast<BatchInst *>(h1);
    int64_t *offs = reinterpret_cast<int64_t *>(h1 + t1_offs);
    offs[0] = 0;
    for (int32_t i = 0; i < n_inst; i++) {
        const BeamletsDev &b = bs[i]->dev;
        offs[i + 1] = offs[i] + b.n;
        const double g0 = b.l0 / b.lam;
        inst[i].b = b;
        inst[i].pl = ps[i]->g;
        inst[i].rec_off = offs[i];
        inst[i].gturns = g0 - nearbyint(g0);
    }
    const BatchInst *dinst = reinterpret_cast<const BatchInst *>(d1);
    const int64_t *doffs = reinterpret_cast<const int64_t *>(d1 + t1_offs);
    HIP_TRY(hipMemcpyAsync(d1, h1, t1_bytes, hipMemcpyHostToDevice, st), "table upload");
    HIP_TRY(hipEventRecord(w.stage_ev, st), "hipEventRecord");
    w.stage_pending = true;
    // [0] status, [1] first bad instance, [2] queue head, [4 ...] per-instance peaks
    uint32_t *flags = static_cast<uint32_t *>(w.flags.p);
    HIP_TRY(launch_batch_clear(flags, n_inst, st), "batch clear launch");
    HIP_TRY(launch_batch_setup(dinst, doffs, n_inst, total, static_cast<Rec32 *>(w.rec.p),
                               static_cast<double *>(w.l5.p), airy ? static_cast<double2 *>(w.e0t.p) : nullptr,
                               flags, reinterpret_cast<int32_t *>(flags + 1), flags + 4, st),
            "batch setup launch");
    HIP_TRY(hipMemcpyAsync(hrb, flags, (4 + (size_t)n_inst) * sizeof(uint32_t), hipMemcpyDeviceToHost, st),
            "status copy");
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    w.stage_pending = false;
    const uint32_t *hflags = reinterpret_cast<const uint32_t *>(hrb), *peaks = hflags + 4;
    const uint32_t stat = hflags[0];
    const int32_t bad = (int32_t)hflags[1];
    if (stat & FLAG_PARALLEL) return fail(GBD_EPARALLEL, "instance %d: a base ray is parallel to the plane", bad);
    if (stat & FLAG_BRANCH) return fail(GBD_EBRANCH, "instance %d: an eigenvalue left the principal branch", bad);
    if (stat & FLAG_NONFINITE) return fail(GBD_EINVAL, "instance %d: non-finite beamlet parameters", bad);
    // an item sums all of its instance's beamlets; the separable form does so
    // in one plain FP32 sum per pixel, so it applies only while every
    // instance fits one segment of the single evaluation (kSepMaxSegLen);
    // the rotor form folds 128-beamlet tile sums and stays accurate at any N
    const int form = pick_form(GBD_MIXED, stat, opts, n_max <= kSepMaxSegLen);
    // the separable form in FP16 halves unless FP32 MFMA is requested (variant 5)
    const bool half = form == 3 && !(opts && opts->variant == 5);
    if (rows == 32 && form != 2) rows = 16;  // 32 rows is a rotor-form shape
    if (form == 2)
        HIP_TRY(launch_batch_sigma(dinst, doffs, n_inst, total, static_cast<const double *>(w.l5.p),
                                   static_cast<Rec32 *>(w.rec.p), st),
                "rotor table launch");

    // evaluation tables; the work list takes instances largest first (LPT),
    // each instance's tiles contiguous and in order
    BatchEval *ev = reinterpret_cast<BatchEval *>(h2);
    int32_t *items = reinterpret_cast<int32_t *>(h2 + t2_items);
    int32_t *e0map = reinterpret_cast<int32_t *>(h2 + t2_e0map);  // normalisation chunk -> instance
    int64_t foff = 0;
    int32_t n_chunks = 0;
    for (int32_t i = 0; i < n_inst; i++) {
        const PlaneGeom &g = ps[i]->g;
        BatchEval &e = ev[i];
        e = BatchEval();
        e.rec_off = offs[i];
        e.n = bs[i]->dev.n;
        e.nx = g.nx;
        e.ny = g.ny;
        if (form == 3) {  // separable form: the single evaluation's workgroup tiles
            Shape sh;
            sh.form = 3;
            sh.half = half;
            sh.rows = kSepTileY;
            sh.waves = kSepWavesX * kSepWavesY;
            int wgx, wgy;
            sep_wg_tile(sh, wgx, wgy);
            e.tiles_x = (g.nx + wgx - 1) / wgx;
            e.tiles_y = (g.ny + wgy - 1) / wgy;
        } else {
            e.tiles_x = (g.nx + 63) / 64;
            e.tiles_y = (g.ny + waves * rows - 1) / (waves * rows);
        }
        e.dx = g.dx;
        e.dy = g.dy;
        e.a0 = -0.5 * (g.nx - 1) * g.dx;
        e.b0 = -0.5 * (g.ny - 1) * g.dy;
        e.field_off = foff;
        foff += (int64_t)g.nx * g.ny;
        e.scale = peaks[i] ? 2 * kSepHalfExp - ((int)peaks[i] - 2048) : 0;  // as a single evaluation's setup
        e.e0_off = n_chunks;
        e.e0_chunks = (int32_t)((e.n + kE0Chunk - 1) / kE0Chunk);
        for (int32_t c = 0; c < e.e0_chunks; c++) e0map[n_chunks++] = i;
    }
    std::vector<int32_t> order(n_inst);
    for (int32_t i = 0; i < n_inst; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return ev[x].n * ((int64_t)ev[x].nx * ev[x].ny) > ev[y].n * ((int64_t)ev[y].nx * ev[y].ny);
    });
    int64_t n_it = 0;
    for (int32_t k = 0; k < n_inst; k++) {
        const int32_t i = order[k];
        ev[i].item_off = n_it;
        const int32_t tiles = ev[i].tiles_x * ev[i].tiles_y;
        for (int32_t t = 0; t < tiles; t++) {
            items[2 * n_it] = i;
            items[2 * n_it + 1] = t;
            n_it++;
        }
    }
    n_items = n_it;
    HIP_TRY(hipMemcpyAsync(d2, h2, t2_e0map + (size_t)n_chunks * sizeof(int32_t), hipMemcpyHostToDevice, st),
            "table upload");
    HIP_TRY(hipEventRecord(w.stage_ev, st), "hipEventRecord");
    w.stage_pending = true;

    BatchArgs a;
    a.inst = reinterpret_cast<const BatchEval *>(d2);
    a.n_inst = n_inst;
    a.items = reinterpret_cast<const int32_t *>(d2 + t2_items);
    a.n_items = (int32_t)n_items;
    a.rec = static_cast<const Rec32 *>(w.rec.p);
    a.e0 = static_cast<const double2 *>(w.e0.p);
    a.airy = airy;
    a.fields = static_cast<float2 *>(fields_out);
    a.part = static_cast<double *>(w.part.p);
    a.counter = flags + 2;
    a.n_zones = n_zones;
    for (int z = 0; z <= kMaxZones; z++)
        a.zone_r2[z] = (z <= n_zones && n_zones > 0) ? zone_edges[z] * zone_edges[z] : 0.0;
    if (airy)
        HIP_TRY(launch_batch_e0(a.inst, n_inst, reinterpret_cast<const int32_t *>(d2 + t2_e0map), n_chunks,
                                static_cast<const double2 *>(w.e0t.p), static_cast<double2 *>(w.e0part.p),
                                static_cast<double2 *>(w.e0.p), st),
                "normalisation launch");
    HIP_TRY(launch_batch_eval(rows, waves, form, half, ctx->cus, a, st), "batch eval launch");
    if (airy) {
        HIP_TRY(launch_batch_finalize(a.inst, n_inst, a.part, n_zones, static_cast<double *>(w.metrics.p), st),
                "finalize launch");
        HIP_TRY(hipMemcpyAsync(metrics_out, w.metrics.p, (size_t)n_inst * (2 + n_zones) * sizeof(double),
                               hipMemcpyDeviceToHost, st),
                "metrics copy");
        HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
        w.stage_pending = false;
    }
    return GBD_OK;
}

int gbd_autotune_batch(gbd_ctx_t ctx, int32_t n_inst, const gbd_beamlets_t *bs, const gbd_plane_t *ps,
                       const float *airy, int64_t airy_bytes, int32_t reps, gbd_eval_opts *best, double *best_ms) {
    if (!ctx || n_inst <= 0 || !bs || !ps || !airy) return fail(GBD_EINVAL, "bad argument");
    if (reps < 1) reps = 1;
    int64_t pairs = 0;
    for (int32_t i = 0; i < n_inst; i++) {
        if (!bs[i] || !ps[i]) return fail(GBD_EINVAL, "instance %d has a NULL handle", i);
        pairs += bs[i]->dev.n * ((int64_t)ps[i]->g.nx * ps[i]->g.ny);
    }
    std::vector<double> metrics((size_t)n_inst * 2);
    static const int rows_c[] = {2, 4, 8, 16, 32}, waves_c[] = {1, 2, 4};
    TuneVal bestv{0, 0, 100, 1e300};
    for (int ri = 0; ri < 5; ri++)
        for (int wi = 0; wi < 3; wi++) {
            gbd_eval_opts o{rows_c[ri], waves_c[wi], 0, 0};
            int rc = gbd_eval_batch(ctx, n_inst, bs, ps, airy, airy_bytes, nullptr, 0, metrics.data(), nullptr, 0, &o);
            if (rc) return rc;
            const auto t0 = std::chrono::steady_clock::now();
            for (int r = 0; r < reps; r++) {
                rc = gbd_eval_batch(ctx, n_inst, bs, ps, airy, airy_bytes, nullptr, 0, metrics.data(), nullptr, 0, &o);
                if (rc) return rc;
            }
            const double ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / reps;
            if (ms < bestv.ms) bestv = TuneVal{rows_c[ri], waves_c[wi], 100, ms};
        }
    ctx->tuned[tune_key(kTuneBatch, GBD_MIXED, pairs, n_inst)] = bestv;
    if (best) *best = gbd_eval_opts{bestv.rows, bestv.waves, 0, 0};
    if (best_ms) *best_ms = bestv.ms;
    return GBD_OK;
}

int gbd_mlp_create(gbd_ctx_t ctx, gbd_mlp_t *out, int32_t n_in, int32_t width, int32_t depth, int32_t max_batch,
                   int mode) {
    if (!ctx || !out) return fail(GBD_EINVAL, "NULL argument");
    if (n_in < 1 || n_in > 64 || width < 1 || width > 1024 || depth < 1 || depth > 8 || max_batch < 1 ||
        max_batch > 65536)
        return fail(GBD_EINVAL, "unsupported network shape (n_in %d, width %d, depth %d, max_batch %d)", n_in, width,
                    depth, max_batch);
    if (mode != GBD_MLP_FP32 && mode != GBD_MLP_BF16) return fail(GBD_EINVAL, "mode must be GBD_MLP_FP32 or GBD_MLP_BF16");
    int rc = ensure_device(ctx);
    if (rc) return rc;
    gbd_mlp_s *m = new (std::nothrow) gbd_mlp_s();
    if (!m) return fail(GBD_ENOMEM, "host allocation failed");
    m->ctx = ctx;
    m->n_in = n_in;
    m->width = width;
    m->depth = depth;
    m->max_batch = max_batch;
    m->mode = mode;
    int64_t k = 0, prev = n_in;
    for (int l = 0; l <= depth; l++) {
        const int64_t o = (l < depth) ? width : 1;
        m->woff.push_back(k);
        k += o * prev;
        m->boff.push_back(k);
        k += o;
        prev = width;
    }
    m->P = k;
    const int64_t act = (int64_t)depth * max_batch * width, bw = (int64_t)max_batch * width;
    const int64_t total = 4 * m->P + 2 * act + 2 * bw + (int64_t)max_batch * (n_in + 3) + 1;
    hipError_t e = hipMalloc(&m->mem, (size_t)total * sizeof(float));
    if (e != hipSuccess) {
        delete m;
        return hip_fail(e, "hipMalloc(mlp)");
    }
    float *q = m->mem;
    m->params = q; q += m->P;
    m->grads = q; q += m->P;
    m->m = q; q += m->P;
    m->v = q; q += m->P;
    m->Z = q; q += act;
    m->H = q; q += act;
    m->dz0 = q; q += bw;
    m->dz1 = q; q += bw;
    m->xb = q; q += (int64_t)max_batch * n_in;
    m->yb = q; q += max_batch;
    m->yhat = q; q += max_batch;
    m->g = q; q += max_batch;
    m->loss = q;
    e = hipMemsetAsync(m->mem, 0, (size_t)total * sizeof(float), ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(m->mem);
        delete m;
        return hip_fail(e, "mlp init");
    }
    *out = m;
    return GBD_OK;
}

void gbd_mlp_free(gbd_mlp_t m) {
    if (!m) return;
    if (m->mem) (void)hipFree(m->mem);
    delete m;
}

int64_t gbd_mlp_num_params(gbd_mlp_t m) { return m ? m->P : (int64_t)fail(GBD_EINVAL, "NULL argument"); }

int gbd_mlp_set_params(gbd_mlp_t m, const float *params, int64_t n) {
    if (!m || !params) return fail(GBD_EINVAL, "NULL argument");
    if (n != m->P) return fail(GBD_EINVAL, "expected %lld parameters, got %lld", (long long)m->P, (long long)n);
    for (int64_t i = 0; i < n; i++)
        if (!std::isfinite(params[i])) return fail(GBD_EINVAL, "non-finite parameter %lld", (long long)i);
    int rc = ensure_device(m->ctx);
    if (rc) return rc;
    hipStream_t st = m->ctx->stream;
    HIP_TRY(hipMemcpyAsync(m->params, params, n * sizeof(float), hipMemcpyHostToDevice, st), "parameter upload");
    HIP_TRY(hipMemsetAsync(m->m, 0, 2 * n * sizeof(float), st), "optimiser reset");  // m and v are adjacent
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    m->step = 0;
    return GBD_OK;
}

static int mlp_copy_out(gbd_mlp_t m, const float *src, float *dst, int64_t n) {
    if (!m || !dst) return fail(GBD_EINVAL, "NULL argument");
    if (n != m->P) return fail(GBD_EINVAL, "expected %lld values, got %lld", (long long)m->P, (long long)n);
    int rc = ensure_device(m->ctx);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyDeviceToHost, m->ctx->stream), "download");
    HIP_TRY(hipStreamSynchronize(m->ctx->stream), "hipStreamSynchronize");
    return GBD_OK;
}

int gbd_mlp_get_params(gbd_mlp_t m, float *params, int64_t n) { return mlp_copy_out(m, m ? m->params : nullptr, params, n); }
int gbd_mlp_get_grads(gbd_mlp_t m, float *grads, int64_t n) { return mlp_copy_out(m, m ? m->grads : nullptr, grads, n); }

// forward over the batch already gathered into m->xb; leaves Z, H, yhat
static int mlp_forward_impl(gbd_mlp_t m, int B) {
    hipStream_t st = m->ctx->stream;
    const int W = m->width;
    const float *in = m->xb;
    int fan = m->n_in;
    for (int l = 0; l < m->depth; l++) {
        MlpGemm g{};
        g.M = B;
        g.N = W;
        g.K = fan;
        g.A = in;
        g.sam = fan;
        g.sak = 1;
        g.B = m->params + m->woff[l];
        g.sbk = 1;
        g.sbn = fan;
        g.bias = m->params + m->boff[l];
        g.C = m->Z + (int64_t)l * m->max_batch * W;
        g.H = m->H + (int64_t)l * m->max_batch * W;
        g.epi = 0;
        HIP_TRY(launch_mlp_gemm(m->mode == GBD_MLP_BF16, g, st), "mlp forward launch");
        in = g.H;
        fan = W;
    }
    HIP_TRY(launch_mlp_head_forward(in, m->params + m->woff[m->depth], m->params + m->boff[m->depth], B, W, m->yhat, st),
            "mlp head launch");
    return GBD_OK;
}

int gbd_mlp_forward(gbd_mlp_t m, const float *x, const int32_t *rows, int32_t batch, float *y) {
    if (!m || !x || !y) return fail(GBD_EINVAL, "NULL argument");
    if (batch < 0 || batch > m->max_batch) return fail(GBD_ERANGE, "batch %d outside [0, %d]", batch, m->max_batch);
    if (batch == 0) return GBD_OK;
    int rc = ensure_device(m->ctx);
    if (rc) return rc;
    hipStream_t st = m->ctx->stream;
    HIP_TRY(launch_mlp_gather(x, nullptr, rows, batch, m->n_in, m->xb, nullptr, st), "mlp gather launch");
    rc = mlp_forward_impl(m, batch);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(y, m->yhat, batch * sizeof(float), hipMemcpyDeviceToDevice, st), "mlp output copy");
    return GBD_OK;
}

int gbd_mlp_backward(gbd_mlp_t m, const float *x, const float *target, const int32_t *rows, int32_t batch,
                     float *loss_dev) {
    if (!m || !x || !target) return fail(GBD_EINVAL, "NULL argument");
    if (batch < 1 || batch > m->max_batch) return fail(GBD_ERANGE, "batch %d outside [1, %d]", batch, m->max_batch);
    int rc = ensure_device(m->ctx);
    if (rc) return rc;
    hipStream_t st = m->ctx->stream;
    const int W = m->width, B = batch, D = m->depth;
    HIP_TRY(launch_mlp_gather(x, target, rows, B, m->n_in, m->xb, m->yb, st), "mlp gather launch");
    rc = mlp_forward_impl(m, B);
    if (rc) return rc;
    const int64_t stride = (int64_t)m->max_batch * W;
    const float *Hlast = m->H + (int64_t)(D - 1) * stride;
    const float *Zlast = m->Z + (int64_t)(D - 1) * stride;
    // head: loss, its gradient, head weights' gradient, dZ of the last hidden layer
    HIP_TRY(launch_mlp_head_backward(m->yhat, m->yb, Hlast, m->params + m->woff[D], Zlast, B, W, m->g, m->loss,
                                     m->grads + m->woff[D], m->dz0, st),
            "mlp head backward launch");
    float *dz = m->dz0, *dz_next = m->dz1;
    for (int l = D - 1; l >= 0; l--) {
        const int fan = (l == 0) ? m->n_in : W;
        const float *Hprev = (l == 0) ? m->xb : m->H + (int64_t)(l - 1) * stride;
        // dW_l[o][i] = sum_b dZ[b][o] Hprev[b][i]
        MlpGemm gw{};
        gw.M = W;
        gw.N = fan;
        gw.K = B;
        gw.A = dz;
        gw.sam = 1;
        gw.sak = W;
        gw.B = Hprev;
        gw.sbk = fan;
        gw.sbn = 1;
        gw.C = m->grads + m->woff[l];
        gw.epi = 2;
        HIP_TRY(launch_mlp_gemm(m->mode == GBD_MLP_BF16, gw, st), "mlp weight-gradient launch");
        HIP_TRY(launch_mlp_colsum(dz, B, W, m->grads + m->boff[l], st), "mlp bias-gradient launch");
        if (l > 0) {
            // dZ_{l-1}[b][i] = (sum_o dZ[b][o] W_l[o][i]) SiLU'(Z_{l-1}[b][i])
            MlpGemm gh{};
            gh.M = B;
            gh.N = W;
            gh.K = W;
            gh.A = dz;
            gh.sam = W;
            gh.sak = 1;
            gh.B = m->params + m->woff[l];
            gh.sbk = W;
            gh.sbn = 1;
            gh.zmul = m->Z + (int64_t)(l - 1) * stride;
            gh.C = dz_next;
            gh.epi = 1;
            HIP_TRY(launch_mlp_gemm(m->mode == GBD_MLP_BF16, gh, st), "mlp backward launch");
            std::swap(dz, dz_next);
        }
    }
    if (loss_dev) HIP_TRY(hipMemcpyAsync(loss_dev, m->loss, sizeof(float), hipMemcpyDeviceToDevice, st), "loss copy");
    return GBD_OK;
}

static bool adamw_args_ok(float lr, float beta1, float beta2, float eps, float weight_decay) {
    return lr >= 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f &&
           weight_decay >= 0.0f;
}

int gbd_mlp_adamw(gbd_mlp_t m, float lr, float beta1, float beta2, float eps, float weight_decay) {
    if (!m) return fail(GBD_EINVAL, "NULL argument");
    if (!adamw_args_ok(lr, beta1, beta2, eps, weight_decay)) return fail(GBD_EINVAL, "invalid AdamW hyper-parameters");
    int rc = ensure_device(m->ctx);
    if (rc) return rc;
    m->step++;
    const float c1 = 1.0f - powf(beta1, (float)m->step), c2 = 1.0f - powf(beta2, (float)m->step);
    HIP_TRY(launch_mlp_adamw(m->params, m->grads, m->m, m->v, m->P, lr, beta1, beta2, eps, weight_decay, c1, c2,
                             m->ctx->stream),
            "adamw launch");
    return GBD_OK;
}

int gbd_mlp_train(gbd_mlp_t m, const float *x, const float *target, const int32_t *rows, int32_t steps, int32_t batch,
                  const float *lr_host, float beta1, float beta2, float eps, float weight_decay, float *loss_sum_dev) {
    if (!m || !x || !target || !rows || !lr_host) return fail(GBD_EINVAL, "NULL argument");
    if (steps < 0) return fail(GBD_EINVAL, "negative step count %d", steps);
    if (batch < 1 || batch > m->max_batch) return fail(GBD_ERANGE, "batch %d outside [1, %d]", batch, m->max_batch);
    // every step's arguments are checked before the first one runs
    for (int32_t s = 0; s < steps; s++)
        if (!adamw_args_ok(lr_host[s], beta1, beta2, eps, weight_decay))
            return fail(GBD_EINVAL, "invalid AdamW hyper-parameters (step %d)", s);
    for (int32_t s = 0; s < steps; s++) {
        int rc = gbd_mlp_backward(m, x, target, rows + (int64_t)s * batch, batch, nullptr);
        if (rc) return rc;
        if (loss_sum_dev) HIP_TRY(launch_mlp_accum(loss_sum_dev, m->loss, m->ctx->stream), "loss sum launch");
        rc = gbd_mlp_adamw(m, lr_host[s], beta1, beta2, eps, weight_decay);
        if (rc) return rc;
    }
    return GBD_OK;
}

}  // extern "C"
