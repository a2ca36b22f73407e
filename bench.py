#!/usr/bin/env python3
"""Benchmark of the plane-evaluation GBD hot path on one MI355X.

One step = one gbd_eval call: the per-beamlet FP64 setup (complex-curvature
law, eigenvalue-branch amplitude, base ray, hit point, phasor coefficients;
with its status check) followed by the N x M mixed-precision evaluation of
the coherent field, on inputs already resident in HBM.  Workload: 51,468 beamlets (256 across a
10 mm f/10 pupil, OF 1.7) onto a 512 x 512 focal-plane detector spanning
+-20 lambda F.  value = N * M / (time per step), beamlet-pixel evaluations/s.

The mixed evaluation takes the library's automatic form: on this workload
(a rotationally symmetric system on a plane normal to the axis, so no
beamlet's phasor has a cross term) the separable matrix form on FP16 MFMA
with every factor split into FP16 hi and lo halves, whose roofline is the
FP16 MFMA peak; the same form on FP32 MFMA (separable_fp32) and the rotor
form, which any plane with cross terms gets (general_form, with its
instruction-mix roofline at nominal and at measured issue rates), are timed
on the same workload beside it.

Also reported: the FP64 form on the same workload (and the mixed/FP64
speed-up), the dominant kernel's live HIP-event duration, point evaluation,
the 441-instance sweep, the ray-traced telescope, higher-order
(Hermite-Gaussian) and truncated (rim-cut) beamlets on the same grid, and
the FP64 CPU oracle timed on a bounded pixel sample (which also gives the mixed form's error against
the oracle there).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

METRIC = "beamlet·pixel evals/s (FP32+FP64-phase vs FP64) at ≤1e-5 rel field err"

# Instruction-mix roofline of the mixed evaluation kernel.  Issue rates in
# lanes per CU per clock from the chip's unit counts: FP64 64 (78.6 TFLOP/s
# FP64 FMA), FP32 128 (157.3 TFLOP/s FP32: reached without packed
# instructions by the two-operand v_fmac_f32 / v_mul_f32, which the
# issue-rate probe measures at 102-107 lanes per CU per nominal clock; its
# three-operand v_fma_f32 loop reaches 58), transcendental 32 (half the FP64 rate;
# probe: 28-29).  The benchmark prices each VALU form at these rates and at
# the probe's measured ones.  Instructions per beamlet-pixel pair for R rows
# per lane (per-lane-beamlet work amortised over the R pixels it serves):
#   stepped form: per pixel 2 transcendental (sin, cos in revolutions) and
#     6 FP32 (2 phase-step FMA, 2 amplitude-step multiply, 2 accumulate FMA);
#     per lane-beamlet 15 FP64 (offsets, phase quadratic, row slope,
#     reductions, conversions), 7 further FP32 (log2-amplitude anchor and
#     ratio; 4 of the per-pixel steps are not needed at the column's ends)
#     and 2 exp2
#   direct form: per pixel 4 FP64 (2 FMA, fract, cvt), 5 FP32 (3 amplitude,
#     2 accumulate), 3 transcendental; per lane-beamlet 10 FP64 and 5 FP32
CUS, CLOCK_HZ = 256, 2.4e9
RATE = {"fp64": 64, "fp32": 128, "trans": 32}


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE (x2.0)
# and WRITE_SIZE (x1.0) runs, scale factors from a plain 256 MiB copy; valid
# only for the kernel and launch they were taken on (else traffic is null).
TRAFFIC = {("airy256_512", 64, 8, 32, 4): (5742.0 * 2.0 + 65536.0 * 1.0) * 1024}


def instruction_mix(rows, variant, hg=False):
    """Instructions per beamlet-pixel pair of the mixed kernel's inner loop
    (per lane and beamlet: an FP64 anchor, then R rows), counted in the
    compiled gfx950 code.  hg: higher-order beamlets (rotor form: the
    Hermite-Gaussian factor's degree-4 row polynomial, 159 FP32 per lane and
    beamlet, then Horner's rule and one more complex product, 12 FP32 per row)."""
    R = float(rows)
    if variant == 3 and hg:
        return {"fp64": 15 / R, "fp32": (20 * R + 159) / R, "trans": 7 / R}
    if variant == 3:  # rotor: 8 FP32 per further row, 7 transcendentals per lane and beamlet
        return {"fp64": 15 / R, "fp32": (8 * R + 13) / R, "trans": 7 / R}
    if variant == 2:  # stepped: sin + cos per pixel
        return {"fp64": 15 / R, "fp32": (6 * R + 7) / R, "trans": (2 * R + 2) / R}
    return {"fp64": (4 * R + 10) / R, "fp32": (5 * R + 5) / R, "trans": 3.0}


def roofline_peak(rows, variant, hg=False, rate=None):
    """Instruction-mix roofline at the nominal issue rates (RATE) or at the
    given measured ones."""
    rate = rate or RATE
    mix = instruction_mix(rows, variant, hg)
    cycles = sum(n / rate[k] for k, n in mix.items())
    return CUS * CLOCK_HZ / cycles, cycles, mix


# Separable (matrix) form: the contraction E = V^T U over beamlets.  Gauss's
# three-product form of the complex product is the algorithm: 3 real
# multiply-adds (6 flops) per beamlet-pixel pair on the matrix cores, plus
# 2 additions per factor (O(N (nx + ny)), not per pair) and 3 per pixel.
# frac = those 6 flops per pair over the FP32 MFMA peak (the MFMA busy
# fraction); the rate of the textbook complex multiply-add (4 real
# multiply-adds, 8 flops) is reported beside it, not as a fraction of peak.
MFMA_FP32_TFLOPS = 157.3
SEP_FLOPS_PER_PAIR = 6.0
SEP_COMPLEX_MADD_FLOPS = 8.0
# the FP64 separable form multiplies in four real FP64 MFMA products
SEP64_FLOPS_PER_PAIR = 8.0
# FP16 halves form (variant 4 for fundamental beamlets): each factor as FP16
# hi + lo, the hi hi, hi lo and lo hi products of the four real products of
# the complex multiply: 12 FP16 multiply-adds (24 flops) per pair on the
# matrix cores, against the FP16 MFMA peak
MFMA_FP16_TFLOPS = 2500.0
SEPH_FLOPS_PER_PAIR = 24.0
# per lane and pass between barriers (16 beamlets x 64 x 32 pixels of one
# wavefront), counted in the compiled loop: 40 FP64, 56 FP32, 24
# transcendental and 62 other VALU instructions (the factors shared by 8
# wavefronts), 96 MFMA 16x16x4
SEP_VALU_PER_PAIR = {"fp64": 40 / 512, "fp32": 56 / 512, "trans": 24 / 512, "other": 62 / 512,
                     "mfma_16x16x4": 96 / 32768}


PROBE_CLASSES = [("fp32_fma", 0, 128), ("fp64_fma", 1, 128), ("sin_f32", 2, 32), ("exp_f32", 3, 32),
                 ("mfma_f32_16x16x4", 4, 4096), ("mfma_f16_16x16x32", 5, 4096), ("mfma_f64_16x16x4", 6, 2048),
                 ("fp32_fmac", 7, 128), ("fp32_mul", 8, 128), ("mfma_f16_16x16x32_with_fp32_fma", 9, 4096)]
MFMA_FLOPS_PER_INSTR = {"mfma_f32_16x16x4": 2048, "mfma_f16_16x16x32": 16384, "mfma_f64_16x16x4": 2048,
                        "mfma_f16_16x16x32_with_fp32_fma": 16384}


def issue_rates(ctx):
    """Measured issue rates (gbd_issue_probe): VALU classes in lane-
    instructions per CU per clock, MFMA classes in TFLOP/s and instructions
    per CU per clock, at the nominal 2.4 GHz clock on 256 CUs."""
    import paper_2404_12454_amd as gbd
    out = {}
    for name, cls, iters in PROBE_CLASSES:
        ms, n = gbd.gbd_issue_probe(ctx, cls, iters)
        if ms < 4.0:  # lengthen to ~5 ms so launch overhead and ramp do not count
            iters = int(iters * min(5.0 / max(ms, 1e-3), 4096.0))
            ms, n = gbd.gbd_issue_probe(ctx, cls, iters)
        per_cu_clk = n / (ms * 1e-3) / (CUS * CLOCK_HZ)
        if name.startswith("mfma"):
            out[name] = {"tflops": n * MFMA_FLOPS_PER_INSTR[name] / (ms * 1e-3) / 1e12,
                         "instr_per_cu_clk": per_cu_clk, "ms": ms, "iters": iters}
        else:
            out[name] = {"lanes_per_cu_clk": 64.0 * per_cu_clk, "ms": ms, "iters": iters}
    # per round: class 5 issues 4 MFMA, class 0 16 FMA, class 9 both; the
    # share of the shorter class's time that class 9 hides (0: the SIMD
    # issues them one after the other, 1: fully overlapped)
    t = {k: out[k]["ms"] / out[k]["iters"] for k in ("mfma_f16_16x16x32", "fp32_fma", "mfma_f16_16x16x32_with_fp32_fma")}
    t5, t0, t9 = t["mfma_f16_16x16x32"], t["fp32_fma"], t["mfma_f16_16x16x32_with_fp32_fma"]
    out["mfma_valu_overlap"] = {"ms_per_round_mfma": t5, "ms_per_round_fma": t0, "ms_per_round_both": t9,
                                "hidden_share": (t5 + t0 - t9) / min(t5, t0)}
    return out


def measured_rate(rates):
    """Issue rates per CU per clock in the roofline's classes from the probe:
    FP32 at the slower of the two-operand multiply and multiply-add (the
    forms the VALU kernels' inner loops use mostly; the probe's
    three-operand v_fma_f32 loop issues at about half their rate), the
    transcendental class at the slower of sin and exp."""
    if not rates:
        return None
    return {"fp64": rates["fp64_fma"]["lanes_per_cu_clk"],
            "fp32": min(rates["fp32_fmac"]["lanes_per_cu_clk"], rates["fp32_mul"]["lanes_per_cu_clk"]),
            "trans": min(rates["sin_f32"]["lanes_per_cu_clk"], rates["exp_f32"]["lanes_per_cu_clk"])}


def roofline(shape, N, M, kernel_ms, hg=False):
    if shape["variant"] == 4:
        achieved = SEPH_FLOPS_PER_PAIR * N * M / (kernel_ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP16_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / MFMA_FP16_TFLOPS, "kernel": "eval_seph_kernel", "kernel_ms": kernel_ms,
                "flops_per_pair": SEPH_FLOPS_PER_PAIR,
                "complex_madd_equiv_tflops": SEP_COMPLEX_MADD_FLOPS * N * M / (kernel_ms * 1e-3) / 1e12}
    if shape["variant"] == 5:
        achieved = SEP_FLOPS_PER_PAIR * N * M / (kernel_ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / MFMA_FP32_TFLOPS, "kernel": "eval_sep_kernel", "kernel_ms": kernel_ms,
                "flops_per_pair": SEP_FLOPS_PER_PAIR,
                "complex_madd_equiv_tflops": SEP_COMPLEX_MADD_FLOPS * N * M / (kernel_ms * 1e-3) / 1e12,
                "instructions_per_pair": SEP_VALU_PER_PAIR}
    achieved = N * M / (kernel_ms * 1e-3)
    peak, cycles, mix = roofline_peak(shape["rows_per_lane"], shape["variant"], hg)
    r = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "evals/s", "frac": achieved / peak,
         "kernel": "eval_mixed_kernel", "kernel_ms": kernel_ms, "cu_cycles_per_pair": cycles,
         "instructions_per_pair": mix}
    if MEASURED_RATE:
        peak_m = roofline_peak(shape["rows_per_lane"], shape["variant"], hg, MEASURED_RATE)[0]
        r.update({"peak_at_measured_rates": peak_m, "frac_at_measured_rates": achieved / peak_m})
    return r


MEASURED_RATE = None  # filled by main() from the issue-rate probe


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the GPU's clocks settle over the first ~15 launches of the evaluation
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="airy256_512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 441-instance batched sweep figure")
    ap.add_argument("--no-point", action="store_true", help="skip the point-evaluation comparison")
    ap.add_argument("--no-telescope", action="store_true", help="skip the ray-traced telescope leg")
    ap.add_argument("--no-hermite", action="store_true", help="skip the higher-order beamlet leg")
    ap.add_argument("--no-truncated", action="store_true", help="skip the truncated-beamlet leg")
    ap.add_argument("--no-aberrated", action="store_true",
                    help="skip the aberrated tilted-plane leg (zern128_1024, the general form)")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--issue-rates-only", action="store_true",
                    help="run only the issue-rate probe and print its rates (for profiling the probe)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device copy (a known-size kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU; multi-GPU runs are not part of it "
              "(the path would shard by pixel rows: every GPU holds all beamlet records and evaluates "
              "its own band of rows, with no reduction)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2404_12454_amd as gbd
    from paper_2404_12454_amd import scenes

    if not os.path.exists(gbd.library_path()):
        from paper_2404_12454_amd import build
        build.build()

    if args.issue_rates_only:
        print(json.dumps({"issue_rates": issue_rates(gbd.Context(0))}), flush=True)
        return
    sc = scenes.config(args.workload)
    N, M = sc.n, sc.plane.npix
    ctx = gbd.Context(0)
    stream = torch.cuda.current_stream()
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, N)
    out = torch.empty((sc.plane.ny, sc.plane.nx), dtype=torch.complex64, device="cuda")
    out64 = torch.empty((sc.plane.ny, sc.plane.nx), dtype=torch.complex128, device="cuda")

    def step(precision, o, ev=None):
        plan.setup(b, p)                      # setup kernel + status sync
        if ev is not None:
            ev[0].record(stream)
        plan.eval(precision, o)
        if ev is not None:
            ev[1].record(stream)

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    global MEASURED_RATE
    rates = issue_rates(ctx)
    MEASURED_RATE = measured_rate(rates)
    for _ in range(args.warmup):
        step(gbd.GBD_MIXED, out)
    torch.cuda.synchronize()

    # the timed steps: one gbd_eval call each (setup, status, evaluation in
    # one library call on the context's own plan)
    for _ in range(2):
        gbd.gbd_eval(ctx, b, p, gbd.GBD_MIXED, out=out)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    ctx.kernel_times()                        # drop pairs from earlier calls
    torch.cuda.synchronize()
    ctx.set_kernel_timing(True)               # HIP events around each step's N x M kernel
    w0 = time.perf_counter()
    t_start.record(stream)
    for i in range(args.steps):
        gbd.gbd_eval(ctx, b, p, gbd.GBD_MIXED, out=out)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ctx.set_kernel_timing(False)
    kernel_ms_each = ctx.kernel_times()
    if len(kernel_ms_each) != args.steps:
        raise RuntimeError(f"{len(kernel_ms_each)} kernel timings for {args.steps} steps")
    kernel_ms = float(np.mean(kernel_ms_each))
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    value = N * M / (ms_step * 1e-3)
    # the evaluation call alone (kernel and segment reduction; HIP events
    # around plan.eval in untimed steps through the plan): the reference the
    # other legs' speed-ups and cost ratios use, measured as they are
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for i in range(args.steps):
        step(gbd.GBD_MIXED, out, evs[i])
    torch.cuda.synchronize()
    eval_ms_mean = float(np.mean([a.elapsed_time(z) for a, z in evs]))

    # FP64 form on the same workload
    step(gbd.GBD_FP64, out64)
    torch.cuda.synchronize()
    ev64 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.fp64_steps)]
    for i in range(args.fp64_steps):
        step(gbd.GBD_FP64, out64, ev64[i])
    torch.cuda.synchronize()
    eval64_ms = float(np.mean([a.elapsed_time(z) for a, z in ev64]))
    shape64 = plan.shape(gbd.GBD_FP64)
    E32 = out.cpu().numpy().astype(np.complex128)
    E64 = out64.cpu().numpy()
    mixed_vs_fp64 = float(np.linalg.norm(E32 - E64) / np.linalg.norm(E64))

    shape = plan.shape(gbd.GBD_MIXED)
    roof = roofline(shape, N, M, kernel_ms)
    # the rest of a step: the setup kernel, its status copy and the host's
    # round trip before the evaluation, and the segment reduction
    roof["step_rest_ms"] = ms_step - kernel_ms
    roof["traffic"] = TRAFFIC.get((args.workload, shape["rows_per_lane"], shape["waves"], shape["segments"],
                                   shape["variant"]))
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {N} beamlets x {sc.plane.nx}x{sc.plane.ny} px, f/10, "
                               f"+-{sc.meta.get('half_span_lamF', 0):g} lamF, mixed precision",
                   "n_beamlets": N, "n_pixels": M, "launch": shape},
        "roofline": roof,
        "eval_call_ms": eval_ms_mean,
        "fp64": fp64_record(shape64, N, M, eval64_ms, eval_ms_mean),
        "err_mixed_vs_fp64_full_grid": mixed_vs_fp64,
        "wall_s_timed": wall,
        "issue_rates": rates,
    }

    if shape["variant"] in (4, 5):
        rec["general_form"] = general_form(plan, N, M, out, stream)
    if shape["variant"] == 4:
        rec["separable_fp32"] = general_form(plan, N, M, out, stream, variant=5)
    if not args.no_aberrated and args.workload != "zern128_1024":
        rec["aberrated"] = aberrated(ctx, stream)
    if not args.no_point:
        rec["point_eval"] = point_eval(ctx, b, p, N * M, eval_ms_mean, eval64_ms)
    if not args.no_sweep:
        rec["sweep"] = sweep(ctx)
    if not args.no_telescope:
        rec["telescope"] = telescope(ctx, stream)
    if not args.no_hermite:
        rec["hermite"] = hermite(ctx, stream, eval_ms_mean)
    if not args.no_truncated:
        rec["truncated"] = truncated(ctx, stream, eval_ms_mean)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(sc, E32, E64)
    print(json.dumps(rec), flush=True)


MFMA_FP64_TFLOPS = 78.6


def fp64_record(shape, N, M, ms, mixed_ms):
    """The FP64 form's figure and roofline: the separable form (the automatic
    one without cross terms; four real FP64 MFMA products per pair) against
    the FP64 MFMA peak at 8 flops per pair;
    the rotor form (the automatic one otherwise, on well-sampled grids)
    against its instruction mix: per further row two complex FP64
    multiply-adds (8 FP64), per lane and beamlet 107 FP64 (anchor exp and
    sine/cosine, rho, 1/rho) and 36 other VALU instructions, counted in the
    compiled loop at 32 rows."""
    r = {"value": N * M / (ms * 1e-3), "eval_ms": ms, "launch": shape, "speedup_mixed_over_fp64": ms / mixed_ms}
    if shape["variant"] == 4:
        achieved = SEP64_FLOPS_PER_PAIR * N * M / (ms * 1e-3) / 1e12
        r.update({"roofline_bound": "mfma", "achieved_tflops": achieved, "roofline_peak_tflops": MFMA_FP64_TFLOPS,
                  "roofline_frac": achieved / MFMA_FP64_TFLOPS})
    if shape["variant"] == 3:
        R = float(shape["rows_per_lane"])
        mix = {"fp64": (8 * R + 107) / R, "fp32": 36 / R}
        peak = CUS * CLOCK_HZ / sum(n / RATE[k] for k, n in mix.items())
        r.update({"roofline_peak": peak, "roofline_frac": r["value"] / peak, "instructions_per_pair": mix})
    return r


def general_form(plan, N, M, out, stream, reps=20, variant=3):
    """The same workload through another form: by default the one that needs
    no separability (rotor, variant 3), what any plane with cross terms
    (tilted, astigmatic) gets; variant 5, the separable form on FP32 MFMA."""
    import numpy as np
    import torch
    import paper_2404_12454_amd as gbd
    o = dict(variant=variant)
    for _ in range(reps):
        plan.eval(gbd.GBD_MIXED, out, opts=o)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, z in evs:
        a.record(stream)
        plan.eval(gbd.GBD_MIXED, out, opts=o)
        z.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(z) for a, z in evs]))
    shape = plan.shape(gbd.GBD_MIXED, opts=o)
    r = roofline(shape, N, M, ms)
    g = {"launch": shape, "eval_ms": ms, "evals_per_s": N * M / (ms * 1e-3), "roofline_frac": r["frac"],
         "roofline_peak": r["peak"], "roofline_bound": r["bound"], "roofline_unit": r["unit"]}
    if "peak_at_measured_rates" in r:
        g.update({"roofline_peak_at_measured_rates": r["peak_at_measured_rates"],
                  "roofline_frac_at_measured_rates": r["frac_at_measured_rates"]})
    return g


def aberrated(ctx, stream, reps=10, reps64=3, oracle_stride=8):
    """The aberrated, tilted-plane workload (zern128_1024: f/4, 12,892
    beamlets with seeded Zernike Z4-Z11 terms, a field angle, the plane tilted
    10 degrees, 1024 x 1024 pixels): cross terms everywhere, so both
    precisions take their general (rotor) forms.  Both fields' error against
    the FP64 oracle on every 8th pixel row (131,072 pixels, ~3 s on 16 host
    threads); oracle_stride 0 skips it."""
    import numpy as np
    import torch
    import paper_2404_12454_amd as gbd
    from paper_2404_12454_amd import scenes
    sc = scenes.config("zern128_1024")
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    N, M = sc.n, sc.plane.npix

    def timed(prec, out, warm, n):
        for _ in range(warm):
            plan.eval(prec, out)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, z in evs:
            a.record(stream)
            plan.eval(prec, out)
            z.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(z) for a, z in evs]))

    out = torch.empty((sc.plane.ny, sc.plane.nx), dtype=torch.complex64, device="cuda")
    out64 = torch.empty((sc.plane.ny, sc.plane.nx), dtype=torch.complex128, device="cuda")
    ms = timed(gbd.GBD_MIXED, out, reps, reps)
    ms64 = timed(gbd.GBD_FP64, out64, 1, reps64)
    E32 = out.cpu().numpy().astype(np.complex128)
    E64 = out64.cpu().numpy()
    shape, shape64 = plan.shape(gbd.GBD_MIXED), plan.shape(gbd.GBD_FP64)
    r = roofline(shape, N, M, ms)
    r64 = fp64_record(shape64, N, M, ms64, ms)
    rec = {"beamlets": N, "npix": [sc.plane.nx, sc.plane.ny], "launch": shape, "eval_ms": ms,
           "evals_per_s": N * M / (ms * 1e-3), "roofline_frac": r["frac"], "roofline_peak": r["peak"],
           "fp64": {"launch": shape64, "eval_ms": ms64, "evals_per_s": N * M / (ms64 * 1e-3),
                    "roofline_frac": r64.get("roofline_frac")},
           "err_mixed_vs_fp64_full_grid": float(np.linalg.norm(E32 - E64) / np.linalg.norm(E64))}
    if "peak_at_measured_rates" in r:
        rec.update({"roofline_peak_at_measured_rates": r["peak_at_measured_rates"],
                    "roofline_frac_at_measured_rates": r["frac_at_measured_rates"]})
    if oracle_stride:
        import oracle
        rows = np.arange(0, sc.plane.ny, oracle_stride)
        iy, ix = np.meshgrid(rows, np.arange(sc.plane.nx), indexing="ij")
        ix, iy = ix.ravel().astype(np.int32), iy.ravel().astype(np.int32)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        ref = oracle.eval_field(sc, pixels=(ix, iy), threads=threads)
        nref = np.linalg.norm(ref)
        rec.update({"oracle_sample": f"every {oracle_stride}th pixel row ({rows.size} rows, {ix.size} px)",
                    "err_mixed_vs_oracle": float(np.linalg.norm(E32[iy, ix] - ref) / nref),
                    "err_fp64_vs_oracle": float(np.linalg.norm(E64[iy, ix] - ref) / nref)})
    return rec


def point_eval(ctx, b, p, pairs, mixed_ms, fp64_ms, reps=2):
    """Point evaluation (every pixel re-propagates every beamlet to its own
    position, FP64) on the same workload: the per-point algorithm the plane
    evaluation replaces, timed on the same GPU."""
    import numpy as np
    import torch
    import paper_2404_12454_amd as gbd
    out = gbd.gbd_eval_point(ctx, b, p)
    t = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        gbd.gbd_eval_point(ctx, b, p, out=out)
        e1.record()
        torch.cuda.synchronize()
        t.append(e0.elapsed_time(e1))
    ms = float(np.median(t))
    return {"ms": ms, "evals_per_s": pairs / (ms * 1e-3), "plane_fp64_speedup": ms / fp64_ms,
            "plane_mixed_speedup": ms / mixed_ms}


def sweep(ctx, reps=3):
    """The parameter sweep in one persistent launch: 441 (OF, q, beamlets
    across) instances, 256 x 256 pixels over +-8 lambda F each, RMS and peak
    error against the Airy pattern per instance (host wall time per call,
    setup and metric read-back included)."""
    import numpy as np
    import torch
    import paper_2404_12454_amd as gbd
    from paper_2404_12454_amd import scenes
    insts = [scenes.airy_scene(na, OF=of, q=q, npix=256, half_span_lamF=8.0) for of, q, na in scenes.sweep_grid()]
    bs = [gbd.beamlets_from_scene(ctx, s) for s in insts]
    ps = [gbd.plane_from_scene(ctx, s) for s in insts]
    m = insts[0].meta
    airy = gbd.gbd_airy(ctx, ps[0], m["D"], m["f"], insts[0].lam)
    metrics, _ = gbd.gbd_eval_batch(ctx, bs, ps, airy=airy)
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        metrics, _ = gbd.gbd_eval_batch(ctx, bs, ps, airy=airy)
        t.append(time.perf_counter() - t0)
    dt = float(np.median(t))
    pairs = sum(s.n for s in insts) * 256 * 256
    best = int(np.argmin(metrics[:, 0]))
    of, q, na = scenes.sweep_grid()[best]
    return {"instances": len(insts), "pairs": pairs, "ms": dt * 1e3, "evals_per_s": pairs / dt,
            "best": {"OF": of, "q": q, "n_across": na, "rms": float(metrics[best, 0]),
                     "peak": float(metrics[best, 1])}}


def telescope(ctx, stream, n_across=128, npix=512, reps=5):
    """The Appendix B telescope with ray-traced inputs: device real-ray trace
    of every beamlet's base ray and 8 parabasal rays (host arrays in and
    out), then the plane evaluation on the image plane (mixed form), its
    error against the obscured-aperture diffraction pattern."""
    import numpy as np
    import torch
    import paper_2404_12454_amd as gbd
    from paper_2404_12454_amd import scenes
    sysd = scenes.hst_rc()
    sc = scenes.rc_scene(n_across, npix=npix, half_span_lamF=16.0)
    args = (sysd["mirrors"], sysd["z_in"], sysd["z_out"], sysd["l0"], sc.r1, sc.th1)
    base, abcd, flags = gbd.gbd_trace(ctx, *args)
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        base, abcd, flags = gbd.gbd_trace(ctx, *args)
        t.append(time.perf_counter() - t0)
    keep = flags == 0
    b = gbd.gbd_beamlets_traced(ctx, int(keep.sum()), sc.lam, sc.l0, sc.r1[keep], sc.th1[keep], sc.w0[keep],
                                sc.amp[keep], sc.path[keep], abcd[keep], base[keep], 1e-7)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, int(keep.sum())).setup(b, p)
    out = torch.empty((npix, npix), dtype=torch.complex64, device="cuda")
    for _ in range(reps):
        plan.eval(gbd.GBD_MIXED, out)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, z in evs:
        a.record(stream)
        plan.eval(gbd.GBD_MIXED, out)
        z.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(z) for a, z in evs]))
    n = int(keep.sum())
    o = gbd.gbd_plane(ctx, sc.plane.origin, sc.plane.normal, sc.plane.xhint, 1, 1, 1e-6, 1e-6)
    E0 = complex(gbd.gbd_eval(ctx, b, o, gbd.GBD_FP64).cpu().numpy()[0, 0])
    E = out.cpu().numpy().astype(np.complex128)
    # figure of merit against the obscured-aperture pattern (scipy J1, on the host)
    import scipy.special
    _, a0, _ = gbd.gbd_trace(ctx, sysd["mirrors"], sysd["z_in"], sysd["z_out"], sysd["l0"], np.zeros((1, 2)))
    f = -1.0 / a0[0, 8]
    eps = sysd["r_obs"] / (sysd["D"] / 2)
    pl = sc.plane
    xa = (np.arange(pl.nx) - (pl.nx - 1) / 2) * pl.dx
    ya = (np.arange(pl.ny) - (pl.ny - 1) / 2) * pl.dy
    v = np.pi * sysd["D"] * np.hypot(*np.meshgrid(xa, ya)) / (sc.lam * f)
    with np.errstate(invalid="ignore", divide="ignore"):
        disc = lambda u: np.where(u > 0, 2 * scipy.special.j1(u) / u, 1.0)
        ref = ((disc(v) - eps * eps * disc(eps * v)) / (1 - eps * eps)) ** 2
    d = np.abs(E) ** 2 / abs(E0) ** 2 - ref
    return {"system": "Appendix B Ritchey-Chretien (f = %.4f m, obscuration %.4f)" % (f, eps),
            "beamlets": n, "vignetted_dropped": int((~keep).sum()), "npix": npix,
            "trace_ms_host_roundtrip": 1e3 * float(np.median(t)), "trace_rays": 9 * sc.n,
            "eval_ms": ms, "evals_per_s": n * npix * npix / (ms * 1e-3), "launch": plan.shape(gbd.GBD_MIXED),
            "rms_vs_obscured_airy": float(np.sqrt(np.mean(d * d))), "peak_vs_obscured_airy": float(np.abs(d).max())}


def hermite(ctx, stream, gauss_ms, n_across=256, npix=512, reps=10):
    """Elegant Hermite-Gaussian beamlets (orders up to 2 per axis, drawn per
    beamlet) on the headline grid: through the ideal lens (no cross terms:
    the separable MFMA form with per-axis factors) and through an added
    rotated cylindrical lens (cross terms: the rotor form with the factor's
    row polynomial), mixed precision, and both in FP64 (separable form on
    FP64 MFMA; FP64 rotor form with the row polynomial)."""
    import numpy as np
    import torch
    import paper_2404_12454_amd as gbd
    from paper_2404_12454_amd import scenes
    res = {}
    for name, kw in (("focal", {}), ("astigmatic", dict(cyl_f=3.0))):
        sc = scenes.hermite_scene(n_across, npix=npix, half_span_lamF=20.0, **kw)
        b = gbd.beamlets_from_scene(ctx, sc)
        p = gbd.plane_from_scene(ctx, sc)
        plan = gbd.Plan(ctx, sc.n).setup(b, p)
        out = torch.empty((npix, npix), dtype=torch.complex64, device="cuda")
        for _ in range(reps):
            plan.eval(gbd.GBD_MIXED, out)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, z in evs:
            a.record(stream)
            plan.eval(gbd.GBD_MIXED, out)
            z.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(z) for a, z in evs]))
        shape = plan.shape(gbd.GBD_MIXED)
        r = {"beamlets": sc.n, "npix": npix, "launch": shape, "eval_ms": ms,
             "evals_per_s": sc.n * npix * npix / (ms * 1e-3)}
        if shape["variant"] in (4, 5):
            r["mfma_frac"] = roofline(shape, sc.n, npix * npix, ms)["frac"]
            r["cost_vs_fundamental"] = ms / gauss_ms
        if shape["variant"] == 4:  # the same on FP32 MFMA (variant 5) for comparison
            o5 = gbd.gbd_eval_opts(variant=5)
            plan.eval(gbd.GBD_MIXED, out, opts=o5)
            e5 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for a, z in e5:
                a.record(stream)
                plan.eval(gbd.GBD_MIXED, out, opts=o5)
                z.record(stream)
            torch.cuda.synchronize()
            ms5 = float(np.mean([a.elapsed_time(z) for a, z in e5]))
            r["separable_fp32"] = {"eval_ms": ms5, "launch": plan.shape(gbd.GBD_MIXED, o5),
                                   "mfma_frac": roofline(plan.shape(gbd.GBD_MIXED, o5), sc.n, npix * npix, ms5)["frac"]}
            plan.eval(gbd.GBD_MIXED, out)  # the automatic form's field, for the FP64 comparison below
        elif shape["variant"] == 3:
            rf = roofline(shape, sc.n, npix * npix, ms, hg=True)
            r["roofline_peak"] = rf["peak"]
            r["roofline_frac"] = rf["frac"]
        # the FP64 form of the same input (separable on FP64 MFMA, or the FP64
        # rotor form with the factor's row polynomial)
        out64 = torch.empty((npix, npix), dtype=torch.complex128, device="cuda")
        plan.eval(gbd.GBD_FP64, out64)
        e64 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for a, z in e64:
            a.record(stream)
            plan.eval(gbd.GBD_FP64, out64)
            z.record(stream)
        torch.cuda.synchronize()
        ms64 = float(np.mean([a.elapsed_time(z) for a, z in e64]))
        E64 = out64.cpu().numpy()
        shape64 = plan.shape(gbd.GBD_FP64)
        r64 = {"launch": shape64, "eval_ms": ms64, "evals_per_s": sc.n * npix * npix / (ms64 * 1e-3),
               "err_mixed_vs_fp64": float(np.linalg.norm(out.cpu().numpy() - E64) / np.linalg.norm(E64))}
        if shape64["variant"] == 4:
            r64["fp64_mfma_frac"] = SEP64_FLOPS_PER_PAIR * sc.n * npix * npix / (ms64 * 1e-3) / 1e12 / MFMA_FP64_TFLOPS
        r["fp64"] = r64
        res[name] = r
    return res


# Truncated-beamlet kernel (eval_cut_mixed_kernel, 2 rows x 4 wavefronts,
# Faddeeva function with N = 16): per lane and beamlet, counted in the
# compiled loop: 215 FP32, 19 FP64, 14 transcendental (exp2, sin, cos twice
# and one reciprocal per pixel) and 10 other VALU instructions for 2 pixels.
CUT_MIX = {"fp64": 19 / 2, "fp32": (215 + 10) / 2, "trans": 14 / 2}


def truncated(ctx, stream, gauss_ms, n_across=256, npix=512, reps=10):
    """The headline pupil with its rim cut: the grid extended past the rim
    and every beamlet within 1.5 w0 of it cut by the rim's tangent.  One
    evaluation = the whole beamlets in their form (separable) + the cut ones
    in their own kernel (complex error function) + the segment reduction.
    Also the RMS error against the Airy pattern, plain grid vs cut rim."""
    import numpy as np
    import torch
    import paper_2404_12454_amd as gbd
    from paper_2404_12454_amd import scenes
    res = {}
    for kind in ("plain", "cut"):
        sc = (scenes.airy_scene(n_across, npix=npix, half_span_lamF=20.0) if kind == "plain" else
              scenes.truncated_airy_scene(n_across, npix=npix, half_span_lamF=20.0))
        b = gbd.beamlets_from_scene(ctx, sc)
        p = gbd.plane_from_scene(ctx, sc)
        plan = gbd.Plan(ctx, sc.n).setup(b, p)
        out = torch.empty((npix, npix), dtype=torch.complex64, device="cuda")
        for _ in range(reps):
            plan.eval(gbd.GBD_MIXED, out)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, z in evs:
            a.record(stream)
            plan.eval(gbd.GBD_MIXED, out)
            z.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(z) for a, z in evs]))
        m = sc.meta
        airy = gbd.gbd_airy(ctx, p, m["D"], m["f"], sc.lam).cpu().numpy().astype(np.float64)
        o = gbd.gbd_plane(ctx, sc.plane.origin, sc.plane.normal, sc.plane.xhint, 1, 1, 1e-6, 1e-6)
        E0 = complex(gbd.gbd_eval(ctx, b, o, gbd.GBD_FP64).cpu().numpy()[0, 0])
        d = np.abs(out.cpu().numpy().astype(np.complex128)) ** 2 / abs(E0) ** 2 - airy
        r = {"beamlets": sc.n, "eval_ms": ms, "evals_per_s": sc.n * npix * npix / (ms * 1e-3),
             "rms_vs_airy": float(np.sqrt(np.mean(d * d))), "peak_vs_airy": float(np.abs(d).max())}
        if kind == "cut":
            n_cut = int(m["n_cut"])
            cycles = sum(v / RATE[k] for k, v in CUT_MIX.items())
            r.update({"cut_beamlets": n_cut, "cut_pairs": n_cut * npix * npix,
                      "cut_kernel_roofline_evals_per_s": CUS * CLOCK_HZ / cycles,
                      "cost_vs_fundamental": ms / gauss_ms})
        res[kind] = r
    return res


def cpu_baseline(sc, E32, E64, stride=2, stride1=64):
    """The FP64 oracle on every 2nd pixel row (a bounded sample of the same
    workload, ~12 s on 16 host threads), all host threads; also the GPU
    fields' error on that sample, and the oracle on one thread over every
    64th row (~6 s)."""
    import numpy as np
    import oracle

    def sample(step):
        rows = np.arange(0, sc.plane.ny, step)
        iy, ix = np.meshgrid(rows, np.arange(sc.plane.nx), indexing="ij")
        return rows, ix.ravel().astype(np.int32), iy.ravel().astype(np.int32)

    ny = sc.plane.ny
    rows, ix, iy = sample(stride)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    ref = oracle.eval_field(sc, pixels=(ix, iy), threads=threads)
    dt = time.perf_counter() - t0
    pairs = sc.n * ix.size
    e32 = E32[iy, ix]
    e64 = E64[iy, ix]
    rows1, ix1, iy1 = sample(stride1)
    t0 = time.perf_counter()
    oracle.eval_field(sc, pixels=(ix1, iy1), threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"every {stride}nd pixel row ({rows.size} of {ny} rows, {ix.size} px x {sc.n} beamlets), "
                      f"{dt:.1f} s",
            "one_thread": {"value": sc.n * ix1.size / dt1, "unit": "evals/s", "cores": 1,
                           "sample": f"every {stride1}th pixel row ({rows1.size} of {ny} rows, {ix1.size} px x "
                                     f"{sc.n} beamlets), {dt1:.1f} s"},
            "err_mixed_vs_oracle": float(np.linalg.norm(e32 - ref) / np.linalg.norm(ref)),
            "err_fp64_vs_oracle": float(np.linalg.norm(e64 - ref) / np.linalg.norm(ref))}


if __name__ == "__main__":
    main()
