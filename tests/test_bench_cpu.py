"""Host logic of the benchmark script, on the CPU: it refuses runs on more
than one GPU before touching a device, and its roofline arithmetic matches
the definitions it states (algorithmic flops per pair over the published
peaks, instruction-mix rooflines from per-pair counts and issue rates)."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_separable_roofline_arithmetic():
    b = load_bench()
    N, M, ms = 51468, 512 * 512, 0.8
    r = b.roofline({"variant": 5, "rows_per_lane": 32, "waves": 8, "segments": 16}, N, M, ms)
    # Gauss's form: three real multiply-adds (6 flops) per pair on the
    # matrix cores; the textbook complex multiply-add (8 flops) only as a rate
    achieved = 6.0 * N * M / (ms * 1e-3) / 1e12
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(achieved, rel=1e-12)
    assert r["frac"] == pytest.approx(achieved / 157.3, rel=1e-12)
    assert r["frac"] <= 1.0
    assert r["complex_madd_equiv_tflops"] == pytest.approx(achieved * 8.0 / 6.0, rel=1e-12)
    # FP16 halves: three hi/lo products of the four real products, 24 flops
    # per pair against the FP16 MFMA peak
    h = b.roofline({"variant": 4, "rows_per_lane": 32, "waves": 8, "segments": 16}, N, M, ms)
    assert h["bound"] == "mfma" and h["peak"] == 2500.0
    assert h["achieved"] == pytest.approx(24.0 * N * M / (ms * 1e-3) / 1e12, rel=1e-12)
    assert h["frac"] == pytest.approx(h["achieved"] / 2500.0, rel=1e-12) and h["frac"] <= 1.0


def test_rotor_instruction_mix_roofline():
    b = load_bench()
    peak, cycles, mix = b.roofline_peak(32, 3)
    # per pair at 32 rows: 8.41 FP32 + 0.47 FP64 + 0.22 transcendental at
    # 128 / 64 / 32 lanes per CU per clock on 256 CUs at 2.4 GHz
    assert mix["fp32"] == pytest.approx(8.41, abs=0.01)
    assert mix["fp64"] == pytest.approx(0.47, abs=0.01)
    assert mix["trans"] == pytest.approx(0.22, abs=0.01)
    assert cycles == pytest.approx(mix["fp32"] / 128 + mix["fp64"] / 64 + mix["trans"] / 32, rel=1e-12)
    assert peak == pytest.approx(256 * 2.4e9 / cycles, rel=1e-12)
    assert peak == pytest.approx(7.70e12, rel=0.005)
    r = b.roofline({"variant": 3, "rows_per_lane": 32, "waves": 4, "segments": 48}, 51468, 512 * 512, 2.6)
    assert r["bound"] == "alu" and r["frac"] == pytest.approx(51468 * 512 * 512 / 2.6e-3 / peak, rel=1e-12)


def test_fp64_records():
    b = load_bench()
    N, M = 51468, 512 * 512
    r4 = b.fp64_record({"variant": 4, "rows_per_lane": 32, "waves": 8, "segments": 16}, N, M, 2.0, 0.8)
    assert r4["roofline_peak_tflops"] == 78.6
    assert r4["roofline_frac"] == pytest.approx(8.0 * N * M / 2.0e-3 / 1e12 / 78.6, rel=1e-12)
    r3 = b.fp64_record({"variant": 3, "rows_per_lane": 32, "waves": 4, "segments": 48}, N, M, 5.9, 0.8)
    # 363 FP64 and 36 other instructions per lane and beamlet at 32 rows
    assert r3["roofline_peak"] == pytest.approx(256 * 2.4e9 / (363 / 32 / 64 + 36 / 32 / 128), rel=1e-12)
