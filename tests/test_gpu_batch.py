"""GPU tests of the batched sweep (one persistent launch over many uneven
instances) and of the Airy reference and its figure of merit.

* reference irradiance vs scipy's J1
* batch fields are bitwise equal to single-instance evaluations with the same
  launch shape and one beamlet segment
* batch metrics (RMS, peak, annular zones) vs the FP64 oracle's field and
  scipy's Airy pattern
* the full 441-instance sweep vs per-instance single evaluations
* error reporting names the failing instance
"""
import math

import numpy as np
import pytest

import oracle
import oracle.metrics as om
import paper_2404_12454_amd as gbd
from paper_2404_12454_amd import scenes
from gbd_testutil import ensure_library

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    ensure_library()
    return gbd.Context(0)


def sweep_scene(na, OF, q, npix=256, span=8.0, npix_y=None):
    return scenes.airy_scene(na, OF=OF, q=q, npix=npix, half_span_lamF=span, npix_y=npix_y)


def test_airy_reference_matches_scipy(ctx):
    import torch
    sc = sweep_scene(16, 1.5, 1.0, npix=101, npix_y=77)
    p = gbd.plane_from_scene(ctx, sc)
    m = sc.meta
    A = gbd.gbd_airy(ctx, p, m["D"], m["f"], sc.lam)
    torch.cuda.synchronize()
    ref = om.airy_irradiance(sc.plane, m["D"], m["f"], sc.lam)
    assert np.abs(A.cpu().numpy() - ref).max() < 2e-7


def small_instances():
    combos = [(8, 1.0, 0.5), (12, 1.7, 1.0), (20, 2.5, 0.75), (16, 1.25, 2.0), (24, 1.5, 1.25), (10, 3.0, 0.5),
              (28, 1.1, 1.0), (6, 2.0, 1.5)]
    return [sweep_scene(na, of, q, npix=90, npix_y=70) for na, of, q in combos]


def test_batch_fields_bitwise_equal_single_instance(ctx):
    import torch
    insts = small_instances()
    bs = [gbd.beamlets_from_scene(ctx, s) for s in insts]
    ps = [gbd.plane_from_scene(ctx, s) for s in insts]
    # variant 4: the separable form in FP16 halves (per-instance scale from the
    # batched setup, as a single evaluation's); 5: on FP32 MFMA
    for rows, waves, variant in ((4, 2, 1), (4, 2, 2), (4, 2, 3), (32, 4, 3), (32, 1, 3), (4, 2, 4), (4, 2, 5)):
        o = dict(rows_per_lane=rows, waves=waves, variant=variant)
        _, fields = gbd.gbd_eval_batch(ctx, bs, ps, fields=True, opts=o)
        for s, b, p, F in zip(insts, bs, ps, fields):
            E = gbd.gbd_eval(ctx, b, p, gbd.GBD_MIXED, opts=dict(o, segments=1))
            torch.cuda.synchronize()
            assert torch.equal(F.cpu().view(torch.float32), E.cpu().view(torch.float32)), o


def test_batch_long_instance_leaves_the_separable_form(ctx):
    """An instance above 16,384 beamlets (160 across: one FP32 MFMA sum would
    exceed the longest the single evaluation allows) sends the batch to the
    rotor form, whose fields equal gbd_eval's rotor form with one segment bit
    for bit and meet the mixed tolerance against the oracle; a request for the
    separable form resolves the same way."""
    import torch
    big = sweep_scene(160, 1.7, 1.0, npix=64, npix_y=48, span=6.0)
    small = sweep_scene(24, 1.5, 1.0, npix=64, npix_y=48, span=6.0)
    assert big.n > 16384
    bs = [gbd.beamlets_from_scene(ctx, s) for s in (big, small)]
    ps = [gbd.plane_from_scene(ctx, s) for s in (big, small)]
    for req in (None, dict(variant=4)):
        _, fields = gbd.gbd_eval_batch(ctx, bs, ps, fields=True, opts=req)
        for s, b, p, F in zip((big, small), bs, ps, fields):
            E = gbd.gbd_eval(ctx, b, p, gbd.GBD_MIXED, opts=dict(rows_per_lane=32, waves=4, segments=1, variant=3))
            torch.cuda.synchronize()
            assert torch.equal(F.cpu().view(torch.float32), E.cpu().view(torch.float32)), (s.n, req)
        got = fields[0].cpu().numpy().astype(np.complex128)
        ref = oracle.eval_field(big)
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"batch instance of {big.n} beamlets, request {req}: rel_l2 {err:.2e}", flush=True)
        assert err <= 1e-5


def test_batch_metrics_match_oracle(ctx):
    import torch
    insts = small_instances()
    m0 = insts[0].meta
    lamF = insts[0].lam * m0["fnum"]
    edges = np.array([0.0, 2.0, 4.0, 6.0]) * lamF
    bs = [gbd.beamlets_from_scene(ctx, s) for s in insts]
    ps = [gbd.plane_from_scene(ctx, s) for s in insts]
    airy = gbd.gbd_airy(ctx, ps[0], m0["D"], m0["f"], insts[0].lam)
    metrics, _ = gbd.gbd_eval_batch(ctx, bs, ps, airy=airy, zone_edges=edges)
    ref_airy = om.airy_irradiance(insts[0].plane, m0["D"], m0["f"], insts[0].lam)
    radius = om.plane_radius(insts[0].plane)
    for s, got in zip(insts, metrics):
        E, E0 = oracle.eval_field(s, extra_point=(0.0, 0.0))
        want = om.airy_metrics(E, E0, ref_airy, radius, edges)
        print(s.meta["n_across"], s.meta["OF"], s.meta["q"], got, want, flush=True)
        np.testing.assert_allclose(got, want, rtol=2e-4, atol=1e-9)


def test_sweep_instances_full_size_match_oracle(ctx):
    """One instance of the 441-instance sweep per beamlet count (208 ...
    12,892 beamlets), each at its full 256 x 256 grid over +-8 lambda F,
    batched as in the sweep (separable form, one FP32 sum per pixel): every
    field pixel within the mixed tolerance of the oracle, and the metrics
    (peak-normalised irradiance, RMS and peak against the Airy pattern)
    within 1e-5 absolute of the oracle's."""
    import torch
    picks = [(1.5, 1.0, 16), (1.75, 0.75, 24), (2.0, 1.25, 32), (1.25, 1.5, 48), (2.5, 0.5, 64), (2.25, 0.75, 96),
             (1.75, 1.0, 128)]
    grid = {tuple(g) for g in scenes.sweep_grid()}
    assert all(p in grid for p in picks)
    insts = [sweep_scene(na, of, q) for of, q, na in picks]
    assert [s.n for s in insts] == [208, 448, 812, 1804, 3228, 7232, 12892]
    bs = [gbd.beamlets_from_scene(ctx, s) for s in insts]
    ps = [gbd.plane_from_scene(ctx, s) for s in insts]
    m0 = insts[0].meta
    airy = gbd.gbd_airy(ctx, ps[0], m0["D"], m0["f"], insts[0].lam)
    metrics, fields = gbd.gbd_eval_batch(ctx, bs, ps, airy=airy, fields=True)
    torch.cuda.synchronize()
    ref_airy = om.airy_irradiance(insts[0].plane, m0["D"], m0["f"], insts[0].lam)
    for s, got, F in zip(insts, metrics, fields):
        E, E0 = oracle.eval_field(s, extra_point=(0.0, 0.0))
        e = F.cpu().numpy().astype(np.complex128)
        err = float(np.linalg.norm(e - E) / np.linalg.norm(E))
        want = om.airy_metrics(E, E0, ref_airy)
        print(f"sweep instance {s.n} beamlets: field rel_l2 {err:.2e}, metrics {got} oracle {want}", flush=True)
        assert err <= 1e-5
        assert np.abs(got - want).max() <= 1e-5


def test_full_sweep_matches_single_instances(ctx):
    """All 441 (OF, q, n_across) instances at 256 x 256 over +-8 lamF in one launch."""
    import time
    import torch
    grid = scenes.sweep_grid()
    insts = [sweep_scene(na, of, q) for of, q, na in grid]
    bs = [gbd.beamlets_from_scene(ctx, s) for s in insts]
    ps = [gbd.plane_from_scene(ctx, s) for s in insts]
    m0 = insts[0].meta
    airy = gbd.gbd_airy(ctx, ps[0], m0["D"], m0["f"], insts[0].lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    metrics, _ = gbd.gbd_eval_batch(ctx, bs, ps, airy=airy)
    dt = time.perf_counter() - t0
    pairs = sum(s.n for s in insts) * 65536
    print(f"sweep: {len(insts)} instances, {pairs:.3e} pairs, {dt * 1e3:.1f} ms, {pairs / dt:.3e} evals/s", flush=True)
    assert np.isfinite(metrics).all()
    A = airy.cpu().numpy().astype(np.float64)
    origin = [None]
    for k in range(0, len(insts), 7):
        s, b = insts[k], bs[k]
        # the batch kernel's form (separable in FP16 halves: the sweep's Airy
        # scenes have no cross terms) with one segment: the same field arithmetic
        E = gbd.gbd_eval(ctx, b, ps[k], gbd.GBD_MIXED, opts=dict(segments=1, variant=4))
        pl = s.plane
        if origin[0] is None:
            origin[0] = gbd.gbd_plane(ctx, pl.origin, pl.normal, pl.xhint, 1, 1, pl.dx, pl.dy)
        E0 = gbd.gbd_eval(ctx, b, origin[0], gbd.GBD_FP64)
        torch.cuda.synchronize()
        want = om.airy_metrics(E.cpu().numpy().astype(np.complex128), complex(E0.cpu().numpy()[0, 0]), A)
        np.testing.assert_allclose(metrics[k], want, rtol=2e-4, atol=1e-9)
    # more beamlets across the pupil gives a smaller error at fixed OF, q
    by = {(of, q, na): m for (of, q, na), m in zip(grid, metrics)}
    for of, q in ((1.5, 1.0), (1.75, 1.0)):
        rms = [by[(of, q, na)][0] for na in scenes.SWEEP_NACROSS]
        assert rms[-1] < rms[0]


def test_batch_names_failing_instance(ctx):
    insts = small_instances()[:4]
    bs = [gbd.beamlets_from_scene(ctx, s) for s in insts]
    ps = [gbd.plane_from_scene(ctx, s) for s in insts]
    one = gbd.gbd_beamlets(ctx, 1, 1e-6, 0.1, [[0.0, 0.0]], None, [1e-3], None, None,
                           scenes.lens_then_distance(0.1, 0.1))
    side = gbd.gbd_plane(ctx, [0, 0, 0], [1, 0, 0], [0, 1, 0], 4, 4, 1e-6, 1e-6)
    bs[2], ps[2] = one, side
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_eval_batch(ctx, bs, ps, fields=True)
    assert e.value.code == -4 and "instance 2" in str(e.value)


def test_batch_autotuner_shape_and_metrics(ctx):
    insts = small_instances()
    bs = [gbd.beamlets_from_scene(ctx, s) for s in insts]
    ps = [gbd.plane_from_scene(ctx, s) for s in insts]
    m0 = insts[0].meta
    airy = gbd.gbd_airy(ctx, ps[0], m0["D"], m0["f"], insts[0].lam)
    ref, _ = gbd.gbd_eval_batch(ctx, bs, ps, airy=airy, opts=dict(rows_per_lane=16, waves=4))
    best, ms = gbd.gbd_autotune_batch(ctx, bs, ps, airy, reps=2)
    print("batch autotuned", best, ms, flush=True)
    assert best["rows_per_lane"] in (2, 4, 8, 16, 32) and best["waves"] in (1, 2, 4) and ms > 0
    got, _ = gbd.gbd_eval_batch(ctx, bs, ps, airy=airy)  # the cached shape
    np.testing.assert_allclose(got, ref, rtol=1e-3, atol=1e-9)


def test_autotuner_picks_a_valid_shape_and_results_hold(ctx, tmp_path):
    import torch
    sc = scenes.zernike_scene(31, n_across=40, npix=300, half_span=60e-6)
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    best, ms = gbd.gbd_autotune(plan, gbd.GBD_MIXED, reps=2)
    print("autotuned", best, ms, flush=True)
    assert best["rows_per_lane"] in (2, 4, 8, 16, 32) and best["waves"] in (1, 2, 4) and ms > 0
    assert plan.shape(gbd.GBD_MIXED) == best          # the cache is used with default opts
    E = plan.eval(gbd.GBD_MIXED)
    torch.cuda.synchronize()
    ref = oracle.eval_field(sc)
    e = E.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(e - ref) / np.linalg.norm(ref) < 1e-5
    path = str(tmp_path / "tune.txt")
    gbd.gbd_autotune_save(ctx, path)
    fresh = gbd.Context(0)
    assert gbd.gbd_autotune_load(fresh, path) >= 1
    plan2 = gbd.Plan(fresh, sc.n).setup(gbd.beamlets_from_scene(fresh, sc), gbd.plane_from_scene(fresh, sc))
    assert plan2.shape(gbd.GBD_MIXED) == best


def test_autotuner_tunes_the_separable_forms_segments(ctx, tmp_path):
    """Where the separable form applies only its segment count is tuned (the
    tile is fixed); the cached choice is used with default opts, survives a
    save and load, and the field still matches the oracle."""
    import torch
    sc = scenes.airy_scene(40, npix=300, npix_y=260, half_span_lamF=10.0)
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    auto = plan.shape(gbd.GBD_MIXED)
    assert auto["variant"] == 4
    best, ms = gbd.gbd_autotune(plan, gbd.GBD_MIXED, reps=2)
    print("separable autotuned", auto, "->", best, ms, flush=True)
    assert best["variant"] == 4 and best["segments"] >= 1 and ms > 0
    assert (best["rows_per_lane"], best["waves"]) == (auto["rows_per_lane"], auto["waves"])
    assert plan.shape(gbd.GBD_MIXED) == best
    E = plan.eval(gbd.GBD_MIXED)
    torch.cuda.synchronize()
    ref = oracle.eval_field(sc)
    e = E.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(e - ref) / np.linalg.norm(ref) < 1e-5
    path = str(tmp_path / "tune_sep.txt")
    gbd.gbd_autotune_save(ctx, path)
    fresh = gbd.Context(0)
    assert gbd.gbd_autotune_load(fresh, path) >= 1
    plan2 = gbd.Plan(fresh, sc.n).setup(gbd.beamlets_from_scene(fresh, sc), gbd.plane_from_scene(fresh, sc))
    assert plan2.shape(gbd.GBD_MIXED) == best


def test_batch_with_an_empty_instance(ctx):
    """An instance without beamlets in the middle of a batch: its field is
    zero, its metrics compare a zero field (RMS of the Airy pattern itself,
    peak its maximum), and the other instances' metrics and fields equal those
    of the batch without it bit for bit (each instance's E(0) chunks and
    item partials are its own)."""
    import torch
    a = sweep_scene(24, 1.5, 1.0, npix=96, npix_y=80, span=6.0)
    b = sweep_scene(40, 1.7, 0.8, npix=96, npix_y=80, span=6.0)
    empty = scenes.Scene(a.lam, a.l0, np.zeros((0, 2)), np.zeros((0, 2)), np.zeros(0) + 1e-3,
                         np.zeros((0, 2)), np.zeros(0), a.abcd, a.plane)
    m = a.meta
    pa = gbd.plane_from_scene(ctx, a)
    airy = gbd.gbd_airy(ctx, pa, m["D"], m["f"], a.lam)
    bs3 = [gbd.beamlets_from_scene(ctx, s) for s in (a, empty, b)]
    ps3 = [gbd.plane_from_scene(ctx, s) for s in (a, empty, b)]
    m3, f3 = gbd.gbd_eval_batch(ctx, bs3, ps3, airy=airy, fields=True)
    m2, f2 = gbd.gbd_eval_batch(ctx, [bs3[0], bs3[2]], [ps3[0], ps3[2]], airy=airy, fields=True)
    torch.cuda.synchronize()
    assert np.array_equal(m3[[0, 2]], m2)
    for F3, F2 in ((f3[0], f2[0]), (f3[2], f2[1])):
        assert torch.equal(F3.cpu().view(torch.float32), F2.cpu().view(torch.float32))
    assert not torch.any(f3[1].cpu().view(torch.float32) != 0)
    A = airy.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(m3[1, 0], np.sqrt(np.mean(A * A)), rtol=1e-6)
    np.testing.assert_allclose(m3[1, 1], A.max(), rtol=1e-6)
