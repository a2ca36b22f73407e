"""GPU parity of the HIP path (called through the C ABI) against the FP64
oracle on the same seeded inputs.

Tolerances (relative L2 field error, raw and global-phase aligned):
  FP64 form  <= 1e-12
  mixed form <= 1e-5   (FP64 phase, FP32 exp2/sin/cos, FP32 compensated sums)
Full-size workloads are checked on pixel samples the oracle computes one by
one, in the launch configuration the benchmark uses, and through symmetry
properties that hold on the whole grid.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2404_12454_amd as gbd
from paper_2404_12454_amd import scenes
from gbd_testutil import ensure_library, rel_l2, rel_l2_phase_aligned

pytestmark = pytest.mark.gpu

TOL = {gbd.GBD_FP64: 1e-12, gbd.GBD_MIXED: 1e-5}
BOTH = [gbd.GBD_FP64, gbd.GBD_MIXED]


@pytest.fixture(scope="module")
def ctx():
    ensure_library()
    return gbd.Context(0)


def run(ctx, sc, precision, opts=None):
    import torch
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    E = gbd.gbd_eval(ctx, b, p, precision, opts=opts)
    torch.cuda.synchronize()
    return E.cpu().numpy()


def check(E, ref, precision, what=""):
    e1, e2 = rel_l2(E, ref), rel_l2_phase_aligned(E, ref)
    print(f"{what} precision={precision} rel_l2={e1:.3e} aligned={e2:.3e}", flush=True)
    assert e1 <= TOL[precision] and e2 <= TOL[precision], (what, e1, e2)


@pytest.mark.parametrize("precision", BOTH)
def test_airy32_64_full_grid(ctx, precision):
    sc = scenes.config("airy32_64")
    check(run(ctx, sc, precision), oracle.eval_field(sc), precision, "airy32_64")


@pytest.mark.parametrize("precision", BOTH)
def test_tilted_aberrated_ragged_grid(ctx, precision):
    """f/4, 1 deg field, Zernike seed 2404, plane tilted 10 deg at +50 um;
    200 x 137 pixels (ragged in both tile directions), 32 across."""
    sc = scenes.zernike_scene(2404, n_across=32, npix=200, half_span=60e-6)
    sc.plane.ny = 137
    check(run(ctx, sc, precision), oracle.eval_field(sc), precision, "zern32_200x137")


SHAPES = [dict(rows_per_lane=r, waves=w, segments=s) for r in (1, 2, 4, 8) for w in (1, 2, 4) for s in (1, 3)]


@pytest.mark.parametrize("precision", BOTH)
def test_every_launch_shape_matches_oracle(ctx, precision):
    sc = scenes.zernike_scene(99, n_across=20, npix=70, half_span=40e-6)
    sc.plane.ny = 45
    ref = oracle.eval_field(sc)
    # FP64: the direct and rotor forms; mixed: direct, stepped and rotor
    variants = (1, 2, 3) if precision == gbd.GBD_MIXED else (1, 3)
    shapes = SHAPES + [dict(rows_per_lane=r, waves=w, segments=s) for r in (16, 32) for w in (1, 2, 4) for s in (1, 3)]
    for v in variants:
        for o in shapes:
            check(run(ctx, sc, precision, opts=dict(o, variant=v)), ref, precision, f"shape {o} variant {v}")


@pytest.mark.parametrize("name", ["airy32_64", "zern128_1024"])
def test_rotor_variant_is_chosen_and_matches_direct(ctx, name):
    """On well-sampled grids with cross terms the automatic mixed form is the
    rotor one (the Airy scene has none and goes to the separable form); the
    rotor and stepped forms agree with the direct form and with the oracle."""
    sc = scenes.config(name)
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    assert plan.shape(gbd.GBD_MIXED)["variant"] == (4 if name.startswith("airy") else 3)
    E3 = plan.eval(gbd.GBD_MIXED, opts=dict(variant=3)).cpu().numpy()
    E2 = plan.eval(gbd.GBD_MIXED, opts=dict(variant=2)).cpu().numpy()
    E1 = plan.eval(gbd.GBD_MIXED, opts=dict(variant=1)).cpu().numpy()
    print(name, "rotor vs direct", rel_l2(E3, E1), "stepped vs direct", rel_l2(E2, E1), flush=True)
    assert rel_l2(E3, E1) < 1e-5
    assert rel_l2(E2, E1) < 1e-5
    if sc.plane.npix <= 4096:
        ref = oracle.eval_field(sc)
        check(E3, ref, gbd.GBD_MIXED, name + " rotor")
        check(E2, ref, gbd.GBD_MIXED, name + " stepped")


def test_separable_form_is_chosen_and_matches_oracle(ctx):
    """A rotationally symmetric system on a plane normal to the axis has no
    cross terms: the automatic mixed form is the separable (MFMA) one; it
    agrees with the oracle and with the rotor form."""
    sc = scenes.config("airy32_64")
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    assert plan.shape(gbd.GBD_MIXED)["variant"] == 4
    E4 = plan.eval(gbd.GBD_MIXED).cpu().numpy()
    E3 = plan.eval(gbd.GBD_MIXED, opts=dict(variant=3)).cpu().numpy()
    print("separable vs rotor", rel_l2(E4, E3), flush=True)
    assert rel_l2(E4, E3) < 1e-5
    check(E4, oracle.eval_field(sc), gbd.GBD_MIXED, "airy32_64 separable")


@pytest.mark.parametrize("variant", [0, 5])
@pytest.mark.parametrize("nx,ny,seg", [(70, 45, 1), (70, 45, 3), (129, 200, 0), (300, 140, 0), (300, 140, 5),
                                       (1, 1, 1), (65, 1, 2), (1, 70, 0)])
def test_separable_form_ragged_defocused_off_axis(ctx, nx, ny, seg, variant):
    """Grids that leave every 16 x 16 block, wavefront and workgroup tile
    partly empty, beamlet counts not a multiple of the quad of beamlets an
    MFMA step takes, a field angle and a defocused plane (strong per-beamlet
    phase slopes); the automatic form (FP16 halves) and the FP32 one (5)."""
    sc = scenes.airy_scene(21, npix=nx, npix_y=ny, half_span_lamF=6.0, field_angle=(1e-3, -5e-4), z0=30e-6)
    assert sc.n % 4 != 0
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    o = dict(segments=seg, variant=variant)
    assert plan.shape(gbd.GBD_MIXED, opts=o)["variant"] == (variant or 4)
    check(plan.eval(gbd.GBD_MIXED, opts=o).cpu().numpy(), oracle.eval_field(sc), gbd.GBD_MIXED,
          f"separable {nx}x{ny} seg {seg} variant {variant or 4}")


@pytest.mark.parametrize("scale,spread", [(1e12, 1.0), (1e-12, 1.0), (1.0, 1e-9), (1e6, 1e-14)])
def test_separable_halves_across_amplitude_ranges(ctx, scale, spread):
    """The FP16 halves form scales each beamlet's factors into FP16's range
    from the setup's bounds: uniform amplitudes far from 1, and half of the
    beamlets weaker by `spread`, on a defocused grid whose envelopes fall
    off across it; against the oracle and the FP32 separable form."""
    sc = scenes.airy_scene(24, npix=96, npix_y=80, half_span_lamF=8.0, z0=200e-6)
    amp = np.asarray(sc.amp, np.float64).reshape(-1, 2) * scale
    amp[::2] *= spread
    sc.amp = amp
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    assert plan.shape(gbd.GBD_MIXED)["variant"] == 4
    E4 = plan.eval(gbd.GBD_MIXED).cpu().numpy()
    E5 = plan.eval(gbd.GBD_MIXED, opts=dict(variant=5)).cpu().numpy()
    ref = oracle.eval_field(sc)
    check(E4, ref, gbd.GBD_MIXED, f"halves amplitude x{scale:g}, spread {spread:g}")
    check(E5, ref, gbd.GBD_MIXED, f"FP32 separable amplitude x{scale:g}, spread {spread:g}")


@pytest.mark.parametrize("precision,variant", [(gbd.GBD_FP64, 4), (gbd.GBD_MIXED, 4), (gbd.GBD_MIXED, 5)])
@pytest.mark.parametrize("n,seg", [(1, 1), (2, 1), (5, 1), (15, 1), (16, 1), (17, 1), (33, 1), (33, 4), (37, 5),
                                   (64, 3), (100, 7)])
def test_separable_form_short_segments(ctx, precision, variant, n, seg):
    """The separable forms take beamlets in passes of four quads (16) between
    barriers: segments shorter than a pass, a pass and a quad, and ragged last
    passes and quads, on a grid smaller than one workgroup tile."""
    full = scenes.airy_scene(21, npix=70, npix_y=45, half_span_lamF=6.0, field_angle=(1e-3, -5e-4), z0=30e-6)
    keep = np.zeros(full.n, bool)
    keep[np.random.default_rng(n).choice(full.n, n, replace=False)] = True
    sc = oracle._subset(full, keep)
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    o = dict(segments=seg, variant=variant)
    assert plan.shape(precision, opts=o)["variant"] == (variant if precision == gbd.GBD_MIXED else 4)
    check(plan.eval(precision, opts=o).cpu().numpy(), oracle.eval_field(sc), precision,
          f"separable n {n} seg {seg} variant {variant}")


def test_consecutive_setups_of_one_plan_keep_their_own_flags(ctx):
    """A plan's setups alternate two device status words, each setup clearing
    the other: flags (cross terms, a refusal) must not carry over to the next
    setup, and a refused setup must not leave stale flags behind."""
    import torch
    airy = scenes.airy_scene(10, npix=40)
    zern = scenes.zernike_scene(7, n_across=10, npix=40, half_span=30e-6)
    n = max(airy.n, zern.n)
    plan = gbd.Plan(ctx, n)
    ba, pa = gbd.beamlets_from_scene(ctx, airy), gbd.plane_from_scene(ctx, airy)
    bz, pz = gbd.beamlets_from_scene(ctx, zern), gbd.plane_from_scene(ctx, zern)
    binv = gbd.gbd_beamlets(ctx, airy.n, airy.lam, airy.l0, airy.r1, airy.th1, airy.w0, airy.amp, airy.path,
                            -np.eye(4))
    ref_a = oracle.eval_field(airy)
    for step in range(5):
        for b, p, variant in ((bz, pz, 3), (ba, pa, 4), (ba, pa, 4), (bz, pz, 3)):
            plan.setup(b, p)
            assert plan.shape(gbd.GBD_MIXED)["variant"] == variant, (step, variant)
        with pytest.raises(gbd.GbdError) as e:
            plan.setup(binv, pa)
        assert e.value.code == -3
        plan.setup(ba, pa)
        assert plan.shape(gbd.GBD_MIXED)["variant"] == 4
        E = plan.eval(gbd.GBD_MIXED)
        torch.cuda.synchronize()
        check(E.cpu().numpy(), ref_a, gbd.GBD_MIXED, f"airy after a refused setup, round {step}")


@pytest.mark.parametrize("precision", BOTH)
def test_reported_shape_is_accepted_back(ctx, precision):
    """The shape gbd_plan_shape reports (for the separable form a fixed tile,
    reported as 32 rows x 8 wavefronts) is accepted as options and gives the
    default evaluation bit for bit; in a VALU form rows and waves are still
    checked."""
    import torch
    for sc in (scenes.airy_scene(12, npix=48), scenes.zernike_scene(5, n_across=12, npix=48)):
        plan = gbd.Plan(ctx, sc.n).setup(gbd.beamlets_from_scene(ctx, sc), gbd.plane_from_scene(ctx, sc))
        shape = plan.shape(precision)
        a = plan.eval(precision).clone()
        b = plan.eval(precision, opts=shape)
        torch.cuda.synchronize()
        assert torch.equal(a.cpu(), b.cpu()), shape
    with pytest.raises(gbd.GbdError) as e:
        plan.eval(precision, opts=dict(rows_per_lane=32, waves=8, variant=3))
    assert e.value.code == -1


@pytest.mark.parametrize("precision", BOTH)
def test_rotor_tables_follow_the_plane(ctx, precision):
    """The rotor forms' sigma^(k^2) tables depend on the plane's row pitch and
    are filled at evaluation: one plan set up in turn on planes of different
    pitch (and the same plane again) gives the oracle's field each time."""
    import torch
    plan = None
    for span in (30e-6, 45e-6, 20e-6, 30e-6):
        sc = scenes.zernike_scene(9, n_across=12, npix=72, half_span=span)
        b, p = gbd.beamlets_from_scene(ctx, sc), gbd.plane_from_scene(ctx, sc)
        plan = plan or gbd.Plan(ctx, sc.n)
        plan.setup(b, p)
        assert plan.shape(precision, dict(variant=3))["variant"] == 3
        E = plan.eval(precision, opts=dict(variant=3))
        torch.cuda.synchronize()
        check(E.cpu().numpy(), oracle.eval_field(sc), precision, f"rotor after re-setup, half span {span}")


def test_separable_form_long_segments_are_split(ctx):
    """823,592 beamlets (1024 across) on 512 x 512 pixels: occupancy alone
    would give 16 segments of 51,474 beamlets summed in FP32; the automatic
    count keeps segments at most 16,384 long, and the field stays within the
    mixed tolerance at sampled pixels."""
    sc = scenes.airy_scene(1024, npix=512, half_span_lamF=20.0)
    b, p = gbd.beamlets_from_scene(ctx, sc), gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    shape = plan.shape(gbd.GBD_MIXED)
    assert shape["variant"] == 4 and shape["segments"] >= -(-sc.n // 16384)
    E = plan.eval(gbd.GBD_MIXED).cpu().numpy().astype(np.complex128)
    rng = np.random.default_rng(8)
    ix = rng.integers(0, 512, 60).astype(np.int32)
    iy = rng.integers(0, 512, 60).astype(np.int32)
    ref = oracle.eval_field(sc, pixels=(ix, iy))
    err = rel_l2(E[iy, ix], ref)
    print(f"1024 across ({sc.n} beamlets), {shape['segments']} segments: rel_l2 {err:.2e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("segments", [1, 5])
def test_separable_explicit_segments_respect_the_fp32_cap(ctx, segments):
    """An explicit segment count that would put more than 16,384 beamlets in
    one FP32 MFMA sum is raised to ceil(N / 16384): 512 across (205,898
    beamlets, 1.4e-5 in one plain FP32 sum) on a 48 x 40 grid, full grid
    against the oracle."""
    sc = scenes.airy_scene(512, npix=48, npix_y=40, half_span_lamF=6.0)
    b, p = gbd.beamlets_from_scene(ctx, sc), gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    o = dict(segments=segments)
    shape = plan.shape(gbd.GBD_MIXED, opts=o)
    floor = -(-sc.n // 16384)
    assert shape["variant"] == 4 and shape["segments"] >= floor, shape
    assert -(-sc.n // shape["segments"]) <= 16384
    E = plan.eval(gbd.GBD_MIXED, opts=o).cpu().numpy()
    check(E, oracle.eval_field(sc), gbd.GBD_MIXED, f"512 across, segments {segments} -> {shape['segments']}")


def test_cross_terms_rule_out_the_separable_form(ctx):
    sc = scenes.zernike_scene(7, n_across=12, npix=40, half_span=30e-6)
    plan = gbd.Plan(ctx, sc.n).setup(gbd.beamlets_from_scene(ctx, sc), gbd.plane_from_scene(ctx, sc))
    assert plan.shape(gbd.GBD_MIXED)["variant"] == 3
    assert plan.shape(gbd.GBD_MIXED, opts=dict(variant=4))["variant"] == 3


def test_steep_grid_falls_back_to_direct(ctx):
    tail = scenes.airy_scene(1, npix=16, half_span_lamF=30.0)
    plan = gbd.Plan(ctx, 1).setup(gbd.beamlets_from_scene(ctx, tail), gbd.plane_from_scene(ctx, tail))
    # no cross terms: the separable form, which needs no curvature bound
    assert plan.shape(gbd.GBD_MIXED)["variant"] == 4
    assert plan.shape(gbd.GBD_MIXED, opts=dict(variant=2))["variant"] == 1
    assert plan.shape(gbd.GBD_MIXED, opts=dict(variant=3))["variant"] == 1
    # 32 rows per lane is a rotor-form shape; the direct form runs 16
    assert plan.shape(gbd.GBD_MIXED, opts=dict(rows_per_lane=32, variant=1))["rows_per_lane"] == 16
    # FP64: the separable form needs no curvature bound, the rotor form does;
    # the FP64 direct form runs at most 8 rows
    assert plan.shape(gbd.GBD_FP64)["variant"] == 4
    assert plan.shape(gbd.GBD_FP64, opts=dict(variant=3))["variant"] == 4
    assert plan.shape(gbd.GBD_FP64, opts=dict(rows_per_lane=32, variant=1))["rows_per_lane"] == 8


@pytest.mark.parametrize("name", ["airy32_64", "zern128_1024"])
def test_fp64_rotor_form_is_chosen_and_matches(ctx, name):
    """The automatic FP64 form: separable (FP64 MFMA) without cross terms,
    else the rotor one (the mixed rotor recurrence in FP64, no per-pixel exp
    or sincospi); both agree with the FP64 direct form to rounding and with
    the oracle."""
    sc = scenes.config(name)
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    shape = plan.shape(gbd.GBD_FP64)
    assert shape["variant"] == (4 if name.startswith("airy") else 3)
    E1 = plan.eval(gbd.GBD_FP64, opts=dict(variant=1)).cpu().numpy()
    for v in ((4, 3) if name.startswith("airy") else (3,)):
        E = plan.eval(gbd.GBD_FP64, opts=dict(variant=v)).cpu().numpy()
        print(name, plan.shape(gbd.GBD_FP64, dict(variant=v)), "FP64 variant", v, "vs direct", rel_l2(E, E1),
              flush=True)
        assert rel_l2(E, E1) < 1e-13
        if sc.plane.npix <= 4096:
            check(E, oracle.eval_field(sc), gbd.GBD_FP64, f"{name} FP64 variant {v}")
        else:
            ix, iy = sample_pixels(sc.plane.nx, sc.plane.ny, 100, 9)
            check(E[iy, ix], oracle.eval_field(sc, pixels=(ix, iy)), gbd.GBD_FP64, f"{name} FP64 variant {v} sampled")


@pytest.mark.parametrize("nx,ny,seg", [(70, 45, 1), (70, 45, 3), (129, 200, 0), (1, 1, 1), (65, 1, 2), (1, 70, 0),
                                       (300, 97, 5)])
def test_fp64_separable_form_ragged_defocused_off_axis(ctx, nx, ny, seg):
    """The FP64 separable form (FP64 MFMA) on grids that leave blocks,
    wavefront and workgroup tiles partly empty, a beamlet count not a multiple
    of K = 4, a field angle and a defocused plane."""
    sc = scenes.airy_scene(21, npix=nx, npix_y=ny, half_span_lamF=6.0, field_angle=(1e-3, -5e-4), z0=30e-6)
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    o = dict(segments=seg)
    assert plan.shape(gbd.GBD_FP64, opts=o)["variant"] == 4
    check(plan.eval(gbd.GBD_FP64, opts=o).cpu().numpy(), oracle.eval_field(sc), gbd.GBD_FP64,
          f"FP64 separable {nx}x{ny} seg {seg}")


@pytest.mark.parametrize("precision", BOTH)
def test_bitwise_run_to_run(ctx, precision):
    for sc in (scenes.zernike_scene(5, n_across=24, npix=96), scenes.airy_scene(24, npix=96)):
        a = run(ctx, sc, precision)
        b = run(ctx, sc, precision)
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def sample_pixels(nx, ny, count, seed):
    rng = np.random.default_rng(seed)
    ix = np.concatenate([rng.integers(0, nx, count), [0, nx - 1, nx // 2, 0, nx - 1]])
    iy = np.concatenate([rng.integers(0, ny, count), [0, ny - 1, ny // 2, ny - 1, 0]])
    return ix.astype(np.int32), iy.astype(np.int32)


@pytest.mark.parametrize("precision", BOTH)
def test_airy256_512_full_size_sampled(ctx, precision):
    """51,468 beamlets on 512 x 512 pixels, default (benchmark) launch shape."""
    sc = scenes.config("airy256_512")
    E = run(ctx, sc, precision)
    ix, iy = sample_pixels(512, 512, 200, 1)
    ref = oracle.eval_field(sc, pixels=(ix, iy))
    check(E[iy, ix], ref, precision, "airy256_512 sampled")
    # whole-grid property: the on-axis pattern is symmetric under x -> -x and y -> -y
    scale = np.abs(E).max()
    assert np.abs(E - E[:, ::-1]).max() <= 4 * TOL[precision] * scale
    assert np.abs(E - E[::-1, :]).max() <= 4 * TOL[precision] * scale


_ZERN_REF = {}


def zern_dense_reference(sc):
    """The oracle on every 8th pixel row of the 1024 x 1024 tilted plane
    (131,072 pixels x 12,892 beamlets), computed once for both precisions."""
    if "ref" not in _ZERN_REF:
        rows = np.arange(0, sc.plane.ny, 8)
        iy, ix = np.meshgrid(rows, np.arange(sc.plane.nx), indexing="ij")
        ix, iy = ix.ravel().astype(np.int32), iy.ravel().astype(np.int32)
        _ZERN_REF["ref"] = (ix, iy, oracle.eval_field(sc, pixels=(ix, iy)))
    return _ZERN_REF["ref"]


@pytest.mark.parametrize("precision", BOTH)
def test_zern128_1024_full_size_sampled(ctx, precision):
    """12,892 aberrated beamlets on a 1024 x 1024 tilted plane in the
    benchmark's launch shape: random pixels and every 8th row against the
    oracle."""
    sc = scenes.config("zern128_1024")
    E = run(ctx, sc, precision)
    ix, iy = sample_pixels(1024, 1024, 200, 2)
    ref = oracle.eval_field(sc, pixels=(ix, iy))
    check(E[iy, ix], ref, precision, "zern128_1024 sampled")
    ix, iy, ref = zern_dense_reference(sc)
    check(E[iy, ix], ref, precision, "zern128_1024 every 8th row")
    assert np.isfinite(E).all()


def test_plan_reuse_and_shape(ctx):
    import torch
    sc = scenes.config("airy32_64")
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.gbd_plan_create(ctx, sc.n)
    plan.setup(b, p)
    shp = plan.shape(gbd.GBD_MIXED)
    assert shp["rows_per_lane"] in (1, 2, 4, 8, 16, 32, 64) and shp["segments"] >= 1
    E1 = plan.eval(gbd.GBD_FP64)
    E2 = plan.eval(gbd.GBD_FP64, opts=dict(rows_per_lane=2, waves=1, segments=5))
    torch.cuda.synchronize()
    ref = oracle.eval_field(sc)
    check(E1.cpu().numpy(), ref, gbd.GBD_FP64, "plan default")
    check(E2.cpu().numpy(), ref, gbd.GBD_FP64, "plan 2x1x5")


def test_edge_cases(ctx):
    import torch
    # empty decomposition: zero field
    sc = scenes.airy_scene(8, npix=5)
    empty = scenes.Scene(sc.lam, sc.l0, np.zeros((0, 2)), np.zeros((0, 2)), np.zeros(0) + 1e-3,
                         np.zeros((0, 2)), np.zeros(0), sc.abcd, sc.plane)
    for prec in BOTH:
        E = run(ctx, empty, prec)
        assert E.shape == (5, 5) and not np.any(E)
    # one pixel, one beamlet; 65 x 1 strip; 1 x 70 column
    for nx, ny in ((1, 1), (65, 1), (1, 70)):
        s = scenes.zernike_scene(8, n_across=6, npix=8, half_span=20e-6)
        s.plane.nx, s.plane.ny = nx, ny
        ref = oracle.eval_field(s)
        for prec in BOTH:
            check(run(ctx, s, prec), ref, prec, f"{nx}x{ny}")
    one = scenes.airy_scene(1, npix=16, half_span_lamF=1.0)
    assert one.n == 1
    for prec in BOTH:
        check(run(ctx, one, prec), oracle.eval_field(one), prec, "single beamlet")
    # every pixel of this grid lies 50 or more e-folds below the spot's peak:
    # FP64 keeps its bar; the mixed form's FP32 log2-amplitude carries an
    # absolute error ~ eps * |log2 amplitude|, so its bound there is 1e-3
    tail = scenes.airy_scene(1, npix=16, half_span_lamF=30.0)
    ref = oracle.eval_field(tail)
    check(run(ctx, tail, gbd.GBD_FP64), ref, gbd.GBD_FP64, "far tail")
    E = run(ctx, tail, gbd.GBD_MIXED)
    assert np.isfinite(E).all() and rel_l2(E, ref) < 1e-3
    # zero-size plane writes nothing and succeeds
    z = scenes.airy_scene(8, npix=4)
    b = gbd.beamlets_from_scene(ctx, z)
    p = gbd.gbd_plane(ctx, z.plane.origin, z.plane.normal, z.plane.xhint, 0, 7, 1e-6, 1e-6)
    out = torch.empty((7, 0), dtype=torch.complex64, device="cuda")
    gbd.gbd_eval(ctx, b, p, gbd.GBD_MIXED, out=out)


def test_errors_are_reported_before_any_write(ctx):
    import torch
    sc = scenes.airy_scene(8, npix=4)
    bad = sc.abcd.copy()
    bad[0, 1] = 0.3
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_beamlets(ctx, sc.n, sc.lam, sc.l0, sc.r1, sc.th1, sc.w0, sc.amp, sc.path, bad)
    assert e.value.code == -2
    w0 = sc.w0.copy()
    w0[2] = -1.0
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_beamlets(ctx, sc.n, sc.lam, sc.l0, sc.r1, sc.th1, w0, sc.amp, sc.path, sc.abcd)
    assert e.value.code == -1
    r1 = sc.r1.copy()
    r1[1, 1] = np.inf
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_beamlets(ctx, sc.n, sc.lam, sc.l0, r1, sc.th1, sc.w0, sc.amp, sc.path, sc.abcd)
    assert e.value.code == -1
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_plane(ctx, [0, 0, 0], [0, 0, 1], [0, 0, 2], 4, 4, 1e-6, 1e-6)
    assert e.value.code == -1
    # plane containing an on-axis base ray
    b1 = gbd.gbd_beamlets(ctx, 1, 1e-6, 0.1, [[0.0, 0.0]], None, [1e-3], None, None,
                          scenes.lens_then_distance(0.1, 0.1))
    side = gbd.gbd_plane(ctx, [0, 0, 0], [1, 0, 0], [0, 1, 0], 4, 4, 1e-6, 1e-6)
    sentinel = torch.full((4, 4), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_eval(ctx, b1, side, gbd.GBD_MIXED, out=sentinel)
    assert e.value.code == -4
    # inverting relay: eigenvalue on the branch cut
    binv = gbd.gbd_beamlets(ctx, sc.n, sc.lam, sc.l0, sc.r1, sc.th1, sc.w0, sc.amp, sc.path, -np.eye(4))
    p = gbd.plane_from_scene(ctx, sc)
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_eval(ctx, binv, p, gbd.GBD_MIXED, out=sentinel)
    assert e.value.code == -3
    torch.cuda.synchronize()
    assert bool((sentinel == (7.0 + 7.0j)).all())
    # output buffer too small; unknown mixed form
    good = gbd.beamlets_from_scene(ctx, sc)
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_eval(ctx, good, p, gbd.GBD_MIXED, out=sentinel, opts=dict(variant=6))
    assert e.value.code == -1
    small = torch.empty((3, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(gbd.GbdError) as e:
        load = gbd.load_library()
        import ctypes
        rc = load.gbd_eval(ctx.handle, good.handle, p.handle, gbd.GBD_FP64, ctypes.c_void_p(small.data_ptr()),
                           small.numel() * 16, None)
        gbd._check(rc)
    assert e.value.code == -7


def test_point_evaluation_matches_oracle_exact_model(ctx):
    """Paraxial point evaluation on a tilted, aberrated plane against the
    oracle's exact per-pixel model (1e-12); on an untilted plane it equals
    plane evaluation."""
    import torch
    sc = scenes.zernike_scene(2404, n_across=24, npix=72, half_span=50e-6)
    sc.plane.ny = 45
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    E = gbd.gbd_eval_point(ctx, b, p).cpu().numpy()
    check(E, oracle.eval_field(sc, model=1), gbd.GBD_FP64, "point tilted")
    flat = scenes.zernike_scene(2404, n_across=24, npix=40, half_span=30e-6, tilt_deg=0.0)
    bf = gbd.beamlets_from_scene(ctx, flat)
    pf = gbd.plane_from_scene(ctx, flat)
    Ep = gbd.gbd_eval_point(ctx, bf, pf).cpu().numpy()
    Epl = gbd.gbd_eval(ctx, bf, pf, gbd.GBD_FP64)
    torch.cuda.synchronize()
    assert rel_l2(Ep, Epl.cpu().numpy()) < 1e-12
    # the plane expansion's error on the tilted grid, measured on the GPU
    Epl_t = gbd.gbd_eval(ctx, b, p, gbd.GBD_FP64)
    torch.cuda.synchronize()
    print("tilted-plane model error vs point evaluation", rel_l2(Epl_t.cpu().numpy(), E), flush=True)
    assert rel_l2(Epl_t.cpu().numpy(), E) < 2e-3


def test_pooled_beamlet_blocks_and_foreign_handles(ctx):
    """A freed beamlet handle's device block serves the context's next handle
    of the same size class (the upload lands after every kernel that read
    the old contents): fields after such reuse equal those of a fresh
    context bit for bit and match the oracle; a handle used with another
    context is refused before anything runs."""
    import torch
    a = scenes.airy_scene(40, npix=96, npix_y=80, half_span_lamF=6.0)
    b = scenes.airy_scene(40, OF=1.3, q=0.8, npix=96, npix_y=80, half_span_lamF=6.0)
    assert a.n == b.n
    p = gbd.plane_from_scene(ctx, b)
    fields = []
    for _ in range(3):
        ba = gbd.beamlets_from_scene(ctx, a)
        gbd.gbd_eval(ctx, ba, gbd.plane_from_scene(ctx, a), gbd.GBD_MIXED)
        del ba  # its block returns to the pool while the evaluation may still run
        bb = gbd.beamlets_from_scene(ctx, b)
        fields.append(gbd.gbd_eval(ctx, bb, p, gbd.GBD_MIXED))
        del bb
    fresh = gbd.Context(0)
    ref_gpu = gbd.gbd_eval(fresh, gbd.beamlets_from_scene(fresh, b), gbd.plane_from_scene(fresh, b), gbd.GBD_MIXED)
    torch.cuda.synchronize()
    for F in fields:
        assert torch.equal(F.cpu().view(torch.float32), ref_gpu.cpu().view(torch.float32))
    ref = oracle.eval_field(b)
    assert rel_l2(fields[-1].cpu().numpy().astype(np.complex128), ref) < 1e-5
    foreign = gbd.beamlets_from_scene(fresh, b)
    sentinel = torch.full((80, 96), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_eval(ctx, foreign, p, gbd.GBD_MIXED, out=sentinel)
    assert e.value.code == -1
    with pytest.raises(gbd.GbdError) as e:
        gbd.Plan(ctx, b.n).setup(foreign, p)
    assert e.value.code == -1
    torch.cuda.synchronize()
    assert bool((sentinel == (7.0 + 7.0j)).all())


def test_eval_launched_ahead_of_the_setup_status():
    """After a successful call gbd_eval launches the next evaluation behind
    its setup with the previous form and FP16 scale, before reading the new
    status.  Across calls that keep them, change the scale, change the form
    (cross terms, higher orders, FP64) or fail, every field equals a first
    call's on a fresh context bit for bit, a failing call (several segments,
    so the launch ahead reaches the guarded reduction) leaves its output
    untouched, and kernel timing keeps one pair per evaluation."""
    import torch
    seg = dict(segments=4)
    airy = scenes.airy_scene(40, npix=96, npix_y=80, half_span_lamF=6.0)
    small = scenes.airy_scene(24, npix=64, half_span_lamF=6.0)
    cases = [(airy, gbd.GBD_MIXED, None),
             (airy, gbd.GBD_MIXED, None),                      # same form and scale: launched ahead
             (scenes.airy_scene(40, OF=1.3, q=0.8, npix=96, npix_y=80, half_span_lamF=6.0), gbd.GBD_MIXED, None),
             (scenes.zernike_scene(5, n_across=12, npix=48), gbd.GBD_MIXED, seg),   # cross terms
             (scenes.hermite_scene(12, npix=64, half_span_lamF=8.0), gbd.GBD_MIXED, None),
             (small, gbd.GBD_FP64, seg),
             (small, gbd.GBD_MIXED, seg)]
    ctx_a = gbd.Context(0)
    ctx_a.set_kernel_timing(True)
    done = 0
    for i, (sc, prec, o) in enumerate(cases):
        b = gbd.beamlets_from_scene(ctx_a, sc)
        p = gbd.plane_from_scene(ctx_a, sc)
        E = gbd.gbd_eval(ctx_a, b, p, prec, opts=o)
        done += 1
        fresh = gbd.Context(0)
        R = gbd.gbd_eval(fresh, gbd.beamlets_from_scene(fresh, sc), gbd.plane_from_scene(fresh, sc), prec, opts=o)
        torch.cuda.synchronize()
        real = torch.float64 if prec == gbd.GBD_FP64 else torch.float32
        assert torch.equal(E.cpu().view(real), R.cpu().view(real)), i
        if i == 2:
            # an inverting relay (eigenvalue on the branch cut) between successful calls
            bad = gbd.gbd_beamlets(ctx_a, sc.n, sc.lam, sc.l0, sc.r1, sc.th1, sc.w0, sc.amp, sc.path, -np.eye(4))
            sentinel = torch.full((sc.plane.ny, sc.plane.nx), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")
            with pytest.raises(gbd.GbdError) as e:
                gbd.gbd_eval(ctx_a, bad, p, gbd.GBD_MIXED, out=sentinel, opts=seg)
            assert e.value.code == -3
            torch.cuda.synchronize()
            assert bool((sentinel == (7.0 + 7.0j)).all())
    assert len(ctx_a.kernel_times()) == done


def test_eval_sequence_moves_the_status_post_between_kernels():
    """One context through a seeded random sequence of gbd_eval calls whose
    forms change from call to call: the separable form in FP16 halves at two
    FP16 scales (its evaluation kernel posts the setup status when launched
    ahead), a plane with cross terms and higher-order beamlets (the post by a
    kernel of its own, ahead of a mispredicted or other form), the FP64
    separable form, and single-segment launches (no launch ahead).  Every
    field equals a fresh context's bit for bit, and kernel timing keeps one
    duration per call."""
    import torch
    seg = dict(segments=4)
    airy = scenes.airy_scene(40, npix=96, npix_y=80, half_span_lamF=6.0)
    airy_b = scenes.airy_scene(40, OF=1.3, q=0.8, npix=96, npix_y=80, half_span_lamF=6.0)
    small = scenes.airy_scene(24, npix=64, half_span_lamF=6.0)
    cases = [(airy, gbd.GBD_MIXED, seg),
             (airy, gbd.GBD_MIXED, dict(segments=1)),
             (airy_b, gbd.GBD_MIXED, seg),
             (scenes.zernike_scene(5, n_across=12, npix=48), gbd.GBD_MIXED, seg),
             (scenes.hermite_scene(12, npix=64, half_span_lamF=8.0), gbd.GBD_MIXED, seg),
             (small, gbd.GBD_FP64, seg)]
    want = []
    for sc, prec, o in cases:
        fresh = gbd.Context(0)
        want.append(gbd.gbd_eval(fresh, gbd.beamlets_from_scene(fresh, sc), gbd.plane_from_scene(fresh, sc), prec,
                                 opts=o))
    rng = np.random.default_rng(2404)
    order = [int(i) for i in rng.integers(0, len(cases), 30)] + [0, 0, 2, 2, 0, 5, 5, 3, 3, 0, 4, 4, 0]
    ctx_a = gbd.Context(0)
    handles = [(gbd.beamlets_from_scene(ctx_a, sc), gbd.plane_from_scene(ctx_a, sc)) for sc, _, _ in cases]
    ctx_a.set_kernel_timing(True)
    got = []
    for i in order:
        b, p = handles[i]
        _, prec, o = cases[i]
        got.append(gbd.gbd_eval(ctx_a, b, p, prec, opts=o))
    torch.cuda.synchronize()
    for k, (i, E) in enumerate(zip(order, got)):
        real = torch.float64 if cases[i][1] == gbd.GBD_FP64 else torch.float32
        assert torch.equal(E.cpu().view(real), want[i].cpu().view(real)), (k, i)
    assert len(ctx_a.kernel_times()) == len(order)


def test_context_on_streams_of_its_own():
    """A context bound to a stream of its own, then rebound to another: the
    evaluations on either stream (the launch ahead of the status included)
    and a beamlet handle created after the switch in a block freed before it
    give the fields of a default context bit for bit."""
    import torch
    a = scenes.airy_scene(40, npix=96, npix_y=80, half_span_lamF=6.0)
    b = scenes.airy_scene(40, OF=1.3, q=0.8, npix=96, npix_y=80, half_span_lamF=6.0)
    ref = gbd.Context(0)
    want = {}
    for name, sc in (("a", a), ("b", b)):
        want[name] = gbd.gbd_eval(ref, gbd.beamlets_from_scene(ref, sc), gbd.plane_from_scene(ref, sc), gbd.GBD_MIXED)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ctx = gbd.Context(0, stream=s1)
    ba = gbd.beamlets_from_scene(ctx, a)
    pa = gbd.plane_from_scene(ctx, a)
    got = [gbd.gbd_eval(ctx, ba, pa, gbd.GBD_MIXED) for _ in range(2)]
    del ba  # its block waits in the pool; the switch below drains s1 first
    ctx.set_stream(s2)
    bb = gbd.beamlets_from_scene(ctx, b)
    got_b = [gbd.gbd_eval(ctx, bb, gbd.plane_from_scene(ctx, b), gbd.GBD_MIXED) for _ in range(2)]
    torch.cuda.synchronize()
    for E in got:
        assert torch.equal(E.cpu().view(torch.float32), want["a"].cpu().view(torch.float32))
    for E in got_b:
        assert torch.equal(E.cpu().view(torch.float32), want["b"].cpu().view(torch.float32))
