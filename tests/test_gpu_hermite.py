"""Higher-order (elegant Hermite-Gaussian) beamlets on the GPU against the
FP64 oracle: FP64 and mixed precision, the direct, rotor and separable mixed
forms in every launch shape, ragged grids, a full-size sampled case, and the
refusals (tilted planes, orders outside 0..2, point evaluation and the
batched sweep)."""
import numpy as np
import pytest

import oracle
import paper_2404_12454_amd as gbd
from paper_2404_12454_amd import scenes

from gbd_testutil import ensure_library, rel_l2

pytestmark = pytest.mark.gpu

TOL = {gbd.GBD_FP64: 1e-12, gbd.GBD_MIXED: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    ensure_library()
    return gbd.Context(0)


def field(ctx, sc, precision, opts=None):
    import torch
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    E = gbd.gbd_eval(ctx, b, p, precision, opts=opts)
    torch.cuda.synchronize()
    return E.cpu().numpy().astype(np.complex128)


def resolved_variant(ctx, sc, opts=None, precision=gbd.GBD_MIXED):
    b = gbd.beamlets_from_scene(ctx, sc)
    p = gbd.plane_from_scene(ctx, sc)
    plan = gbd.Plan(ctx, sc.n).setup(b, p)
    return plan.shape(precision, opts)["variant"]


SCENES = {
    # rotationally symmetric: no cross terms, the separable form applies
    "focal": dict(n_across=20, npix=100, npix_y=77),
    "defocus": dict(n_across=20, npix=100, npix_y=77, z0=2e-3, half_span_lamF=14.0),
    # rotated cylindrical lens: non-diagonal blocks, rotor form
    "astig": dict(n_across=20, npix=100, npix_y=77, cyl_f=3.0, half_span_lamF=12.0),
    # astigmatic and defocused: the rotor form over broad spots
    "astig_defocus": dict(n_across=20, npix=100, npix_y=77, cyl_f=3.0, half_span_lamF=16.0, z0=1.5e-3),
}


@pytest.mark.parametrize("precision", [gbd.GBD_FP64, gbd.GBD_MIXED])
@pytest.mark.parametrize("name", list(SCENES))
def test_hermite_beamlets_match_oracle(ctx, name, precision):
    sc = scenes.hermite_scene(**SCENES[name])
    ref = oracle.eval_field(sc)
    E = field(ctx, sc, precision)
    err = rel_l2(E, ref)
    print(f"hermite {name} precision {precision}: n {sc.n} variant {resolved_variant(ctx, sc)} rel_l2 {err:.2e}",
          flush=True)
    assert err < TOL[precision]


def test_hermite_forms_resolve(ctx):
    sym = scenes.hermite_scene(12, npix=64)
    astig = scenes.hermite_scene(12, npix=64, cyl_f=3.0)
    # mixed: the separable form of higher-order beamlets in FP16 halves (4),
    # or on FP32 MFMA on request (5)
    assert resolved_variant(ctx, sym) == 4
    assert resolved_variant(ctx, sym, dict(variant=4)) == 4
    assert resolved_variant(ctx, sym, dict(variant=5)) == 5
    assert resolved_variant(ctx, astig) == 3
    # the stepped form does not carry the Hermite-Gaussian factor
    assert resolved_variant(ctx, sym, dict(variant=2)) == 1
    assert resolved_variant(ctx, sym, dict(variant=3)) == 3
    assert resolved_variant(ctx, astig, dict(variant=4)) == 3
    # FP64: separable without cross terms, else the rotor form (16 rows at
    # most with the higher-order factor)
    assert resolved_variant(ctx, sym, precision=gbd.GBD_FP64) == 4
    assert resolved_variant(ctx, astig, precision=gbd.GBD_FP64) == 3
    assert resolved_variant(ctx, astig, dict(variant=1), precision=gbd.GBD_FP64) == 1
    b = gbd.beamlets_from_scene(ctx, astig)
    plan64 = gbd.Plan(ctx, astig.n).setup(b, gbd.plane_from_scene(ctx, astig))
    assert plan64.shape(gbd.GBD_FP64, dict(rows_per_lane=32, waves=4, variant=3))["rows_per_lane"] == 16
    assert resolved_variant(ctx, sym, dict(variant=3), precision=gbd.GBD_FP64) == 3
    assert resolved_variant(ctx, sym, dict(variant=1), precision=gbd.GBD_FP64) == 1
    b = gbd.beamlets_from_scene(ctx, astig)
    plan = gbd.Plan(ctx, astig.n).setup(b, gbd.plane_from_scene(ctx, astig))
    assert plan.shape(gbd.GBD_MIXED, dict(rows_per_lane=32, waves=4, variant=3))["rows_per_lane"] == 32
    assert plan.shape(gbd.GBD_MIXED, dict(rows_per_lane=32, waves=4, variant=1))["rows_per_lane"] == 16


@pytest.mark.parametrize("variant", [1, 3, 4, 5])
@pytest.mark.parametrize("rows,waves,segments", [(1, 1, 1), (2, 2, 3), (4, 4, 2), (8, 1, 5), (16, 4, 1), (16, 2, 7),
                                                 (32, 4, 3), (32, 1, 1)])
def test_hermite_mixed_shapes(ctx, variant, rows, waves, segments):
    sc = scenes.hermite_scene(14, npix=90, npix_y=70, seed=11)
    ref = oracle.eval_field(sc)
    E = field(ctx, sc, gbd.GBD_MIXED, dict(rows_per_lane=rows, waves=waves, segments=segments, variant=variant))
    assert rel_l2(E, ref) < 1e-5


@pytest.mark.parametrize("rows,waves,segments", [(1, 1, 1), (2, 4, 3), (4, 2, 1), (8, 4, 4), (16, 4, 2), (16, 1, 5),
                                                 (32, 2, 1)])
def test_hermite_fp64_rotor_form(ctx, rows, waves, segments):
    """The FP64 rotor form with the higher-order factor's row polynomial
    (astigmatic, cross terms) in every launch shape, against the oracle and
    against the FP64 direct form."""
    sc = scenes.hermite_scene(14, npix=90, npix_y=70, seed=12, cyl_f=4.0, half_span_lamF=12.0)
    ref = oracle.eval_field(sc)
    E3 = field(ctx, sc, gbd.GBD_FP64, dict(rows_per_lane=rows, waves=waves, segments=segments, variant=3))
    E1 = field(ctx, sc, gbd.GBD_FP64, dict(variant=1))
    print(f"hermite FP64 rotor {rows}x{waves} seg {segments}: vs oracle {rel_l2(E3, ref):.2e}, "
          f"vs direct {rel_l2(E3, E1):.2e}", flush=True)
    assert rel_l2(E3, ref) < 1e-12
    assert rel_l2(E3, E1) < 1e-13


@pytest.mark.parametrize("rows,waves,segments", [(1, 1, 1), (2, 4, 3), (4, 2, 1), (8, 4, 4)])
def test_hermite_fp64_shapes(ctx, rows, waves, segments):
    sc = scenes.hermite_scene(14, npix=90, npix_y=70, seed=12, cyl_f=4.0, half_span_lamF=12.0)
    ref = oracle.eval_field(sc)
    E = field(ctx, sc, gbd.GBD_FP64, dict(rows_per_lane=rows, waves=waves, segments=segments))
    assert rel_l2(E, ref) < 1e-12


@pytest.mark.parametrize("nx,ny,seg", [(90, 70, 1), (90, 70, 3), (33, 17, 2), (130, 129, 7), (1, 1, 1)])
def test_hermite_fp64_separable_form(ctx, nx, ny, seg):
    """The FP64 separable form with the per-axis Hermite-Gaussian factors on
    ragged grids and segment counts, defocused, against the oracle and
    against the FP64 direct form."""
    sc = scenes.hermite_scene(14, npix=nx, npix_y=ny, seed=13, z0=1e-3, half_span_lamF=12.0)
    ref = oracle.eval_field(sc)
    E4 = field(ctx, sc, gbd.GBD_FP64, dict(variant=4, segments=seg))
    E1 = field(ctx, sc, gbd.GBD_FP64, dict(variant=1))
    print(f"hermite FP64 separable {nx}x{ny} seg {seg}: vs oracle {rel_l2(E4, ref):.2e}, "
          f"vs direct {rel_l2(E4, E1):.2e}", flush=True)
    assert rel_l2(E4, ref) < 1e-12
    assert rel_l2(E4, E1) < 1e-13


@pytest.mark.parametrize("precision", [gbd.GBD_FP64, gbd.GBD_MIXED])
def test_zero_orders_are_the_gaussian_beamlets_bitwise(ctx, precision):
    import torch
    sc = scenes.hermite_scene(16, npix=80)
    sc.order = np.zeros_like(sc.order)
    p = gbd.plane_from_scene(ctx, sc)
    bh = gbd.beamlets_from_scene(ctx, sc)
    bg = gbd.gbd_beamlets(ctx, sc.n, sc.lam, sc.l0, sc.r1, sc.th1, sc.w0, sc.amp, sc.path, sc.abcd)
    Eh = gbd.gbd_eval(ctx, bh, p, precision)
    Eg = gbd.gbd_eval(ctx, bg, p, precision)
    torch.cuda.synchronize()
    assert torch.equal(Eh.cpu(), Eg.cpu())


def test_single_order_beamlet_and_tiny_grids(ctx):
    """One beamlet of each order, and grids smaller than one tile."""
    for order in ((0, 1), (2, 0), (1, 2), (2, 2)):
        sc = scenes.hermite_scene(2, npix=5, npix_y=3, half_span_lamF=3.0)
        sc.order = np.array([order] * sc.n, np.int32)
        ref = oracle.eval_field(sc)
        for prec in (gbd.GBD_FP64, gbd.GBD_MIXED):
            assert rel_l2(field(ctx, sc, prec), ref) < TOL[prec], (order, prec)


@pytest.mark.parametrize("precision", [gbd.GBD_FP64, gbd.GBD_MIXED])
def test_hermite_full_size_sampled(ctx, precision):
    """51,468 higher-order beamlets (256 across) on 512 x 512, default launch
    shape, against the oracle at sampled pixels."""
    sc = scenes.hermite_scene(256, npix=512, half_span_lamF=20.0)
    E = field(ctx, sc, precision)
    rng = np.random.default_rng(5)
    ix = np.concatenate([rng.integers(0, 512, 150), [0, 511, 256]]).astype(np.int32)
    iy = np.concatenate([rng.integers(0, 512, 150), [511, 0, 256]]).astype(np.int32)
    ref = oracle.eval_field(sc, pixels=(ix, iy))
    err = rel_l2(E[iy, ix], ref)
    print(f"hermite 256 across sampled, precision {precision}: rel_l2 {err:.2e}", flush=True)
    assert err < TOL[precision]
    assert np.isfinite(E).all()


def test_hermite_refusals(ctx):
    sc = scenes.hermite_scene(8, npix=16)
    b = gbd.beamlets_from_scene(ctx, sc)
    # a plane tilted against the axis
    t = np.radians(3.0)
    tilted = gbd.gbd_plane(ctx, [0, 0, 0], [0, np.sin(t), np.cos(t)], [1, 0, 0], 16, 16, 1e-6, 1e-6)
    for prec in (gbd.GBD_FP64, gbd.GBD_MIXED):
        with pytest.raises(gbd.GbdError) as e:
            gbd.gbd_eval(ctx, b, tilted, prec)
        assert e.value.code == -1
    # orders outside 0..2
    bad = sc.order.copy()
    bad[3, 1] = 3
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_beamlets_hg(ctx, sc.n, sc.lam, sc.l0, sc.r1, sc.th1, sc.w0, sc.amp, sc.path, sc.abcd, bad)
    assert e.value.code == -1 and "order[3][1]" in str(e.value)
    bad[3, 1] = -1
    with pytest.raises(gbd.GbdError):
        gbd.gbd_beamlets_hg(ctx, sc.n, sc.lam, sc.l0, sc.r1, sc.th1, sc.w0, sc.amp, sc.path, sc.abcd, bad)
    # point evaluation and the batched sweep take fundamental beamlets only
    p = gbd.plane_from_scene(ctx, sc)
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_eval_point(ctx, b, p)
    assert e.value.code == -1
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_eval_batch(ctx, [b], [p], fields=True)
    assert e.value.code == -1
    # an empty decomposition is fine
    e0 = gbd.gbd_beamlets_hg(ctx, 0, sc.lam, sc.l0, np.zeros((0, 2)), None, [1e-3], None, None, sc.abcd, None)
    E = gbd.gbd_eval(ctx, e0, p, gbd.GBD_MIXED)
    import torch
    torch.cuda.synchronize()
    assert not E.cpu().numpy().any()


@pytest.mark.parametrize("variant", [4, 5])
def test_hermite_separable_halves_wide_spots_and_orders(ctx, variant):
    """The separable form in FP16 halves (4) against the FP32 one (5) and the
    oracle where the axis polynomials reach far: order 2 on both axes, a
    defocused plane (broad spots, large g at the grid's edge), a multi-tile
    ragged grid; the setup's bound of each factor with its polynomial keeps
    every factor inside FP16's range."""
    sc = scenes.hermite_scene(16, npix=300, npix_y=140, z0=3e-3, half_span_lamF=24.0, seed=3)
    sc.order = np.array([(2, 2)] * sc.n, np.int32)
    ref = oracle.eval_field(sc)
    assert resolved_variant(ctx, sc, dict(variant=variant)) == variant
    E = field(ctx, sc, gbd.GBD_MIXED, dict(variant=variant))
    err = rel_l2(E, ref)
    print(f"hermite (2, 2) defocused variant {variant}: rel_l2 {err:.2e}", flush=True)
    assert np.isfinite(E).all()
    assert err < 1e-5

