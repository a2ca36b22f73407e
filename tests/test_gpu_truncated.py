"""Truncated beamlets on the GPU against the FP64 oracle: the cut beamlets'
own kernel (complex error function) beside every form of the whole ones,
FP64 and mixed, ragged grids, all beamlets cut, complementary edges, a
full-size sampled case, the Airy improvement, and the refusals."""
import numpy as np
import pytest

import oracle
import paper_2404_12454_amd as gbd
from oracle import metrics as om
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


SCENES = {
    "focal": dict(n_across=20, npix=100, npix_y=77, half_span_lamF=8.0),
    "defocus": dict(n_across=20, npix=100, npix_y=77, half_span_lamF=14.0, z0=2e-3),
    "wide_reach": dict(n_across=14, npix=90, npix_y=70, half_span_lamF=10.0, reach=2.5, OF=2.2),
}


@pytest.mark.parametrize("precision", [gbd.GBD_FP64, gbd.GBD_MIXED])
@pytest.mark.parametrize("name", list(SCENES))
def test_truncated_beamlets_match_oracle(ctx, name, precision):
    sc = scenes.truncated_airy_scene(**SCENES[name])
    ref = oracle.eval_field(sc)
    E = field(ctx, sc, precision)
    err = rel_l2(E, ref)
    print(f"truncated {name} precision {precision}: n {sc.n}, cut {sc.meta['n_cut']}: rel_l2 {err:.2e}", flush=True)
    assert err < TOL[precision]


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
@pytest.mark.parametrize("rows,waves,segments", [(1, 1, 1), (4, 2, 3), (16, 4, 2), (32, 4, 5)])
def test_whole_beamlet_forms_beside_the_cut_kernel(ctx, variant, rows, waves, segments):
    sc = scenes.truncated_airy_scene(14, npix=90, npix_y=70, half_span_lamF=8.0)
    ref = oracle.eval_field(sc)
    E = field(ctx, sc, gbd.GBD_MIXED, dict(rows_per_lane=rows, waves=waves, segments=segments, variant=variant))
    assert rel_l2(E, ref) < 1e-5


@pytest.mark.parametrize("rows,waves,segments", [(1, 1, 1), (4, 4, 3), (8, 2, 1)])
def test_fp64_shapes_beside_the_cut_kernel(ctx, rows, waves, segments):
    sc = scenes.truncated_airy_scene(14, npix=90, npix_y=70, half_span_lamF=8.0, z0=1e-3)
    ref = oracle.eval_field(sc)
    E = field(ctx, sc, gbd.GBD_FP64, dict(rows_per_lane=rows, waves=waves, segments=segments))
    assert rel_l2(E, ref) < 1e-12


def test_every_beamlet_cut_and_complementary_edges(ctx):
    """No whole beamlets (the cut kernel alone), and edges (e, t), (-e, -t)
    adding up to the whole beamlets."""
    sc = scenes.airy_scene(10, npix=48, npix_y=40, half_span_lamF=6.0)
    rng = np.random.default_rng(3)
    ang = rng.uniform(-np.pi, np.pi, sc.n)
    e = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    t = (e * sc.r1).sum(1) + rng.uniform(-1, 1, sc.n) * sc.w0[0]
    whole = field(ctx, sc, gbd.GBD_FP64)
    for prec in (gbd.GBD_FP64, gbd.GBD_MIXED):
        sc.edge = np.column_stack([e, t])
        Ea = field(ctx, sc, prec)
        assert rel_l2(Ea, oracle.eval_field(sc)) < TOL[prec]
        sc.edge = np.column_stack([-e, -t])
        Eb = field(ctx, sc, prec)
        assert rel_l2(Ea + Eb, whole) < TOL[prec] * 2
    sc.edge = None


@pytest.mark.parametrize("precision", [gbd.GBD_FP64, gbd.GBD_MIXED])
def test_zero_edges_are_the_whole_beamlets_bitwise(ctx, precision):
    import torch
    sc = scenes.airy_scene(16, npix=80)
    p = gbd.plane_from_scene(ctx, sc)
    bt = gbd.gbd_beamlets_truncated(ctx, sc.n, sc.lam, sc.l0, sc.r1, sc.th1, sc.w0, sc.amp, sc.path, sc.abcd,
                                    np.zeros((sc.n, 3)))
    bg = gbd.beamlets_from_scene(ctx, sc)
    Et = gbd.gbd_eval(ctx, bt, p, precision)
    Eg = gbd.gbd_eval(ctx, bg, p, precision)
    torch.cuda.synchronize()
    assert torch.equal(Et.cpu(), Eg.cpu())


@pytest.mark.parametrize("precision", [gbd.GBD_FP64, gbd.GBD_MIXED])
def test_truncated_full_size_sampled(ctx, precision):
    """256 across with the rim cut (51,468 + rim beamlets) on 512 x 512,
    default launch shapes, against the oracle at sampled pixels."""
    sc = scenes.truncated_airy_scene(256, npix=512, half_span_lamF=20.0)
    E = field(ctx, sc, precision)
    rng = np.random.default_rng(6)
    ix = np.concatenate([rng.integers(0, 512, 120), [0, 511, 256]]).astype(np.int32)
    iy = np.concatenate([rng.integers(0, 512, 120), [511, 0, 256]]).astype(np.int32)
    ref = oracle.eval_field(sc, pixels=(ix, iy))
    err = rel_l2(E[iy, ix], ref)
    print(f"truncated 256 across ({sc.n} beamlets, {sc.meta['n_cut']} cut), precision {precision}: "
          f"rel_l2 {err:.2e}", flush=True)
    assert err < TOL[precision]
    assert np.isfinite(E).all()


def test_cut_rim_images_closer_to_airy(ctx):
    """On the GPU, 64 across at 256 x 256 over +-8 lambda F: the cut rim's
    RMS error against the Airy pattern is far below the plain grid's."""
    res = {}
    for kind in ("plain", "cut"):
        sc = (scenes.airy_scene(64, OF=1.2, npix=256, half_span_lamF=8.0) if kind == "plain" else
              scenes.truncated_airy_scene(64, OF=1.2, npix=256, half_span_lamF=8.0))
        m = sc.meta
        E = field(ctx, sc, gbd.GBD_MIXED)
        one = scenes.Plane(sc.plane.origin, sc.plane.normal, sc.plane.xhint, 1, 1, 1e-6, 1e-6)
        import copy
        s1 = copy.copy(sc)
        s1.plane = one
        E0 = complex(field(ctx, s1, gbd.GBD_FP64)[0, 0])
        ref = om.airy_irradiance(sc.plane, m["D"], m["f"], sc.lam)
        res[kind] = om.airy_metrics(E, E0, ref)
    print(f"RMS vs Airy, 64 across OF 1.2: plain {res['plain'][0]:.3e}, cut rim {res['cut'][0]:.3e}", flush=True)
    assert res["cut"][0] < res["plain"][0] / 10


def test_truncated_refusals(ctx):
    sc = scenes.truncated_airy_scene(8, npix=16)
    b = gbd.beamlets_from_scene(ctx, sc)
    t = np.radians(3.0)
    tilted = gbd.gbd_plane(ctx, [0, 0, 0], [0, np.sin(t), np.cos(t)], [1, 0, 0], 16, 16, 1e-6, 1e-6)
    for prec in (gbd.GBD_FP64, gbd.GBD_MIXED):
        with pytest.raises(gbd.GbdError) as e:
            gbd.gbd_eval(ctx, b, tilted, prec)
        assert e.value.code == -1
    bad = sc.edge.copy()
    bad[5, :2] = (0.6, 0.7)
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_beamlets_truncated(ctx, sc.n, sc.lam, sc.l0, sc.r1, sc.th1, sc.w0, sc.amp, sc.path, sc.abcd, bad)
    assert e.value.code == -1 and "edge[5]" in str(e.value)
    p = gbd.plane_from_scene(ctx, sc)
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_eval_point(ctx, b, p)
    assert e.value.code == -1
    with pytest.raises(gbd.GbdError) as e:
        gbd.gbd_eval_batch(ctx, [b], [p], fields=True)
    assert e.value.code == -1
