"""Pins of the oracle's truncated beamlets (a Gaussian beamlet whose input
envelope is cut by a straight edge, kept where e . r <= t), one of the
Collins-integral solutions Sec. 2.1 names as usable in beamlet
decomposition.  The oracle forms the propagated beamlet as the Gaussian
field times erfc(zeta) / 2 with zeta linear in the offset from the base ray;
every pin here is independent of that construction:

T1  1-D Collins quadrature of the cut input (Gauss-Legendre up to the edge)
    through lens + distance: decentred, tilted, edges on either side of the
    centre, near field, focal plane and beyond
T2  2-D Collins quadrature, oblique edge, through a rotated cylindrical +
    spherical lens (non-diagonal blocks)
T3  complementary edges (e, t) and (-e, -t) add up to the whole beamlet
T4  an edge far outside the envelope leaves the beamlet whole; one far on
    the other side removes it
T5  input validation: edge normals not of unit length, a plane tilted
    against the axis, edges combined with higher orders
"""
import math

import numpy as np
import pytest

import oracle
from paper_2404_12454_amd import scenes


def cut_scene(lam, w0, abcd, edge, r1=(0.0, 0.0), th1=(0.0, 0.0), W=0.0, amp=(1.0, 0.0),
              origin=(0.0, 0.0, 0.0), normal=(0.0, 0.0, 1.0), npix=12, dx=1e-6):
    plane = scenes.Plane(np.array(origin, float), np.array(normal, float), np.array([1.0, 0, 0]),
                         npix, npix, dx, dx)
    sc = scenes.Scene(lam, 0.0, np.array([r1], float), np.array([th1], float), np.array([w0], float),
                      np.array([amp], float), np.array([W], float), np.asarray(abcd, float).reshape(1, 16), plane)
    sc.edge = np.array([edge], float)
    return sc


def coords(pl):
    a = (np.arange(pl.nx) - (pl.nx - 1) / 2.0) * pl.dx + pl.origin[0]
    b = (np.arange(pl.ny) - (pl.ny - 1) / 2.0) * pl.dy + pl.origin[1]
    return np.meshgrid(a, b, indexing="xy")


def gauss_legendre(lo, hi, panels=400, order=24):
    """Composite Gauss-Legendre nodes and weights on [lo, hi]."""
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(lo, hi, panels + 1)
    h = np.diff(edges) / 2
    mid = (edges[:-1] + edges[1:]) / 2
    return (mid[:, None] + h[:, None] * x[None, :]).ravel(), (h[:, None] * w[None, :]).ravel()


def collins_1d(x2, x1c, w0, th, A, B, D, lam, upper=None, span=12):
    """sqrt(i / (lam B)) * integral over x <= upper (default: the whole line)
    of e^(-(x - x1c)^2 / w0^2 - i k th (x - x1c)) against the Collins kernel
    e^(-i k/2 [A/B x^2 - 2 x x2 / B + D/B x2^2])."""
    k = 2 * math.pi / lam
    hi = x1c + span * w0 if upper is None else upper
    x, wq = gauss_legendre(x1c - span * w0, hi)
    g = np.exp(-((x - x1c) / w0) ** 2 - 1j * k * th * (x - x1c)) * wq
    kern = np.exp(-0.5j * k * (A / B * x[None, :] ** 2 - 2 * x[None, :] * np.asarray(x2)[:, None] / B
                                + D / B * np.asarray(x2)[:, None] ** 2))
    return (kern * g[None, :]).sum(1) * np.sqrt(1j / (lam * B))


# ---------------------------------------------------------------- T1 ----------
@pytest.mark.parametrize("d", [0.03, 0.2, 0.23, 0.6])
@pytest.mark.parametrize("cut", [-0.7, 0.0, 0.5, 1.5])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_t1_lens_distance_collins_quadrature(d, cut, sign):
    """Edge normal +-x at t = e . c + cut w0; lens f = 0.2 m then d (d = f is
    the focal plane, 0.03 m the near field where the edge's Fresnel fringes
    show)."""
    lam, w0, f = 0.8e-6, 0.5e-3, 0.2
    k = 2 * math.pi / lam
    M = scenes.lens_then_distance(f, d)
    A, B, D = M[0, 0], M[0, 2], M[2, 2]
    x1, y1, tx, ty, W = 0.7e-3, -0.4e-3, 1.5e-3, -0.8e-3, 0.3e-6
    t = sign * x1 + cut * w0
    r2 = (A * x1 + B * tx, A * y1 + B * ty)
    spot = max(w0 * abs(A), lam * B / (math.pi * w0)) * 3
    sc = cut_scene(lam, w0, M, (sign, 0.0, t), r1=(x1, y1), th1=(tx, ty), W=W, origin=(r2[0], r2[1], 0),
                   npix=12, dx=2 * spot / 12)
    E = oracle.eval_field(sc)
    X, Y = coords(sc.plane)
    if sign > 0:
        Ix = collins_1d(X[0], x1, w0, tx, A, B, D, lam, upper=t)
    else:   # keep -x <= t: mirror the problem, x -> -x
        Ix = collins_1d(-X[0], -x1, w0, -tx, A, B, D, lam, upper=t)
    Iy = collins_1d(Y[:, 0], y1, w0, ty, A, B, D, lam)
    ref = np.exp(-1j * k * W) * Iy[:, None] * Ix[None, :]
    err = np.linalg.norm(E - ref) / np.linalg.norm(ref)
    assert err < 1e-9, err


# ---------------------------------------------------------------- T2 ----------
@pytest.mark.parametrize("angle,cut", [(0.6, 0.3), (2.2, -0.4), (-1.0, 1.0)])
def test_t2_oblique_edge_nonseparable_2d_quadrature(angle, cut):
    lam, w0 = 1e-6, 0.25e-3
    k = 2 * math.pi / lam
    th = 0.4
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    C = -np.eye(2) / 0.5 - R @ np.diag([1 / 0.8, 0]) @ R.T
    d = 0.12
    M = np.block([[np.eye(2) + d * C, d * np.eye(2)], [C, np.eye(2)]])
    r1, th1 = np.array([0.3e-3, 0.1e-3]), np.array([0.5e-3, -0.2e-3])
    e = np.array([math.cos(angle), math.sin(angle)])
    m_ = np.array([-e[1], e[0]])
    t = e @ r1 + cut * w0
    r2 = M[:2, :2] @ r1 + M[:2, 2:] @ th1
    sc = cut_scene(lam, w0, M, (e[0], e[1], t), r1=tuple(r1), th1=tuple(th1), amp=(0.5, 0.5),
                   origin=(r2[0], r2[1], 0.0), npix=8, dx=40e-6)
    E = oracle.eval_field(sc)
    # quadrature in the edge frame: u = e . (x - c) up to the edge, v along it
    u, wu = gauss_legendre(-12 * w0, t - e @ r1, panels=60, order=20)
    v = np.linspace(-12 * w0, 12 * w0, 801)
    hv = v[1] - v[0]
    U, V = np.meshgrid(u, v, indexing="ij")
    X1 = r1[0] + U * e[0] + V * m_[0]
    Y1 = r1[1] + U * e[1] + V * m_[1]
    E1 = (0.5 + 0.5j) * np.exp(-(U * U + V * V) / w0 ** 2) \
        * np.exp(-1j * k * (th1[0] * (X1 - r1[0]) + th1[1] * (Y1 - r1[1]))) * wu[:, None] * hv
    Binv = np.linalg.inv(M[:2, 2:])
    BA = Binv @ M[:2, :2]
    DB = M[2:, 2:] @ Binv
    q11 = BA[0, 0] * X1 * X1 + 2 * BA[0, 1] * X1 * Y1 + BA[1, 1] * Y1 * Y1
    pref = 1j / (lam * math.sqrt(np.linalg.det(M[:2, 2:])))
    X, Y = coords(sc.plane)
    ref = np.empty_like(E)
    for iy in range(sc.plane.ny):
        for ix in range(sc.plane.nx):
            p = np.array([X[iy, ix], Y[iy, ix]])
            cross = Binv @ p
            S = 0.5 * (q11 - 2 * (X1 * cross[0] + Y1 * cross[1]) + p @ DB @ p)
            ref[iy, ix] = pref * np.sum(E1 * np.exp(-1j * k * S))
    err = np.linalg.norm(E - ref) / np.linalg.norm(ref)
    assert err < 1e-9, err


# ---------------------------------------------------------------- T3 ----------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_t3_complementary_edges_add_to_the_whole_beamlet(seed):
    rng = np.random.default_rng(seed)
    Hm = rng.normal(size=(2, 2)) * 8.0
    Hm = 0.5 * (Hm + Hm.T)
    M = scenes.lens_then_distance(1e300, rng.uniform(0.02, 0.3)) @ scenes.thin_plate(Hm)
    lam, w0 = 1e-6, 0.3e-3
    r1, th1 = (1e-4, -2e-4), (1e-3, 0.0)
    b = oracle.beamlet(lam, r1, th1, w0, 0.0, M)
    ang = rng.uniform(-math.pi, math.pi)
    e = (math.cos(ang), math.sin(ang))
    t = e[0] * r1[0] + e[1] * r1[1] + rng.uniform(-1, 1) * w0
    kw = dict(r1=r1, th1=th1, amp=(0.6, 0.8), origin=(b["r2"][0], b["r2"][1], 0.0), npix=24, dx=20e-6)
    Ea = oracle.eval_field(cut_scene(lam, w0, M, (e[0], e[1], t), **kw))
    Eb = oracle.eval_field(cut_scene(lam, w0, M, (-e[0], -e[1], -t), **kw))
    whole = cut_scene(lam, w0, M, (0.0, 0.0, 0.0), **kw)
    Ew = oracle.eval_field(whole)
    assert np.linalg.norm(Ea + Eb - Ew) / np.linalg.norm(Ew) < 1e-12
    whole.edge = None
    assert np.array_equal(Ew, oracle.eval_field(whole))


# ---------------------------------------------------------------- T4 ----------
def test_t4_edges_far_from_the_envelope():
    lam, w0 = 1e-6, 0.3e-3
    M = scenes.lens_then_distance(0.2, 0.21)
    kw = dict(r1=(2e-4, 0.0), npix=16, dx=8e-6)
    Ew = oracle.eval_field(cut_scene(lam, w0, M, (0.0, 0.0, 0.0), **kw))
    Eo = oracle.eval_field(cut_scene(lam, w0, M, (0.6, 0.8, 0.6 * 2e-4 + 12 * w0), **kw))
    Ei = oracle.eval_field(cut_scene(lam, w0, M, (0.6, 0.8, 0.6 * 2e-4 - 12 * w0), **kw))
    assert np.linalg.norm(Eo - Ew) / np.linalg.norm(Ew) < 1e-12
    assert np.abs(Ei).max() < 1e-12 * np.abs(Ew).max()


# ---------------------------------------------------------------- T5 ----------
def test_t5_invalid_edges_and_planes():
    M = scenes.lens_then_distance(0.2, 0.2)
    with pytest.raises(RuntimeError):
        oracle.eval_field(cut_scene(1e-6, 1e-3, M, (0.6, 0.6, 0.0)))
    with pytest.raises(RuntimeError):
        oracle.eval_field(cut_scene(1e-6, 1e-3, M, (1.0, 0.0, 0.0), normal=(0.0, math.sin(0.1), math.cos(0.1))))
    sc = cut_scene(1e-6, 1e-3, M, (1.0, 0.0, 0.0))
    sc.order = np.array([[1, 0]], np.int32)
    with pytest.raises(RuntimeError):
        oracle.eval_field(sc)


# ---------------------------------------------------------------- T6 ----------
@pytest.mark.parametrize("n_across,OF", [(16, 1.7), (32, 1.2), (32, 2.2)])
def test_t6_cut_beamlets_at_the_rim_approach_the_airy_pattern(n_across, OF):
    """A hard-edged circular pupil decomposed with the beamlets near the rim
    cut by the rim's tangent (and the grid extended past the rim) images
    much closer to the Airy pattern (scipy's J1) than the plain
    decomposition of the same pupil, OF and count: what truncated beamlets
    are for (Sec. 7.1)."""
    from oracle import metrics as om
    plain = scenes.airy_scene(n_across, OF=OF, npix=64, half_span_lamF=8.0)
    m = plain.meta
    ref = om.airy_irradiance(plain.plane, m["D"], m["f"], plain.lam)
    E, E0 = oracle.eval_field(plain, extra_point=(0.0, 0.0))
    cut = scenes.truncated_airy_scene(n_across, OF=OF, npix=64, half_span_lamF=8.0)
    Et, Et0 = oracle.eval_field(cut, extra_point=(0.0, 0.0))
    rms_plain = om.airy_metrics(E, E0, ref)[0]
    rms_cut = om.airy_metrics(Et, Et0, ref)[0]
    assert rms_cut < rms_plain / 5, (rms_plain, rms_cut)
