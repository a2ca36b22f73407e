"""Pins of the oracle's higher-order (elegant Hermite-Gaussian) beamlets, one
of the Collins-integral solutions Sec. 2.1 names as usable in beamlet
decomposition.  A beamlet of orders (m, n) launches
    H_m(u_x) H_n(u_y) e^(-|u|^2) e^(-i k th1 . (r - r1)),  u = (r - r1) / w0,
and is carried as the Gaussian beamlet's field times a polynomial in the
offset from the base ray.  Every pin below is independent of that
construction:

H1  identity system: the launched field itself (Hermite polynomials from scipy)
H2  free space: the textbook elegant Hermite-Gaussian beam,
    prod (q0/q)^((m+1)/2) H_m(x sqrt(i k / 2q)) e^(-i k x^2 / 2q)
H3  lens + distance, decentred and tilted: 1-D quadrature of the Collins
    integral of the launched field, per axis
H4  rotated cylindrical + spherical lens (non-diagonal blocks, so the cross
    term of the second-derivative matrix matters): 2-D quadrature of the
    Collins integral
H5  energy through a general astigmatic system equals the launched energy,
    sqrt(pi/2) w0 c_m per axis with c_0 = c_1 = 1, c_2 = 3
H6  input validation: orders outside 0..2, a plane tilted against the axis
"""
import math

import numpy as np
import pytest
import scipy.special

import oracle
from paper_2404_12454_amd import scenes

ORDERS = [(0, 1), (1, 0), (1, 1), (2, 0), (0, 2), (2, 1), (1, 2), (2, 2)]


def hg_scene(lam, w0, abcd, order, r1=(0.0, 0.0), th1=(0.0, 0.0), W=0.0, amp=(1.0, 0.0),
             origin=(0.0, 0.0, 0.0), normal=(0.0, 0.0, 1.0), npix=16, dx=1e-6):
    plane = scenes.Plane(np.array(origin, float), np.array(normal, float), np.array([1.0, 0, 0]),
                         npix, npix, dx, dx)
    sc = scenes.Scene(lam, 0.0, np.array([r1], float), np.array([th1], float), np.array([w0], float),
                      np.array([amp], float), np.array([W], float), np.asarray(abcd, float).reshape(1, 16), plane)
    sc.order = np.array([order], np.int32)
    return sc


def coords(pl):
    a = (np.arange(pl.nx) - (pl.nx - 1) / 2.0) * pl.dx + pl.origin[0]
    b = (np.arange(pl.ny) - (pl.ny - 1) / 2.0) * pl.dy + pl.origin[1]
    return np.meshgrid(a, b, indexing="xy")


def hermite(m, u):
    """Physicists' Hermite polynomial H_m (numpy's series form takes complex u)."""
    if np.iscomplexobj(u):
        return np.polynomial.hermite.hermval(u, [0.0] * m + [1.0])
    return scipy.special.eval_hermite(m, u)


def free_space(d):
    return scenes.lens_then_distance(1e300, d)


def launched(X, Y, order, r1, th1, w0, lam):
    k = 2 * math.pi / lam
    u, v = (X - r1[0]) / w0, (Y - r1[1]) / w0
    return hermite(order[0], u) * hermite(order[1], v) * np.exp(-(u * u + v * v)) \
        * np.exp(-1j * k * (th1[0] * (X - r1[0]) + th1[1] * (Y - r1[1])))


# ---------------------------------------------------------------- H1 ----------
@pytest.mark.parametrize("order", ORDERS)
def test_h1_identity_system_returns_the_launched_field(order):
    lam, w0 = 0.8e-6, 40e-6
    r1, th1 = (7e-6, -5e-6), (2e-3, -1e-3)
    sc = hg_scene(lam, w0, np.eye(4), order, r1=r1, th1=th1, npix=24, dx=8e-6)
    E = oracle.eval_field(sc)
    X, Y = coords(sc.plane)
    ref = launched(X, Y, order, r1, th1, w0, lam)
    assert np.abs(E - ref).max() < 1e-12 * np.abs(ref).max()


def test_h1_order_zero_is_the_gaussian_beamlet():
    lam, w0 = 1e-6, 0.3e-3
    M = scenes.lens_then_distance(0.2, 0.15)
    sc = hg_scene(lam, w0, M, (0, 0), r1=(1e-4, 2e-4), th1=(1e-3, 0.0), dx=10e-6)
    E = oracle.eval_field(sc)
    sc.order = None
    assert np.array_equal(E, oracle.eval_field(sc))


# ---------------------------------------------------------------- H2 ----------
@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("z", [0.03, 0.5, 3.0])
def test_h2_free_space_elegant_hermite_gaussian(order, z):
    lam, w0 = 1e-6, 0.3e-3
    k = 2 * math.pi / lam
    zR = math.pi * w0 ** 2 / lam
    q0, q = 1j * zR, z + 1j * zR
    wz = w0 * math.sqrt(1 + (z / zR) ** 2)
    sc = hg_scene(lam, w0, free_space(z), order, npix=20, dx=4 * wz / 20)
    E = oracle.eval_field(sc)
    X, Y = coords(sc.plane)
    alpha = np.sqrt(1j * k / (2 * q))
    s = np.sqrt(q0 / q)
    turns = z / lam - round(z / lam)      # e^(-i k z), reduced before scaling by 2 pi
    ref = np.exp(-2j * math.pi * turns) * s ** (order[0] + 1) * s ** (order[1] + 1) \
        * hermite(order[0], alpha * X) * hermite(order[1], alpha * Y) * np.exp(-1j * k * (X * X + Y * Y) / (2 * q))
    assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-12


# ---------------------------------------------------------------- H3 ----------
def collins_1d_hg(x2, m, x1c, w0, th, A, B, D, lam, npts=40001, span=12):
    """sqrt(i / (lam B)) * integral of the launched 1-D field
    H_m(u) e^(-u^2) e^(-i k th (x - x1c)), u = (x - x1c) / w0, against the
    Collins kernel e^(-i k/2 [A/B x^2 - 2 x x2 / B + D/B x2^2]), trapezoid rule."""
    k = 2 * math.pi / lam
    x = np.linspace(x1c - span * w0, x1c + span * w0, npts)
    h = x[1] - x[0]
    u = (x - x1c) / w0
    g = hermite(m, u) * np.exp(-u * u - 1j * k * th * (x - x1c))
    out = np.empty(len(x2), complex)
    for i, xx in enumerate(x2):
        kern = np.exp(-0.5j * k * (A / B * x * x - 2 * x * xx / B + D / B * xx * xx))
        out[i] = np.sum(g * kern) * h
    return out * np.sqrt(1j / (lam * B))


@pytest.mark.parametrize("order", [(1, 0), (2, 1), (0, 2), (2, 2)])
@pytest.mark.parametrize("d", [0.23, 0.2])
def test_h3_lens_distance_collins_quadrature(order, d):
    """Lens f = 0.2 m then d (d = f: the focal plane, where the beamlet is
    the Fourier transform of the launched field), decentred and tilted."""
    lam, w0, f = 0.8e-6, 0.5e-3, 0.2
    k = 2 * math.pi / lam
    M = scenes.lens_then_distance(f, d)
    A, B, D = M[0, 0], M[0, 2], M[2, 2]
    x1, y1, tx, ty, W = 0.7e-3, -0.4e-3, 1.5e-3, -0.8e-3, 0.3e-6
    r2 = (A * x1 + B * tx, A * y1 + B * ty)
    spot = max(w0 * abs(A), lam * B / (math.pi * w0)) * 3
    sc = hg_scene(lam, w0, M, order, r1=(x1, y1), th1=(tx, ty), W=W, origin=(r2[0], r2[1], 0), npix=12,
                  dx=2 * spot / 12)
    E = oracle.eval_field(sc)
    X, Y = coords(sc.plane)
    Ix = collins_1d_hg(X[0], order[0], x1, w0, tx, A, B, D, lam)
    Iy = collins_1d_hg(Y[:, 0], order[1], y1, w0, ty, A, B, D, lam)
    ref = np.exp(-1j * k * W) * Iy[:, None] * Ix[None, :]
    assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-10


# ---------------------------------------------------------------- H4 ----------
@pytest.mark.parametrize("order", [(1, 1), (2, 1), (2, 2)])
def test_h4_nonseparable_system_2d_quadrature(order):
    lam, w0 = 1e-6, 0.25e-3
    k = 2 * math.pi / lam
    th = 0.4
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    C = -np.eye(2) / 0.5 - R @ np.diag([1 / 0.8, 0]) @ R.T
    d = 0.12
    M = np.block([[np.eye(2) + d * C, d * np.eye(2)], [C, np.eye(2)]])
    r1, th1 = (0.3e-3, 0.1e-3), (0.5e-3, -0.2e-3)
    r2 = M[:2, :2] @ r1 + M[:2, 2:] @ th1
    sc = hg_scene(lam, w0, M, order, r1=r1, th1=th1, amp=(0.5, 0.5), origin=(r2[0], r2[1], 0.0), npix=8,
                  dx=40e-6)
    E = oracle.eval_field(sc)
    n = 801
    x = np.linspace(-2.4e-3, 2.4e-3, n)
    h = x[1] - x[0]
    X1, Y1 = np.meshgrid(x, x, indexing="xy")
    E1 = (0.5 + 0.5j) * launched(X1, Y1, order, r1, th1, w0, lam)
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
            ref[iy, ix] = pref * np.sum(E1 * np.exp(-1j * k * S)) * h * h
    assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-9


# ---------------------------------------------------------------- H5 ----------
@pytest.mark.parametrize("seed,order", [(0, (1, 2)), (1, (2, 2)), (2, (2, 0))])
def test_h5_energy_through_astigmatic_system(seed, order):
    rng = np.random.default_rng(seed)
    Hm = rng.normal(size=(2, 2)) * 8.0
    Hm = 0.5 * (Hm + Hm.T)
    M = free_space(rng.uniform(0.02, 0.3)) @ scenes.thin_plate(Hm)
    lam, w0 = 1e-6, 0.3e-3
    r1, th1 = (1e-4, -2e-4), (1e-3, 0.0)
    b = oracle.beamlet(lam, r1, th1, w0, 0.0, M)
    Wm = np.linalg.inv(-b["Qinv"].imag * math.pi / lam)
    ext = 8 * math.sqrt(np.linalg.eigvalsh(Wm).max())
    n = 200
    sc = hg_scene(lam, w0, M, order, r1=r1, th1=th1, amp=(0.6, 0.8), origin=(b["r2"][0], b["r2"][1], 0.0),
                  npix=n, dx=2 * ext / n)
    E = oracle.eval_field(sc)
    energy = (np.abs(E) ** 2).sum() * sc.plane.dx * sc.plane.dy
    c = {0: 1.0, 1: 1.0, 2: 3.0}
    want = (math.pi / 2) * w0 ** 2 * c[order[0]] * c[order[1]]
    assert abs(energy / want - 1) < 1e-10


# ---------------------------------------------------------------- H6 ----------
def test_h6_invalid_orders_and_tilted_plane():
    M = scenes.lens_then_distance(0.2, 0.2)
    for bad in ((3, 0), (0, -1)):
        sc = hg_scene(1e-6, 1e-3, M, bad)
        with pytest.raises(RuntimeError):
            oracle.eval_field(sc)
    # the plane-evaluation field of a higher-order beamlet is exact only on
    # planes normal to the axis; a tilted plane is refused there but point
    # evaluation (exact at every pixel) accepts it
    sc = hg_scene(1e-6, 1e-3, M, (1, 0), normal=(0.0, math.sin(0.1), math.cos(0.1)), dx=5e-6)
    with pytest.raises(RuntimeError):
        oracle.eval_field(sc)
    assert np.isfinite(oracle.eval_field(sc, model=1)).all()


def test_h6_point_evaluation_agrees_on_a_normal_plane():
    """On a plane normal to the axis the plane-evaluation field of a
    higher-order beamlet is the exact one that point evaluation computes."""
    M = scenes.lens_then_distance(0.2, 0.19)
    sc = hg_scene(1e-6, 0.4e-3, M, (2, 1), r1=(0.2e-3, 0.1e-3), th1=(0.3e-3, 0.0), dx=6e-6,
                  origin=(0.0, 0.0, 0.004))
    E0, E1 = oracle.eval_field(sc), oracle.eval_field(sc, model=1)
    assert np.linalg.norm(E0 - E1) / np.linalg.norm(E1) < 1e-12
