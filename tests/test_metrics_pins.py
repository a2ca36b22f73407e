"""Pins of the Airy figure of merit (oracle/metrics.py) against facts fixed
outside it: the textbook zeros and ring maxima of the Airy pattern, Bessel's
integral for J1 (an evaluation that shares nothing with scipy's), and fields
whose peak-normalised irradiance error has a closed form.

The figure of merit is the one of the Airy experiments (Sec. 4.2) and of the
parameter search (Sec. 6): the irradiance of the coherent sum, normalised by
its value on axis, against the Airy pattern (2 J1(v)/v)^2 of the circular
pupil, v = pi D r / (lambda f); RMS and peak of the difference over the
detector, and the RMS over annular zones.

A wrong radius scale (D/2 for D, a missing pi, lambda for lambda f) moves
the zeros; a normalisation by E(0) instead of |E(0)|^2, a signed peak or a
mean without the square root changes the closed-form answers.
"""
import math

import numpy as np
import pytest

from oracle import metrics as om
from paper_2404_12454_amd import scenes

# Airy pattern landmarks in v = pi D r / (lambda f): the zeros of J1
# (Abramowitz & Stegun, Table 9.5, j_{1,s}) and the first ring maximum at
# the first zero of J2 (j_{2,1}; the derivative of J1(v)/v is -J2(v)/v),
# whose relative irradiance Born & Wolf (Principles of Optics, Sec. 8.5.2)
# tabulate as 0.0175.
J1_ZEROS = (3.831705970207512, 7.015586669815619, 10.173468135062722)
RING1_V, RING1_I = 5.135622301840683, 0.0175


def bessel_j1(x):
    """J1 from Bessel's integral J1(x) = (1/2pi) int_{-pi}^{pi} cos(t - x sin t) dt
    (the integrand is periodic, so the trapezoid rule converges
    geometrically; 256 nodes give full FP64 accuracy for x < 40)."""
    t = -math.pi + 2 * math.pi * np.arange(256) / 256
    x = np.asarray(x, np.float64)[..., None]
    return np.mean(np.cos(t - x * np.sin(t)), axis=-1)


def radial_plane(radii, dx=None):
    """A 1-row plane whose pixels (nx odd, centred on the origin) sit at the
    given distances on the +x axis: pixel (nx-1)/2 + i is at i dx, so a
    single radius r is placed with nx = 3 and dx = r."""
    return scenes.Plane(np.zeros(3), np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]), 3, 1,
                        float(radii), float(radii))


D, F, LAM = 10e-3, 100e-3, 1e-6          # the f/10, 1 um system of the Airy workloads
LAMF = LAM * F / D                       # lambda F = 10 um


@pytest.mark.parametrize("v", J1_ZEROS)
def test_airy_irradiance_vanishes_at_the_dark_rings(v):
    """First dark ring at r = 1.2197 lambda F (v = 3.8317), then 2.2331 and
    3.2383 lambda F: the pattern must vanish there, and not a pixel off."""
    r = v / math.pi * LAMF
    a = om.airy_irradiance(radial_plane(r), D, F, LAM)
    assert a.shape == (1, 3)
    assert abs(a[0, 1] - 1.0) < 1e-15          # the origin pixel: 1 on axis
    assert a[0, 2] < 1e-20 and a[0, 0] < 1e-20  # r and -r
    # 1 % off the zero the pattern is clearly nonzero (the test resolves the scale)
    off = om.airy_irradiance(radial_plane(1.01 * r), D, F, LAM)[0, 2]
    assert off > 1e-7


def test_airy_irradiance_first_ring_maximum():
    """The first bright ring peaks at r = 1.6347 lambda F with 1.750 % of the
    central irradiance."""
    r = RING1_V / math.pi * LAMF
    assert abs(r / LAMF - 1.6347) < 1e-4
    a = om.airy_irradiance(radial_plane(r), D, F, LAM)[0, 2]
    assert abs(a - RING1_I) < 5e-6
    assert abs(a - (2 * float(bessel_j1(RING1_V)) / RING1_V) ** 2) < 1e-15
    # a maximum: both neighbours lower
    for s in (0.99, 1.01):
        assert om.airy_irradiance(radial_plane(s * r), D, F, LAM)[0, 2] < a


def test_airy_irradiance_matches_bessel_integral_on_a_grid():
    """Every pixel of a 2-D grid against (2 J1(v)/v)^2 with J1 from Bessel's
    integral, v computed from the pixel position written out here, and the
    Taylor expansion 1 - v^2/4 + 5 v^4/192 near the axis."""
    pl = scenes.Plane(np.zeros(3), np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]), 21, 17,
                      0.73 * LAMF, 0.61 * LAMF)
    a = om.airy_irradiance(pl, D, F, LAM)
    xs = (np.arange(21) - 10) * 0.73 * LAMF
    ys = (np.arange(17) - 8) * 0.61 * LAMF
    for iy, y in enumerate(ys):
        for ix, x in enumerate(xs):
            v = math.pi * D * math.hypot(x, y) / (LAM * F)
            ref = 1.0 if v == 0 else (2 * float(bessel_j1(v)) / v) ** 2
            assert abs(a[iy, ix] - ref) < 1e-14, (ix, iy, a[iy, ix], ref)
    # near the axis
    r = 1e-3 * LAMF
    v = math.pi * r / LAMF
    assert abs(om.airy_irradiance(radial_plane(r), D, F, LAM)[0, 2] - (1 - v * v / 4 + 5 * v ** 4 / 192)) < 1e-15


def test_airy_irradiance_scales_with_the_f_number_only():
    """At fixed lambda F the pattern is the same for any (D, f) pair."""
    pl = scenes.Plane(np.zeros(3), np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]), 15, 15,
                      0.4 * LAMF, 0.4 * LAMF)
    a = om.airy_irradiance(pl, D, F, LAM)
    b = om.airy_irradiance(pl, 2 * D, 2 * F, LAM)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)
    # and moves outwards in proportion to lambda F
    c = om.airy_irradiance(radial_plane(2 * J1_ZEROS[0] / math.pi * LAMF), D, F, 2 * LAM)[0, 2]
    assert c < 1e-20


def test_airy_metrics_zero_for_the_exact_field_with_any_phase():
    """E = sqrt(Airy) e^{i phi(x, y)}, E(0) of any modulus and phase: the
    peak-normalised irradiance is the Airy pattern, so both metrics vanish."""
    pl = scenes.Plane(np.zeros(3), np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]), 33, 31,
                      0.35 * LAMF, 0.35 * LAMF)
    airy = om.airy_irradiance(pl, D, F, LAM)
    rng = np.random.default_rng(5)
    E0 = 3.7 * np.exp(1.3j)
    E = E0 * np.sqrt(airy) * np.exp(2j * math.pi * rng.random(airy.shape))
    m = om.airy_metrics(E, E0, airy)
    assert m[0] < 1e-15 and m[1] < 1e-15


def test_airy_metrics_closed_forms():
    """A reference of 1/4 everywhere and a field with |E/E(0)|^2 = 1/2 on one
    half of the pixels and 1/4 on the other: difference 1/4 on half the
    pixels, RMS sqrt(1/2 * 1/16) = 0.176777, peak 1/4.  A field 10 % too
    bright everywhere (|E|^2 = 1.1 |E(0)|^2 airy) gives RMS 0.1 sqrt(mean
    airy^2) and peak 0.1 max airy; one too dark by the same gives the same
    (the peak is of the absolute difference)."""
    ny, nx = 6, 8
    airy = np.full((ny, nx), 0.25)
    E0 = 2.0 * np.exp(-0.4j)               # normalisation by |E(0)|^2, not by E(0)
    E = np.full((ny, nx), 1.0 + 0j) * abs(E0) / 2  # |E/E0|^2 = 1/4
    E[:, : nx // 2] *= math.sqrt(2.0)      # 1/2 on the left half
    m = om.airy_metrics(E, E0, airy)
    assert abs(m[0] - math.sqrt(0.5 / 16)) < 1e-15
    assert abs(m[1] - 0.25) < 1e-15

    rng = np.random.default_rng(1)
    airy = rng.random((ny, nx))
    for s in (1.1, 0.9):
        E = abs(E0) * np.sqrt(s * airy)
        m = om.airy_metrics(E, E0, airy)
        assert abs(m[0] - 0.1 * math.sqrt(np.mean(airy ** 2))) < 1e-15
        assert abs(m[1] - 0.1 * airy.max()) < 1e-15


def test_airy_metrics_zones():
    """Zone RMS over r in [edge_k, edge_k+1): with the difference equal to
    k + 1 on zone k (and 0 beyond the last edge), zone k's RMS is k + 1; a
    zone holding no pixel reports 0."""
    pl = scenes.Plane(np.zeros(3), np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]), 41, 41, 1.0, 1.0)
    r = om.plane_radius(pl)
    edges = np.array([0.0, 5.0, 10.0, 15.0, 15.5])
    zone = np.digitize(r, edges) - 1        # 0 ... 3 inside, 4 beyond the last edge
    assert ((r >= 15.0) & (r < 15.5)).any()  # every zone holds pixels on this grid
    d = np.where(zone < 4, zone + 1.0, 0.0)
    m = om.airy_metrics(np.sqrt(d), 1.0, np.zeros_like(r), radius=r, zone_edges=edges)
    assert len(m) == 2 + 4
    np.testing.assert_allclose(m[2:], [1.0, 2.0, 3.0, 4.0], rtol=0, atol=1e-15)
    assert abs(m[0] - math.sqrt(np.mean(d * d))) < 1e-15 and m[1] == 4.0
    m2 = om.airy_metrics(np.sqrt(d), 1.0, np.zeros_like(r), radius=r, zone_edges=np.array([100.0, 200.0]))
    assert m2[2] == 0.0
