"""Pins of the oracle's real-ray trace through conic mirrors (the traced base
rays and differential ABCD matrices of Sec. 2.2, on the Appendix B
telescope).  Each pin is a closed form that a plausible mistake in the
tracer (intersection root, surface normal, reflection, output frame, path
length, finite differences) would break."""
import math

import numpy as np
import pytest

import oracle
from paper_2404_12454_amd import scenes


def on_axis_rays(r_in, r_out, n=40):
    r = np.linspace(r_in, r_out, n)
    phi = np.linspace(0.0, 2 * np.pi, n, endpoint=False)
    return np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)


def test_paraboloid_focuses_every_axial_ray_with_equal_path():
    """k = -1: rays parallel to the axis meet at the focus z = R / 2 and, by
    Fermat, all reach it with the same optical path (plane wave -> point)."""
    R = -2.0
    mirrors = [[0.0, R, -1.0, 0.0, 10.0]]
    z_in, z_f = -3.0, R / 2.0
    l0 = (0.0 - z_in) + (0.0 - z_f)
    r1 = on_axis_rays(0.05, 0.9)       # up to f/0.55: far from paraxial
    base, _, flags = oracle.trace(mirrors, z_in, z_f, l0, r1)
    assert not flags.any()
    assert np.abs(base[:, :2]).max() < 1e-12
    assert np.abs(base[:, 4]).max() < 1e-12


def test_sphere_marginal_focus_matches_closed_form():
    """k = 0: a ray at height h crosses the axis at z = R (1 - 1 / (2 cos a)),
    sin a = h / |R| (spherical aberration of a concave mirror)."""
    R = -2.0
    z_in, z_out = -3.0, -0.5
    h = np.array([0.05, 0.3, 0.6, 0.9])
    r1 = np.stack([h, np.zeros_like(h)], axis=1)
    base, _, flags = oracle.trace([[0.0, R, 0.0, 0.0, 10.0]], z_in, z_out, 0.0, r1)
    assert not flags.any()
    # one reflection: the output frame is turned by pi about x, so the global
    # direction is (l, -m, -n); the ray x(z) = x2 + (z - z_out) l / n_global
    l = base[:, 2]
    n_glob = -np.sqrt(1.0 - l ** 2 - base[:, 3] ** 2)
    z_cross = z_out - base[:, 0] * n_glob / l
    alpha = np.arcsin(h / abs(R))
    want = R * (1.0 - 1.0 / (2.0 * np.cos(alpha)))
    np.testing.assert_allclose(z_cross, want, rtol=0, atol=1e-12)


def cassegrain(R1=-11.04, z2=-4.90607, z_img=1.50013):
    """Classical Cassegrain: paraboloid primary (focus F1 = R1 / 2); the
    hyperboloid secondary's foci z2 + R2 / (1 +- e) are put at F1 and at the
    image, which makes every axial ray meet there exactly."""
    a, b = R1 / 2.0 - z2, z_img - z2
    e = (b - a) / (a + b)
    R2 = a * (1.0 + e)
    return np.array([[0.0, R1, -1.0, 0.0, 1.2], [z2, R2, -e * e, 0.0, 0.2]]), z_img


def test_cassegrain_conjugate_foci_image_axial_rays_perfectly():
    mirrors, z_img = cassegrain()
    z_in = -5.0
    l0 = (0.0 - z_in) + (0.0 - mirrors[1, 0]) + (z_img - mirrors[1, 0])
    r1 = on_axis_rays(0.15, 1.19)
    base, abcd, flags = oracle.trace(mirrors, z_in, z_img, l0, r1)
    assert not flags.any()
    assert np.abs(base[:, :2]).max() < 1e-12     # every ray through the image point
    assert np.ptp(base[:, 4]) < 1e-12              # and with one optical path (Fermat)
    # the secondary's radius comes out at the telescope's 1.358 m
    assert abs(mirrors[1, 1] + 1.358) < 1e-3


def paraxial_matrix(sysd):
    """Unfolded paraxial (x, l) matrix: spaces S(t) = [[1, t], [0, 1]] (t the
    path), mirror reflecting light that travels +z: [[1, 0], [2 c, 1]],
    travelling -z: [[1, 0], [-2 c, 1]] (c = 1/R in the global frame)."""
    (z1, R1, *_), (z2, R2, *_) = sysd["mirrors"]
    S = lambda t: np.array([[1.0, t], [0.0, 1.0]])
    M = lambda c, s: np.array([[1.0, 0.0], [2.0 * c * s, 1.0]])
    return S(sysd["z_out"] - z2) @ M(1.0 / R2, -1) @ S(z1 - z2) @ M(1.0 / R1, +1) @ S(z1 - sysd["z_in"])


def test_axial_differential_matrix_is_the_paraxial_system_matrix():
    sysd = scenes.hst_rc()
    base, abcd, flags = oracle.trace(sysd["mirrors"], sysd["z_in"], sysd["z_out"], sysd["l0"], np.zeros((1, 2)))
    assert flags[0] == 0
    Mx = paraxial_matrix(sysd)
    M = abcd[0].reshape(4, 4)
    want = np.zeros((4, 4))
    want[np.ix_([0, 2], [0, 2])] = Mx
    want[np.ix_([1, 3], [1, 3])] = Mx
    np.testing.assert_allclose(M, want, rtol=0, atol=1e-7 * np.abs(want).max())
    efl = -1.0 / Mx[1, 0]
    assert abs(efl - 57.6) < 0.05                  # HST: f/24 on 2.4 m
    assert abs(base[0, 4]) < 1e-12                   # the axial ray's path is l0


def test_plane_mirror_folds_space_and_turns_the_output_frame():
    """One flat mirror: free space of length 2 unfolded, output frame turned
    by pi about x: (x, y, l, m) -> (x + 2 l / n, -(y + 2 m / n), l, -m)."""
    r1 = np.array([[0.1, -0.2], [0.0, 0.0]])
    th1 = np.array([[0.03, 0.02], [0.0, 0.0]])
    base, abcd, flags = oracle.trace([[0.0, 0.0, 0.0, 0.0, 10.0]], -1.0, -1.0, 2.0, r1, th1)
    assert not flags.any()
    n = np.sqrt(1.0 - th1[:, 0] ** 2 - th1[:, 1] ** 2)
    np.testing.assert_allclose(base[:, 0], r1[:, 0] + 2 * th1[:, 0] / n, atol=1e-14)
    np.testing.assert_allclose(base[:, 1], -(r1[:, 1] + 2 * th1[:, 1] / n), atol=1e-14)
    np.testing.assert_allclose(base[:, 2:4], th1 * [1, -1], atol=1e-15)
    np.testing.assert_allclose(base[:, 4], 2.0 / n - 2.0, atol=1e-14)
    np.testing.assert_allclose(abcd[1].reshape(4, 4), [[1, 0, 2, 0], [0, -1, 0, -2], [0, 0, 1, 0], [0, 0, 0, -1]],
                               atol=1e-9)


@pytest.mark.parametrize("field", [(0.0, 0.0), (2e-4, -1e-4)])
def test_telescope_differential_matrices_are_symplectic(field):
    """Direction cosines are canonical: the exact ray map is symplectic, the
    central differences are within their truncation/rounding error of it."""
    sysd = scenes.hst_rc()
    sc = scenes.rc_scene(24, field_angle=field)
    base, abcd, flags = oracle.trace(sysd["mirrors"], sysd["z_in"], sysd["z_out"], sysd["l0"], sc.r1, sc.th1)
    assert not flags.any()
    J = np.block([[np.zeros((2, 2)), np.eye(2)], [-np.eye(2), np.zeros((2, 2))]])
    worst = 0.0
    for m in abcd:
        M = m.reshape(4, 4)
        worst = max(worst, np.abs(M.T @ J @ M - J).max() / (np.abs(M).max() ** 2))
    assert worst < 1e-8, worst


def test_base_override_with_paraxial_values_reproduces_the_abcd_field():
    """The traced-base-ray input path: handing the oracle the base ray that
    the ab/cd laws give (r2M = A r1 + B th1, th2M = C r1 + D th1) and the
    eikonal of Euler's relation as its path, (th2M . r2M - th1 . r1) / 2,
    must reproduce the field of the plain ABCD input."""
    sc = scenes.zernike_scene(11, n_across=10, npix=24, half_span=25e-6)
    E0 = oracle.eval_field(sc)
    M = sc.abcd if sc.abcd.shape[0] == sc.n else np.repeat(sc.abcd, sc.n, axis=0)
    M = M.reshape(-1, 4, 4)
    v1 = np.concatenate([sc.r1, sc.th1], axis=1)
    v2 = np.einsum("nij,nj->ni", M, v1)
    L = 0.5 * (np.sum(v2[:, 2:] * v2[:, :2], axis=1) - np.sum(sc.th1 * sc.r1, axis=1))
    sc.base = np.concatenate([v2, L[:, None]], axis=1)
    E1 = oracle.eval_field(sc)
    assert np.linalg.norm(E1 - E0) / np.linalg.norm(E0) < 1e-12
    # a traced path differing by half a wave flips that beamlet's sign
    sc.base[3, 4] += 0.5 * sc.lam
    E2 = oracle.eval_field(sc)
    assert np.linalg.norm(E2 - E0) / np.linalg.norm(E0) > 1e-3


def test_annular_airy_reference_reduces_to_the_airy_pattern():
    """The obscured-aperture reference at eps -> 0 is the Airy pattern, with
    its first zero at v = 3.8317 (r = 1.2197 lambda F); with an obscuration
    the first zero moves inwards; it is 1 on axis."""
    from oracle import metrics as om
    pl = scenes.airy_scene(8, npix=65, half_span_lamF=6.0).plane
    a = om.airy_irradiance(pl, 10e-3, 100e-3, 1e-6)
    np.testing.assert_allclose(om.annular_airy_irradiance(pl, 10e-3, 100e-3, 1e-6, 0.0), a, atol=1e-15)
    lamF = 10e-6
    r0 = 3.831705970207512 / np.pi * lamF

    def at(r, eps):
        p1 = scenes.Plane(np.zeros(3), np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0]), 3, 1, r, r)
        return om.annular_airy_irradiance(p1, 10e-3, 100e-3, 1e-6, eps)[0, 2]

    assert at(r0, 0.0) < 1e-20
    # with eps = 0.33 the first zero lies inside r0: the pattern changes sign
    # between 0.8 r0 and r0 (its amplitude, the square root with sign, is
    # found by bisection on the irradiance's minimum)
    rs = np.linspace(0.8 * r0, r0, 2001)
    vals = np.array([at(r, 0.33) for r in rs])
    k = int(np.argmin(vals))
    assert 0 < k < len(rs) - 1 and vals[k] < 1e-6 and at(r0, 0.33) > 1e-4
    c = pl.nx // 2
    assert abs(om.annular_airy_irradiance(pl, 10e-3, 100e-3, 1e-6, 0.3)[c, c] - 1.0) < 1e-12
