"""Seeded synthetic inputs for plane-evaluation Gaussian beamlet decomposition.

This module builds *inputs only*: pupil sample positions, waists, amplitudes,
input optical paths, per-beamlet 4x4 ray-transfer (ABCD) matrices and detector
planes.  It contains none of the propagation arithmetic (no complex curvature,
no Collins solution, no field sums), so both the HIP library and the FP64
oracle can consume exactly the same arrays.

Conventions (metres, paraxial slopes, ray vector order (x, y, theta_x, theta_y)):

* Pupil decomposition (Sec. 6, overlap-factor equation): a square, cell-centred
  grid of ``n_across`` samples over the aperture width ``D`` with spacing
  ``s = D / n_across``; samples with ``x^2 + y^2 <= (D/2)^2`` are kept.  The
  overlap factor gives the waist ``w0 = OF * s / 2``; the sweep's waist/spacing
  ratio ``q`` multiplies it (``w0 = OF * q * s / 2``).
* System matrix of a thin lens of focal length f followed by a distance d
  (Sec. 4.1, lens-then-distance system-matrix equation).
* Detector plane: origin, normal, an x-hint vector, a cell-centred nx x ny
  pixel grid of pitch (dx, dy).
* Aberrations: Noll-normalised Zernike Z4..Z11 on rho = r/(D/2); the path
  W(r) = lam sum c_i Z_i + theta_field . r is expanded to second order about
  each beamlet centre r_j and carried as the ABCD ``M_sys @ [[I, 0], [H_j, I]]``
  (H_j = Hess W(r_j); symplectic because H_j is symmetric) together with the
  pre-plate slope grad W(r_j) - H_j r_j and piston W(r_j) - r_j.H_j r_j / 2.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Scene", "Plane", "pupil_grid", "lens_then_distance", "thin_plate",
    "airy_scene", "zernike_scene", "config", "sweep_grid", "surrogate_draws",
    "NOLL", "zernike_poly", "hst_rc", "annulus_grid", "rc_scene",
]


@dataclass
class Plane:
    """Detector plane: pixel (ix, iy) sits at origin + a*e1 + b*e2 with
    a = (ix - (nx-1)/2)*dx, b = (iy - (ny-1)/2)*dy; e1 is xhint projected
    onto the plane, e2 = normal x e1.  Output arrays are [ny][nx]."""
    origin: np.ndarray
    normal: np.ndarray
    xhint: np.ndarray
    nx: int
    ny: int
    dx: float
    dy: float

    @property
    def npix(self) -> int:
        return int(self.nx) * int(self.ny)


@dataclass
class Scene:
    """Beamlet decomposition handed to both the library and the oracle.

    r1   [n,2]  beamlet centres in the input plane (m)
    (abcd and base may come from a ray tracer: rc_scene leaves them None)
    th1  [n,2]  beamlet base-ray slopes in the input plane (rad, paraxial)
    w0   [n]    1/e field waist radius in the input plane (m)
    amp  [n,2]  complex amplitude (re, im)
    path [n]    input optical path W_j (m)
    abcd [k,16] row-major 4x4 ray-transfer matrix, k == 1 (shared) or n
    """
    lam: float
    l0: float
    r1: np.ndarray
    th1: np.ndarray
    w0: np.ndarray
    amp: np.ndarray
    path: np.ndarray
    abcd: Optional[np.ndarray]
    plane: Plane
    meta: dict = field(default_factory=dict)
    # traced inputs (filled by a ray tracer, not by this module):
    # base [n,5] = output-plane base ray (x, y, l, m, optical path - l0), and the
    # symplectic tolerance the differential (finite-difference) matrices get
    base: Optional[np.ndarray] = None
    sympl_tol: Optional[float] = None
    # elegant Hermite-Gaussian orders [n,2] (m, n) in 0..2 per beamlet, or None (Gaussian)
    order: Optional[np.ndarray] = None
    # truncating edges [n,3] = (e_x, e_y, t): beamlet j keeps e . r <= t of its input
    # envelope (e a unit vector; e = (0, 0) leaves the beamlet whole), or None
    edge: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.r1.shape[0])

    @property
    def shared_abcd(self) -> bool:
        return self.abcd.shape[0] == 1


@functools.lru_cache(maxsize=64)
def _pupil_grid(n_across: int, D: float) -> tuple[np.ndarray, float]:
    s = D / n_across
    c = (np.arange(n_across) - (n_across - 1) / 2.0) * s
    yy, xx = np.meshgrid(c, c, indexing="ij")
    keep = xx * xx + yy * yy <= (D / 2.0) ** 2
    r1 = np.stack([xx[keep], yy[keep]], axis=1).astype(np.float64)
    r1.flags.writeable = False
    return r1, s


def pupil_grid(n_across: int, D: float) -> tuple[np.ndarray, float]:
    """Cell-centred square grid clipped to the circular aperture of diameter D.
    Returns (r1 [n,2] in row-major order of (iy, ix), spacing s): a fresh copy
    of a cached grid (the parameter sweeps draw the same few grids many times)."""
    r1, s = _pupil_grid(int(n_across), float(D))
    return np.array(r1, dtype=np.float64, order="C"), s


def lens_then_distance(f: float, d: float) -> np.ndarray:
    """4x4 row-major ray-transfer matrix: thin lens f, then free space d."""
    I = np.eye(2)
    lens = np.eye(4)
    lens[2:, :2] = -I / f
    dist = np.eye(4)
    dist[:2, 2:] = d * I
    return dist @ lens


def thin_plate(H: np.ndarray) -> np.ndarray:
    """4x4 matrix of a thin phase plate whose path has Hessian H (2x2 symmetric)."""
    I = np.eye(2)
    Z = np.zeros((2, 2))
    return np.block([[I, Z], [H, I]])


def _plane(origin, normal, xhint, nx, ny, dx, dy) -> Plane:
    return Plane(np.asarray(origin, np.float64), np.asarray(normal, np.float64),
                 np.asarray(xhint, np.float64), int(nx), int(ny), float(dx), float(dy))


def airy_scene(n_across: int, *, D: float = 10e-3, fnum: float = 10.0, lam: float = 1e-6,
               OF: float = 1.7, q: float = 1.0, npix: int = 64, half_span_lamF: float = 5.0,
               field_angle=(0.0, 0.0), z0: float = 0.0, npix_y: Optional[int] = None) -> Scene:
    """Ideal-lens focal-plane scene (the Airy experiments): unit amplitudes,
    optional field angle (plane-wave tilt), detector at axial offset z0 from the
    focal plane, centred on f*field_angle, spanning +-half_span (lambda*F)."""
    f = fnum * D
    r1, s = pupil_grid(n_across, D)
    n = r1.shape[0]
    w0 = OF * q * s / 2.0
    tf = np.asarray(field_angle, np.float64)
    th1 = np.tile(tf, (n, 1))
    amp = np.zeros((n, 2))
    amp[:, 0] = 1.0
    path = r1 @ tf                    # tilted plane wave: path theta_f . r
    abcd = lens_then_distance(f, f).reshape(1, 16)
    lamF = lam * fnum
    ny = npix if npix_y is None else npix_y
    dx = 2.0 * half_span_lamF * lamF / npix
    dy = 2.0 * half_span_lamF * lamF / ny
    plane = _plane((f * tf[0], f * tf[1], z0), (0.0, 0.0, 1.0), (1.0, 0.0, 0.0), npix, ny, dx, dy)
    return Scene(lam, f, r1, np.ascontiguousarray(th1), np.full(n, w0), amp, path, abcd, plane,
                 meta=dict(kind="airy", n_across=n_across, D=D, f=f, fnum=fnum, OF=OF, q=q,
                           s=s, half_span_lamF=half_span_lamF))


# --- Zernike polynomials (Noll 1976 ordering and normalisation) -------------
# Each polynomial in the normalised Cartesian pupil coordinates (u, v) = (x, y)/R
# as {(pu, pv): coefficient}.
def _p(*terms):
    out = {}
    for c, pu, pv in terms:
        out[(pu, pv)] = out.get((pu, pv), 0.0) + c
    return out


_S3, _S5, _S6, _S8 = math.sqrt(3), math.sqrt(5), math.sqrt(6), math.sqrt(8)
NOLL = {
    4: _p((2 * _S3, 2, 0), (2 * _S3, 0, 2), (-_S3, 0, 0)),                 # defocus
    5: _p((2 * _S6, 1, 1)),                                                # astig sin 2t
    6: _p((_S6, 2, 0), (-_S6, 0, 2)),                                      # astig cos 2t
    7: _p((3 * _S8, 2, 1), (3 * _S8, 0, 3), (-2 * _S8, 0, 1)),             # coma sin t
    8: _p((3 * _S8, 3, 0), (3 * _S8, 1, 2), (-2 * _S8, 1, 0)),             # coma cos t
    9: _p((3 * _S8, 2, 1), (-_S8, 0, 3)),                                  # trefoil sin 3t
    10: _p((_S8, 3, 0), (-3 * _S8, 1, 2)),                                 # trefoil cos 3t
    11: _p((6 * _S5, 4, 0), (12 * _S5, 2, 2), (6 * _S5, 0, 4),
           (-6 * _S5, 2, 0), (-6 * _S5, 0, 2), (_S5, 0, 0)),               # spherical
}


def zernike_poly(coeffs: dict, u: np.ndarray, v: np.ndarray, du: int = 0, dv: int = 0) -> np.ndarray:
    """Evaluate d^(du+dv)/du^du dv^dv of sum_i coeffs[i] * Z_i at (u, v)."""
    out = np.zeros(np.broadcast(u, v).shape)
    for j, c in coeffs.items():
        for (pu, pv), a in NOLL[j].items():
            if pu < du or pv < dv:
                continue
            k = a * c * math.perm(pu, du) * math.perm(pv, dv)
            out = out + k * u ** (pu - du) * v ** (pv - dv)
    return out


def zernike_scene(seed: int = 2404, *, n_across: int = 128, D: float = 10e-3, fnum: float = 4.0,
                  lam: float = 1e-6, OF: float = 1.7, field_deg: float = 1.0, tilt_deg: float = 10.0,
                  defocus: float = 50e-6, npix: int = 1024, half_span: float = 128e-6,
                  sigma_waves: Optional[float] = None) -> Scene:
    """Aberrated off-axis system on a tilted detector.

    Seeded draw (numpy PCG64): sigma ~ U[0.05, 0.5] waves RMS (unless given),
    c ~ N(0,1)^8 rescaled to |c| = sigma, W(r) = lam * sum_i c_i Z_i(r/(D/2)).
    Field angle about x, detector tilted about x and offset along z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sigma = rng.uniform(0.05, 0.5) if sigma_waves is None else float(sigma_waves)
    c = rng.standard_normal(8)
    c = c * (sigma / np.linalg.norm(c))
    coeffs = {j: float(cj) for j, cj in zip(range(4, 12), c)}
    f = fnum * D
    R = D / 2.0
    r1, s = pupil_grid(n_across, D)
    n = r1.shape[0]
    u, v = r1[:, 0] / R, r1[:, 1] / R
    W = lam * zernike_poly(coeffs, u, v)
    gx = lam * zernike_poly(coeffs, u, v, 1, 0) / R
    gy = lam * zernike_poly(coeffs, u, v, 0, 1) / R
    hxx = lam * zernike_poly(coeffs, u, v, 2, 0) / R ** 2
    hxy = lam * zernike_poly(coeffs, u, v, 1, 1) / R ** 2
    hyy = lam * zernike_poly(coeffs, u, v, 0, 2) / R ** 2
    tf = np.array([0.0, math.radians(field_deg)])
    # The plate [[I,0],[H,I]] acts about the axis (theta' = theta + H r); the
    # local expansion W(r_j) + g.(r - r_j) + (r - r_j)^T H (r - r_j)/2 is
    # reproduced by the pre-plate slope g - H r_j and piston
    # W(r_j) - r_j^T H r_j / 2 (the base ray leaves the plate with slope g).
    g = np.stack([tf[0] + gx, tf[1] + gy], axis=1)
    Hr = np.stack([hxx * r1[:, 0] + hxy * r1[:, 1], hxy * r1[:, 0] + hyy * r1[:, 1]], axis=1)
    th1 = g - Hr
    path = W + r1 @ tf - 0.5 * (r1 * Hr).sum(axis=1)
    Msys = lens_then_distance(f, f)
    abcd = np.empty((n, 16))
    for j in range(n):
        H = np.array([[hxx[j], hxy[j]], [hxy[j], hyy[j]]])
        abcd[j] = (Msys @ thin_plate(H)).reshape(16)
    amp = np.zeros((n, 2))
    amp[:, 0] = 1.0
    t = math.radians(tilt_deg)
    dxy = 2.0 * half_span / npix
    plane = _plane((0.0, f * tf[1], defocus), (0.0, -math.sin(t), math.cos(t)), (1.0, 0.0, 0.0),
                   npix, npix, dxy, dxy)
    return Scene(lam, f, r1, np.ascontiguousarray(th1), np.full(n, OF * s / 2.0), amp,
                 np.ascontiguousarray(path), abcd, plane,
                 meta=dict(kind="zernike", seed=seed, sigma_waves=sigma, coeffs=coeffs, n_across=n_across,
                           D=D, f=f, fnum=fnum, OF=OF, s=s, field_deg=field_deg, tilt_deg=tilt_deg))


# --- Named workloads ---------------------------------------------------------
def hermite_scene(n_across: int = 32, *, seed: int = 7, D: float = 10e-3, fnum: float = 10.0, lam: float = 1e-6,
                  OF: float = 1.7, npix: int = 128, half_span_lamF: float = 8.0, cyl_f: Optional[float] = None,
                  cyl_angle: float = 0.5, z0: float = 0.0, npix_y: Optional[int] = None,
                  max_order: int = 2) -> Scene:
    """Higher-order beamlets on the pupil grid of airy_scene: every beamlet
    draws its Hermite-Gaussian orders (m, n) uniformly from 0..max_order and
    a unit-modulus amplitude of uniform phase (seeded), through an ideal lens
    of focal length fnum * D, detector normal to the axis at z0 from the
    focal plane.  cyl_f adds a thin cylindrical lens of that focal length
    whose power axis is turned by cyl_angle (rad), in contact with the
    lens: the system is then astigmatic with non-diagonal blocks."""
    f = fnum * D
    r1, sp = pupil_grid(n_across, D)
    n = r1.shape[0]
    rng = np.random.default_rng(seed)
    order = rng.integers(0, max_order + 1, size=(n, 2)).astype(np.int32)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n)
    amp = np.stack([np.cos(ph), np.sin(ph)], axis=1)
    M = lens_then_distance(f, f)
    if cyl_f is not None:
        c, s_ = np.cos(cyl_angle), np.sin(cyl_angle)
        R = np.array([[c, -s_], [s_, c]])
        M = M @ thin_plate(-R @ np.diag([1.0 / cyl_f, 0.0]) @ R.T)
    lamF = lam * fnum
    ny = npix if npix_y is None else npix_y
    plane = _plane((0.0, 0.0, z0), (0.0, 0.0, 1.0), (1.0, 0.0, 0.0), npix, ny,
                   2.0 * half_span_lamF * lamF / npix, 2.0 * half_span_lamF * lamF / ny)
    sc = Scene(lam, f, r1, np.zeros((n, 2)), np.full(n, OF * sp / 2.0), amp, np.zeros(n), M.reshape(1, 16), plane,
               meta=dict(kind="hermite", n_across=n_across, D=D, f=f, fnum=fnum, OF=OF, seed=seed, cyl_f=cyl_f,
                         half_span_lamF=half_span_lamF))
    sc.order = order
    return sc


def truncated_airy_scene(n_across: int, *, D: float = 10e-3, fnum: float = 10.0, lam: float = 1e-6,
                         OF: float = 1.7, npix: int = 64, half_span_lamF: float = 5.0, reach: float = 1.5,
                         z0: float = 0.0, npix_y: Optional[int] = None) -> Scene:
    """The Airy experiment with a hard-edged pupil: the cell-centred grid of
    airy_scene extended to centres within reach * w0 outside the aperture,
    and every beamlet whose centre lies within reach * w0 of the rim cut by
    the rim's tangent at the nearest rim point (edge normal r / |r|, t = D/2).
    Unit amplitudes, ideal lens, detector at z0 from the focal plane."""
    f = fnum * D
    s = D / n_across
    w0 = OF * s / 2.0
    K = int(np.ceil(reach * w0 / s)) + 1      # lattice rows beyond the pupil grid
    c = (np.arange(-K, n_across + K) - (n_across - 1) / 2.0) * s
    yy, xx = np.meshgrid(c, c, indexing="ij")
    rr = np.hypot(xx, yy)
    keep = rr <= D / 2.0 + reach * w0
    r1 = np.ascontiguousarray(np.stack([xx[keep], yy[keep]], axis=1))
    rho = rr[keep]
    n = r1.shape[0]
    edge = np.zeros((n, 3))
    cut = rho > D / 2.0 - reach * w0
    edge[cut, 0] = r1[cut, 0] / rho[cut]
    edge[cut, 1] = r1[cut, 1] / rho[cut]
    edge[cut, 2] = D / 2.0
    amp = np.zeros((n, 2))
    amp[:, 0] = 1.0
    lamF = lam * fnum
    ny = npix if npix_y is None else npix_y
    plane = _plane((0.0, 0.0, z0), (0.0, 0.0, 1.0), (1.0, 0.0, 0.0), npix, ny,
                   2.0 * half_span_lamF * lamF / npix, 2.0 * half_span_lamF * lamF / ny)
    sc = Scene(lam, f, r1, np.zeros((n, 2)), np.full(n, w0), amp, np.zeros(n),
               lens_then_distance(f, f).reshape(1, 16), plane,
               meta=dict(kind="truncated_airy", n_across=n_across, D=D, f=f, fnum=fnum, OF=OF, s=s, reach=reach,
                         half_span_lamF=half_span_lamF, n_cut=int(cut.sum())))
    sc.edge = edge
    return sc


def config(name: str) -> Scene:
    """Named workloads:

    airy32_64     32 across (812 beamlets), 64x64, +-5 lamF, f/10, FP64 form
    airy256_512   256 across (51,468 beamlets), 512x512, +-20 lamF, f/10
    zern128_1024  f/4, field 1 deg, Zernike seed 2404, plane tilted 10 deg,
                  +50 um, 128 across (12,892 beamlets), 1024x1024, +-128 um
    """
    if name == "airy32_64":
        return airy_scene(32, OF=1.7, npix=64, half_span_lamF=5.0)
    if name == "airy256_512":
        return airy_scene(256, OF=1.7, npix=512, half_span_lamF=20.0)
    if name == "zern128_1024":
        return zernike_scene(2404)
    raise KeyError(name)


SWEEP_OF = tuple(1.0 + 0.25 * i for i in range(9))
SWEEP_Q = tuple(0.5 + 0.25 * i for i in range(7))
SWEEP_NACROSS = (16, 24, 32, 48, 64, 96, 128)


def sweep_grid():
    """The 9 x 7 x 7 = 441 (OF, q, n_across) instances of the parameter sweep,
    each an f/10, lambda = 1 um focal-plane Airy scene at 256x256, +-8 lamF."""
    return [(of, q, na) for na in SWEEP_NACROSS for of in SWEEP_OF for q in SWEEP_Q]


def surrogate_draws(n: int = 20000, seed: int = 12454, counts=None):
    """Seeded uniform draws of the surrogate's inputs:
    OF ~ U[1,3], q ~ U[0.5,2], beamlets across uniform over ``counts`` (a
    list of integers, e.g. the candidate pool's), or, with counts None,
    ln n_across ~ U[ln 16, ln 128] rounded; F# ~ U[4,20],
    ln lam ~ U[ln 0.4 um, ln 2.0 um].  Returns [n,5] float64 columns
    (OF, q, n_across, fnum, lam)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    of = rng.uniform(1.0, 3.0, n)
    q = rng.uniform(0.5, 2.0, n)
    if counts is None:
        na = np.rint(np.exp(rng.uniform(math.log(16), math.log(128), n)))
    else:
        na = np.asarray(counts, np.float64)[rng.integers(0, len(counts), n)]
    fn = rng.uniform(4.0, 20.0, n)
    lam = np.exp(rng.uniform(math.log(0.4e-6), math.log(2.0e-6), n))
    return np.stack([of, q, na, fn, lam], axis=1)


# --- Appendix B telescope (ray-traced inputs) --------------------------------

def hst_rc(k1: float = -1.00230, k2: float = -1.49686, z_in: float = -5.0) -> dict:
    """The Ritchey-Chretien telescope of Appendix B in the global frame (z the
    axis, light from -z; radii signed by where the centre of curvature lies:
    R < 0 means it is on the -z side of the vertex).  The table gives the
    primary as concave (R 11.04 m) and the secondary as convex (R 1.358 m)
    towards the light that reaches them; the primary faces -z, the secondary
    +z, so both centres of curvature lie on the -z side: R1 = -11.04,
    R2 = -1.358.  Secondary 4.90607 m in front of the primary, image 6.40620 m
    behind the secondary; clear diameters 2.4 m and 0.28112 m.  The
    decomposition plane z_in sits in front of the secondary; mirrors are rows
    (z_vertex, R, k, r_min, r_max)."""
    z2 = -4.90607
    z_img = z2 + 6.40620
    D, d2 = 2.4, 0.28112
    mirrors = np.array([[0.0, -11.0400, k1, 0.0, D / 2.0],
                        [z2, -1.35800, k2, 0.0, d2 / 2.0]], np.float64)
    return dict(mirrors=mirrors, z_in=float(z_in), z_out=float(z_img), D=D, r_obs=d2 / 2.0,
                l0=float((0.0 - z_in) + (0.0 - z2) + (z_img - z2)))


def annulus_grid(n_across: int, D: float, r_in: float) -> tuple[np.ndarray, float]:
    """The cell-centred square grid of pupil_grid, keeping r_in <= r <= D/2."""
    r1, s = pupil_grid(n_across, D)
    rr = np.hypot(r1[:, 0], r1[:, 1])
    return np.ascontiguousarray(r1[rr >= r_in]), s


def rc_scene(n_across: int = 128, *, lam: float = 1e-6, OF: float = 1.7, field_angle=(0.0, 0.0),
             npix: int = 512, half_span_lamF: float = 16.0, system: Optional[dict] = None) -> Scene:
    """Beamlets on the annular entrance pupil of the Appendix B telescope
    (outer diameter 2.4 m, obscured by the secondary's 0.28112 m), unit
    amplitudes, w0 = OF s / 2, base-ray direction cosines = field angle;
    the detector is the image plane (the trace's output plane), normal to
    the axis, npix^2 pixels over +-half_span_lamF lambda F with F the
    nominal f/24.  abcd and base are left to a ray tracer."""
    sys_ = system or hst_rc()
    r1, s = annulus_grid(n_across, sys_["D"], sys_["r_obs"])
    n = r1.shape[0]
    th1 = np.tile(np.asarray(field_angle, np.float64), (n, 1))
    w0 = np.full(n, OF * s / 2.0)
    amp = np.zeros((n, 2))
    amp[:, 0] = 1.0
    lamF = lam * 24.0
    pitch = 2.0 * half_span_lamF * lamF / npix
    pl = _plane([0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0], npix, npix, pitch, pitch)
    return Scene(lam, sys_["l0"], r1, th1, w0, amp, np.zeros(n), None, pl,
                 meta=dict(n_across=n_across, OF=OF, D=sys_["D"], r_obs=sys_["r_obs"], fnum=24.0,
                           half_span_lamF=half_span_lamF, system=sys_, field_angle=tuple(field_angle)))
