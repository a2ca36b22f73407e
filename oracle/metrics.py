"""FP64 figures of merit of the Airy experiments (Sec. 4.2, Sec. 6).

TEST INFRASTRUCTURE (see the package docstring).

* airy_irradiance: the analytic Airy pattern of an unobscured circular pupil
  of diameter D focused at focal length f, (2 J1(v)/v)^2 with
  v = pi D r / (lambda f), r the distance from the plane origin (J1 from
  scipy.special).
* airy_metrics: RMS (over all pixels) and peak of |E/E(0)|^2 - airy, and the
  RMS over annular zones r in [edge_k, edge_{k+1}).
"""
import numpy as np
import scipy.special


def plane_radius(plane):
    a = (np.arange(plane.nx) - (plane.nx - 1) / 2.0) * plane.dx
    b = (np.arange(plane.ny) - (plane.ny - 1) / 2.0) * plane.dy
    A, B = np.meshgrid(a, b, indexing="xy")
    return np.hypot(A, B)


def airy_irradiance(plane, D, f, lam):
    v = np.pi * D * plane_radius(plane) / (lam * f)
    with np.errstate(invalid="ignore", divide="ignore"):
        amp = np.where(v > 0, 2.0 * scipy.special.j1(v) / v, 1.0)
    return amp * amp


def annular_airy_irradiance(plane, D, f, lam, eps):
    """Peak-normalised irradiance of a uniformly lit annulus of outer
    diameter D and obscuration ratio eps (inner / outer radius) in the focal
    plane of focal length f: the field is the outer disc's Airy amplitude
    minus the inner disc's, each 2 J1(u) / u scaled by its area,
    [(2 J1(v)/v - eps^2 2 J1(eps v)/(eps v)) / (1 - eps^2)]^2, v = pi D r / (lam f)."""
    v = np.pi * D * plane_radius(plane) / (lam * f)

    def disc(u):
        with np.errstate(invalid="ignore", divide="ignore"):
            return np.where(u > 0, 2.0 * scipy.special.j1(u) / u, 1.0)

    amp = (disc(v) - eps * eps * disc(eps * v)) / (1.0 - eps * eps)
    return amp * amp


def airy_metrics(E, E0, airy, radius=None, zone_edges=None):
    d = np.abs(E) ** 2 / abs(E0) ** 2 - airy
    out = [float(np.sqrt(np.mean(d * d))), float(np.abs(d).max())]
    if zone_edges is not None:
        for lo, hi in zip(zone_edges[:-1], zone_edges[1:]):
            m = (radius >= lo) & (radius < hi)
            out.append(float(np.sqrt(np.mean(d[m] ** 2))) if m.any() else 0.0)
    return np.array(out)
