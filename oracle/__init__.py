"""FP64 CPU oracle for plane-evaluation Gaussian beamlet decomposition.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  The product path
(``paper_2404_12454_amd``) never imports it, and the two share no code; the
only common module is the seeded input generator, which holds no propagation
arithmetic.

``gbd_oracle.c`` is a plain, slow, direct FP64 implementation (libm exp/sin/
cos, no fast-math, OpenMP over pixels); ``raytrace.c`` the plain FP64
sequential real-ray trace through conic mirrors that gives traced base rays
and differential ABCD matrices.  ``metrics`` and ``mlp`` hold the FP64
figures of merit and the surrogate's reference network in numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gbd_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "raytrace.c")]
_LIB = os.path.join(_HERE, "libgbd_oracle.so")
_lib = None

ERRORS = {0: "ok", -1: "EINVAL", -2: "ENOTSYMPLECTIC", -3: "EBRANCH", -4: "EPARALLEL"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code} ({ERRORS.get(code, '?')})")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc -O2 -fopenmp (no fast-math)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", *_SRCS, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_eval.restype = ctypes.c_int
        lib.oracle_eval.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, P, P, P, ctypes.c_int64,
                                    P, P, P, ctypes.c_int, P, P, P, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int64, P, P, ctypes.c_int, P, P, P]
        lib.oracle_eval_base.restype = ctypes.c_int
        lib.oracle_eval_base.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, P, P, P, ctypes.c_int64,
                                         P, P, P, ctypes.c_int, P, ctypes.c_double, P, P, P, P, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int64, P, P,
                                         ctypes.c_int, P, P, P]
        lib.oracle_trunc_terms.restype = ctypes.c_int
        lib.oracle_trunc_terms.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, P, P, P,
                                           ctypes.c_int64, P, P, P, ctypes.c_int, P, P, P, P, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int64, P, P,
                                           P, P]
        lib.oracle_trace.restype = ctypes.c_int
        lib.oracle_trace.argtypes = [ctypes.c_int32, P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int64, P, P, ctypes.c_double, ctypes.c_double, P, P, P]
        lib.oracle_beamlet.restype = ctypes.c_int
        lib.oracle_beamlet.argtypes = [ctypes.c_double, P, P, ctypes.c_double, ctypes.c_double, P,
                                       ctypes.c_double, P]
        lib.oracle_set_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_symplectic_ok.restype = ctypes.c_int
        lib.oracle_symplectic_ok.argtypes = [P]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _subset(scene, keep):
    """The scene restricted to the beamlets where keep is True."""
    import copy
    s = copy.copy(scene)
    for name in ("r1", "th1", "amp", "path"):
        setattr(s, name, np.ascontiguousarray(np.asarray(getattr(scene, name))[keep]))
    w0 = np.atleast_1d(scene.w0)
    s.w0 = np.ascontiguousarray(w0 if w0.size == 1 else w0[keep])
    abcd = np.asarray(scene.abcd).reshape(-1, 16)
    s.abcd = np.ascontiguousarray(abcd if abcd.shape[0] == 1 else abcd[keep])
    s.edge = None
    return s


def _truncated_field(scene, edge, pixels, plane):
    """Sum over truncated beamlets of E_j * erfc(zeta_j) / 2 (see
    oracle_trunc_terms), formed with the scaled complex error function
    erfcx(z) = e^(z^2) erfc(z) so that large |zeta| neither overflows nor
    underflows: for Re zeta >= 0 the term is e^(log E - zeta^2) erfcx(zeta) / 2,
    else E - e^(log E - zeta^2) erfcx(-zeta) / 2."""
    import scipy.special
    lib = _load()
    r1, th1, w0, amp, path, abcd = (_f64(scene.r1), _f64(scene.th1), _f64(scene.w0), _f64(scene.amp),
                                    _f64(scene.path), _f64(scene.abcd))
    shared = 1 if abcd.shape[0] == 1 else 0
    n = scene.n
    if pixels is not None:
        ix = np.ascontiguousarray(pixels[0], dtype=np.int32).ravel()
        iy = np.ascontiguousarray(pixels[1], dtype=np.int32).ravel()
        m = ix.size
    else:
        ix = iy = None
        m = plane.nx * plane.ny
    logE = np.empty((m, n, 2))
    zeta = np.empty((m, n, 2))
    rc = lib.oracle_trunc_terms(n, scene.lam, scene.l0, _ptr(r1), _ptr(th1), _ptr(w0), w0.size, _ptr(amp),
                                _ptr(path), _ptr(abcd), shared, _ptr(_f64(edge)), _ptr(_f64(plane.origin)),
                                _ptr(_f64(plane.normal)), _ptr(_f64(plane.xhint)), plane.nx, plane.ny, plane.dx,
                                plane.dy, m, _ptr(ix), _ptr(iy), _ptr(logE), _ptr(zeta))
    if rc != 0:
        raise OracleError(rc)
    lg = logE.view(np.complex128)[..., 0]
    z = zeta.view(np.complex128)[..., 0]
    pos = z.real >= 0
    zz = np.where(pos, z, -z)
    half = 0.5 * np.exp(lg - zz * zz) * scipy.special.erfcx(zz)
    terms = np.where(pos, half, np.exp(lg) - half)
    return terms.sum(axis=1)


def eval_field(scene, model: int = 0, pixels: Optional[tuple] = None, extra_point=None,
               threads: Optional[int] = None):
    """Coherent field of ``scene`` on its detector plane, complex128.

    model 0 = plane-evaluation, model 1 = exact paraxial point evaluation.
    pixels = (ix, iy) int arrays for a sample of pixels, else the full
    [ny][nx] grid.  extra_point = (a, b) plane coordinates also evaluated
    (returned second).  Truncated beamlets (scene.edge rows with a nonzero
    edge normal) are summed by _truncated_field, on planes normal to the
    axis, where both models coincide."""
    edge = getattr(scene, "edge", None)
    if edge is not None:
        edge = np.ascontiguousarray(edge, dtype=np.float64).reshape(-1, 3)
        if getattr(scene, "order", None) is not None or getattr(scene, "base", None) is not None:
            raise OracleError(-1)
        cut = (edge[:, 0] != 0.0) | (edge[:, 1] != 0.0)
        E = eval_field(_subset(scene, ~cut), model, pixels, None, threads) if (~cut).any() else None
        Et = _truncated_field(_subset(scene, cut), edge[cut], pixels, scene.plane)
        Et = Et.reshape(E.shape) if E is not None else (Et if pixels is not None else
                                                         Et.reshape(scene.plane.ny, scene.plane.nx))
        E = Et if E is None else E + Et
        if extra_point is None:
            return E
        pl = scene.plane
        e1 = np.asarray(pl.xhint, float) - np.dot(pl.xhint, pl.normal) / np.dot(pl.normal, pl.normal) * np.asarray(pl.normal, float)
        e1 = e1 / np.linalg.norm(e1)
        nrm = np.asarray(pl.normal, float) / np.linalg.norm(pl.normal)
        e2 = np.cross(nrm, e1)
        import copy
        one = copy.copy(scene)
        one.plane = type(pl)(np.asarray(pl.origin, float) + extra_point[0] * e1 + extra_point[1] * e2, pl.normal,
                             pl.xhint, 1, 1, pl.dx, pl.dy)
        return E, complex(eval_field(one, model, None, None, threads)[0, 0])
    lib = _load()
    pl = scene.plane
    r1, th1, w0, amp, path, abcd = (_f64(scene.r1), _f64(scene.th1), _f64(scene.w0), _f64(scene.amp),
                                    _f64(scene.path), _f64(scene.abcd))
    shared = 1 if abcd.shape[0] == 1 else 0
    if pixels is not None:
        ix = np.ascontiguousarray(pixels[0], dtype=np.int32).ravel()
        iy = np.ascontiguousarray(pixels[1], dtype=np.int32).ravel()
        m = ix.size
        out = np.empty(2 * m)
    else:
        ix = iy = None
        m = pl.nx * pl.ny
        out = np.empty(2 * m)
    ep = _f64(extra_point)
    oe = np.zeros(2) if ep is not None else None
    if threads is not None:
        lib.oracle_set_threads(int(threads))
    base = _f64(getattr(scene, "base", None))
    tol = getattr(scene, "sympl_tol", None) or 1e-10
    order = getattr(scene, "order", None)
    order = None if order is None else np.ascontiguousarray(order, dtype=np.int32).reshape(-1, 2)
    rc = lib.oracle_eval_base(scene.n, scene.lam, scene.l0, _ptr(r1), _ptr(th1), _ptr(w0), w0.size, _ptr(amp),
                              _ptr(path), _ptr(abcd), shared, _ptr(base), float(tol), _ptr(order),
                              _ptr(_f64(pl.origin)),
                              _ptr(_f64(pl.normal)), _ptr(_f64(pl.xhint)), pl.nx, pl.ny, pl.dx, pl.dy, m,
                              _ptr(ix), _ptr(iy), model, _ptr(out), _ptr(ep), _ptr(oe))
    if rc != 0:
        raise OracleError(rc)
    E = out.view(np.complex128)
    if pixels is None:
        E = E.reshape(pl.ny, pl.nx)
    if ep is not None:
        return E, complex(oe[0], oe[1])
    return E


def beamlet(lam, r1, th1, w0, W, abcd, z=0.0):
    """One beamlet propagated by abcd extended with free space z.
    Returns dict(Qinv [2,2] complex, gamma, r2 [2], th2 [2], tau)."""
    lib = _load()
    out = np.empty(15)
    rc = lib.oracle_beamlet(float(lam), _ptr(_f64(r1)), _ptr(_f64(th1)), float(w0), float(W),
                            _ptr(_f64(np.asarray(abcd).reshape(16))), float(z), _ptr(out))
    if rc != 0:
        raise OracleError(rc)
    Q = (out[0:8:2] + 1j * out[1:8:2]).reshape(2, 2)
    return dict(Qinv=Q, gamma=complex(out[8], out[9]), r2=out[10:12].copy(), th2=out[12:14].copy(), tau=out[14])


def set_threads(n: int = 0) -> int:
    """Set the oracle's OpenMP thread count (0 keeps it); returns the count in use."""
    return int(_load().oracle_set_threads(int(n)))


def symplectic_ok(abcd) -> bool:
    return bool(_load().oracle_symplectic_ok(_ptr(_f64(np.asarray(abcd).reshape(16)))))


TRACE_FLAGS = {1: "vignetted", 2: "missed", 4: "backward"}


def trace(mirrors, z_in: float, z_out: float, l0: float, r1, th1=None, dr: float = 1e-5, dth: float = 1e-7):
    """Real-ray trace through conic mirrors (rows (z_vertex, R, k, r_min,
    r_max)): returns base [n,5] = (x2, y2, l2, m2, optical path - l0) on the
    plane z_out, the central-difference differential matrices abcd [n,16]
    (parabasal offsets dr in position, dth in direction cosine) and the
    per-ray flags [n] (TRACE_FLAGS bits)."""
    lib = _load()
    mir = _f64(np.asarray(mirrors, np.float64).reshape(-1, 5))
    r1 = _f64(np.asarray(r1).reshape(-1, 2))
    n = r1.shape[0]
    th = None if th1 is None else _f64(np.asarray(th1).reshape(-1, 2))
    base = np.empty((n, 5))
    abcd = np.empty((n, 16))
    flags = np.empty(n, np.int32)
    rc = lib.oracle_trace(mir.shape[0], _ptr(mir), float(z_in), float(z_out), float(l0), n, _ptr(r1), _ptr(th),
                          float(dr), float(dth), _ptr(base), _ptr(abcd), _ptr(flags))
    if rc != 0:
        raise OracleError(rc)
    return base, abcd, flags
