"""MI355X plane-evaluation Gaussian beamlet decomposition (arXiv:2404.12454).

Thin ctypes binding of the C ABI in ``include/gbd.h``: argument marshalling
only.  Every step of the computation runs in the HIP library ``libgbd.so``
built in-tree for gfx950 (``python -m paper_2404_12454_amd.build``); there is
no CPU fallback, and calls fail loudly when the library is missing.  PyTorch
supplies device memory (output tensors) and the HIP stream.

Names follow the C ABI: ``gbd_ctx_create``, ``gbd_beamlets``, ``gbd_plane``,
``gbd_eval``, ``gbd_plan_create``, ``gbd_plan_setup``, ``gbd_plan_eval``,
``gbd_plan_shape``.  Handles are small Python objects that free their C
handle when collected.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

__all__ = [
    "GBD_FP64", "GBD_MIXED", "GbdError", "gbd_eval_opts", "library_path", "load_library",
    "gbd_ctx_create", "gbd_beamlets", "gbd_plane", "gbd_eval", "gbd_plan_create", "gbd_plan_setup",
    "gbd_plan_eval", "gbd_plan_eval_noalloc", "gbd_plan_shape", "gbd_issue_probe", "gbd_airy", "gbd_eval_batch", "gbd_eval_point", "gbd_autotune", "gbd_autotune_batch",
    "gbd_autotune_save", "gbd_autotune_load", "GBD_MLP_FP32", "GBD_MLP_BF16", "Mlp", "gbd_mlp_create", "beamlets_from_scene", "plane_from_scene",
    "gbd_trace", "gbd_beamlets_traced", "gbd_beamlets_hg", "gbd_beamlets_truncated",
    "Context", "Beamlets", "Plane", "Plan",
]

GBD_FP64 = 0
GBD_MIXED = 1
GBD_MLP_FP32 = 0
GBD_MLP_BF16 = 1
ERRORS = {0: "GBD_OK", -1: "GBD_EINVAL", -2: "GBD_ENOTSYMPLECTIC", -3: "GBD_EBRANCH", -4: "GBD_EPARALLEL",
          -5: "GBD_ENOMEM", -6: "GBD_EHIP", -7: "GBD_ERANGE"}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgbd.so")
_lib = None


def library_path() -> str:
    return _LIB_PATH


class GbdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class gbd_eval_opts(ctypes.Structure):
    _fields_ = [("rows_per_lane", ctypes.c_int32), ("waves", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("variant", ctypes.c_int32)]


def load_library():
    """Load the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -m paper_2404_12454_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "gbd_ctx_create": (ctypes.c_int, [PP, ctypes.c_int, P]),
        "gbd_ctx_set_stream": (ctypes.c_int, [P, P]),
        "gbd_ctx_destroy": (None, [P]),
        "gbd_ctx_set_kernel_timing": (ctypes.c_int, [P, ctypes.c_int]),
        "gbd_ctx_kernel_times": (ctypes.c_int, [P, P, I32, P]),
        "gbd_trace": (ctypes.c_int, [P, I32, P, D, D, D, I64, P, P, D, D, P, P, P]),
        "gbd_beamlets_traced": (ctypes.c_int, [P, PP, I64, D, D, P, P, P, I64, P, P, P, P, D]),
        "gbd_last_error": (ctypes.c_char_p, []),
        "gbd_beamlets": (ctypes.c_int, [P, PP, I64, D, D, P, P, P, I64, P, P, P, I64]),
        "gbd_beamlets_hg": (ctypes.c_int, [P, PP, I64, D, D, P, P, P, I64, P, P, P, I64, P]),
        "gbd_beamlets_truncated": (ctypes.c_int, [P, PP, I64, D, D, P, P, P, I64, P, P, P, I64, P]),
        "gbd_beamlets_free": (None, [P]),
        "gbd_plane": (ctypes.c_int, [P, PP, P, P, P, I32, I32, D, D]),
        "gbd_plane_free": (None, [P]),
        "gbd_eval": (ctypes.c_int, [P, P, P, ctypes.c_int, P, I64, P]),
        "gbd_plan_create": (ctypes.c_int, [P, PP, I64]),
        "gbd_plan_setup": (ctypes.c_int, [P, P, P, P]),
        "gbd_plan_eval": (ctypes.c_int, [P, P, ctypes.c_int, P, I64, P]),
        "gbd_plan_eval_noalloc": (ctypes.c_int, [P, P, ctypes.c_int, P, I64, P]),
        "gbd_plan_free": (None, [P]),
        "gbd_plan_shape": (ctypes.c_int, [P, P, ctypes.c_int, P, P]),
        "gbd_airy": (ctypes.c_int, [P, P, D, D, D, P, I64]),
        "gbd_eval_point": (ctypes.c_int, [P, P, P, P, I64]),
        "gbd_autotune": (ctypes.c_int, [P, P, ctypes.c_int, I32, P, P]),
        "gbd_mlp_create": (ctypes.c_int, [P, PP, I32, I32, I32, I32, ctypes.c_int]),
        "gbd_mlp_free": (None, [P]),
        "gbd_mlp_num_params": (I64, [P]),
        "gbd_mlp_set_params": (ctypes.c_int, [P, P, I64]),
        "gbd_mlp_get_params": (ctypes.c_int, [P, P, I64]),
        "gbd_mlp_get_grads": (ctypes.c_int, [P, P, I64]),
        "gbd_mlp_forward": (ctypes.c_int, [P, P, P, I32, P]),
        "gbd_mlp_backward": (ctypes.c_int, [P, P, P, P, I32, P]),
        "gbd_mlp_adamw": (ctypes.c_int, [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float]),
        "gbd_mlp_train": (ctypes.c_int, [P, P, P, P, I32, I32, P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, P]),
        "gbd_autotune_batch": (ctypes.c_int, [P, I32, P, P, P, I64, I32, P, P]),
        "gbd_autotune_save": (ctypes.c_int, [P, ctypes.c_char_p]),
        "gbd_autotune_load": (ctypes.c_int, [P, ctypes.c_char_p]),
        "gbd_eval_batch": (ctypes.c_int, [P, I32, P, P, P, I64, P, I32, P, P, I64, P]),
        "gbd_issue_probe": (ctypes.c_int, [P, I32, I32, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise GbdError(rc, load_library().gbd_last_error().decode(errors="replace"))


def _f64(a) -> Optional[np.ndarray]:
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data  # the caller keeps the array alive over the call


def _handles(objs) -> np.ndarray:
    """The objects' C handles as one array of pointers."""
    return np.fromiter((o.hv for o in objs), dtype=np.uintp, count=len(objs))


class Context:
    """A library context bound to one device and one HIP stream (default:
    torch's current stream on that device)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load_library()
        self.device = int(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib.gbd_ctx_create(ctypes.byref(h), self.device, ctypes.c_void_p(self.stream.cuda_stream)))
        self.handle = h

    def set_stream(self, stream):
        self.stream = stream
        _check(load_library().gbd_ctx_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)))

    def set_kernel_timing(self, enable: bool = True):
        """Record HIP events around each evaluation's N x M kernel."""
        _check(load_library().gbd_ctx_set_kernel_timing(self.handle, 1 if enable else 0))

    def kernel_times(self, cap: int = 4096) -> list:
        """Durations (ms) of the kernels timed since the last call, oldest first."""
        buf = np.zeros(cap, dtype=np.float32)
        n = ctypes.c_int32()
        _check(load_library().gbd_ctx_kernel_times(self.handle, _p(buf), cap, ctypes.byref(n)))
        return [float(v) for v in buf[:min(n.value, cap)]]

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load_library().gbd_ctx_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gbd_ctx_create(device: int = 0, stream=None) -> Context:
    return Context(device, stream)


class Beamlets:
    def __init__(self, handle, n):
        self.handle, self.n = handle, n
        self.hv = handle.value or 0  # the handle as an int, for handle arrays

    def __del__(self):
        try:
            if self.handle.value:
                load_library().gbd_beamlets_free(self.handle)
        except Exception:
            pass


class Plane:
    def __init__(self, handle, nx, ny):
        self.handle, self.nx, self.ny = handle, nx, ny
        self.hv = handle.value or 0

    def __del__(self):
        try:
            if self.handle.value:
                load_library().gbd_plane_free(self.handle)
        except Exception:
            pass


def gbd_beamlets(ctx: Context, n: int, lam: float, l0: float, r1, th1=None, w0=None, amp=None, path=None,
                 abcd=None) -> Beamlets:
    """Validate, copy and upload a beamlet decomposition (see gbd.h)."""
    r1, th1, w0, amp, path, abcd = map(_f64, (r1, th1, w0, amp, path, abcd))
    w0 = np.atleast_1d(w0) if w0 is not None else None
    abcd = None if abcd is None else abcd.reshape(-1, 16)
    h = ctypes.c_void_p()
    _check(load_library().gbd_beamlets(ctx.handle, ctypes.byref(h), int(n), float(lam), float(l0), _p(r1), _p(th1),
                                       _p(w0), 0 if w0 is None else w0.size, _p(amp), _p(path), _p(abcd),
                                       0 if abcd is None else abcd.shape[0]))
    return Beamlets(h, int(n))


def gbd_beamlets_hg(ctx: Context, n: int, lam: float, l0: float, r1, th1, w0, amp, path, abcd, order) -> Beamlets:
    """Elegant Hermite-Gaussian beamlets of orders order [n,2] in 0..2 (see gbd.h)."""
    r1, th1, w0, amp, path, abcd = map(_f64, (r1, th1, w0, amp, path, abcd))
    w0 = np.atleast_1d(w0) if w0 is not None else None
    abcd = None if abcd is None else abcd.reshape(-1, 16)
    order = None if order is None else np.ascontiguousarray(np.asarray(order).reshape(-1, 2), dtype=np.int32)
    h = ctypes.c_void_p()
    _check(load_library().gbd_beamlets_hg(ctx.handle, ctypes.byref(h), int(n), float(lam), float(l0), _p(r1),
                                          _p(th1), _p(w0), 0 if w0 is None else w0.size, _p(amp), _p(path),
                                          _p(abcd), 0 if abcd is None else abcd.shape[0], _p(order)))
    return Beamlets(h, int(n))


def gbd_beamlets_truncated(ctx: Context, n: int, lam: float, l0: float, r1, th1, w0, amp, path, abcd,
                           edge) -> Beamlets:
    """Beamlets whose input envelopes are cut by straight edges, edge [n,3] =
    (e_x, e_y, t) keeping e . r <= t (e = (0, 0): whole) (see gbd.h)."""
    r1, th1, w0, amp, path, abcd, edge = map(_f64, (r1, th1, w0, amp, path, abcd, edge))
    w0 = np.atleast_1d(w0) if w0 is not None else None
    abcd = None if abcd is None else abcd.reshape(-1, 16)
    edge = None if edge is None else edge.reshape(-1, 3)
    h = ctypes.c_void_p()
    _check(load_library().gbd_beamlets_truncated(ctx.handle, ctypes.byref(h), int(n), float(lam), float(l0), _p(r1),
                                                 _p(th1), _p(w0), 0 if w0 is None else w0.size, _p(amp), _p(path),
                                                 _p(abcd), 0 if abcd is None else abcd.shape[0], _p(edge)))
    return Beamlets(h, int(n))


def gbd_plane(ctx: Context, origin, normal, xhint, nx: int, ny: int, dx: float, dy: float) -> Plane:
    o, n, x = _f64(origin), _f64(normal), _f64(xhint)
    h = ctypes.c_void_p()
    _check(load_library().gbd_plane(ctx.handle, ctypes.byref(h), _p(o), _p(n), _p(x), int(nx), int(ny),
                                    float(dx), float(dy)))
    return Plane(h, int(nx), int(ny))


def gbd_trace(ctx: Context, mirrors, z_in: float, z_out: float, l0: float, r1, th1=None, dr: float = 1e-5,
              dth: float = 1e-7):
    """Real-ray trace through conic mirrors on the device (see gbd.h): returns
    base [n,5], abcd [n,16] and flags [n] as host arrays."""
    mir = _f64(np.asarray(mirrors, np.float64).reshape(-1, 5))
    r1 = _f64(np.asarray(r1).reshape(-1, 2))
    th = None if th1 is None else _f64(np.asarray(th1).reshape(-1, 2))
    n = r1.shape[0]
    base = np.empty((n, 5))
    abcd = np.empty((n, 16))
    flags = np.empty(n, np.int32)
    _check(load_library().gbd_trace(ctx.handle, mir.shape[0], _p(mir), float(z_in), float(z_out), float(l0), n,
                                    _p(r1), _p(th), float(dr), float(dth), _p(base), _p(abcd), _p(flags)))
    return base, abcd, flags


def gbd_beamlets_traced(ctx: Context, n: int, lam: float, l0: float, r1, th1, w0, amp, path, abcd, base,
                        sympl_tol: float = 1e-7) -> Beamlets:
    """Beamlets with traced base rays and differential matrices (see gbd.h)."""
    r1, th1, w0, amp, path, abcd, base = map(_f64, (r1, th1, w0, amp, path, abcd, base))
    w0 = np.atleast_1d(w0)
    h = ctypes.c_void_p()
    _check(load_library().gbd_beamlets_traced(ctx.handle, ctypes.byref(h), int(n), float(lam), float(l0), _p(r1),
                                              _p(th1), _p(w0), w0.size, _p(amp), _p(path),
                                              _p(abcd.reshape(-1, 16)), _p(base.reshape(-1, 5)), float(sympl_tol)))
    return Beamlets(h, int(n))


def beamlets_from_scene(ctx: Context, s) -> Beamlets:
    if getattr(s, "edge", None) is not None:
        if getattr(s, "base", None) is not None or getattr(s, "order", None) is not None:
            raise ValueError("truncated beamlets take neither traced inputs nor higher orders")
        return gbd_beamlets_truncated(ctx, s.n, s.lam, s.l0, s.r1, s.th1, s.w0, s.amp, s.path, s.abcd, s.edge)
    if getattr(s, "order", None) is not None:
        if getattr(s, "base", None) is not None:
            raise ValueError("traced inputs of higher-order beamlets are not supported")
        return gbd_beamlets_hg(ctx, s.n, s.lam, s.l0, s.r1, s.th1, s.w0, s.amp, s.path, s.abcd, s.order)
    if getattr(s, "base", None) is not None:
        return gbd_beamlets_traced(ctx, s.n, s.lam, s.l0, s.r1, s.th1, s.w0, s.amp, s.path, s.abcd, s.base,
                                   s.sympl_tol or 1e-7)
    return gbd_beamlets(ctx, s.n, s.lam, s.l0, s.r1, s.th1, s.w0, s.amp, s.path, s.abcd)


def plane_from_scene(ctx: Context, s) -> Plane:
    pl = s.plane
    return gbd_plane(ctx, pl.origin, pl.normal, pl.xhint, pl.nx, pl.ny, pl.dx, pl.dy)


def _opts(opts) -> Optional[gbd_eval_opts]:
    if opts is None:
        return None
    if isinstance(opts, gbd_eval_opts):
        return opts
    return gbd_eval_opts(int(opts.get("rows_per_lane", 0)), int(opts.get("waves", 0)),
                         int(opts.get("segments", 0)), int(opts.get("variant", 0)))


def _out_tensor(ctx: Context, plane_nx: int, plane_ny: int, precision: int, out):
    import torch
    dt = torch.complex128 if precision == GBD_FP64 else torch.complex64
    if out is None:
        out = torch.empty((plane_ny, plane_nx), dtype=dt, device=f"cuda:{ctx.device}")
    if out.dtype != dt or not out.is_contiguous() or out.device.type != "cuda":
        raise ValueError(f"out must be a contiguous {dt} CUDA tensor")
    return out


def gbd_eval(ctx: Context, beamlets: Beamlets, plane: Plane, precision: int = GBD_MIXED, out=None, opts=None):
    """Field [ny, nx] on the plane (complex128 for GBD_FP64, complex64 for
    GBD_MIXED), written asynchronously on the context stream."""
    out = _out_tensor(ctx, plane.nx, plane.ny, precision, out)
    o = _opts(opts)
    _check(load_library().gbd_eval(ctx.handle, beamlets.handle, plane.handle, int(precision),
                                   ctypes.c_void_p(out.data_ptr()), out.numel() * out.element_size(),
                                   None if o is None else ctypes.byref(o)))
    return out


def gbd_eval_point(ctx: Context, beamlets: Beamlets, plane: Plane, out=None):
    """Point evaluation (paraxial, FP64): complex128 [ny, nx]; synchronises."""
    out = _out_tensor(ctx, plane.nx, plane.ny, GBD_FP64, out)
    _check(load_library().gbd_eval_point(ctx.handle, beamlets.handle, plane.handle, ctypes.c_void_p(out.data_ptr()),
                                         out.numel() * out.element_size()))
    return out


class Plan:
    """Per-beamlet records for one (beamlets, plane) pair, re-usable across
    evaluations (gbd_plan_* of the C ABI)."""

    def __init__(self, ctx: Context, capacity: int):
        self.ctx = ctx
        self.capacity = int(capacity)
        h = ctypes.c_void_p()
        _check(load_library().gbd_plan_create(ctx.handle, ctypes.byref(h), self.capacity))
        self.handle = h
        self.nx = self.ny = 0

    def setup(self, beamlets: Beamlets, plane: Plane):
        _check(load_library().gbd_plan_setup(self.ctx.handle, self.handle, beamlets.handle, plane.handle))
        self.nx, self.ny = plane.nx, plane.ny
        return self

    def eval(self, precision: int = GBD_MIXED, out=None, opts=None):
        out = _out_tensor(self.ctx, self.nx, self.ny, precision, out)
        o = _opts(opts)
        _check(load_library().gbd_plan_eval(self.ctx.handle, self.handle, int(precision),
                                            ctypes.c_void_p(out.data_ptr()), out.numel() * out.element_size(),
                                            None if o is None else ctypes.byref(o)))
        return out

    def eval_noalloc(self, precision: int = GBD_MIXED, out=None, opts=None):
        """gbd_plan_eval_noalloc: partial sums in the library's static device
        buffer; ``out`` should be pre-allocated by callers that cannot allocate."""
        out = _out_tensor(self.ctx, self.nx, self.ny, precision, out)
        o = _opts(opts)
        _check(load_library().gbd_plan_eval_noalloc(self.ctx.handle, self.handle, int(precision),
                                                    ctypes.c_void_p(out.data_ptr()), out.numel() * out.element_size(),
                                                    None if o is None else ctypes.byref(o)))
        return out

    def shape(self, precision: int = GBD_MIXED, opts=None) -> dict:
        o = _opts(opts)
        r = gbd_eval_opts()
        _check(load_library().gbd_plan_shape(self.ctx.handle, self.handle, int(precision),
                                             None if o is None else ctypes.byref(o), ctypes.byref(r)))
        return dict(rows_per_lane=r.rows_per_lane, waves=r.waves, segments=r.segments, variant=r.variant)

    def __del__(self):
        try:
            if self.handle.value:
                load_library().gbd_plan_free(self.handle)
        except Exception:
            pass


def gbd_plan_create(ctx: Context, capacity: int) -> Plan:
    return Plan(ctx, capacity)


def gbd_plan_setup(plan: Plan, beamlets: Beamlets, plane: Plane) -> Plan:
    return plan.setup(beamlets, plane)


def gbd_plan_eval(plan: Plan, precision: int = GBD_MIXED, out=None, opts=None):
    return plan.eval(precision, out, opts)


def gbd_issue_probe(ctx: Context, cls: int, iters: int):
    """(milliseconds, wavefront-instructions) of one timed launch of the
    issue-rate probe for instruction class ``cls`` (see include/gbd.h)."""
    ms, n = ctypes.c_double(), ctypes.c_double()
    _check(load_library().gbd_issue_probe(ctx.handle, int(cls), int(iters), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def gbd_plan_eval_noalloc(plan: Plan, precision: int = GBD_MIXED, out=None, opts=None):
    return plan.eval_noalloc(precision, out, opts)


def gbd_plan_shape(plan: Plan, precision: int = GBD_MIXED, opts=None) -> dict:
    return plan.shape(precision, opts)


def gbd_airy(ctx: Context, plane: Plane, D: float, f: float, lam: float, out=None):
    """Reference irradiance (2 J1(v)/v)^2 on the plane grid, float32 [ny, nx] on the device."""
    import torch
    if out is None:
        out = torch.empty((plane.ny, plane.nx), dtype=torch.float32, device=f"cuda:{ctx.device}")
    if out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 CUDA tensor")
    _check(load_library().gbd_airy(ctx.handle, plane.handle, float(D), float(f), float(lam),
                                   ctypes.c_void_p(out.data_ptr()), out.numel() * 4))
    return out


def gbd_eval_batch(ctx: Context, beamlets, planes, airy=None, zone_edges=None, fields: bool = False, opts=None):
    """Evaluate many instances in one persistent launch (mixed precision).

    Returns (metrics, fields): metrics is a float64 array [n_inst, 2 + n_zones]
    (RMS, peak, zone RMS...) when ``airy`` (a float32 [ny, nx] device tensor)
    is given, else None; fields is a list of complex64 [ny_i, nx_i] device
    tensors (views of one allocation) when ``fields`` is true, else None."""
    import torch
    n = len(beamlets)
    if len(planes) != n:
        raise ValueError("beamlets and planes differ in length")
    hb, hp = _handles(beamlets), _handles(planes)
    ze = None if zone_edges is None else _f64(zone_edges)
    nz = 0 if ze is None else ze.size - 1
    metrics = np.zeros((n, 2 + nz)) if airy is not None else None
    fbuf = None
    if fields:
        total = sum(p.nx * p.ny for p in planes)
        fbuf = torch.empty(max(total, 1), dtype=torch.complex64, device=f"cuda:{ctx.device}")
    o = _opts(opts)
    _check(load_library().gbd_eval_batch(
        ctx.handle, n, _p(hb), _p(hp), None if airy is None else ctypes.c_void_p(airy.data_ptr()),
        0 if airy is None else airy.numel() * 4, _p(ze), nz, _p(metrics),
        None if fbuf is None else ctypes.c_void_p(fbuf.data_ptr()), 0 if fbuf is None else fbuf.numel() * 8,
        None if o is None else ctypes.byref(o)))
    out_fields = None
    if fbuf is not None:
        out_fields, off = [], 0
        for p in planes:
            m = p.nx * p.ny
            out_fields.append(fbuf[off:off + m].view(p.ny, p.nx))
            off += m
    return metrics, out_fields


def gbd_autotune(plan: Plan, precision: int = GBD_MIXED, reps: int = 3):
    """Time every launch shape for this plan; the fastest is cached in the
    context and returned as (opts dict, ms per evaluation)."""
    best = gbd_eval_opts()
    ms = ctypes.c_double()
    _check(load_library().gbd_autotune(plan.ctx.handle, plan.handle, int(precision), int(reps), ctypes.byref(best),
                                       ctypes.byref(ms)))
    return dict(rows_per_lane=best.rows_per_lane, waves=best.waves, segments=best.segments,
                variant=best.variant), ms.value


def gbd_autotune_batch(ctx: Context, beamlets, planes, airy, reps: int = 2):
    n = len(beamlets)
    hb, hp = _handles(beamlets), _handles(planes)
    best = gbd_eval_opts()
    ms = ctypes.c_double()
    _check(load_library().gbd_autotune_batch(ctx.handle, n, _p(hb), _p(hp), ctypes.c_void_p(airy.data_ptr()), airy.numel() * 4,
                                             int(reps), ctypes.byref(best), ctypes.byref(ms)))
    return dict(rows_per_lane=best.rows_per_lane, waves=best.waves), ms.value


def gbd_autotune_save(ctx: Context, path: str):
    _check(load_library().gbd_autotune_save(ctx.handle, os.fsencode(path)))


def gbd_autotune_load(ctx: Context, path: str) -> int:
    rc = load_library().gbd_autotune_load(ctx.handle, os.fsencode(path))
    if rc < 0:
        _check(rc)
    return rc


class Mlp:
    """Surrogate network handle (gbd_mlp_* of the C ABI): n_in -> width (SiLU)
    x depth -> 1, parameters/gradients/AdamW state on the device."""

    def __init__(self, ctx: Context, n_in: int = 5, width: int = 128, depth: int = 3, max_batch: int = 256,
                 mode: int = GBD_MLP_BF16):
        self.ctx = ctx
        self.n_in, self.width, self.depth, self.max_batch, self.mode = n_in, width, depth, max_batch, mode
        h = ctypes.c_void_p()
        _check(load_library().gbd_mlp_create(ctx.handle, ctypes.byref(h), n_in, width, depth, max_batch, mode))
        self.handle = h
        self.num_params = int(load_library().gbd_mlp_num_params(h))

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(load_library().gbd_mlp_set_params(self.handle, _p(p), p.size))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.num_params, np.float32)
        _check(load_library().gbd_mlp_get_params(self.handle, _p(p), p.size))
        return p

    def get_grads(self) -> np.ndarray:
        g = np.empty(self.num_params, np.float32)
        _check(load_library().gbd_mlp_get_grads(self.handle, _p(g), g.size))
        return g

    def forward(self, x, rows=None, batch=None, out=None):
        """x: device float32 [*, n_in]; rows: optional device int32 indices."""
        import torch
        batch = int(rows.numel() if rows is not None else (x.shape[0] if batch is None else batch))
        if out is None:
            out = torch.empty(batch, dtype=torch.float32, device=x.device)
        _check(load_library().gbd_mlp_forward(self.handle, ctypes.c_void_p(x.data_ptr()),
                                              None if rows is None else ctypes.c_void_p(rows.data_ptr()), batch,
                                              ctypes.c_void_p(out.data_ptr())))
        return out

    def backward(self, x, target, rows=None, loss_out=None):
        batch = int(rows.numel() if rows is not None else x.shape[0])
        _check(load_library().gbd_mlp_backward(self.handle, ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(target.data_ptr()),
                                               None if rows is None else ctypes.c_void_p(rows.data_ptr()), batch,
                                               None if loss_out is None else ctypes.c_void_p(loss_out.data_ptr())))

    def adamw(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        _check(load_library().gbd_mlp_adamw(self.handle, float(lr), float(beta1), float(beta2), float(eps),
                                            float(weight_decay)))

    def train(self, x, target, rows, lrs, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, loss_sum=None):
        """len(lrs) steps of backward on rows[s] then adamw(lrs[s]) in one
        call; rows: device int32 [steps, batch]; loss_sum: optional device
        float32 [1] that each step's loss is added to."""
        lr = np.ascontiguousarray(lrs, dtype=np.float32)
        steps, batch = int(rows.shape[0]), int(rows.shape[1])
        if lr.size != steps:
            raise ValueError(f"{lr.size} learning rates for {steps} steps")
        _check(load_library().gbd_mlp_train(self.handle, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(target.data_ptr()), ctypes.c_void_p(rows.data_ptr()),
                                            steps, batch, _p(lr), float(beta1), float(beta2), float(eps),
                                            float(weight_decay),
                                            None if loss_sum is None else ctypes.c_void_p(loss_sum.data_ptr())))

    def __del__(self):
        try:
            if self.handle.value:
                load_library().gbd_mlp_free(self.handle)
        except Exception:
            pass


def gbd_mlp_create(ctx: Context, n_in=5, width=128, depth=3, max_batch=256, mode=GBD_MLP_BF16) -> Mlp:
    return Mlp(ctx, n_in, width, depth, max_batch, mode)
