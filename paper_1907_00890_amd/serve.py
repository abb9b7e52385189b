"""Python binding of the continuous-batching request loop (include/vofserve.h).

Argument marshalling only: admission, batching, lanes and plan residency are
the library's scheduler thread; every solve runs in its HIP kernels.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import ExtendFields

_p = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_ll = ctypes.c_longlong

VP_EAGAIN, VP_ETOOBIG, VP_ECANCELED, VP_ETIMEDOUT = -5, -6, -7, -8
SOLVE, EXTEND = 0, 1
FAULT_LAUNCH, FAULT_PLAN = 0, 1


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", _ll), ("lanes", _i), ("max_batch", _i), ("max_pending", _i),
                ("dry_run", _i), ("dry_run_us", _d)]


class Request(ctypes.Structure):
    _fields_ = [("kind", _i), ("precision", _i), ("nx", _i), ("ny", _i), ("nz", _i),
                ("dx", _d), ("dy", _d), ("dz", ctypes.POINTER(_d)), ("bc", ctypes.c_char_p),
                ("rhs", _p), ("sol", _p), ("ext", ExtendFields), ("queue_timeout_ms", _d)]


class Result(ctypes.Structure):
    _fields_ = [("status", _i), ("batch", _i), ("lane", _i), ("t_submit_us", _d),
                ("t_dispatch_us", _d), ("t_done_us", _d)]


class Stats(ctypes.Structure):
    _fields_ = [(n, _ll) for n in (
        "submitted", "rejected", "completed", "failed", "cancelled", "timed_out", "batches",
        "batched_requests", "plans_created", "plans_evicted", "plans_resident", "bytes_resident",
        "bytes_peak", "pending", "running")]


SIGNATURES = {
    "vp_server_now_us": (_d, []),
    "vp_server_create": (_p, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_i)]),
    "vp_server_submit": (_i, [_p, ctypes.POINTER(Request), ctypes.POINTER(_ll)]),
    "vp_server_prewarm": (_i, [_p, ctypes.POINTER(Request), _i, _d, ctypes.POINTER(_i)]),
    "vp_server_wait": (_i, [_p, _ll, _d, ctypes.POINTER(Result)]),
    "vp_server_cancel": (_i, [_p, _ll]),
    "vp_server_drain": (_i, [_p, _d]),
    "vp_server_get_stats": (_i, [_p, ctypes.POINTER(Stats)]),
    "vp_server_inject": (_i, [_p, _i, _i]),
    "vp_server_destroy": (None, [_p]),
}

_lib_ = _lib.lib
for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(_lib_, _name)
    _f.restype = _res
    _f.argtypes = _args


class ServeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        names = {VP_EAGAIN: "queue full / not ready", VP_ETOOBIG: "plan above the memory budget",
                 VP_ECANCELED: "cancelled", VP_ETIMEDOUT: "queue timeout"}
        msg = names.get(status) or _lib_.poisson_strerror(status).decode(errors="replace")
        super().__init__(f"{where}: status {status} ({msg})")


def now_us() -> float:
    """The server clock (monotonic, microseconds)."""
    return _lib_.vp_server_now_us()


class Grid:
    """A request's grid: nx, ny, nz, dx, dy, dz (nz widths) and bc."""

    def __init__(self, nx, ny, nz, dx, dy, dz, bc):
        import numpy as np
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy = float(dx), float(dy)
        self.dz = np.ascontiguousarray(np.asarray(dz, dtype=np.float64).reshape(-1))
        self.bc = str(bc).upper()
        self.shape = (self.nz, self.ny, self.nx)


class Server:
    """Continuous-batching server on the current ROCm device.

    hbm_budget: device bytes its resident plans may hold; lanes: HIP streams;
    max_batch: requests per launch; max_pending: queue bound (submit raises
    ServeError(VP_EAGAIN) beyond it); dry_run: host logic only (no device
    calls, each batch takes dry_run_us).
    """

    def __init__(self, hbm_budget, lanes=4, max_batch=8, max_pending=4096, dry_run=False,
                 dry_run_us=0.0):
        cfg = ServerConfig(int(hbm_budget), int(lanes), int(max_batch), int(max_pending),
                           int(bool(dry_run)), float(dry_run_us))
        st = _i(0)
        h = _lib_.vp_server_create(ctypes.byref(cfg), ctypes.byref(st))
        if not h:
            raise ServeError(st.value, "vp_server_create")
        self._h = _p(h)
        self.dry_run = bool(dry_run)
        self._keep = {}  # ticket -> objects that must outlive the request

    # -- low level: raw pointers ------------------------------------------------
    def submit_raw(self, kind, grid: Grid, precision="fp64", rhs=0, sol=0, ext=None,
                   timeout_ms=0.0, keep=()):
        """Submit with integer device addresses (ext: dict of ExtendFields names)."""
        r = Request()
        r.kind = int(kind)
        r.precision = _lib.PRECISION[precision]
        r.nx, r.ny, r.nz = grid.nx, grid.ny, grid.nz
        r.dx, r.dy = grid.dx, grid.dy
        r.dz = grid.dz.ctypes.data_as(ctypes.POINTER(_d))
        bc = grid.bc.encode()
        r.bc = bc
        r.rhs = rhs or None
        r.sol = sol or None
        for name, val in (ext or {}).items():
            setattr(r.ext, name, val or None)
        r.queue_timeout_ms = float(timeout_ms)
        t = _ll(0)
        s = _lib_.vp_server_submit(self._h, ctypes.byref(r), ctypes.byref(t))
        if s != 0:
            raise ServeError(s, "vp_server_submit")
        self._keep[t.value] = (grid, keep)
        return t.value

    # -- tensors -----------------------------------------------------------------
    @staticmethod
    def _ptr(t, shape, name, optional=False):
        import torch
        if t is None:
            if optional:
                return 0
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a torch tensor on a ROCm device")
        if t.dtype != torch.float64 or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous float64 with shape {shape}")
        return t.data_ptr()

    def submit_solve(self, grid: Grid, rhs, sol, precision="fp64", timeout_ms=0.0):
        """Queue sol = L^+ rhs; returns a ticket."""
        return self.submit_raw(SOLVE, grid, precision, rhs=self._ptr(rhs, grid.shape, "rhs"),
                               sol=self._ptr(sol, grid.shape, "sol"), timeout_ms=timeout_ms,
                               keep=(rhs, sol))

    def submit_extend(self, grid: Grid, u, v, w, src, out, q=None, gamma=None, phi=None,
                      precision="fp64", timeout_ms=0.0):
        """Queue a liquid-velocity extension (outputs out = (ue, ve, we), optional
        gamma = (ug, vg, wg) with q, phi); returns a ticket."""
        sh = grid.shape
        ext = {"u": self._ptr(u, sh, "u"), "v": self._ptr(v, sh, "v"), "w": self._ptr(w, sh, "w"),
               "src": self._ptr(src, sh, "src"), "phi": self._ptr(phi, sh, "phi", optional=True)}
        for names, ts in ((("ue", "ve", "we"), out), (("qx", "qy", "qz"), q),
                          (("ug", "vg", "wg"), gamma)):
            for n, t in zip(names, ts or (None, None, None)):
                ext[n] = self._ptr(t, sh, n, optional=ts is None)
        return self.submit_raw(EXTEND, grid, precision, ext=ext, timeout_ms=timeout_ms,
                               keep=(u, v, w, src, out, q, gamma, phi))

    def prewarm(self, grid: Grid, precision="fp64", instances=1, timeout_ms=-1.0) -> int:
        """Make `instances` plans of this class resident before traffic; returns
        how many were created."""
        r = Request()
        r.precision = _lib.PRECISION[precision]
        r.nx, r.ny, r.nz = grid.nx, grid.ny, grid.nz
        r.dx, r.dy = grid.dx, grid.dy
        r.dz = grid.dz.ctypes.data_as(ctypes.POINTER(_d))
        bc = grid.bc.encode()
        r.bc = bc
        made = _i(0)
        s = _lib_.vp_server_prewarm(self._h, ctypes.byref(r), int(instances), float(timeout_ms),
                                    ctypes.byref(made))
        if s != 0:
            raise ServeError(s, "vp_server_prewarm")
        return made.value

    def wait(self, ticket, timeout_ms=-1.0):
        """The request's result as a dict, or None if it has not ended in time."""
        res = Result()
        s = _lib_.vp_server_wait(self._h, int(ticket), float(timeout_ms), ctypes.byref(res))
        if s == VP_EAGAIN:
            return None
        if s != 0:
            raise ServeError(s, "vp_server_wait")
        self._keep.pop(int(ticket), None)
        return {"status": res.status, "batch": res.batch, "lane": res.lane,
                "t_submit_us": res.t_submit_us, "t_dispatch_us": res.t_dispatch_us,
                "t_done_us": res.t_done_us}

    def cancel(self, ticket):
        s = _lib_.vp_server_cancel(self._h, int(ticket))
        if s != 0:
            raise ServeError(s, "vp_server_cancel")

    def drain(self, timeout_ms=-1.0) -> bool:
        return _lib_.vp_server_drain(self._h, float(timeout_ms)) == 0

    def stats(self) -> dict:
        st = Stats()
        s = _lib_.vp_server_get_stats(self._h, ctypes.byref(st))
        if s != 0:
            raise ServeError(s, "vp_server_get_stats")
        return {n: getattr(st, n) for n, _ in Stats._fields_}

    def inject(self, fault, count=1):
        s = _lib_.vp_server_inject(self._h, int(fault), int(count))
        if s != 0:
            raise ServeError(s, "vp_server_inject")

    def close(self):
        if getattr(self, "_h", None):
            _lib_.vp_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
