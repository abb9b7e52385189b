"""MI355X-native Poisson / projection / liquid-velocity-extension path.

Python binding of libvofpoisson (include/vofpoisson.h): torch tensors in and
out (device memory and streams only), all arithmetic in the library's HIP
kernels for gfx950.  Fields are float64 tensors of shape (nz, ny, nx) on a
ROCm device, contiguous (x fastest).
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import VofPoissonError, check  # noqa: F401

__all__ = ["Plan", "VofPoissonError", "footprint", "version"]


def version() -> str:
    return _lib.lib.vofpoisson_version().decode()


def footprint(nx: int, ny: int, nz: int, precision: str = "fp64", max_batch: int = 1) -> int:
    """Device bytes a plan of this shape holds."""
    return int(_lib.lib.poisson_plan_footprint(nx, ny, nz, _lib.PRECISION[precision], max_batch))


def kernel_class_names():
    return [_lib.lib.poisson_kernel_class_name(i).decode() for i in range(_lib.NUM_KERNEL_CLASSES)]


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A solve plan: grid, boundary conditions, device tables and workspace.

    nx, ny: transform lengths, 2^k in [8, 1024], 3 * 2^k in [24, 768] or
    5 * 2^k in [40, 640]; nz in [1, 1024] (>= 3 when z is periodic); dz: nz
    cell widths (z may be stretched); bc: three letters (x, y, z, both ends
    alike) or six (x-, x+, y-, y+, z-, z+) from 'P' (periodic, both ends of a
    direction), 'N' (wall, zero normal gradient) and 'D' (outflow, p = 0 on
    the boundary face); every direction takes P or any pair of N and D (NN,
    DD, ND, DN).  precision: 'fp64' or 'mixed'.
    """

    def __init__(self, nx, ny, nz, dx, dy, dz, bc, precision="fp64", max_batch=1):
        import numpy as np
        dz = np.ascontiguousarray(np.asarray(dz, dtype=np.float64).reshape(-1))
        if dz.shape != (nz,):
            raise ValueError("dz must have nz entries")
        self.shape = (int(nz), int(ny), int(nx))
        self.bc = str(bc).upper()
        self.precision = precision
        self.max_batch = int(max_batch)
        self._dz = dz
        status = ctypes.c_int(0)
        h = _lib.lib.poisson_plan_create(
            int(nx), int(ny), int(nz), float(dx), float(dy),
            dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.bc.encode(),
            _lib.PRECISION[precision], int(max_batch), ctypes.byref(status))
        if not h:
            raise VofPoissonError(status.value, "poisson_plan_create")
        self._h = ctypes.c_void_p(h)

    # -- helpers --------------------------------------------------------------
    def _ptr(self, t, name, optional=False):
        import torch
        if t is None:
            if optional:
                return None
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a torch tensor on a ROCm device")
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64")
        if tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.shape}")
        return ctypes.c_void_p(t.data_ptr())

    def _lower(self, planes, name):
        """vp_lower_faces from (x, y, z) device planes or None entries; None if
        planes is None."""
        import torch
        if planes is None:
            return None
        nz, ny, nx = self.shape
        shapes = ((nz, ny), (nz, nx), (ny, nx))
        ptrs = []
        for t, shp in zip(planes, shapes):
            if t is None:
                ptrs.append(None)
                continue
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or \
                    t.dtype != torch.float64 or tuple(t.shape) != shp or not t.is_contiguous():
                raise ValueError(f"{name}: planes are contiguous float64 device tensors shaped "
                                 f"{shapes}")
            ptrs.append(t.data_ptr())
        return ctypes.byref(_lib.LowerFaces(*ptrs))

    def _new(self, like):
        import torch
        return torch.empty(self.shape, dtype=torch.float64, device=like.device)

    # -- entry points ---------------------------------------------------------
    def solve(self, rhs, out=None, stream=None):
        """out = L^+ rhs (zero volume-weighted mean); out may be rhs."""
        if out is None:
            out = self._new(rhs)
        check(_lib.lib.poisson_solve(self._h, self._ptr(rhs, "rhs"), self._ptr(out, "out"),
                                     _stream_ptr(stream)), "poisson_solve")
        return out

    def solve_noalloc(self, rhs, out=None, stream=None):
        """As solve, with the spectrum in the library's static device array
        (poisson_solve_noalloc: no allocation; FP64 plans of at most
        2^23 points; overlapping calls on one GPU race)."""
        if out is None:
            out = self._new(rhs)
        check(_lib.lib.poisson_solve_noalloc(self._h, self._ptr(rhs, "rhs"),
                                             self._ptr(out, "out"), _stream_ptr(stream)),
              "poisson_solve_noalloc")
        return out

    def solve_batched(self, rhs_list, out_list=None, stream=None):
        n = len(rhs_list)
        if out_list is None:
            out_list = [self._new(r) for r in rhs_list]
        arr_in = (ctypes.c_void_p * n)(*[self._ptr(r, "rhs").value for r in rhs_list])
        arr_out = (ctypes.c_void_p * n)(*[self._ptr(o, "out").value for o in out_list])
        check(_lib.lib.poisson_solve_batched(self._h, n, arr_in, arr_out, _stream_ptr(stream)),
              "poisson_solve_batched")
        return out_list

    def extend_batched(self, items, stream=None):
        """Batched extension: items is a list of dicts with keys u, v, w, src and
        optionally q (3 tensors), out (3), gamma (3), phi.  Missing outputs are
        allocated; returns a list of (ue, ve, we, ug, vg, wg, phi) per item."""
        n = len(items)
        arr = (_lib.ExtendFields * max(n, 1))()
        results = []
        for k, it in enumerate(items):
            u = it["u"]
            out = it.get("out") or (self._new(u), self._new(u), self._new(u))
            q = it.get("q")
            gamma = it.get("gamma")
            if q is not None and gamma is None:
                gamma = (self._new(u), self._new(u), self._new(u))
            phi = it.get("phi")
            if phi is None and self.precision == "mixed":
                phi = self._new(u)
            qs = (None, None, None) if q is None else q
            gs = (None, None, None) if gamma is None else gamma
            f = arr[k]
            f.u, f.v, f.w = (self._ptr(it[c], c).value for c in ("u", "v", "w"))
            f.src = self._ptr(it["src"], "src").value
            f.qx, f.qy, f.qz = (getattr(self._ptr(t, "q", optional=True), "value", None)
                                for t in qs)
            f.ue, f.ve, f.we = (self._ptr(t, "out").value for t in out)
            f.ug, f.vg, f.wg = (getattr(self._ptr(t, "gamma", optional=True), "value", None)
                                for t in gs)
            f.phi = getattr(self._ptr(phi, "phi", optional=True), "value", None)
            results.append((*out, *gs, phi))
        check(_lib.lib.extend_liquid_velocity_batched(self._h, n, arr, _stream_ptr(stream)),
              "extend_liquid_velocity_batched")
        return results

    def device_bytes(self) -> int:
        return int(_lib.lib.poisson_plan_device_bytes(self._h))

    def project(self, u, v, w, phat, rho, rho0, src, dt, p=None, lower=None, stream=None):
        """In-place projection of (u, v, w) = u*; returns (u, v, w, p).  `lower`:
        (x, y, z) planes of the faces at -1/2 of lower outflow ends (None
        elsewhere), updated in place (project_lf)."""
        if p is None:
            p = self._new(u)
        args = [self._h, self._ptr(u, "u"), self._ptr(v, "v"), self._ptr(w, "w")]
        rest = [self._ptr(phat, "phat"), self._ptr(rho, "rho"), float(rho0),
                self._ptr(src, "src", optional=True), float(dt), self._ptr(p, "p"),
                _stream_ptr(stream)]
        if lower is None:
            check(_lib.lib.project(*args, *rest), "project")
        else:
            check(_lib.lib.project_lf(*args, self._lower(lower, "lower"), *rest), "project_lf")
        return u, v, w, p

    def extend(self, u, v, w, src, q=None, out=None, gamma=None, phi=None, lower=None,
               lower_out=None, stream=None):
        """u_1^e = u - G phi (phi = L^+ src), u_Gamma = u_1^e - q.

        Returns (ue, ve, we, ug, vg, wg, phi); the u_Gamma entries are None
        without q.  `lower` / `lower_out`: (x, y, z) planes of u and of u_1^e
        (= u_Gamma) on the faces at -1/2 of lower outflow ends
        (extend_liquid_velocity_lf).
        """
        if out is None:
            out = (self._new(u), self._new(u), self._new(u))
        if q is not None and gamma is None:
            gamma = (self._new(u), self._new(u), self._new(u))
        if phi is None and self.precision == "mixed":
            phi = self._new(u)
        qs = (None, None, None) if q is None else q
        gs = (None, None, None) if gamma is None else gamma
        args = [self._h, self._ptr(u, "u"), self._ptr(v, "v"), self._ptr(w, "w"),
                self._ptr(src, "src")]
        qa = [self._ptr(t, "q", optional=True) for t in qs]
        oa = [self._ptr(t, "out") for t in out]
        ga = [self._ptr(t, "gamma", optional=True) for t in gs]
        tail = [self._ptr(phi, "phi", optional=True), _stream_ptr(stream)]
        if lower is None and lower_out is None:
            check(_lib.lib.extend_liquid_velocity(*args, *qa, *oa, *ga, *tail),
                  "extend_liquid_velocity")
        else:
            check(_lib.lib.extend_liquid_velocity_lf(
                args[0], args[1], args[2], args[3], self._lower(lower, "lower"), args[4], *qa, *oa,
                self._lower(lower_out, "lower_out"), *ga, *tail), "extend_liquid_velocity_lf")
        return (*out, *gs, phi)

    def interface_terms(self, C, mdot, rho1, rho2, phase=1, out=None, stream=None):
        """(s, qx, qy, qz): the Stefan source mdot (1/rho2 - 1/rho1)|grad C| at
        centres and (mdot/rho_e) n on faces, grad C by Youngs' differences;
        rho_e = rho1 (phase 1, liquid extension) or rho2 (phase 2, boiling)."""
        if out is None:
            out = tuple(self._new(C) for _ in range(4))
        args = [self._h, self._ptr(C, "C"), self._ptr(mdot, "mdot"), float(rho1), float(rho2),
                int(phase)]
        args += [self._ptr(t, "out") for t in out]
        check(_lib.lib.interface_terms(*args, _stream_ptr(stream)), "interface_terms")
        return tuple(out)

    def advect(self, C, ug, vg, wg, dt, beta=1.0, deflation=True, out=None, lower=None,
               stream=None):
        """C^{n+1} from C^n and the interface velocity on the faces (vof_advect:
        directional split, MTHINC flux, volume deflation when `deflation`);
        `lower`: the interface velocity's (x, y, z) planes at lower outflow ends."""
        if out is None:
            out = self._new(C)
        check(_lib.lib.vof_advect(self._h, self._ptr(C, "C"), self._ptr(ug, "ug"),
                                  self._ptr(vg, "vg"), self._ptr(wg, "wg"),
                                  self._lower(lower, "lower"), float(dt), float(beta),
                                  1 if deflation else 0, self._ptr(out, "out"),
                                  _stream_ptr(stream)), "vof_advect")
        return out

    def step(self, u, v, w, phat, rho, rho0, src_p, dt, src_ext, p=None, phi=None, q=None,
             out=None, gamma=None, lower=None, lower_e=None, stream=None):
        """One time step: projection of (u, v, w) = u* (in place) and extension of the
        projected velocity.  Returns (u, v, w, p, phi, ue, ve, we, ug, vg, wg); ue.. are
        None unless `out` is given, ug.. None without q.  `lower` (in u*, out u^{n+1})
        and `lower_e` (out u_1^e = u_Gamma): (x, y, z) planes of the faces at -1/2 of
        lower outflow ends (vof_step_lf)."""
        if p is None:
            p = self._new(u)
        if phi is None:
            phi = self._new(u)
        if q is not None and gamma is None:
            gamma = (self._new(u), self._new(u), self._new(u))
        qs = (None, None, None) if q is None else q
        es = (None, None, None) if out is None else out
        gs = (None, None, None) if gamma is None else gamma
        head = [self._h, self._ptr(u, "u"), self._ptr(v, "v"), self._ptr(w, "w")]
        mid = [self._ptr(phat, "phat"), self._ptr(rho, "rho"), float(rho0),
               self._ptr(src_p, "src_p", optional=True), float(dt), self._ptr(p, "p"),
               self._ptr(src_ext, "src_ext")]
        mid += [self._ptr(t, "q", optional=True) for t in qs]
        ea = [self._ptr(t, "out", optional=True) for t in es]
        tail = [self._ptr(t, "gamma", optional=True) for t in gs]
        tail += [self._ptr(phi, "phi"), _stream_ptr(stream)]
        if lower is None and lower_e is None:
            check(_lib.lib.vof_step(*head, *mid, *ea, *tail), "vof_step")
        else:
            check(_lib.lib.vof_step_lf(*head, self._lower(lower, "lower"), *mid, *ea,
                                       self._lower(lower_e, "lower_e"), *tail), "vof_step_lf")
        return (u, v, w, p, phi, *es, *gs)

    def step_interface(self, u, v, w, phat, rho, rho0, C, mdot, rho1, rho2, dt, phase=1,
                       p=None, phi=None, s=None, out=None, gamma=None, stream=None):
        """One time step with the interface terms formed inside its first and last
        passes (vof_step_interface): s from C and mdot in the right-hand-side pass
        (returned; the Stefan potential's right-hand side), q in the epilogue.
        Returns (u, v, w, p, phi, s, ue, ve, we, ug, vg, wg); ue.. are None unless
        `out` is given.  Same bits as interface_terms followed by step."""
        if p is None:
            p = self._new(u)
        if phi is None:
            phi = self._new(u)
        if s is None:
            s = self._new(u)
        if gamma is None:
            gamma = (self._new(u), self._new(u), self._new(u))
        es = (None, None, None) if out is None else out
        args = [self._h, self._ptr(u, "u"), self._ptr(v, "v"), self._ptr(w, "w"),
                self._ptr(phat, "phat"), self._ptr(rho, "rho"), float(rho0), self._ptr(C, "C"),
                self._ptr(mdot, "mdot"), float(rho1), float(rho2), int(phase), float(dt),
                self._ptr(p, "p"), self._ptr(s, "s")]
        args += [self._ptr(t, "out", optional=True) for t in es]
        args += [self._ptr(t, "gamma") for t in gamma]
        args += [self._ptr(phi, "phi"), _stream_ptr(stream)]
        check(_lib.lib.vof_step_interface(*args), "vof_step_interface")
        return (u, v, w, p, phi, s, *es, *gamma)

    def set_mixed(self, dc_steps: int, tol=None):
        """Mixed plans: at most dc_steps FP64 defect-correction steps, stopping per
        member once the estimated error is at most tol (tol <= 0: every step)."""
        check(_lib.lib.poisson_plan_set_mixed(self._h, int(dc_steps)), "poisson_plan_set_mixed")
        if tol is not None:
            check(_lib.lib.poisson_plan_set_mixed_tol(self._h, float(tol)),
                  "poisson_plan_set_mixed_tol")

    def mixed_report(self, n: int = 1, stream=None):
        """[(steps taken, last error estimate)] of the n members of the last mixed call."""
        steps = (ctypes.c_int * n)()
        est = (ctypes.c_double * n)()
        check(_lib.lib.poisson_plan_mixed_report(self._h, int(n), steps, est, _stream_ptr(stream)),
              "poisson_plan_mixed_report")
        return [(steps[i], est[i]) for i in range(n)]

    def last_mean(self, stream=None) -> float:
        out = ctypes.c_double(0.0)
        check(_lib.lib.poisson_plan_last_mean(self._h, ctypes.byref(out), _stream_ptr(stream)),
              "poisson_plan_last_mean")
        return out.value

    TUNING_KEYS = ("x_radix", "y_radix", "z_lines", "stencil_planes", "z_spectral", "z_radix",
                   "y_lines", "z_spectral_lines", "stream_planes", "stream_tiled", "rhs_tiled",
                   "epilogue_tiled",
                   "epilogue_planes", "interface_planes", "z_segment", "interface_tile")
    AUTOTUNED_KEYS = TUNING_KEYS[:8]

    def tune(self, key: str, value: int):
        """Launch-shape knob (see poisson_plan_tune); results do not change."""
        check(_lib.lib.poisson_plan_tune(self._h, key.encode(), int(value)), "poisson_plan_tune")

    def tuning(self) -> dict:
        """Current value of every tuning key."""
        out = {}
        for k in self.TUNING_KEYS:
            v = ctypes.c_int(0)
            check(_lib.lib.poisson_plan_get_tuning(self._h, k.encode(), ctypes.byref(v)),
                  "poisson_plan_get_tuning")
            out[k] = v.value
        return out

    def autotune(self, batch: int = 1, stream=None) -> dict:
        """Time every candidate of each tuning key on this plan's workspace and keep
        the fastest (see poisson_plan_autotune); returns the chosen values, with the
        z segment length that the autotuner picks together with z_lines."""
        chosen = (ctypes.c_int * 8)()
        check(_lib.lib.poisson_plan_autotune(self._h, int(batch), _stream_ptr(stream), chosen),
              "poisson_plan_autotune")
        out = dict(zip(self.AUTOTUNED_KEYS, list(chosen)))
        v = ctypes.c_int(0)
        check(_lib.lib.poisson_plan_get_tuning(self._h, b"z_segment", ctypes.byref(v)),
              "poisson_plan_get_tuning")
        out["z_segment"] = v.value
        return out

    def set_profiling(self, enable=True, classes=None):
        """Bracket kernel launches of this plan with HIP events: every class when
        `classes` is None, else only the named classes (see kernel_class_names)."""
        if not enable:
            mask = 0
        elif classes is None:
            mask = -1
        else:
            names = kernel_class_names()
            mask = 0
            for c in classes:
                mask |= 1 << names.index(c)
        check(_lib.lib.poisson_plan_set_profiling(self._h, int(mask)),
              "poisson_plan_set_profiling")

    def kernel_times(self):
        """{class name: (total ms, launches)} for the launches recorded since
        the last call (waits for them to finish)."""
        n = _lib.NUM_KERNEL_CLASSES
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        check(_lib.lib.poisson_plan_kernel_times(self._h, ms, cnt, n), "poisson_plan_kernel_times")
        out = {}
        for i in range(n):
            if cnt[i]:
                out[_lib.lib.poisson_kernel_class_name(i).decode()] = (ms[i], cnt[i])
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib.poisson_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
