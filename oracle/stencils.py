"""Second-order marker-and-cell stencils (section 3, staggered finite differences).

Array layout (nz, ny, nx); u[k, j, i] on face i+1/2, v on j+1/2, w on k+1/2.
Every direction has n+1 faces, -1/2 .. n-1/2; the arrays hold the n faces
+1/2 .. n-1/2, so the face at -1/2 is implicit: the wrapped last face
(periodic) or a wall with zero normal velocity.

* G(p): face gradient (p[i+1] - p[i]) / dx on face i+1/2 (in z the centre
  distance dzc).  On a wall face ('N') it is zero (the homogeneous Neumann
  pressure condition of section 3.2); on an outflow face ('D', p = 0 on the
  face, half a cell from the centre) it is (0 - p[n-1]) / (dx / 2) at the
  upper end and (p[0] - 0) / (dx / 2) at the lower end.
* D(u): cell divergence (u[i+1/2] - u[i-1/2]) / dx + ... + (w[k+1/2] -
  w[k-1/2]) / dzf[k].
* L_h = D(G(.)): the 7-point Laplacian whose discrete Poisson equation the
  paper's direct solver inverts.
* face_density: arithmetic mean of the two adjacent cell densities, the
  reading used for rho at velocity points in the split of section 3.2; on a
  boundary face, the inner cell's density.

An outflow at a lower end ('D' at x-, y- or z-) has a face at -1/2 whose
velocity the n-face layout does not hold: it travels as a separate plane per
direction, ``lower = (u_lo, v_lo, w_lo)`` shaped (nz, ny), (nz, nx) and
(ny, nx) (None for a direction without a lower outflow), which ``div`` takes
and ``grad_lower`` / ``face_density_lower`` complete.
"""
from __future__ import annotations

import numpy as np


def _spacings(g, axis):
    """(interior centre distances of faces 1/2 .. n-3/2, wrap distance, lower
    half width, upper half width), shaped to broadcast along ``axis``."""
    n = (g.nx, g.ny, g.nz)[2 - axis]
    if axis == 2:
        return np.full(n - 1, g.dx), g.dx, 0.5 * g.dx, 0.5 * g.dx
    if axis == 1:
        return np.full(n - 1, g.dy), g.dy, 0.5 * g.dy, 0.5 * g.dy
    dzf = g.dzf
    return 0.5 * (dzf[:-1] + dzf[1:]), 0.5 * (dzf[-1] + dzf[0]), 0.5 * dzf[0], 0.5 * dzf[-1]


def _ends(g, axis):
    return g.ends[2 - axis]


def _as_axis0(a, axis):
    return np.moveaxis(a, axis, 0)


def _bcast(v, ndim):
    return np.asarray(v).reshape((-1,) + (1,) * (ndim - 1))


def grad_all_faces(p, g, axis):
    """Gradient along ``axis`` on all n+1 faces -1/2 .. n-1/2 (the first
    axis of the result is the face index)."""
    q = _as_axis0(p, axis)
    n = q.shape[0]
    inner, wrap, h_lo, h_hi = _spacings(g, axis)
    lo, hi = _ends(g, axis)
    out = np.zeros((n + 1,) + q.shape[1:], dtype=q.dtype)
    if n > 1:
        out[1:n] = (q[1:] - q[:-1]) / _bcast(inner, q.ndim)
    if lo == "P":
        out[0] = (q[0] - q[n - 1]) / wrap
        out[n] = out[0]
    else:
        if lo == "D":
            out[0] = (q[0] - 0.0) / h_lo
        if hi == "D":
            out[n] = (0.0 - q[n - 1]) / h_hi
    return out


def div_all_faces(faces, g, axis):
    """(F[i+1] - F[i]) / width_i from the n+1 face values of ``axis``, moved
    back to the field layout."""
    n = faces.shape[0] - 1
    width = {2: np.full(n, g.dx), 1: np.full(n, g.dy), 0: g.dzf}[axis]
    d = (faces[1:] - faces[:-1]) / _bcast(width, faces.ndim)
    return np.moveaxis(d, 0, axis)


def grad(p, g):
    """G(p) -> (gx, gy, gz) on the stored faces +1/2 .. n-1/2."""
    p = np.asarray(p)
    if p.dtype != np.longdouble:
        p = p.astype(np.float64, copy=False)
    return tuple(np.moveaxis(grad_all_faces(p, g, axis)[1:], 0, axis) for axis in (2, 1, 0))


def _lower_index(axis):
    return {2: 0, 1: 1, 0: 2}[axis]


def div(u, v, w, g, lower=None):
    """D(u, v, w) at cell centres from the stored faces; `lower` holds the
    velocities on the faces at -1/2 of the directions with an outflow at
    their lower end (see the module docstring)."""
    out = None
    for arr, axis in ((u, 2), (v, 1), (w, 0)):
        lo, _ = _ends(g, axis)
        q = _as_axis0(np.asarray(arr), axis)
        faces = np.zeros((q.shape[0] + 1,) + q.shape[1:], dtype=np.result_type(q, np.float64))
        faces[1:] = q
        if lo == "D":
            plane = None if lower is None else lower[_lower_index(axis)]
            if plane is None:
                raise ValueError("an outflow at the lower end needs its face's velocity "
                                 "(the layout stores no face at -1/2)")
            faces[0] = plane
        if lo == "P":
            faces[0] = q[-1]
        term = div_all_faces(faces, g, axis)
        out = term if out is None else out + term
    return out


def grad_lower(p, g):
    """G(p) on the faces at -1/2 of the directions with a lower outflow end
    ((p_0 - 0) / (h / 2)), as (x, y, z) planes; None elsewhere."""
    p = np.asarray(p)
    if p.dtype != np.longdouble:
        p = p.astype(np.float64, copy=False)
    return tuple(grad_all_faces(p, g, axis)[0] if _ends(g, axis)[0] == "D" else None
                 for axis in (2, 1, 0))


def face_density_lower(rho, g):
    """rho on the faces at -1/2 of the directions with a lower outflow end:
    the inner (first) cell's density, as (x, y, z) planes; None elsewhere."""
    rho = np.asarray(rho, dtype=np.float64)
    return tuple(np.take(rho, 0, axis=axis) if _ends(g, axis)[0] == "D" else None
                 for axis in (2, 1, 0))


def lap(p, g):
    """L_h p = D(G(p)) with every boundary face, lower outflow faces included."""
    p = np.asarray(p)
    if p.dtype != np.longdouble:
        p = p.astype(np.float64, copy=False)
    out = None
    for axis in (2, 1, 0):
        term = div_all_faces(grad_all_faces(p, g, axis), g, axis)
        out = term if out is None else out + term
    return out


def face_density(rho, g):
    """rho on faces: (rho[i] + rho[i+1]) / 2; on a boundary face, the inner cell's rho."""
    rho = np.asarray(rho, dtype=np.float64)
    out = []
    for axis in (2, 1, 0):
        lo, _ = _ends(g, axis)
        if lo == "P" and rho.shape[axis] > 1:
            rf = 0.5 * (rho + np.roll(rho, -1, axis=axis))
        else:
            rf = rho.copy()
            n = rho.shape[axis]
            a = [slice(None)] * 3
            b = [slice(None)] * 3
            a[axis] = slice(0, n - 1)
            b[axis] = slice(1, n)
            rf[tuple(a)] = 0.5 * (rho[tuple(a)] + rho[tuple(b)])
        out.append(rf)
    return tuple(out)
