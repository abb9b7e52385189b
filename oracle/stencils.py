"""Second-order marker-and-cell stencils (section 3, staggered finite differences).

Array layout (nz, ny, nx); u[k, j, i] on face i+1/2, v on j+1/2, w on k+1/2.

* G(p): face gradient.  (p[i+1] - p[i]) / dx on face i+1/2, periodic wrap or,
  with walls, zero on the wall face (zero normal gradient, the homogeneous
  Neumann pressure condition of section 3.2).  In z the distance is dzc.
* D(u): cell divergence.  (u[i+1/2] - u[i-1/2]) / dx + ... + (w[k+1/2] -
  w[k-1/2]) / dzf[k], with the face at -1/2 wrapped (periodic) or zero (wall).
* L_h = D(G(.)): the 7-point Laplacian whose discrete Poisson equation the
  paper's direct solver inverts.
* face_density: arithmetic mean of the two adjacent cell densities, the
  reading used for rho at velocity points in the split of section 3.2.
"""
from __future__ import annotations

import numpy as np


def _forward_diff(p, axis, h, letter):
    """(p[i+1] - p[i]) / h along ``axis``; wall face (last index) = 0 for N."""
    if letter == "P":
        return (np.roll(p, -1, axis=axis) - p) / h
    out = np.zeros_like(p)
    n = p.shape[axis]
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    lo[axis] = slice(0, n - 1)
    hi[axis] = slice(1, n)
    out[tuple(lo)] = (p[tuple(hi)] - p[tuple(lo)]) / (
        h if np.ndim(h) == 0 else h[tuple(lo)])
    return out


def _backward_face(u, axis, letter):
    """Face value at i-1/2 for each cell i: wrapped, or zero at the wall."""
    if letter == "P":
        return np.roll(u, 1, axis=axis)
    out = np.zeros_like(u)
    n = u.shape[axis]
    dst = [slice(None)] * 3
    src = [slice(None)] * 3
    dst[axis] = slice(1, n)
    src[axis] = slice(0, n - 1)
    out[tuple(dst)] = u[tuple(src)]
    return out


def grad(p, g):
    """G(p) -> (gx, gy, gz) on faces."""
    p = np.asarray(p, dtype=np.float64)
    gx = _forward_diff(p, 2, g.dx, g.bc[0])
    gy = _forward_diff(p, 1, g.dy, g.bc[1])
    if g.bc[2] == "P":
        gz = (np.roll(p, -1, axis=0) - p) / g.dzc[:, None, None]
    else:
        gz = _forward_diff(p, 0, g.dzc[:, None, None], "N")
    return gx, gy, gz


def div(u, v, w, g):
    """D(u, v, w) at cell centres."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    dxu = (u - _backward_face(u, 2, g.bc[0])) / g.dx
    dyv = (v - _backward_face(v, 1, g.bc[1])) / g.dy
    dzw = (w - _backward_face(w, 0, g.bc[2])) / g.dzf[:, None, None]
    return dxu + dyv + dzw


def lap(p, g):
    """L_h p = D(G(p))."""
    return div(*grad(p, g), g)


def face_density(rho, g):
    """rho on faces: (rho[i] + rho[i+1]) / 2; on a wall face, the inner cell's rho."""
    rho = np.asarray(rho, dtype=np.float64)
    out = []
    for axis, letter in ((2, g.bc[0]), (1, g.bc[1]), (0, g.bc[2])):
        if letter == "P" and rho.shape[axis] > 1:
            rf = 0.5 * (rho + np.roll(rho, -1, axis=axis))
        else:
            rf = rho.copy()
            n = rho.shape[axis]
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[axis] = slice(0, n - 1)
            hi[axis] = slice(1, n)
            rf[tuple(lo)] = 0.5 * (rho[tuple(lo)] + rho[tuple(hi)])
        out.append(rf)
    return tuple(out)
