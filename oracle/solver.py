"""Plain FP64 spectral Poisson solve, projection and extension (test oracle).

The paper (section 3.2) solves the constant-coefficient second-order
finite-difference Poisson equation with an FFT-based direct method and
(section 3.6) re-uses it for the Stefan-flow potential.  A direct method
reaches exactly the solution of the discrete problem, so the oracle is that
definition computed in the most transparent way available:

1. x and y: library transforms that diagonalise the 1-D second difference
   under each pair of end conditions (scipy.fft, orthonormal):
     periodic                      complex DFT   -(4/h^2) sin^2(pi m / n)
     wall / wall        (N N)      DCT-II        -(4/h^2) sin^2(pi m / (2n))
     outflow / outflow  (D D)      DST-II        -(4/h^2) sin^2(pi (m+1) / (2n))
     wall / outflow     (N D)      DCT-IV        -(4/h^2) sin^2(pi (2m+1) / (4n))
     outflow / wall     (D N)      DST-IV        -(4/h^2) sin^2(pi (2m+1) / (4n))
   (outflow: p = 0 on the boundary face, half a cell beyond the last centre).
2. z: the tridiagonal z operator A = W^-1 S (S symmetric, W = diag(dzf)) is
   diagonalised by the generalised symmetric eigenproblem S v = mu W v
   (scipy.linalg.eigh), so (A + lambda I)^-1 = V diag(1/(mu+lambda)) V^T W.
   No tridiagonal sweep is used anywhere in the oracle.
3. Without an outflow end the operator is singular.  Its single zero
   eigenvalue (the constant mode, reached only on the (kx, ky) = (0, 0) line)
   is dropped: this is the W-weighted pseudo-inverse.  The volume-weighted
   mean is also subtracted explicitly from the right-hand side before, and
   from the solution after, so that a large constant offset cannot leak
   through the numerically computed null vector.  With an outflow end every
   eigenvalue is negative and the plain inverse is taken (no mean removed,
   no gauge).
4. Inverse transforms.
5. One step of iterative refinement: the residual of the discrete equation,
   f - mean_W(f) - L_h p, is evaluated in extended precision (numpy
   longdouble) and its solution added.  The eigenvector route alone loses
   accuracy on long, strongly stretched z lines (relative errors up to ~1e-11
   at nz = 600-1024, where the condition number of the z operator is ~1e5-1e6);
   one refinement step brings it to the accuracy of the discrete solution
   (a second step changes it by ~1e-17).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

from .grid import Grid
from .stencils import grad, div, lap, face_density, grad_lower, face_density_lower


def _pair(ends):
    return (ends, ends) if isinstance(ends, str) and len(ends) == 1 else tuple(ends)


def eigenvalues_1d(n: int, h: float, ends) -> np.ndarray:
    """Eigenvalues of the 1-D second difference in the library transform's
    order; ``ends`` is a letter (both ends) or a (lower, upper) pair."""
    lo, hi = _pair(ends)
    m = np.arange(n, dtype=np.float64)
    if lo == "P":
        arg = np.pi * m / n
    elif lo == "N" and hi == "N":
        arg = np.pi * m / (2.0 * n)
    elif lo == "D" and hi == "D":
        arg = np.pi * (m + 1.0) / (2.0 * n)
    else:
        arg = np.pi * (2.0 * m + 1.0) / (4.0 * n)
    return -(4.0 / (h * h)) * np.sin(arg) ** 2


def z_operator_dense(g: Grid):
    """S (symmetric) and W = diag(dzf) with A_z = W^-1 S the z second difference.

    Row k of A_z: [(p[k+1]-p[k]) / dzc[k] - (p[k]-p[k-1]) / dzc[k-1]] / dzf[k],
    with zero flux through walls, wrapped couplings when z is periodic, and
    through an outflow face the flux (0 - p) / (dzf / 2) of the end cell.
    """
    nz = g.nz
    S = np.zeros((nz, nz))
    for k in range(nz - 1):
        c = 1.0 / g.dzc[k]
        S[k, k + 1] += c
        S[k + 1, k] += c
        S[k, k] -= c
        S[k + 1, k + 1] -= c
    if g.ends[2][0] == "P":
        c = 1.0 / g.dzc[nz - 1]
        S[nz - 1, 0] += c
        S[0, nz - 1] += c
        S[nz - 1, nz - 1] -= c
        S[0, 0] -= c
    lo, hi = g.ends[2]
    if lo == "D":
        S[0, 0] -= 2.0 / g.dzf[0]
    if hi == "D":
        S[nz - 1, nz - 1] -= 2.0 / g.dzf[nz - 1]
    return S, np.diag(g.dzf)


# (lower, upper) -> (library transform, type); periodic uses the complex DFT
_R2R = {("N", "N"): ("dct", 2), ("D", "D"): ("dst", 2), ("N", "D"): ("dct", 4),
        ("D", "N"): ("dst", 4)}


def _fwd(a, axis, ends):
    if ends[0] == "P":
        return np.fft.fft(a, axis=axis)
    kind, t = _R2R[tuple(ends)]
    f = sfft.dct if kind == "dct" else sfft.dst
    return f(a, type=t, norm="ortho", axis=axis)


def _inv(a, axis, ends):
    if ends[0] == "P":
        return np.fft.ifft(a, axis=axis)
    kind, t = _R2R[tuple(ends)]
    f = sfft.idct if kind == "dct" else sfft.idst
    return f(a, type=t, norm="ortho", axis=axis)


def _spectral(fc, g: Grid):
    """Eigen-decomposition solve of L_h p = fc for a compatible fc (steps 1-4)."""
    F = fc.astype(np.complex128)
    ex, ey, ez = g.ends
    F = _fwd(F, 2, ex)
    F = _fwd(F, 1, ey)
    lam = (eigenvalues_1d(g.ny, g.dy, ey)[:, None]
           + eigenvalues_1d(g.nx, g.dx, ex)[None, :]).reshape(-1)

    S, W = z_operator_dense(g)
    mu, V = sla.eigh(S, W)

    B = F.reshape(g.nz, -1)
    C = V.T @ (g.dzf[:, None] * B)
    den = mu[:, None] + lam[None, :]
    inv = np.zeros_like(den)
    nonzero = np.ones_like(den, dtype=bool)
    if g.singular:
        null = int(np.argmin(np.abs(mu)))
        # the constant mode is the only (numerically) zero eigenvalue
        rest = np.delete(np.abs(mu), null)
        if rest.size and not np.abs(mu[null]) < 1e-6 * rest.min():
            raise RuntimeError("z operator has no isolated null mode")
        nonzero[null, 0] = False  # line (0, 0): lam == 0 exactly
    inv[nonzero] = 1.0 / den[nonzero]
    P = (V @ (C * inv)).reshape(g.shape)

    P = _inv(P, 1, ey)
    P = _inv(P, 2, ex)
    return P.real.copy()


def _lap_extended(p, g: Grid):
    """L_h p evaluated in numpy longdouble (the same stencil, wider arithmetic)."""
    return lap(np.asarray(p, dtype=np.longdouble), g)


def solve(f, g: Grid, return_mean: bool = False):
    """FP64 solution of the discrete Poisson equation.

    Without an outflow end: p with L_h p = f - mean_W(f) and sum(dV p) = 0.
    With one: p = L_h^-1 f (the mean returned is then 0).
    """
    f = np.asarray(f, dtype=np.float64)
    if f.shape != g.shape:
        raise ValueError(f"rhs shape {f.shape} != grid {g.shape}")
    # the definition: right-hand side minus its volume-weighted mean
    fbar = g.weighted_mean(f) if g.singular else 0.0
    fc = f - fbar
    p = _spectral(fc, g)
    # step 5: one refinement step with an extended-precision residual
    r = (fc.astype(np.longdouble) - _lap_extended(p, g)).astype(np.float64)
    if g.singular:
        r -= g.weighted_mean(r)
    p = p + _spectral(r, g)
    if g.singular:
        # the gauge: zero volume-weighted mean (removes only round-off here)
        p -= g.weighted_mean(p)
    if return_mean:
        return p, fbar
    return p


def _has_lower_outflow(g: Grid):
    return any(lo == "D" for lo, _ in g.ends)


def _check_lower(g: Grid, lower):
    if lower is None:
        if _has_lower_outflow(g):
            raise ValueError("an outflow at a lower end needs the velocities of its faces at -1/2 "
                             "(`lower`)")
        return
    for (lo, _), plane in zip(g.ends, lower):
        if (lo == "D") != (plane is not None):
            raise ValueError("`lower` holds a plane exactly for the directions with a lower outflow")


def assemble_pressure_rhs(ustar, vstar, wstar, phat, rho, rho0, src, dt, g: Grid, lower=None):
    """Right-hand side b of L_h p = b (section 3.2, pressure equation x rho0).

    b = rho0 D[(1/rho0 - 1/rho_f) G p_hat] + (rho0/dt) (D u* - s), with
    s = mdot (1/rho2 - 1/rho1) delta_Gamma the phase-change source; `lower`
    holds u* on the faces at -1/2 of lower outflow ends.
    """
    gx, gy, gz = grad(phat, g)
    rfx, rfy, rfz = face_density(rho, g)
    cx = (1.0 / rho0 - 1.0 / rfx) * gx
    cy = (1.0 / rho0 - 1.0 / rfy) * gy
    cz = (1.0 / rho0 - 1.0 / rfz) * gz
    clow = None
    if lower is not None:
        gl = grad_lower(phat, g)
        rl = face_density_lower(rho, g)
        clow = tuple(None if a is None else (1.0 / rho0 - 1.0 / r) * a for a, r in zip(gl, rl))
    return (rho0 * div(cx, cy, cz, g, clow)
            + (rho0 / dt) * (div(ustar, vstar, wstar, g, lower) - src))


def project(ustar, vstar, wstar, phat, rho, rho0, src, dt, g: Grid, lower=None):
    """Pressure-split projection step (section 3.2).

    Returns (u, v, w, p): p solves L_h p = b (assemble_pressure_rhs) and
    u^{n+1} = u* - dt [ (1/rho0) G p + (1/rho_f - 1/rho0) G p_hat ].  With an
    outflow at a lower end, `lower` holds u* on the faces at -1/2 (planes,
    see ``oracle.stencils``) and the result gains a fifth entry, u^{n+1} on
    those faces (rho there is the first cell's).
    """
    _check_lower(g, lower)
    b = assemble_pressure_rhs(ustar, vstar, wstar, phat, rho, rho0, src, dt, g, lower)
    p = solve(b, g)
    gpx, gpy, gpz = grad(p, g)
    ghx, ghy, ghz = grad(phat, g)
    rfx, rfy, rfz = face_density(rho, g)
    u = ustar - dt * (gpx / rho0 + (1.0 / rfx - 1.0 / rho0) * ghx)
    v = vstar - dt * (gpy / rho0 + (1.0 / rfy - 1.0 / rho0) * ghy)
    w = wstar - dt * (gpz / rho0 + (1.0 / rfz - 1.0 / rho0) * ghz)
    if lower is None:
        return u, v, w, p
    gpl, ghl, rl = grad_lower(p, g), grad_lower(phat, g), face_density_lower(rho, g)
    new_lower = tuple(None if a is None else a - dt * (b_ / rho0 + (1.0 / r - 1.0 / rho0) * c)
                      for a, b_, c, r in zip(lower, gpl, ghl, rl))
    return u, v, w, p, new_lower


def extend(u, v, w, src, g: Grid, q=None, lower=None):
    """Liquid-velocity extension and interface velocity (section 3.6).

    phi solves L_h phi = s (the Stefan potential, s = mdot (1/rho2 - 1/rho1)|grad C|),
    u_1^e = u - G phi and, when q = (mdot/rho1) n on faces is given,
    u_Gamma = u_1^e - q.  Returns (ue, ve, we, ug, vg, wg, phi); the u_Gamma
    entries are None without q.  With an outflow at a lower end, `lower`
    holds u on the faces at -1/2 and the result gains an eighth entry, u_1^e
    on those faces; u_Gamma equals it there (q is zero on a non-periodic
    boundary face).
    """
    _check_lower(g, lower)
    phi = solve(src, g)
    gx, gy, gz = grad(phi, g)
    ue, ve, we = u - gx, v - gy, w - gz
    if q is None:
        out = (ue, ve, we, None, None, None, phi)
    else:
        out = (ue, ve, we, ue - q[0], ve - q[1], we - q[2], phi)
    if lower is None:
        return out
    gl = grad_lower(phi, g)
    return out + (tuple(None if a is None else a - b for a, b in zip(lower, gl)),)
