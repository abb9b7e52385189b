"""VoF advection of section 3.1 (test oracle, FP64): directional splitting with
the MTHINC flux and the implicit volume-deflation correction.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What it computes.  Eq. (cadv), dC/dt + div(u_G H) = C div(u_G), advanced from
C^n to C^{n+1} with the interface velocity u_G of section 3.6 by

* eq. (fluxes): three one-dimensional sweeps, x then y then z, each implicit
  in its own result through the divergence of that velocity component:
      C*   = C^n  - (f_{i+1/2} - f_{i-1/2}) / dx + dt C*   (u_{i+1/2} - u_{i-1/2}) / dx
      C**  = C*   - (g_{j+1/2} - g_{j-1/2}) / dy + dt C**  (v_{j+1/2} - v_{j-1/2}) / dy
      C*** = C**  - (h_{k+1/2} - h_{k-1/2}) / dz + dt C*** (w_{k+1/2} - w_{k-1/2}) / dz
  where f is computed from C^n, g from C* and h from C**;
* eq. (final_corr_1) / (final_corr_2): with F = C* du/dx + C** dv/dy + C*** dw/dz
  (the divided differences above),
      C^{n+1} = C*** - dt F                                  (final_corr_1, the
                                                              original method),
      C^{n+1} = C*** - dt F + dt C^{n+1} div_h(u_G)           (final_corr_2, the
                                                              paper's deflation),
  div_h the cell divergence of the stored face velocities.

The flux (Ii et al., "An interface capturing method with a continuous
function: the THINC method with multi-dimensional reconstruction",
J. Comput. Phys. 231 (2012); the paper only cites it).  Reading, linear
(normal-only) reconstruction:

1. In a cell with local coordinates X = (x - x_c)/dx, Y, Z in [-1/2, 1/2]
   the indicator is H(X) = 1/2 (1 + tanh(beta (m . X + d))), m the unit
   normal in those coordinates pointing towards increasing C:
   m = (dx g_x, dy g_y, dz_k g_z) / |.|, g the Youngs gradient of C at the
   cell centre (the corner construction of ``oracle.interface``); beta is
   the sharpness parameter (an input; 1 by default).
2. Only cells with EPS < C < 1 - EPS and a gradient above rounding level,
   |(dx g_x, dy g_y, dz_k g_z)| > GRAD_MIN (the change of C across the cell),
   are reconstructed; any other cell is uniform, H = C (a normal drawn from
   rounding noise would otherwise reconstruct a profile in a constant
   field).  Ghost cells beyond a non-periodic end are uniform with the end
   cell's C.
3. d is fixed by the cell's volume: the integral of H over the cell equals C.
   Here it is found by bisection (the definition: d is the root of that
   monotone equation).
4. The integral of H over a box of the cell (the cell itself, or the part a
   face sweeps in one step) is semi-analytical: exact along the dominant
   axis a (the first of x, y, z whose |m| is within a factor 1 - 1e-9 of the
   largest; the tolerance keeps the choice away from rounding ties),
       int_{s0}^{s1} H ds = (s1 - s0)/2
            + [ln cosh(beta (m_a s1 + A)) - ln cosh(beta (m_a s0 + A))] / (2 beta m_a),
   A = d + m . (transverse coordinates), and by 2-point Gauss-Legendre
   quadrature in each of the two other axes over the box's extent.
5. The flux through a face with velocity V in a sweep along an axis of
   upwind-cell width h: xi = |V| dt / h (clamped to [0, 1]: one step moves
   at most one cell); the swept box is the last xi of the upwind cell along
   the axis, X in [1/2 - xi, 1/2] for V >= 0 (upwind: the lower cell), or
   [-1/2, -1/2 + xi] for V < 0 (the upper cell), the full extent in the other
   axes; the flux is sign(V) h times the box integral (V dt C for a uniform
   cell).

Boundaries: periodic faces wrap; the lower face of a wall direction is
implicit with zero velocity, the stored upper face is taken as stored (the
caller keeps it zero at a wall); an outflow end takes its face velocity (the
stored last face at an upper end, the plane of `lower` at a lower end, as in
``oracle.stencils``), inflow through it carrying the ghost's C.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid
from .interface import youngs_gradient

EPS = 1e-8            # reconstruction band: EPS < C < 1 - EPS
GRAD_MIN = 1e-12      # and a change of C across the cell above this
AXIS_TOL = 1e-9       # dominant-axis tie tolerance
_GAUSS = 0.5 / np.sqrt(3.0)  # 2-point Gauss-Legendre nodes on [-1/2, 1/2]: +-1/(2 sqrt 3)

_AX = {"x": 2, "y": 1, "z": 0}  # array axis of each direction (arrays are (nz, ny, nx))


def _lncosh(x):
    a = np.abs(x)
    return a + np.log1p(np.exp(-2.0 * a)) - np.log(2.0)


def normals(C, g: Grid):
    """(m, |g_h|): the unit normal m in cell coordinates, components (x, y, z)
    each shaped like C, from the Youngs gradient g, and the magnitude of
    g_h = (dx g_x, dy g_y, dz_k g_z); m is zero where g_h is."""
    gx, gy, gz = youngs_gradient(C, g)
    hx = g.dx * gx
    hy = g.dy * gy
    hz = g.dzf[:, None, None] * gz
    mag = np.sqrt(hx * hx + hy * hy + hz * hz)
    safe = np.where(mag > 0.0, mag, 1.0)
    on = mag > 0.0
    return (np.where(on, hx / safe, 0.0), np.where(on, hy / safe, 0.0),
            np.where(on, hz / safe, 0.0)), mag


def dominant_axis(m):
    """Index 0, 1, 2 (x, y, z) of the dominant component of each normal, the
    first whose magnitude is at least (1 - AXIS_TOL) times the largest."""
    a = np.abs(np.stack(m))
    big = a.max(axis=0) * (1.0 - AXIS_TOL)
    out = np.full(a.shape[1:], 2, dtype=np.int64)
    out = np.where(a[1] >= big, 1, out)
    out = np.where(a[0] >= big, 0, out)
    return out


class Geometry:
    """Per-cell quantities of the semi-analytical integral that do not depend
    on d or on the box: the dominant axis a, the two transverse axes t1 < t2
    and the components of m along them (m: (3, n), x-y-z order)."""

    def __init__(self, m):
        m = np.asarray(m, dtype=np.float64)
        n = m.shape[1]
        self.idx = np.arange(n)
        self.a = dominant_axis(m)
        self.t1 = np.where(self.a == 0, 1, 0)
        self.t2 = np.where(self.a == 2, 1, 2)
        self.ma = m[self.a, self.idx]
        self.m1 = m[self.t1, self.idx]
        self.m2 = m[self.t2, self.idx]


def box_integral(m, d, lo, hi, beta, geo=None):
    """Integral of H = 1/2 (1 + tanh(beta (m . X + d))) over the boxes
    [lo, hi] (normalised coordinates), semi-analytically (step 4).

    m: (3, n) normals, d: (n,), lo / hi: (3, n) box corners, x-y-z order;
    geo: Geometry(m), if already at hand."""
    G = Geometry(m) if geo is None else geo
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    idx = G.idx
    c1 = 0.5 * (lo[G.t1, idx] + hi[G.t1, idx])
    r1 = hi[G.t1, idx] - lo[G.t1, idx]
    c2 = 0.5 * (lo[G.t2, idx] + hi[G.t2, idx])
    r2 = hi[G.t2, idx] - lo[G.t2, idx]
    s0 = lo[G.a, idx]
    s1 = hi[G.a, idx]
    total = np.zeros(idx.shape[0])
    for p in (-1.0, 1.0):
        for q in (-1.0, 1.0):
            y = c1 + p * _GAUSS * r1  # nodes c +- r / (2 sqrt 3)
            z = c2 + q * _GAUSS * r2
            A = d + G.m1 * y + G.m2 * z
            J = 0.5 * (s1 - s0) + (_lncosh(beta * (G.ma * s1 + A))
                                   - _lncosh(beta * (G.ma * s0 + A))) / (2.0 * beta * G.ma)
            total = total + 0.25 * r1 * r2 * J
    return total


def solve_d(m, C, beta, iters=64):
    """d with box_integral(m, d, cell) = C, by bisection (step 3).  m: (3, n).
    The bracket [-(2 + 25/beta), 2 + 25/beta] holds the root for every C in
    the band (at its ends H differs from 0 or 1 by less than 1e-21 over the
    cell); 64 halvings take it below the spacing of doubles."""
    n = m.shape[1]
    geo = Geometry(m)
    lo = np.full((3, n), -0.5)
    hi = np.full((3, n), 0.5)
    span = 2.0 + 25.0 / beta
    a = np.full(n, -span)
    b = np.full(n, span)
    for _ in range(iters):
        mid = 0.5 * (a + b)
        below = box_integral(m, mid, lo, hi, beta, geo) < C
        a = np.where(below, mid, a)
        b = np.where(below, b, mid)
    return 0.5 * (a + b)


def _band(C, mag):
    return (C > EPS) & (C < 1.0 - EPS) & (mag > GRAD_MIN)


def _face_velocities(V, g: Grid, direction: str, lower_plane=None):
    """Velocities of the n+1 faces -1/2 .. n-1/2 along `direction` (first
    array axis = face index), from the stored n faces (and, at a lower
    outflow end, the plane of the face at -1/2)."""
    ax = _AX[direction]
    lo, _ = g.ends[{"x": 0, "y": 1, "z": 2}[direction]]
    q = np.moveaxis(np.asarray(V, dtype=np.float64), ax, 0)
    faces = np.zeros((q.shape[0] + 1,) + q.shape[1:])
    faces[1:] = q
    if lo == "D":
        if lower_plane is None:
            raise ValueError("an outflow at the lower end needs its face's velocity "
                             "(the layout stores no face at -1/2)")
        faces[0] = lower_plane
    if lo == "P":
        faces[0] = q[-1]
    return faces


def sweep(C, V, direction: str, dt: float, g: Grid, beta: float = 1.0, lower_plane=None):
    """One split step of eq. (fluxes) along `direction` ('x', 'y' or 'z').
    Returns (C_new, delta) with delta = (V_{+1/2} - V_{-1/2}) / h at every cell."""
    C = np.asarray(C, dtype=np.float64)
    ax = _AX[direction]
    d_idx = {"x": 0, "y": 1, "z": 2}[direction]
    periodic = g.ends[d_idx][0] == "P"
    n = C.shape[ax]
    if direction == "x":
        widths = np.full(n, g.dx)
    elif direction == "y":
        widths = np.full(n, g.dy)
    else:
        widths = g.dzf.copy()

    # reconstruction of every cell of the sweep's input
    m, mag = normals(C, g)
    band = _band(C, mag)
    d = np.zeros(C.shape)
    if band.any():
        mb = np.stack([c[band] for c in m])
        d[band] = solve_d(mb, C[band], beta)

    # faces -1/2 .. n-1/2 along the axis: velocity, upwind cell
    Vf = _face_velocities(V, g, direction, lower_plane)  # (n+1, ...) along axis 0
    Cm = np.moveaxis(C, ax, 0)
    mm = [np.moveaxis(c, ax, 0) for c in m]
    dm = np.moveaxis(d, ax, 0)
    bm = np.moveaxis(band, ax, 0)
    flux = np.zeros_like(Vf)
    for f in range(n + 1):
        vel = Vf[f]
        below, above = f - 1, f  # the cells on either side of face f
        if periodic:
            below %= n
            above %= n
        pos = vel >= 0.0
        # V >= 0: the upwind cell is the one below, its last xi is swept;
        # V < 0: the cell above, its first xi
        for side, sel, from_below in ((below, pos, True), (above, ~pos, False)):
            if not sel.any():
                continue
            if side < 0 or side >= n:  # ghost: uniform with the end cell's C
                cell = 0 if side < 0 else n - 1
                h = widths[cell]
                xi = np.clip(np.abs(vel[sel]) * dt / h, 0.0, 1.0)
                flux[f][sel] = np.sign(vel[sel]) * h * xi * Cm[cell][sel]
                continue
            h = widths[side]
            xi = np.clip(np.abs(vel) * dt / h, 0.0, 1.0)
            val = np.sign(vel) * h * xi * Cm[side]  # uniform cells
            rec = sel & bm[side]
            if rec.any():
                k = int(rec.sum())
                lo = np.full((3, k), -0.5)
                hi = np.full((3, k), 0.5)
                a3 = 2 - ax  # x-y-z order index of this axis
                xr = xi[rec]
                if from_below:
                    lo[a3] = 0.5 - xr
                else:
                    hi[a3] = -0.5 + xr
                mk = np.stack([c[side][rec] for c in mm])
                val[rec] = np.sign(vel[rec]) * h * box_integral(mk, dm[side][rec], lo, hi, beta)
            flux[f][sel] = val[sel]
    hw = widths.reshape((-1,) + (1,) * (C.ndim - 1))
    delta = (Vf[1:] - Vf[:-1]) / hw
    Cn = (Cm - (flux[1:] - flux[:-1]) / hw) / (1.0 - dt * delta)
    return np.moveaxis(Cn, 0, ax), np.moveaxis(delta, 0, ax)


def advect(C, ug, vg, wg, dt: float, g: Grid, beta: float = 1.0, deflation: bool = True,
           return_stages: bool = False, lower=None):
    """C^{n+1} from C^n and the interface velocity (ug, vg, wg) on the faces:
    eq. (fluxes) then eq. (final_corr_2) (deflation=True, the paper's method)
    or eq. (final_corr_1) (deflation=False); `lower` holds the interface
    velocity on the faces at -1/2 of lower outflow ends (x, y, z planes)."""
    lw = (None, None, None) if lower is None else lower
    C1, dx_ = sweep(C, ug, "x", dt, g, beta, lw[0])
    C2, dy_ = sweep(C1, vg, "y", dt, g, beta, lw[1])
    C3, dz_ = sweep(C2, wg, "z", dt, g, beta, lw[2])
    F = C1 * dx_ + C2 * dy_ + C3 * dz_
    if deflation:
        Cn = (C3 - dt * F) / (1.0 - dt * (dx_ + dy_ + dz_))
    else:
        Cn = C3 - dt * F
    if return_stages:
        return Cn, (C1, C2, C3)
    return Cn
