"""Pins of the oracle's VoF advection (section 3.1: eqs. cadv, fluxes,
final_corr_1, final_corr_2; MTHINC flux of Ii et al. 2012), from facts that do
not come from the oracle itself:

* the volume balance of the split scheme, exact for any face velocities
  (periodic and wall ends, stretched z): sum dV C^{n+1} (1 - dt div u) =
  sum dV C^n with the deflation step, sum dV C^{n+1} = sum dV C^n without;
* a constant field stays constant under any velocity with the deflation step
  (and is scaled by 1 - dt div u without it);
* a one-dimensional field: the THINC profile's volume equation and swept-box
  integrals in closed form (the volume equation is solved for d exactly),
  written out in a scalar loop, both velocity signs, walls, periodic and
  outflow ends with inflow through the outflow face;
* a uniform velocity of one cell per step moves any field by exactly one cell
  (the swept box is the whole upwind cell, whose integral is its C);
* the semi-analytical box integral against a dense tensor Gauss rule: exact
  for normals along an axis, within the 2-point rule's error otherwise;
* exchanging the x and y (or x and z) axes of a cubic grid together with the
  velocity components exchanges the result; mirroring x with u reversed
  mirrors it.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import advection as adv
import vofsynth


def _grid(n, bc, nz=None, stretched=False, lz=1.0):
    nz = n if nz is None else nz
    dzf = vofsynth.stretched_dz(nz, lz, 1.5) if stretched else vofsynth.uniform_dz(nz, lz)
    return oracle.Grid(n, n, nz, 1.0 / n, 1.0 / n, dzf, bc)


def _faces(g, seed, scale):
    u, v, w = vofsynth.random_faces(g.shape, seed, g.bc)
    return u * scale, v * scale, w * scale


def _cfl_dt(g, u, v, w, cfl):
    """A time step moving at most `cfl` of a cell per step (the flux takes the
    swept part of one upwind cell)."""
    h = min(g.dx, g.dy, float(g.dzf.min()))
    vmax = max(np.abs(a).max() for a in (u, v, w))
    return cfl * h / vmax


def _sphere(g, seed, radius=0.25):
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=seed, radius=radius)
    return C


@pytest.mark.parametrize("bc,stretched", [("PPP", False), ("NNN", False), ("PPN", True),
                                           ("NPN", True)])
@pytest.mark.parametrize("deflation", [True, False])
def test_volume_balance(bc, stretched, deflation):
    g = _grid(16, bc, nz=12, stretched=stretched)
    C = _sphere(g, 3)
    u, v, w = _faces(g, 4, 0.4)
    dt = _cfl_dt(g, u, v, w, 0.8)
    Cn = adv.advect(C, u, v, w, dt, g, deflation=deflation)
    dv = g.cell_volume()
    div = oracle.div(u, v, w, g)
    before = float((C * dv).sum())
    after = float((Cn * (1.0 - dt * div) * dv).sum()) if deflation else float((Cn * dv).sum())
    assert abs(after - before) <= 1e-13 * before
    # the scheme does change the field
    assert np.abs(Cn - C).max() > 1e-3


@pytest.mark.parametrize("c", [0.0, 1.0, 0.37])
def test_constant_field_kept_by_deflation(c):
    g = _grid(12, "PPN", nz=10, stretched=True)
    C = np.full(g.shape, c)
    u, v, w = _faces(g, 7, 0.5)
    dt = _cfl_dt(g, u, v, w, 0.9)
    Cn = adv.advect(C, u, v, w, dt, g, deflation=True)
    assert np.abs(Cn - c).max() <= 1e-14
    C0 = adv.advect(C, u, v, w, dt, g, deflation=False)
    div = oracle.div(u, v, w, g)
    assert np.abs(C0 - c * (1.0 - dt * div)).max() <= 1e-13


# ---------------------------------------------------------------------------
# one-dimensional closed form
# ---------------------------------------------------------------------------
def _lncosh(x):
    return math.log(math.cosh(x))


def _d_closed(C, beta):
    """Root d of 1/2 + [lncosh(b(d + 1/2)) - lncosh(b(d - 1/2))] / (2b) = C."""
    R = math.exp(beta * (2.0 * C - 1.0))
    b = math.exp(beta)
    return math.log((R * b - 1.0) / (b - R)) / (2.0 * beta)


def _box_1d(m, d, s0, s1, beta):
    return 0.5 * (s1 - s0) + (_lncosh(beta * (m * s1 + d)) - _lncosh(beta * (m * s0 + d))) / (
        2.0 * beta * m)


def _loop_1d(c, vel_faces, dt, h, ends, beta):
    """x-only field c[i] and face velocities vel_faces[f], f = 0..n (face f
    at i = f - 1/2): one sweep written out cell by cell."""
    n = len(c)
    lo, hi = ends
    per = lo == "P"

    def cell(i):
        if per:
            return c[i % n]
        return c[min(max(i, 0), n - 1)]

    def flux(f):
        V = vel_faces[f]
        if V == 0.0:
            return 0.0
        up = f - 1 if V >= 0 else f
        if not per and (up < 0 or up >= n):  # ghost: uniform, the end cell's C
            xi = min(abs(V) * dt / h, 1.0)
            return math.copysign(1.0, V) * h * xi * cell(up)
        ui = up % n if per else up
        cu = c[ui]
        xi = min(abs(V) * dt / h, 1.0)
        grad = cell(ui + 1) - cell(ui - 1)  # twice the cell-scaled gradient
        if not (adv.EPS < cu < 1.0 - adv.EPS) or abs(0.5 * grad) <= adv.GRAD_MIN:
            return V / abs(V) * h * xi * cu
        m = 1.0 if grad > 0 else -1.0
        d = _d_closed(cu, beta)
        if V >= 0:
            I = _box_1d(m, d, 0.5 - xi, 0.5, beta)
        else:
            I = _box_1d(m, d, -0.5, -0.5 + xi, beta)
        return math.copysign(1.0, V) * h * I

    out = np.zeros(n)
    for i in range(n):
        delta = (vel_faces[i + 1] - vel_faces[i]) / h
        out[i] = (c[i] - (flux(i + 1) - flux(i)) / h) / (1.0 - dt * delta)
    return out


@pytest.mark.parametrize("bc", ["PPP", "NPP", "NDPPPP"])
@pytest.mark.parametrize("beta", [1.0, 2.5])
def test_one_dimensional_closed_form(bc, beta):
    n = 24
    g = oracle.Grid(n, 3, 3, 1.0 / n, 1.0 / 3, np.full(3, 1.0 / 3), bc)
    x = (np.arange(n) + 0.5) / n
    c = 0.5 * (1 - np.tanh((np.abs(x - 0.45) - 0.2) / 0.04))
    c[3] = 1.0  # a cell outside the band
    r = np.random.default_rng(9)
    ux = r.uniform(-0.9, 0.9, n)  # stored faces i+1/2
    lo, hi = g.ends[0]
    if lo == "N":
        ux[-1] = 0.0 if hi == "N" else ux[-1]
    if hi == "D":
        ux[-1] = -0.7  # inflow through the outflow face
    dt = 0.6 / n
    C = np.broadcast_to(c[None, None, :], g.shape).copy()
    U = np.broadcast_to(ux[None, None, :], g.shape).copy()
    Z = np.zeros(g.shape)
    Cn = adv.advect(C, U, Z, Z, dt, g, beta=beta)
    faces = np.concatenate([[ux[-1] if lo == "P" else 0.0], ux])
    want = _loop_1d(c, faces, dt, 1.0 / n, (lo, hi), beta)
    assert np.abs(Cn - want[None, None, :]).max() <= 1e-13
    assert np.abs(want - c).max() > 1e-2


@pytest.mark.parametrize("axis", ["x", "y", "z"])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_one_cell_per_step_shifts_exactly(axis, sign):
    n = 16
    g = _grid(n, "PPP")
    C = _sphere(g, 11)
    dt = 0.01
    vel = sign * (1.0 / n) / dt
    u, v, w = (np.full(g.shape, vel if a == axis else 0.0) for a in "xyz")
    Cn = adv.advect(C, u, v, w, dt, g)
    ax = {"x": 2, "y": 1, "z": 0}[axis]
    assert np.abs(Cn - np.roll(C, int(sign), axis=ax)).max() <= 1e-13


def _dense_integral(m, d, lo, hi, beta, q=48):
    xg, wg = np.polynomial.legendre.leggauss(q)
    pts, wts = [], []
    for a in range(3):
        pts.append(0.5 * (lo[a] + hi[a]) + 0.5 * (hi[a] - lo[a]) * xg)
        wts.append(0.5 * (hi[a] - lo[a]) * wg)
    X, Y, Z = np.meshgrid(*pts, indexing="ij")
    W = wts[0][:, None, None] * wts[1][None, :, None] * wts[2][None, None, :]
    H = 0.5 * (1.0 + np.tanh(beta * (m[0] * X + m[1] * Y + m[2] * Z + d)))
    return float((W * H).sum())


@pytest.mark.parametrize("beta", [1.0, 2.0])
def test_box_integral_against_dense_rule(beta):
    r = np.random.default_rng(5)
    worst = 0.0
    for trial in range(40):
        if trial < 6:  # along an axis: the transverse integrand is constant
            m = np.zeros(3)
            m[trial % 3] = 1.0 if trial < 3 else -1.0
        else:
            m = r.standard_normal(3)
            m /= np.linalg.norm(m)
        d = r.uniform(-1.0, 1.0)
        lo = r.uniform(-0.5, 0.0, 3)
        hi = r.uniform(0.0, 0.5, 3)
        got = adv.box_integral(m[:, None], np.array([d]), lo[:, None], hi[:, None], beta)[0]
        ref = _dense_integral(m, d, lo, hi, beta)
        if trial < 6:
            assert abs(got - ref) <= 1e-13, trial
        else:
            worst = max(worst, abs(got - ref))
    # 2-point Gauss in the two transverse axes, whose slopes beta |m_t| are at
    # most beta / sqrt(2): the rule's error stays orders below a flux
    assert worst <= 2e-4 * beta ** 2


def test_volume_equation_solved():
    r = np.random.default_rng(6)
    m = r.standard_normal((3, 50))
    m /= np.linalg.norm(m, axis=0)
    C = r.uniform(1e-6, 1 - 1e-6, 50)
    for beta in (1.0, 3.0):
        d = adv.solve_d(m, C, beta)
        full = adv.box_integral(m, d, np.full((3, 50), -0.5), np.full((3, 50), 0.5), beta)
        assert np.abs(full - C).max() <= 2e-15


@pytest.mark.parametrize("pair", [(2, 1), (2, 0)])
def test_axis_exchange(pair):
    n = 14
    g = _grid(n, "PPP")
    C = _sphere(g, 21, radius=0.3)
    r = np.random.default_rng(22)
    vel = r.uniform(-0.8, 0.8, g.shape) * (1.0 / n) / 0.02
    dt = 0.02
    Z = np.zeros(g.shape)
    comps = {2: 0, 1: 1, 0: 2}  # array axis -> velocity component index (u, v, w)
    a, b = pair
    va = [Z, Z, Z]
    va[comps[a]] = vel
    res_a = adv.advect(C, *va, dt, g)
    Ct = np.swapaxes(C, a, b)
    vb = [Z, Z, Z]
    vb[comps[b]] = np.swapaxes(vel, a, b)
    res_b = adv.advect(Ct, *vb, dt, g)
    assert np.abs(np.swapaxes(res_b, a, b) - res_a).max() <= 1e-13
    assert np.abs(res_a - C).max() > 1e-2


def test_mirror_in_x():
    n = 16
    g = _grid(n, "PPP")
    C = _sphere(g, 31)
    r = np.random.default_rng(32)
    u = r.uniform(-0.8, 0.8, g.shape) * (1.0 / n) / 0.02
    v = r.uniform(-0.8, 0.8, g.shape) * (1.0 / n) / 0.02
    w = r.uniform(-0.8, 0.8, g.shape) * (1.0 / n) / 0.02
    dt = 0.02
    res = adv.advect(C, u, v, w, dt, g)
    # face i+1/2 maps to face (n-2-i)+1/2; u changes sign, v and w are mirrored cells
    idx = (n - 2 - np.arange(n)) % n
    um = -u[:, :, idx]
    resm = adv.advect(C[:, :, ::-1], um, v[:, :, ::-1], w[:, :, ::-1], dt, g)
    assert np.abs(resm[:, :, ::-1] - res).max() <= 1e-12


def test_lower_outflow_refused():
    g = oracle.Grid(8, 8, 8, 0.125, 0.125, np.full(8, 0.125), "DNPPNN")
    z = np.zeros(g.shape)
    with pytest.raises(ValueError):
        adv.advect(z, z, z, z, 0.1, g)


def test_normal_in_cell_coordinates_stretched():
    """A linear field C = a x + b y + c z (inside the band) on a stretched z
    grid: the Youngs gradient is exact away from the boundary, so the normal
    in cell coordinates is (dx a, dy b, dz_k c) normalised, cell by cell."""
    nx, ny, nz = 8, 7, 12
    dzf = vofsynth.stretched_dz(nz, 1.0, 1.5)
    g = oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, "NNN")
    zc = np.cumsum(dzf) - 0.5 * dzf
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    a, b, c = 0.11, -0.07, 0.23
    C = 0.3 + a * x[None, None, :] + b * y[None, :, None] + c * zc[:, None, None]
    (mx, my, mz), mag = adv.normals(C, g)
    inner = (slice(1, -1),) * 3
    for k in range(1, nz - 1):
        h = np.array([g.dx * a, g.dy * b, dzf[k] * c])
        want = h / np.linalg.norm(h)
        got = np.stack([mx[k], my[k], mz[k]])[:, 1:-1, 1:-1]
        assert np.abs(got - want[:, None, None]).max() <= 1e-12, k
        assert np.abs(mag[k][1:-1, 1:-1] - np.linalg.norm(h)).max() <= 1e-13
    assert np.all(adv.dominant_axis((mx, my, mz))[inner] >= 0)


def test_one_dimensional_lower_outflow_inflow():
    """x ends outflow (lower) and wall (upper): inflow through the face at
    -1/2 (velocity from its plane, > 0) carries the ghost's C (the first
    cell's, uniform); the 1-D loop with that face."""
    n = 24
    g = oracle.Grid(n, 3, 3, 1.0 / n, 1.0 / 3, np.full(3, 1.0 / 3), "DNPPPP")
    x = (np.arange(n) + 0.5) / n
    c = 0.5 * (1 - np.tanh((x - 0.35) / 0.05))
    r = np.random.default_rng(19)
    ux = r.uniform(0.05, 0.9, n)
    ux[-1] = 0.0  # the wall
    ulo = 0.6     # inflow through the lower outflow face
    dt = 0.6 / n
    C = np.broadcast_to(c[None, None, :], g.shape).copy()
    U = np.broadcast_to(ux[None, None, :], g.shape).copy()
    Z = np.zeros(g.shape)
    lower = (np.full((g.nz, g.ny), ulo), None, None)
    Cn = adv.advect(C, U, Z, Z, dt, g, lower=lower)
    faces = np.concatenate([[ulo], ux])
    want = _loop_1d(c, faces, dt, 1.0 / n, ("D", "N"), 1.0)
    assert np.abs(Cn - want[None, None, :]).max() <= 1e-13
