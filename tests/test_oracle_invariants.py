"""Exact invariants of the projection and the extension (oracle, CPU).

* Projection (section 3.2): after the correction the discrete divergence
  equals the phase-change source minus its volume-weighted mean,
  D u^{n+1} = s - mean_W(s) (zero when s = 0).
* Extension (section 3.6): u_1^e is divergence-free by construction.  With
  u = u_sol + G psi and s := L_h psi, the extension recovers u_sol exactly and
  phi = psi - mean_W(psi).  With u_sol = 0 this is the static evaporating
  droplet of section 4.1, where u_1^e vanishes and u_Gamma = -(mdot/rho1) n.
"""
import numpy as np
import pytest

import oracle
import vofsynth


def _grid(name):
    if name == "ppp32":
        return oracle.Grid.from_config(vofsynth.config("ppp32"))
    if name == "ppn48s":
        return oracle.Grid(48, 32, 40, 1 / 48, 1 / 32, vofsynth.stretched_dz(40, 1.0, 1.5), "PPN")
    if name == "npn":
        return oracle.Grid(32, 16, 24, 1 / 32, 1 / 16, vofsynth.stretched_dz(24, 1.0, 1.2), "NPN")
    raise KeyError(name)


@pytest.mark.parametrize("name", ["ppp32", "ppn48s", "npn"])
@pytest.mark.parametrize("with_source", [False, True])
def test_projection_divergence(name, with_source):
    g = _grid(name)
    us, vs, ws = vofsynth.random_faces(g.shape, 1, g.bc)
    phat = vofsynth.gaussian_field(g.shape, 21)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=2)
    rho1, rho2 = 1000.0, 1.0
    rho = rho1 * C + rho2 * (1 - C)
    rho0 = min(rho1, rho2)
    if with_source:
        mag, _ = vofsynth.grad_mag_central(C, g.dx, g.dy, g.dzf, g.bc)
        s = 1e-2 * mag
    else:
        s = np.zeros(g.shape)
    dt = 0.37
    u, v, w, p = oracle.project(us, vs, ws, phat, rho, rho0, s, dt, g)
    d = oracle.div(u, v, w, g)
    target = s - g.weighted_mean(s)
    scale = np.abs(oracle.div(us, vs, ws, g)).max()
    assert np.abs(d - target).max() <= 1e-12 * scale
    # gauge of the pressure
    assert abs((p * g.cell_volume()).sum()) <= 1e-12 * np.abs(p * g.cell_volume()).sum()


@pytest.mark.parametrize("name", ["ppp32", "ppn48s", "npn"])
@pytest.mark.parametrize("static", [False, True])
def test_extension_recovers_solenoidal(name, static):
    g = _grid(name)
    if static:
        usol = [np.zeros(g.shape) for _ in range(3)]
    else:
        usol = vofsynth.solenoidal_faces(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc, seed=3)
        assert np.abs(oracle.div(*usol, g)).max() < 1e-9 * np.abs(usol[0]).max() / g.dx
    psi = vofsynth.gaussian_field(g.shape, 4)
    gpsi = oracle.grad(psi, g)
    u = [a + b for a, b in zip(usol, gpsi)]
    s = oracle.lap(psi, g)
    q = vofsynth.random_faces(g.shape, 5, g.bc)
    ue, ve, we, ug, vg, wg, phi = oracle.extend(u[0], u[1], u[2], s, g, q=q)
    scale = max(np.abs(a).max() for a in u)
    for a, b in zip((ue, ve, we), usol):
        assert np.abs(a - b).max() <= 1e-11 * scale
    psic = psi - g.weighted_mean(psi)
    assert np.abs(phi - psic).max() <= 1e-11 * np.abs(psic).max()
    for a, b, c in zip((ug, vg, wg), (ue, ve, we), q):
        assert np.array_equal(a, b - c)
    dmax = np.abs(oracle.div(ue, ve, we, g)).max()
    assert dmax <= 1e-10 * scale / min(g.dx, g.dy, g.dzf.min())


def test_projection_constant_density_ignores_phat():
    """rho == const: the split terms cancel, u^{n+1} does not depend on p_hat."""
    g = _grid("ppn48s")
    us, vs, ws = vofsynth.random_faces(g.shape, 1, g.bc)
    s = np.zeros(g.shape)
    rho = np.full(g.shape, 7.0)
    a = oracle.project(us, vs, ws, vofsynth.gaussian_field(g.shape, 8), rho, 1.0, s, 0.5, g)
    b = oracle.project(us, vs, ws, np.zeros(g.shape), rho, 1.0, s, 0.5, g)
    for x, y in zip(a[:3], b[:3]):
        assert np.abs(x - y).max() <= 1e-11 * np.abs(us).max()


def test_projection_layered_closed_form():
    """Fields varying along x only (periodic): D u = 0 forces a uniform u whose
    value is -dt times the face mean of (1/rho_f - 1/rho0) dp_hat/dx, with
    rho_f the mean of the two cells sharing the face."""
    nx, ny, nz = 16, 4, 4
    g = oracle.Grid(nx, ny, nz, 1 / nx, 1 / ny, np.full(nz, 1 / nz), "PPP")
    r = np.random.default_rng(31)
    rx = r.uniform(1.0, 50.0, nx)
    px = r.standard_normal(nx)
    rho = np.broadcast_to(rx[None, None, :], g.shape).copy()
    phat = np.broadcast_to(px[None, None, :], g.shape).copy()
    z = np.zeros(g.shape)
    dt = 0.25
    u, v, w, p = oracle.project(z, z, z, phat, rho, 1.0, z, dt, g)
    terms = [(1.0 / (0.5 * (rx[i] + rx[(i + 1) % nx])) - 1.0) * (px[(i + 1) % nx] - px[i]) * nx
             for i in range(nx)]
    expect = -dt * sum(terms) / nx
    assert np.allclose(u, expect, rtol=0, atol=1e-11 * abs(expect))
    assert np.abs(v).max() < 1e-12 and np.abs(w).max() < 1e-12
