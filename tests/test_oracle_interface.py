"""Pins of the oracle's interface terms (Youngs gradient of C, the Stefan
source s and the interface-velocity jump q on faces), from facts that do not
come from the oracle itself:

* a triple loop over cells with the (1, 2, 1) transverse weights written out
  (uniform grids) and with one-sided z differences (stretched z);
* exactness on linear fields away from the boundary, on any z spacing;
* a field varying along x only gives n = (+-1, 0, 0) and no y / z flux;
* reflection symmetry of a centred sphere, and periodic shift invariance;
* q on a face is the mean of the two cells' (mdot / rho1) n, and 0 on a
  non-periodic boundary face.
"""
import numpy as np
import pytest

import oracle
import oracle.interface as oi
import vofsynth

W = (1.0, 2.0, 1.0)


def _idx(n, i, periodic):
    if periodic:
        return i % n
    return min(max(i, 0), n - 1)  # mirrored ghost = the end cell's value


def loop_gradient(C, g):
    nz, ny, nx = C.shape
    px, py, pz = (e[0] == "P" for e in g.ends)
    dzf = g.dzf
    out = np.zeros((3,) + C.shape)

    def c(k, j, i):
        return C[_idx(nz, k, pz), _idx(ny, j, py), _idx(nx, i, px)]

    def dz_between(k0, k1):  # centre distance of neighbours k0 < k1 (ghosts copy widths)
        return 0.5 * (dzf[_idx(nz, k0, pz)] + dzf[_idx(nz, k1, pz)])

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                gx = gy = gz = 0.0
                for a in (-1, 0, 1):
                    for b in (-1, 0, 1):
                        w = W[a + 1] * W[b + 1] / 16.0
                        gx += w * (c(k + a, j + b, i + 1) - c(k + a, j + b, i - 1)) / (2 * g.dx)
                        gy += w * (c(k + a, j + 1, i + b) - c(k + a, j - 1, i + b)) / (2 * g.dy)
                        up = (c(k + 1, j + a, i + b) - c(k, j + a, i + b)) / dz_between(k, k + 1)
                        dn = (c(k, j + a, i + b) - c(k - 1, j + a, i + b)) / dz_between(k - 1, k)
                        gz += w * 0.5 * (up + dn)
                out[:, k, j, i] = gx, gy, gz
    return out


@pytest.mark.parametrize("bc,stretched", [("PPP", False), ("NNN", True), ("PNN", True),
                                           ("DDD", False), ("NNNNND", True), ("NPP", False)])
def test_loop_weights(bc, stretched):
    nx, ny, nz = 6, 5, 7
    dzf = np.random.default_rng(1).uniform(0.05, 0.2, nz) if stretched else np.full(nz, 0.1)
    g = oracle.Grid(nx, ny, nz, 0.13, 0.21, dzf, bc)
    C = np.random.default_rng(2).uniform(0.0, 1.0, g.shape)
    ref = loop_gradient(C, g)
    got = oi.youngs_gradient(C, g)
    for a, b in zip(got, ref):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_linear_field_exact():
    nx, ny, nz = 10, 9, 12
    dzf = vofsynth.stretched_dz(nz, 1.0, 1.5)
    g = oracle.Grid(nx, ny, nz, 0.1, 0.07, dzf, "NNN")
    zc = np.cumsum(dzf) - 0.5 * dzf
    x = (np.arange(nx) + 0.5) * g.dx
    y = (np.arange(ny) + 0.5) * g.dy
    C = 0.3 * x[None, None, :] - 1.7 * y[None, :, None] + 2.9 * zc[:, None, None]
    gx, gy, gz = oi.youngs_gradient(C, g)
    inner = (slice(1, -1),) * 3
    assert np.allclose(gx[inner], 0.3, rtol=0, atol=1e-12)
    assert np.allclose(gy[inner], -1.7, rtol=0, atol=1e-12)
    assert np.allclose(gz[inner], 2.9, rtol=0, atol=1e-12)


def test_one_dimensional_interface():
    g = oracle.Grid(16, 8, 8, 1 / 16, 1 / 8, np.full(8, 1 / 8), "NPP")
    x = (np.arange(16) + 0.5) / 16
    C = np.broadcast_to((0.5 * (1 - np.tanh((x - 0.43) / 0.05)))[None, None, :], g.shape).copy()
    mdot = np.full(g.shape, 0.02)
    s, qx, qy, qz, mag = oi.interface_terms(C, mdot, 1000.0, 1.0, g)
    gx, gy, gz = oi.youngs_gradient(C, g)
    assert np.abs(gy).max() == 0 and np.abs(gz).max() == 0
    on = mag > 0
    assert np.allclose(np.abs(gx[on]), mag[on], rtol=1e-15, atol=0)
    assert np.abs(qy).max() == 0 and np.abs(qz).max() == 0
    # q_x is the face mean of +mdot/rho1: C falls along +x, so the normal
    # into phase 2 is n_x = +1
    a = np.where(on, 0.02 / 1000.0, 0.0)
    assert np.allclose(qx[:, :, :-1], 0.5 * (a[:, :, :-1] + a[:, :, 1:]), rtol=1e-14, atol=0)
    assert np.all(qx[:, :, -1] == 0.0)  # wall face
    assert np.allclose(s, 0.02 * (1.0 - 1e-3) * mag, rtol=1e-15, atol=0)


def test_sphere_reflection_symmetry():
    n = 16
    g = oracle.Grid(n, n, n, 1 / n, 1 / n, np.full(n, 1 / n), "NNN")
    c = (np.arange(n) + 0.5) / n - 0.5
    r = np.sqrt(c[None, None, :] ** 2 + c[None, :, None] ** 2 + c[:, None, None] ** 2)
    C = 0.5 * (1 - np.tanh((r - 0.3) / 0.06))
    gx, gy, gz = oi.youngs_gradient(C, g)
    assert np.allclose(gx, -gx[:, :, ::-1], rtol=0, atol=1e-12)
    assert np.allclose(gy, -gy[:, ::-1, :], rtol=0, atol=1e-12)
    assert np.allclose(gz, -gz[::-1, :, :], rtol=0, atol=1e-12)
    # the sphere's gradient points inwards (C falls outwards)
    assert np.all(gx[:, :, n // 2:] <= 1e-12)


def test_periodic_shift_invariance():
    g = oracle.Grid(8, 12, 10, 0.1, 0.1, np.full(10, 0.1), "PPP")
    C = np.random.default_rng(5).uniform(size=g.shape)
    mdot = np.random.default_rng(6).uniform(0.5, 1.5, size=g.shape)
    shift = (3, -2, 5)
    a = oi.interface_terms(C, mdot, 10.0, 1.0, g)
    b = oi.interface_terms(np.roll(C, shift, axis=(0, 1, 2)), np.roll(mdot, shift, axis=(0, 1, 2)),
                           10.0, 1.0, g)
    for x, y in zip(a, b):
        assert np.allclose(np.roll(x, shift, axis=(0, 1, 2)), y, rtol=1e-13, atol=1e-15)
    # periodic: the last face is a real face, the mean with the wrapped cell
    gx, _, _ = oi.youngs_gradient(C, g)
    mag = a[4]
    ax = -mdot / 10.0 * gx / mag
    assert np.allclose(a[1][:, :, -1], 0.5 * (ax[:, :, -1] + ax[:, :, 0]), rtol=1e-13, atol=0)


def test_vapour_phase_jump():
    """Boiling: the interface velocity follows the vapour (q = (mdot/rho2) n);
    the source and the normal are unchanged, q scales by rho1 / rho2, and
    u_Gamma from either phase's extension is the same field (the velocity
    jump mdot (1/rho2 - 1/rho1) n lies between the two extensions)."""
    g = oracle.Grid(12, 10, 8, 0.1, 0.1, np.full(8, 0.1), "PNN")
    C, _ = vofsynth.sphere_vof(12, 10, 8, 0.1, 0.1, np.full(8, 0.1), seed=4)
    mdot = np.random.default_rng(8).uniform(0.5, 1.5, g.shape)
    rho1, rho2 = 800.0, 2.0
    liq = oi.interface_terms(C, mdot, rho1, rho2, g, phase=1)
    vap = oi.interface_terms(C, mdot, rho1, rho2, g, phase=2)
    assert np.array_equal(liq[0], vap[0]) and np.array_equal(liq[4], vap[4])
    for a, b in zip(liq[1:4], vap[1:4]):
        assert np.allclose(b, a * (rho1 / rho2), rtol=1e-13, atol=0)
    with pytest.raises(ValueError):
        oi.interface_terms(C, mdot, rho1, rho2, g, phase=3)


def test_evaporating_sphere_recedes():
    """A resting liquid sphere (phase 1, C = 1 inside) evaporating at mdot > 0:
    the one-fluid velocity is the pure Stefan flow u = G psi with L psi = s,
    so the liquid extension is zero and u_Gamma = -q.  The jump condition of
    section 2 (n into phase 2) makes the interface recede into the liquid at
    mdot / rho1: u_Gamma . r_hat < 0 at every face the interface crosses,
    close to -mdot / rho1 where the interface is thin."""
    n = 24
    h = 1.0 / n
    g = oracle.Grid(n, n, n, h, h, np.full(n, h), "NNN")
    c = (np.arange(n) + 0.5) * h - 0.5
    x, y, z = c[None, None, :], c[None, :, None], c[:, None, None]
    r = np.sqrt(x * x + y * y + z * z)
    C = 0.5 * (1 - np.tanh((r - 0.3) / (1.5 * h)))
    rho1, rho2, mdot0 = 1000.0, 1.0, 0.5
    mdot = np.full(g.shape, mdot0)
    s, qx, qy, qz, mag = oi.interface_terms(C, mdot, rho1, rho2, g)
    psi = oracle.solve(s, g)
    u = oracle.grad(psi, g)
    ue, ve, we, ug, vg, wg, _ = oracle.extend(*u, s, g, q=(qx, qy, qz))
    assert max(np.abs(a).max() for a in (ue, ve, we)) <= 1e-12 * max(np.abs(a).max() for a in u)
    # radial component of u_Gamma at the faces (face centres' radial direction)
    xf, yf, zf = x + 0.5 * h, y + 0.5 * h, z + 0.5 * h
    ur_x = ug * xf / np.sqrt(xf * xf + y * y + z * z)
    ur_y = vg * yf / np.sqrt(x * x + yf * yf + z * z)
    ur_z = wg * zf / np.sqrt(x * x + y * y + zf * zf)
    band = np.abs(r - 0.3) < 1.5 * h  # cells the interface crosses
    for comp in (ur_x, ur_y, ur_z):
        sel = band & (np.abs(comp) > 1e-3 * mdot0 / rho1)
        assert sel.sum() > 100
        assert np.all(comp[sel] < 0.0)
    # the velocity of the interface along the normal: u_Gamma . n = -mdot/rho1
    # at the centres of the band (q averaged back from the faces)
    qc = (0.5 * (qx + np.roll(qx, 1, axis=2)), 0.5 * (qy + np.roll(qy, 1, axis=1)),
          0.5 * (qz + np.roll(qz, 1, axis=0)))
    qr = (qc[0] * x + qc[1] * y + qc[2] * z) / r
    thin = np.abs(r - 0.3) < 0.5 * h
    assert np.allclose(-qr[thin], -mdot0 / rho1, rtol=0.05, atol=0)
