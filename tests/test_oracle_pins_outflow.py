"""Pins of the FP64 oracle with outflow ends (p = 0 on the boundary face).

The zero-pressure outflow boundaries of the cases of section 4 make the
discrete Laplacian non-singular.  Facts that do not come from the oracle:

* brute force: the operator assembled entry by entry with a mirrored ghost
  (p_ghost = -p, so p = 0 on the face half a cell out) and solved with
  numpy.linalg.solve -- every end combination, stretched z;
* closed-form eigenfunctions of the staggered second difference with
  outflow/outflow, wall/outflow and outflow/wall ends (sines and
  quarter-wave cosines);
* a z-only right-hand side through scipy.linalg.solve_banded;
* second-order convergence to continuous solutions with p = 0 on the
  boundary, which fixes the face at half a cell beyond the last centre;
* pointwise stencils with an outflow face at the upper end, and the exact
  divergence after a projection (no mean removed).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import vofsynth

# 3 letters: both ends of x, y, z alike; 6 letters: x-, x+, y-, y+, z-, z+
BCS = ["DDD", "NNNNND", "PPNDDN", "DNNDPP", "PDN", "NDPPDD", "DNPPND"]


def ends_of(bc):
    if len(bc) == 3:
        return [(c, c) for c in bc]
    return [(bc[2 * a], bc[2 * a + 1]) for a in range(3)]


def loop_laplacian(nx, ny, nz, dx, dy, dzf, bc):
    """The 7-point operator row by row: a neighbour across a wall contributes
    nothing, across a periodic end the wrapped cell, across an outflow face
    the ghost -p (face value zero), i.e. -2 p / h^2 on the diagonal."""
    ex, ey, ez = ends_of(bc)
    n = nx * ny * nz
    A = np.zeros((n, n))

    def idx(i, j, k):
        return i + nx * (j + ny * k)

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = idx(i, j, k)
                for d in (-1, 1):
                    end = 0 if d < 0 else 1
                    ii = i + d
                    if 0 <= ii < nx or ex[end] == "P":
                        A[r, idx(ii % nx, j, k)] += 1.0 / dx**2
                        A[r, r] -= 1.0 / dx**2
                    elif ex[end] == "D":
                        A[r, r] -= 2.0 / dx**2
                    jj = j + d
                    if 0 <= jj < ny or ey[end] == "P":
                        A[r, idx(i, jj % ny, k)] += 1.0 / dy**2
                        A[r, r] -= 1.0 / dy**2
                    elif ey[end] == "D":
                        A[r, r] -= 2.0 / dy**2
                    kk = k + d
                    if 0 <= kk < nz or ez[end] == "P":
                        face = k if d > 0 else k - 1
                        dist = 0.5 * (dzf[face % nz] + dzf[(face + 1) % nz])
                        A[r, idx(i, j, kk % nz)] += 1.0 / (dzf[k] * dist)
                        A[r, r] -= 1.0 / (dzf[k] * dist)
                    elif ez[end] == "D":
                        A[r, r] -= 1.0 / (dzf[k] * 0.5 * dzf[k])
    return A


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("stretched", [False, True])
def test_brute_force_dense(bc, stretched):
    nx, ny, nz = 8, 6, 7
    dx, dy = 0.13, 0.21
    dzf = (np.random.default_rng(3).uniform(0.05, 0.2, nz) if stretched else np.full(nz, 0.1))
    g = oracle.Grid(nx, ny, nz, dx, dy, dzf, bc)
    assert not g.singular
    A = loop_laplacian(nx, ny, nz, dx, dy, dzf, bc)
    f = vofsynth.gaussian_field(g.shape, 11)  # any right-hand side: no compatibility
    ref = np.linalg.solve(A, f.reshape(-1)).reshape(g.shape)
    p, fbar = oracle.solve(f, g, return_mean=True)
    assert fbar == 0.0
    assert np.abs(p - ref).max() <= 1e-12 * np.abs(ref).max()
    # the operator itself, applied to a random field
    q = vofsynth.gaussian_field(g.shape, 12)
    lq = oracle.lap(q, g)
    assert np.abs(lq - (A @ q.reshape(-1)).reshape(g.shape)).max() <= 1e-12 * np.abs(lq).max()


def mode(n, h, ends, m):
    """Discrete eigenfunction (at centres i + 1/2) and eigenvalue."""
    c = np.arange(n) + 0.5
    lo, hi = ends
    if (lo, hi) == ("D", "D"):
        return np.sin(np.pi * (m + 1) * c / n), -(4 / h**2) * np.sin(np.pi * (m + 1) / (2 * n)) ** 2
    lam = -(4 / h**2) * np.sin(np.pi * (2 * m + 1) / (4 * n)) ** 2
    if (lo, hi) == ("N", "D"):
        return np.cos(np.pi * (2 * m + 1) * c / (2 * n)), lam
    if (lo, hi) == ("D", "N"):
        return np.sin(np.pi * (2 * m + 1) * c / (2 * n)), lam
    if (lo, hi) == ("N", "N"):
        return np.cos(np.pi * m * c / n), -(4 / h**2) * np.sin(np.pi * m / (2 * n)) ** 2
    return np.cos(2 * np.pi * m * c / n), -(4 / h**2) * np.sin(np.pi * m / n) ** 2


@pytest.mark.parametrize("bc", BCS)
def test_eigenfunctions(bc):
    nx, ny, nz = 16, 12, 10
    hx, hy, hz = 0.07, 0.11, 0.05
    ex, ey, ez = ends_of(bc)
    g = oracle.Grid(nx, ny, nz, hx, hy, np.full(nz, hz), bc)
    for mx, my, mz in ((3, 1, 2), (0, 0, 0), (nx - 1, ny - 1, nz - 1)):
        fx, lx = mode(nx, hx, ex, mx)
        fy, ly = mode(ny, hy, ey, my)
        fz, lz = mode(nz, hz, ez, mz)
        p_exact = fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
        lam = lx + ly + lz
        p = oracle.solve(lam * p_exact, g)
        assert np.abs(p - p_exact).max() <= 1e-12, (mx, my, mz)


@pytest.mark.parametrize("ends", [("D", "D"), ("N", "D"), ("D", "N")])
def test_z_only_rhs_solve_banded(ends):
    """f(z) only: the x/y-constant mode reduces to one tridiagonal system,
    solved here by scipy's banded LU (x, y periodic)."""
    nx, ny, nz = 4, 4, 50
    dzf = vofsynth.stretched_dz(nz, 1.0, 1.5)
    bc = "PPPP" + ends[0] + ends[1]
    g = oracle.Grid(nx, ny, nz, 0.25, 0.25, dzf, bc)
    fz = np.random.default_rng(9).standard_normal(nz)
    f = np.broadcast_to(fz[:, None, None], g.shape).copy()
    dzc = 0.5 * (dzf[:-1] + dzf[1:])
    ab = np.zeros((3, nz))
    for k in range(nz):
        if k + 1 < nz:
            ab[0, k + 1] = 1.0 / (dzf[k] * dzc[k])  # super-diagonal of row k
            ab[1, k] -= 1.0 / (dzf[k] * dzc[k])
        if k > 0:
            ab[2, k - 1] = 1.0 / (dzf[k] * dzc[k - 1])  # sub-diagonal of row k
            ab[1, k] -= 1.0 / (dzf[k] * dzc[k - 1])
    if ends[0] == "D":
        ab[1, 0] -= 2.0 / dzf[0] ** 2
    if ends[1] == "D":
        ab[1, nz - 1] -= 2.0 / dzf[nz - 1] ** 2
    ref = sla.solve_banded((1, 1), ab, fz)
    p = oracle.solve(f, g)
    assert np.abs(p - ref[:, None, None]).max() <= 1e-12 * np.abs(ref).max()


def _centres(n, length=1.0):
    return (np.arange(n) + 0.5) * (length / n)


@pytest.mark.parametrize("case", ["DDD", "container"])
def test_second_order_convergence(case):
    """Continuous solutions vanishing on the outflow faces: the discrete error
    falls by 4 per halving of h only if the outflow face is placed half a cell
    beyond the last centre."""
    errs = []
    for n in (8, 16, 32):
        x, y, z = _centres(n), _centres(n), _centres(n)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        if case == "DDD":
            bc = "DDD"
            exact = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
            f = -3 * np.pi**2 * exact
        else:  # walls on the sides and the bottom, outflow at the top
            bc = "NNNNND"
            exact = np.cos(np.pi * X) * np.cos(np.pi * Y) * np.cos(np.pi * Z / 2)
            f = -(2 * np.pi**2 + np.pi**2 / 4) * exact
        g = oracle.Grid(n, n, n, 1 / n, 1 / n, np.full(n, 1 / n), bc)
        p = oracle.solve(f, g)
        errs.append(np.abs(p - exact).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.8 < r2 < 4.2, errs


def test_stencils_pointwise_upper_outflow():
    """Face gradient and divergence at every point, written as loops, for
    outflow at the upper ends of y and z (walls at x, the lower y end and the
    lower z end)."""
    bc = "NNNDND"
    nx, ny, nz = 5, 4, 6
    dx, dy = 0.3, 0.2
    dzf = np.random.default_rng(2).uniform(0.1, 0.3, nz)
    g = oracle.Grid(nx, ny, nz, dx, dy, dzf, bc)
    p = vofsynth.gaussian_field(g.shape, 1)
    u, v, w = (vofsynth.gaussian_field(g.shape, s) for s in (2, 3, 4))
    gx, gy, gz = oracle.grad(p, g)
    d = oracle.div(u, v, w, g)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                ex = (p[k, j, i + 1] - p[k, j, i]) / dx if i + 1 < nx else 0.0
                ey = (p[k, j + 1, i] - p[k, j, i]) / dy if j + 1 < ny else -p[k, j, i] / (dy / 2)
                if k + 1 < nz:
                    ez = (p[k + 1, j, i] - p[k, j, i]) / (0.5 * (dzf[k] + dzf[k + 1]))
                else:
                    ez = -p[k, j, i] / (dzf[k] / 2)
                assert np.isclose(gx[k, j, i], ex, rtol=1e-14, atol=0)
                assert np.isclose(gy[k, j, i], ey, rtol=1e-14, atol=0)
                assert np.isclose(gz[k, j, i], ez, rtol=1e-14, atol=1e-300)
                um = u[k, j, i - 1] if i > 0 else 0.0
                vm = v[k, j - 1, i] if j > 0 else 0.0
                wm = w[k - 1, j, i] if k > 0 else 0.0
                ed = (u[k, j, i] - um) / dx + (v[k, j, i] - vm) / dy + (w[k, j, i] - wm) / dzf[k]
                assert np.isclose(d[k, j, i], ed, rtol=1e-13, atol=1e-13)


def test_lower_outflow_refused_by_face_stencils():
    g = oracle.Grid(8, 8, 8, 0.1, 0.1, np.full(8, 0.1), "NNNNDN")
    z = np.zeros(g.shape)
    with pytest.raises(ValueError):
        oracle.div(z, z, z, g)
    with pytest.raises(ValueError):
        oracle.project(z, z, z, z, z + 1, 1.0, z, 0.1, g)
    with pytest.raises(ValueError):
        oracle.extend(z, z, z, z, g)
    # the solve itself is defined
    assert np.abs(oracle.solve(z + 1, g)).max() > 0


@pytest.mark.parametrize("bc", ["NNNNND", "PPPPND", "NDNDND", "NDPPNN"])
def test_projection_exact_divergence(bc):
    """With an outflow end the correction meets D u^{n+1} = s exactly: no
    mean is removed from the source (the outflow face carries the net flux)."""
    g = oracle.Grid(24, 16, 20, 1 / 24, 1 / 16, vofsynth.stretched_dz(20, 1.0, 1.3), bc)
    us, vs, ws = vofsynth.random_faces(g.shape, 1, g.bc)
    phat = vofsynth.gaussian_field(g.shape, 21)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=2)
    rho = 1000.0 * C + 1.0 * (1 - C)
    mag, _ = vofsynth.grad_mag_central(C, g.dx, g.dy, g.dzf, g.bc)
    s = 1e-2 * mag
    assert g.weighted_mean(s) > 0
    u, v, w, p = oracle.project(us, vs, ws, phat, rho, 1.0, s, 0.37, g)
    d = oracle.div(u, v, w, g)
    scale = np.abs(oracle.div(us, vs, ws, g)).max()
    assert np.abs(d - s).max() <= 1e-12 * scale


def test_static_extension_with_outflow():
    """u = G psi with psi = 0 on the outflow faces and s = L_h psi: the
    extension returns phi = psi (no gauge) and u_1^e = 0."""
    g = oracle.Grid(16, 16, 24, 1 / 16, 1 / 16, vofsynth.stretched_dz(24, 1.0, 1.2), "NNNNND")
    psi = vofsynth.gaussian_field(g.shape, 4)
    u = oracle.grad(psi, g)
    s = oracle.lap(psi, g)
    ue, ve, we, *_, phi = oracle.extend(u[0], u[1], u[2], s, g)
    assert np.abs(phi - psi).max() <= 1e-11 * np.abs(psi).max()
    scale = max(np.abs(a).max() for a in u)
    for a in (ue, ve, we):
        assert np.abs(a).max() <= 1e-11 * scale


@pytest.mark.parametrize("shape,bc", [((24, 4, 3), "PPNNND"), ((4, 24, 3), "NNPPDD"),
                                      ((40, 3, 3), "DDNNNN"), ((3, 40, 4), "NNNDPP"),
                                      ((24, 3, 4), "NDNNPP"), ((6, 12, 5), "DNDDNN")],
                         ids=lambda c: c if isinstance(c, str) else "x".join(map(str, c)))
def test_brute_force_dense_odd_lengths(shape, bc):
    """Lengths with an odd factor (3 * 2^k, 5 * 2^k, as the GPU transforms
    take them) and every transform type: the oracle's spectral solve equals
    the dense solve of the loop-built operator."""
    nx, ny, nz = shape
    dzf = np.random.default_rng(5).uniform(0.05, 0.2, nz)
    g = oracle.Grid(nx, ny, nz, 0.11, 0.17, dzf, bc)
    A = loop_laplacian(nx, ny, nz, 0.11, 0.17, dzf, bc)
    f = vofsynth.gaussian_field(g.shape, 13)
    if g.singular:
        pytest.skip("every direction closed: covered by the periodic / wall pins")
    ref = np.linalg.solve(A, f.reshape(-1)).reshape(g.shape)
    p = oracle.solve(f, g)
    assert np.abs(p - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("axis,bc", [(2, "NDPPPP"), (1, "PPNDNN"), (0, "PPPPND")])
def test_projection_layered_outflow_face_density(axis, bc):
    """Density and p_hat varying along a direction with a wall at its lower end
    and an outflow at its upper end, u* = 0, s = 0: the projected velocity
    is divergence-free and zero on the wall, hence zero on every face of that
    direction, so the split correction balances face by face:
        G p / rho0 = -(1/rho_f - 1/rho0) G p_hat.
    On the outflow face (p = p_hat = 0 on the face, half a cell beyond the
    last centre) this gives p_last = -(rho0/rho_out - 1) p_hat_last, which
    fixes the density taken on that face (the end cell's); inward,
    p_i = p_{i+1} + rho0 (1/rho_f - 1/rho0)(p_hat_{i+1} - p_hat_i) with rho_f
    the mean of the two cells.  Written here in a loop, independently of the
    oracle's stencils (stretched cells along z)."""
    n = 12
    shape = [3, 4, 5]
    shape[axis] = n
    nz, ny, nx = shape
    dzf = (np.random.default_rng(40).uniform(0.5, 1.5, nz) / nz if axis == 0
           else np.full(nz, 1.0 / nz))
    g = oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, bc)
    r = np.random.default_rng(41 + axis)
    rl = r.uniform(1.0, 50.0, n)
    pl = r.standard_normal(n)
    bshape = [1, 1, 1]
    bshape[axis] = n
    rho = np.broadcast_to(rl.reshape(bshape), g.shape).copy()
    phat = np.broadcast_to(pl.reshape(bshape), g.shape).copy()
    z = np.zeros(g.shape)
    rho0 = 1.0
    u, v, w, p = oracle.project(z, z, z, phat, rho, rho0, z, 0.4, g)
    expect = np.zeros(n)
    expect[n - 1] = -(rho0 / rl[n - 1] - 1.0) * pl[n - 1]
    for i in range(n - 2, -1, -1):
        rf = 0.5 * (rl[i] + rl[i + 1])
        expect[i] = expect[i + 1] + rho0 * (1.0 / rf - 1.0 / rho0) * (pl[i + 1] - pl[i])
    want = np.broadcast_to(expect.reshape(bshape), g.shape)
    assert np.abs(p - want).max() <= 1e-11 * np.abs(expect).max()
    for vel in (u, v, w):
        assert np.abs(vel).max() <= 1e-10 * np.abs(pl).max() * n


def _lower_planes(g, seed):
    """Random velocities on the faces at -1/2 of the lower outflow ends."""
    r = np.random.default_rng(seed)
    shapes = ((g.nz, g.ny), (g.nz, g.nx), (g.ny, g.nx))
    return tuple(r.standard_normal(shp) if lo == "D" else None
                 for (lo, _), shp in zip(g.ends, shapes))


def test_stencils_pointwise_lower_outflow():
    """Outflow at every end ('DDD'): the face gradient on the faces at -1/2
    is (p_0 - 0) / (h / 2) and the divergence reads those faces from their
    planes, written as loops (stretched z)."""
    nx, ny, nz = 5, 4, 6
    dx, dy = 0.3, 0.2
    dzf = np.random.default_rng(12).uniform(0.1, 0.3, nz)
    g = oracle.Grid(nx, ny, nz, dx, dy, dzf, "DDD")
    p = vofsynth.gaussian_field(g.shape, 11)
    gxl, gyl, gzl = oracle.grad_lower(p, g)
    ul, vl, wl = _lower_planes(g, 13)
    u, v, w = (vofsynth.gaussian_field(g.shape, s) for s in (14, 15, 16))
    d = oracle.div(u, v, w, g, (ul, vl, wl))
    for k in range(nz):
        for j in range(ny):
            assert np.isclose(gxl[k, j], p[k, j, 0] / (dx / 2), rtol=1e-15, atol=0)
            for i in range(nx):
                if j == 0:
                    assert np.isclose(gyl[k, i], p[k, 0, i] / (dy / 2), rtol=1e-15, atol=0)
                if k == 0:
                    assert np.isclose(gzl[j, i], p[0, j, i] / (dzf[0] / 2), rtol=1e-15, atol=0)
                um = u[k, j, i - 1] if i > 0 else ul[k, j]
                vm = v[k, j - 1, i] if j > 0 else vl[k, i]
                wm = w[k - 1, j, i] if k > 0 else wl[j, i]
                ed = (u[k, j, i] - um) / dx + (v[k, j, i] - vm) / dy + (w[k, j, i] - wm) / dzf[k]
                assert np.isclose(d[k, j, i], ed, rtol=1e-13, atol=1e-13)
    rl = oracle.face_density_lower(np.arange(g.nx * g.ny * g.nz, dtype=float).reshape(g.shape), g)
    assert np.array_equal(rl[0], np.arange(g.nx * g.ny * g.nz, dtype=float).reshape(g.shape)[:, :, 0])


@pytest.mark.parametrize("bc", ["DDD", "DNDNDN", "DDPPND", "NNDNPP"])
def test_projection_exact_divergence_lower_faces(bc):
    """Lower outflow ends (the box of section 4 with zero-pressure outflow on
    every side, 'DDD', among them): with the faces at -1/2 carried as planes,
    the projection meets D u^{n+1} = s exactly, lower faces included."""
    g = oracle.Grid(24, 16, 20, 1 / 24, 1 / 16, vofsynth.stretched_dz(20, 1.0, 1.3), bc)
    us, vs, ws = vofsynth.random_faces(g.shape, 1, g.bc)
    lower = _lower_planes(g, 7)
    phat = vofsynth.gaussian_field(g.shape, 21)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=2)
    rho = 1000.0 * C + 1.0 * (1 - C)
    mag, _ = vofsynth.grad_mag_central(C, g.dx, g.dy, g.dzf, g.bc)
    s = 1e-2 * mag
    u, v, w, p, low = oracle.project(us, vs, ws, phat, rho, 1.0, s, 0.37, g, lower=lower)
    d = oracle.div(u, v, w, g, low)
    scale = np.abs(oracle.div(us, vs, ws, g, lower)).max()
    assert np.abs(d - s).max() <= 1e-12 * scale
    # the lower faces did change, by the correction with p = 0 on the face
    gpl, ghl = oracle.grad_lower(p, g), oracle.grad_lower(phat, g)
    rl = oracle.face_density_lower(rho, g)
    for a, b, gp, gh, r in zip(low, lower, gpl, ghl, rl):
        if a is not None:
            want = b - 0.37 * (gp / 1.0 + (1.0 / r - 1.0) * gh)
            assert np.abs(a - want).max() <= 1e-13 * np.abs(want).max()


def test_static_extension_lower_outflow():
    """'DDD': u = G psi on every face (the lower faces from their planes) and
    s = L_h psi: the extension returns phi = psi and u_1^e = 0, lower faces
    included."""
    g = oracle.Grid(16, 12, 20, 1 / 16, 1 / 12, vofsynth.stretched_dz(20, 1.0, 1.2), "DDD")
    psi = vofsynth.gaussian_field(g.shape, 4)
    u = oracle.grad(psi, g)
    lower = oracle.grad_lower(psi, g)
    s = oracle.lap(psi, g)
    out = oracle.extend(u[0], u[1], u[2], s, g, lower=lower)
    ue, ve, we, phi, low = out[0], out[1], out[2], out[6], out[7]
    assert np.abs(phi - psi).max() <= 1e-11 * np.abs(psi).max()
    scale = max(np.abs(a).max() for a in u)
    for a in (ue, ve, we) + tuple(low):
        assert np.abs(a).max() <= 1e-11 * scale


@pytest.mark.parametrize("axis,bc", [(2, "DNPPPP"), (0, "PPPPDN")])
def test_projection_layered_lower_outflow_face_density(axis, bc):
    """The layered closed form of the upper-outflow test, mirrored: a wall at
    the upper end and an outflow at the lower end, u* = 0 (lower face too),
    s = 0.  Every face velocity stays zero, so on the lower outflow face
    p_0 = -(rho0/rho_0 - 1) p_hat_0 (rho of the first cell on that face) and
    p_{i+1} = p_i - rho0 (1/rho_f - 1/rho0)(p_hat_{i+1} - p_hat_i)."""
    n = 12
    shape = [3, 4, 5]
    shape[axis] = n
    nz, ny, nx = shape
    dzf = (np.random.default_rng(44).uniform(0.5, 1.5, nz) / nz if axis == 0
           else np.full(nz, 1.0 / nz))
    g = oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, bc)
    r = np.random.default_rng(45 + axis)
    rl = r.uniform(1.0, 50.0, n)
    pl = r.standard_normal(n)
    bshape = [1, 1, 1]
    bshape[axis] = n
    rho = np.broadcast_to(rl.reshape(bshape), g.shape).copy()
    phat = np.broadcast_to(pl.reshape(bshape), g.shape).copy()
    z = np.zeros(g.shape)
    lower = tuple(None if lo != "D" else np.zeros(
        {0: (g.nz, g.ny), 1: (g.nz, g.nx), 2: (g.ny, g.nx)}[d]) for d, (lo, _) in enumerate(g.ends))
    rho0 = 1.0
    u, v, w, p, low = oracle.project(z, z, z, phat, rho, rho0, z, 0.4, g, lower=lower)
    expect = np.zeros(n)
    expect[0] = -(rho0 / rl[0] - 1.0) * pl[0]
    for i in range(n - 1):
        rf = 0.5 * (rl[i] + rl[i + 1])
        expect[i + 1] = expect[i] - rho0 * (1.0 / rf - 1.0 / rho0) * (pl[i + 1] - pl[i])
    want = np.broadcast_to(expect.reshape(bshape), g.shape)
    assert np.abs(p - want).max() <= 1e-11 * np.abs(expect).max()
    for vel in (u, v, w) + tuple(a for a in low if a is not None):
        assert np.abs(vel).max() <= 1e-10 * np.abs(pl).max() * n
