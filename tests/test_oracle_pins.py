"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* closed-form discrete eigenfunctions of the staggered second difference
  (sin/cos modes; every P/N combination, non-cubic, dx != dy != dz);
* second-order convergence to the continuous eigenfunction;
* brute force: the Laplacian assembled entry by entry in plain loops, and
  the bordered dense system [L 1; dV^T 0] solved with numpy.linalg.solve;
* library special cases: a z-only right-hand side through
  scipy.linalg.solve_banded, a one-cell slab through numpy.fft.fft2, and
  the periodic uniform grid through numpy.fft.fftn divided by the FFT of the
  7-point stencil;
* residual, gauge (zero volume-weighted mean) and shift invariance.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import vofsynth

BCS = ["PPP", "PPN", "PNP", "NPP", "PNN", "NPN", "NNP", "NNN"]


# ----------------------------------------------------------------------------
# brute-force dense operator, written entry by entry (independent of oracle/)
# ----------------------------------------------------------------------------
def loop_laplacian(nx, ny, nz, dx, dy, dzf, bc):
    n = nx * ny * nz
    A = np.zeros((n, n))

    def idx(i, j, k):
        return i + nx * (j + ny * k)

    def zdist(face):  # distance between centres across face `face` + 1/2
        k0, k1 = face % nz, (face + 1) % nz
        return 0.5 * (dzf[k0] + dzf[k1])

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = idx(i, j, k)
                for d in (-1, 1):
                    ii = i + d
                    if 0 <= ii < nx or bc[0] == "P":
                        A[r, idx(ii % nx, j, k)] += 1.0 / dx**2
                        A[r, r] -= 1.0 / dx**2
                    jj = j + d
                    if 0 <= jj < ny or bc[1] == "P":
                        A[r, idx(i, jj % ny, k)] += 1.0 / dy**2
                        A[r, r] -= 1.0 / dy**2
                    kk = k + d
                    if 0 <= kk < nz or bc[2] == "P":
                        face = k if d == 1 else k - 1
                        c = 1.0 / (dzf[k] * zdist(face))
                        A[r, idx(i, j, kk % nz)] += c
                        A[r, r] -= c
    return A


def bordered_solve(A, f, dv):
    """Solve L p + mu 1 = f, dV^T p = 0 densely."""
    n = A.shape[0]
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A
    M[:n, n] = 1.0
    M[n, :n] = dv
    rhs = np.concatenate([f, [0.0]])
    sol = np.linalg.solve(M, rhs)
    return sol[:n], sol[n]


def random_dz(nz, seed):
    r = np.random.default_rng(seed).uniform(0.5, 2.0, size=nz)
    return r / r.sum()


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("stretched", [False, True])
def test_brute_force_dense(bc, stretched):
    nx, ny, nz = 8, 4, 6
    dx, dy = 1.0 / nx, 0.7 / ny
    dzf = random_dz(nz, 7) * 1.3 if stretched else np.full(nz, 1.3 / nz)
    g = oracle.Grid(nx, ny, nz, dx, dy, dzf, bc)
    A = loop_laplacian(nx, ny, nz, dx, dy, dzf, bc)
    f = np.random.default_rng(3).standard_normal(g.shape)
    dv = np.broadcast_to(g.cell_volume(), g.shape).reshape(-1)
    p_ref, mu = bordered_solve(A, f.reshape(-1), dv)
    p = oracle.solve(f, g)
    err = np.linalg.norm(p.reshape(-1) - p_ref) / np.linalg.norm(p_ref)
    assert err < 1e-12, err
    # the multiplier of the bordered system is the volume-weighted mean of f
    assert abs(mu - g.weighted_mean(f)) < 1e-12 * np.abs(f).max()
    # the oracle's stencils agree with the loop-built operator entry by entry
    q = np.random.default_rng(4).standard_normal(g.shape)
    lq = oracle.lap(q, g).reshape(-1)
    assert np.allclose(lq, A @ q.reshape(-1), rtol=0, atol=1e-12 * np.abs(A).max())


def loop_grad_div(nx, ny, nz, dx, dy, dzf, bc, p, u, v, w):
    """Face gradient and cell divergence written point by point."""
    gx = np.zeros((nz, ny, nx)); gy = np.zeros_like(gx); gz = np.zeros_like(gx)
    d = np.zeros_like(gx)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if i + 1 < nx or bc[0] == "P":
                    gx[k, j, i] = (p[k, j, (i + 1) % nx] - p[k, j, i]) / dx
                if j + 1 < ny or bc[1] == "P":
                    gy[k, j, i] = (p[k, (j + 1) % ny, i] - p[k, j, i]) / dy
                if k + 1 < nz or bc[2] == "P":
                    kk = (k + 1) % nz
                    gz[k, j, i] = (p[kk, j, i] - p[k, j, i]) / (0.5 * (dzf[k] + dzf[kk]))
                um = u[k, j, i - 1] if (i > 0 or bc[0] == "P") else 0.0
                vm = v[k, j - 1, i] if (j > 0 or bc[1] == "P") else 0.0
                wm = w[k - 1, j, i] if (k > 0 or bc[2] == "P") else 0.0
                d[k, j, i] = ((u[k, j, i] - um) / dx + (v[k, j, i] - vm) / dy
                              + (w[k, j, i] - wm) / dzf[k])
    return (gx, gy, gz), d


@pytest.mark.parametrize("bc", ["PPN", "NPN", "PNP", "NNN"])
def test_stencils_pointwise(bc):
    nx, ny, nz = 6, 4, 5
    dx, dy = 0.3, 0.2
    dzf = random_dz(nz, 9)
    g = oracle.Grid(nx, ny, nz, dx, dy, dzf, bc)
    r = np.random.default_rng(11)
    p, u, v, w = (r.standard_normal(g.shape) for _ in range(4))
    (gx, gy, gz), d = loop_grad_div(nx, ny, nz, dx, dy, dzf, bc, p, u, v, w)
    ox, oy, oz = oracle.grad(p, g)
    assert np.allclose(ox, gx, atol=1e-13) and np.allclose(oy, gy, atol=1e-13)
    assert np.allclose(oz, gz, atol=1e-12)
    assert np.allclose(oracle.div(u, v, w, g), d, atol=1e-12)


# ----------------------------------------------------------------------------
# closed-form discrete eigenfunctions
# ----------------------------------------------------------------------------
def _mode(n, h, letter, m):
    x = (np.arange(n) + 0.5) * h
    L = n * h
    if letter == "P":
        return np.sin(2.0 * np.pi * m * x / L), -(4.0 / h**2) * np.sin(np.pi * m / n) ** 2
    return np.cos(np.pi * m * x / L), -(4.0 / h**2) * np.sin(np.pi * m / (2 * n)) ** 2


def test_eigenfunction_config0_value():
    """sin(2 pi x) cos(4 pi y) sin(2 pi z) on 32^3, L = 1: p = f / Lambda."""
    n, h = 32, 1.0 / 32
    x = (np.arange(n) + 0.5) * h
    f = (np.sin(2 * np.pi * x)[None, None, :] * np.cos(4 * np.pi * x)[None, :, None]
         * np.sin(2 * np.pi * x)[:, None, None])
    lam = -(4.0 / h**2) * (2 * np.sin(np.pi / n) ** 2 + np.sin(2 * np.pi / n) ** 2)
    assert abs(lam - (-234.5982088852528)) < 1e-9
    g = oracle.Grid(n, n, n, h, h, np.full(n, h), "PPP")
    p = oracle.solve(f, g)
    err = np.linalg.norm(p - f / lam) / np.linalg.norm(f / lam)
    assert err < 1e-13, err


@pytest.mark.parametrize("bc", BCS)
def test_eigenfunction_all_bcs(bc):
    nx, ny, nz = 16, 8, 12
    hx, hy, hz = 1.0 / nx, 0.5 / ny, 2.0 / nz
    fx, lx = _mode(nx, hx, bc[0], 3)
    fy, ly = _mode(ny, hy, bc[1], 1)
    fz, lz = _mode(nz, hz, bc[2], 2)
    f = fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    g = oracle.Grid(nx, ny, nz, hx, hy, np.full(nz, hz), bc)
    p = oracle.solve(f, g)
    lam = lx + ly + lz
    err = np.linalg.norm(p - f / lam) / np.linalg.norm(f / lam)
    assert err < 1e-13, err


def test_second_order_convergence():
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        f = (np.sin(2 * np.pi * x)[None, None, :] * np.cos(4 * np.pi * x)[None, :, None]
             * np.sin(2 * np.pi * x)[:, None, None])
        g = oracle.Grid(n, n, n, h, h, np.full(n, h), "PPP")
        p = oracle.solve(f, g)
        exact = f / (-24.0 * np.pi**2)
        errs.append(np.abs(p - exact).max() / np.abs(exact).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.9 < r2 < 4.1, errs


# ----------------------------------------------------------------------------
# library special cases
# ----------------------------------------------------------------------------
def ld_pinned_thomas(fz, dzf, periodic):
    """Textbook Thomas sweep in numpy longdouble on the pinned 1-D problem
    (p0 = 0, rows 1..nz-1, then the weighted mean removed)."""
    L = np.longdouble
    nz = len(fz)
    dzf_l = dzf.astype(L)
    fc = fz.astype(L) - (fz.astype(L) * dzf_l).sum() / dzf_l.sum()
    dzc = (dzf_l + np.roll(dzf_l, -1)) / 2
    lo = np.zeros(nz, L); up = np.zeros(nz, L)
    for k in range(nz):
        if k + 1 < nz or periodic:
            up[k] = 1 / (dzf_l[k] * dzc[k])
        if k > 0 or periodic:
            lo[k] = 1 / (dzf_l[k] * dzc[k - 1])
    di = -(lo + up)
    cp = np.zeros(nz, L); dp = np.zeros(nz, L); x = np.zeros(nz, L)
    for k in range(1, nz):
        den = di[k] - (lo[k] * cp[k - 1] if k > 1 else 0)
        cp[k] = up[k] / den
        dp[k] = (fc[k] - (lo[k] * dp[k - 1] if k > 1 else 0)) / den
    x[nz - 1] = dp[nz - 1]
    for k in range(nz - 2, 0, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    x -= (x * dzf_l).sum() / dzf_l.sum()
    return x.astype(np.float64)


@pytest.mark.parametrize("zbc", ["N", "P"])
@pytest.mark.parametrize("nz", [600, 1024])
def test_z_only_rhs_long_lines(zbc, nz):
    """Long, ill-conditioned z lines against an extended-precision sweep."""
    dzf = vofsynth.stretched_dz(nz, 1.0, 1.5) if zbc == "N" else np.full(nz, 1.0 / nz)
    g = oracle.Grid(4, 4, nz, 0.25, 0.25, dzf, "PP" + zbc)
    fz = np.random.default_rng(nz).standard_normal(nz)
    p = oracle.solve(np.broadcast_to(fz[:, None, None], g.shape).copy(), g)
    ref = ld_pinned_thomas(fz, dzf, zbc == "P")
    assert np.abs(p[:, 0, 0] - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("zbc", ["N", "P"])
def test_z_only_rhs_solve_banded(zbc):
    nx, ny, nz = 4, 4, 40
    dzf = vofsynth.stretched_dz(nz, 1.0, 1.5) if zbc == "N" else np.full(nz, 1.0 / nz)
    g = oracle.Grid(nx, ny, nz, 0.25, 0.25, dzf, "PP" + zbc)
    fz = np.random.default_rng(5).standard_normal(nz)
    f = np.broadcast_to(fz[:, None, None], g.shape).copy()
    p = oracle.solve(f, g)
    # textbook route: remove the weighted mean, pin p0 = 0, solve the rest banded
    fc = fz - (fz * dzf).sum() / dzf.sum()
    dzc = 0.5 * (dzf + np.roll(dzf, -1))
    lo = np.zeros(nz); di = np.zeros(nz); up = np.zeros(nz)
    for k in range(nz):
        if k + 1 < nz or zbc == "P":
            up[k] = 1.0 / (dzf[k] * dzc[k])
        if k > 0 or zbc == "P":
            lo[k] = 1.0 / (dzf[k] * dzc[k - 1])
        di[k] = -(up[k] + lo[k])
    m = nz - 1  # unknowns p1..p_{nz-1}
    ab = np.zeros((3, m))
    ab[0, 1:] = up[1:m]
    ab[1, :] = di[1:]
    ab[2, :-1] = lo[2:]
    q = sla.solve_banded((1, 1), ab, fc[1:])
    pz = np.concatenate([[0.0], q])
    pz -= (pz * dzf).sum() / dzf.sum()
    assert np.allclose(p, pz[:, None, None], rtol=0, atol=1e-12 * np.abs(pz).max())


def test_slab_fft2():
    nx, ny = 64, 32
    dx, dy = 1.0 / nx, 0.5 / ny
    g = oracle.Grid(nx, ny, 1, dx, dy, [1.0 / 1024], "PPN")
    f = np.random.default_rng(6).standard_normal(g.shape)
    p = oracle.solve(f, g)
    kern = np.zeros((ny, nx))
    kern[0, 0] = -2 / dx**2 - 2 / dy**2
    kern[0, 1] = kern[0, -1] = 1 / dx**2
    kern[1, 0] = kern[-1, 0] = 1 / dy**2
    sym = np.fft.fft2(kern).real
    F = np.fft.fft2(f[0])
    sym[0, 0] = np.inf
    ref = np.fft.ifft2(F / sym).real
    assert np.allclose(p[0], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_periodic_fftn():
    nx, ny, nz = 32, 16, 24
    dx, dy, dz = 1.0 / nx, 2.0 / ny, 1.5 / nz
    g = oracle.Grid(nx, ny, nz, dx, dy, np.full(nz, dz), "PPP")
    f = np.random.default_rng(8).standard_normal(g.shape)
    kern = np.zeros(g.shape)
    kern[0, 0, 0] = -2 / dx**2 - 2 / dy**2 - 2 / dz**2
    kern[0, 0, 1] = kern[0, 0, -1] = 1 / dx**2
    kern[0, 1, 0] = kern[0, -1, 0] = 1 / dy**2
    kern[1, 0, 0] = kern[-1, 0, 0] = 1 / dz**2
    sym = np.fft.fftn(kern).real
    sym[0, 0, 0] = np.inf
    ref = np.fft.ifftn(np.fft.fftn(f) / sym).real
    p = oracle.solve(f, g)
    assert np.allclose(p, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


# ----------------------------------------------------------------------------
# residual, gauge and shift invariance on configuration-like sizes
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name,stretch", [("ppp32", None), ("ppn64s", 1.5), ("nnn", None)])
def test_residual_gauge_shift(name, stretch):
    if name == "ppp32":
        cfg = vofsynth.config("ppp32")
        g = oracle.Grid.from_config(cfg)
    elif name == "ppn64s":
        dzf = vofsynth.stretched_dz(64, 1.0, stretch)
        g = oracle.Grid(64, 64, 64, 1 / 64, 1 / 64, dzf, "PPN")
    else:
        g = oracle.Grid(32, 16, 24, 1 / 32, 1 / 16, vofsynth.stretched_dz(24, 1.0, 1.2), "NNN")
    f = vofsynth.gaussian_field(g.shape, 0)
    p = oracle.solve(f, g)
    r = oracle.lap(p, g) - (f - g.weighted_mean(f))
    assert np.linalg.norm(r) / np.linalg.norm(f) < 1e-12
    dv = g.cell_volume()
    assert abs((p * dv).sum()) < 1e-13 * np.abs(p * dv).sum()
    p2 = oracle.solve(f + 3.25, g)
    assert np.allclose(p2, p, rtol=0, atol=1e-12 * np.abs(p).max())


@pytest.mark.parametrize("shape,bc", [((24, 4, 3), "PPN"), ((4, 24, 3), "NPN"),
                                      ((40, 3, 4), "PNN"), ((3, 40, 4), "NNP"),
                                      ((12, 20, 3), "PPP"), ((48, 3, 3), "NNN")],
                         ids=lambda c: c if isinstance(c, str) else "x".join(map(str, c)))
def test_brute_force_dense_odd_lengths(shape, bc):
    """Lengths with an odd factor (3 * 2^k, 5 * 2^k, as the GPU transforms
    take them) with periodic and wall ends: the oracle's solve equals the
    bordered dense solve of the loop-built operator."""
    nx, ny, nz = shape
    dx, dy = 1.0 / nx, 0.7 / ny
    dzf = random_dz(nz, 9) * 1.1
    g = oracle.Grid(nx, ny, nz, dx, dy, dzf, bc)
    A = loop_laplacian(nx, ny, nz, dx, dy, dzf, bc)
    f = np.random.default_rng(6).standard_normal(g.shape)
    dv = np.broadcast_to(g.cell_volume(), g.shape).reshape(-1)
    p_ref, _ = bordered_solve(A, f.reshape(-1), dv)
    p = oracle.solve(f, g)
    err = np.linalg.norm(p.reshape(-1) - p_ref) / np.linalg.norm(p_ref)
    assert err < 1e-12, err
