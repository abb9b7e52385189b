"""GPU parity with outflow ends (p = 0 on the boundary face): the HIP path
through the C ABI against the FP64 oracle.

Outflow at both ends of x or y runs the sine transform (the cosine transform
of the sign-alternated line); a wall at one end and an outflow at the other
runs the quarter-wave cosine transform (DCT-IV through a half-length complex
FFT; reversed lines for an outflow at the lower end); in z the tridiagonal
pass takes an outflow at either end (extra diagonal term of the end row) and
the spectral z pass an outflow at both ends.  With an outflow end the operator is non-singular: no
mean is removed, and the mixed chain corrects without removing means.

Tolerances: FP64 relative L2 <= 1e-12; mixed precision <= 1e-10.
"""
import numpy as np
import pytest

import oracle
import vofsynth

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1907_00890_amd  # noqa: F401  (fails loudly without the library)
    return torch


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def _grid(nx, ny, nz, bc, beta=None):
    dzf = vofsynth.uniform_dz(nz, 1.0) if beta is None else vofsynth.stretched_dz(nz, 1.0, beta)
    return oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, bc)


def _plan(g, precision="fp64", max_batch=1):
    from paper_1907_00890_amd import Plan
    return Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc, precision=precision,
                max_batch=max_batch)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


SOLVE_CASES = [
    # (nx, ny, nz, bc, beta)
    (32, 32, 32, "DDD", None),           # outflow on every side
    (64, 32, 40, "DDD", 1.5),            # stretched z, ragged segments
    (32, 32, 48, "NNNNND", None),        # container: walls, outflow at the top
    (64, 64, 40, "NNNNND", 1.3),
    (16, 32, 24, "PPPPDN", 1.2),         # outflow at the bottom only
    (128, 16, 17, "DPN", None),          # x outflow, y periodic, z walls
    (16, 128, 9, "PDP", None),           # y outflow, periodic z
    (1024, 8, 5, "DDNNDD", None),        # longest x line, z outflow both ends
    (8, 1024, 4, "NNDDND", None),        # longest y line
    (16, 8, 600, "PPPPND", 1.5),         # long stretched z line
    (8, 8, 1024, "PPD", None),           # longest z, spectral z DST
    (32, 16, 1, "PPD", None),            # one-cell slab, outflow both z faces
    (32, 16, 1, "DDN", None),
    (16, 16, 2, "NNNNDN", None),
    # a wall and an outflow in x or y (quarter-wave transforms), every length
    (8, 16, 12, "NDPPNN", None),
    (16, 8, 12, "DNNDNN", 1.2),
    (32, 64, 10, "NDDNPP", None),
    (64, 32, 20, "DNPPND", 1.4),
    (128, 16, 9, "NDNNNN", None),
    (256, 8, 7, "DNNNDD", None),
    (512, 16, 3, "NDPPPP", None),
    (1024, 8, 5, "DNNDNN", None),
    (16, 128, 9, "PPNDNN", None),
    (8, 256, 5, "NNDNND", None),
    (16, 512, 4, "PPDNDD", None),
    (8, 1024, 3, "DDNDNN", None),
]


@pytest.mark.parametrize("case", SOLVE_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_solve_parity(torch_dev, case):
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 300 + nx + ny + nz)  # non-zero mean: no compatibility
    ref, fbar = oracle.solve(f, g, return_mean=True)
    assert fbar == 0.0
    plan = _plan(g)
    p = plan.solve(_dev(torch, f))
    torch.cuda.synchronize()
    err = rel_l2(p.cpu().numpy(), ref)
    print(f"outflow solve {case}: rel L2 {err:.3e}")
    assert err <= FP64_TOL, err
    assert plan.last_mean() == 0.0


def test_closed_form_sine_modes(torch_dev):
    """Outflow on every side, uniform grid: a product of discrete sine modes
    is an eigenfunction, p = f / Lambda (closed form, not the oracle)."""
    torch = torch_dev
    n, h = 32, 1.0 / 32
    c = np.arange(n) + 0.5
    mx, my, mz = 2, 5, n - 1
    sx = np.sin(np.pi * (mx + 1) * c / n)
    sy = np.sin(np.pi * (my + 1) * c / n)
    sz = np.sin(np.pi * (mz + 1) * c / n)
    lam = sum(-(4 / h**2) * np.sin(np.pi * (m + 1) / (2 * n)) ** 2 for m in (mx, my, mz))
    p_exact = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    g = _grid(n, n, n, "DDD")
    p = _plan(g).solve(_dev(torch, lam * p_exact)).cpu().numpy()
    assert np.abs(p - p_exact).max() <= 1e-12


@pytest.mark.parametrize("case", [(32, 32, 32, "DDD", None), (16, 64, 512, "NNNNDD", None),
                                  (64, 16, 8, "DPD", None), (8, 8, 1024, "PPD", None)],
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_z_spectral_matches_tridiagonal(torch_dev, case):
    """Uniform z with outflow at both z ends: the spectral z pass (sine
    transform, both radix schedules) and the tridiagonal pass agree to
    rounding and match the oracle."""
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 41 + nz)
    ref = oracle.solve(f, g)
    plan = _plan(g)
    assert plan.tuning()["z_spectral"] == 1
    got = {}
    for spec, radix in ((0, 16), (1, 16), (1, 8)):
        plan.tune("z_spectral", spec)
        plan.tune("z_radix", radix)
        got[(spec, radix)] = plan.solve(_dev(torch, f)).cpu().numpy()
    for key, p in got.items():
        assert rel_l2(p, ref) <= FP64_TOL, key
        assert rel_l2(p, got[(0, 16)]) <= 1e-13, key


def test_z_spectral_refused_for_one_outflow_end(torch_dev):
    from paper_1907_00890_amd import VofPoissonError
    plan = _plan(_grid(32, 32, 32, "NNNNND"))
    assert plan.tuning()["z_spectral"] == 0
    with pytest.raises(VofPoissonError):
        plan.tune("z_spectral", 1)


@pytest.mark.parametrize("case", [(32, 32, 32, "DDD", None), (64, 32, 40, "NNNNND", 1.5),
                                  (16, 16, 64, "PPPPDN", None), (64, 32, 24, "NDDNND", 1.3),
                                  (1024, 16, 4, "DNNDPP", None), (16, 1024, 4, "NDDNNN", None)],
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_radix8_and_mixed(torch_dev, case):
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 17)
    ref = oracle.solve(f, g)
    plan = _plan(g)
    plan.tune("x_radix", 8)
    plan.tune("y_radix", 8)
    assert rel_l2(plan.solve(_dev(torch, f)).cpu().numpy(), ref) <= FP64_TOL
    mixed = _plan(g, precision="mixed")
    mixed.set_mixed(3, tol=0.0)
    err = rel_l2(mixed.solve(_dev(torch, f)).cpu().numpy(), ref)
    print(f"outflow mixed {case}: rel L2 {err:.3e}")
    assert err <= MIXED_TOL, err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_equals_single(torch_dev, prec):
    torch = torch_dev
    g = _grid(32, 16, 24, "NDDNND", 1.4)
    n = 3
    fs = [vofsynth.gaussian_field(g.shape, 60 + i) for i in range(n)]
    plan = _plan(g, precision=prec, max_batch=n)
    singles = [plan.solve(_dev(torch, f)).cpu().numpy() for f in fs]
    outs = plan.solve_batched([_dev(torch, f) for f in fs])
    torch.cuda.synchronize()
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    for a, b, f in zip(outs, singles, fs):
        assert np.array_equal(a.cpu().numpy(), b)
        assert rel_l2(b, oracle.solve(f, g)) <= tol


def _step_inputs(g, seed=2):
    us, vs, ws = vofsynth.random_faces(g.shape, seed + 1, g.bc)
    phat = vofsynth.gaussian_field(g.shape, seed + 20)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=seed)
    rho = 1000.0 * C + 1.0 * (1 - C)
    mag, _ = vofsynth.grad_mag_central(C, g.dx, g.dy, g.dzf, g.bc)
    q = vofsynth.interface_normal_faces(C, g.dx, g.dy, g.dzf, g.bc, 1e-5)
    return us, vs, ws, phat, rho, 1.0, 1e-2 * mag, 0.3, q


STEP_CASES = [((64, 64, 64), "NNNNND", None), ((64, 32, 48), "PPPPND", 1.5),
              ((32, 32, 32), "NNPPND", None), ((64, 64, 32), "NDNDND", 1.2),
              ((128, 16, 16), "NDPPNN", None)]


@pytest.mark.parametrize("shape,bc,beta", STEP_CASES)
def test_project_and_step_upper_outflow(torch_dev, shape, bc, beta):
    """Outflow at the top (the container of section 4): projection, extension
    and the fused step against the oracle, and D u^{n+1} = s exactly."""
    torch = torch_dev
    g = _grid(*shape, bc, beta)
    us, vs, ws, phat, rho, rho0, s, dt, q = _step_inputs(g)
    u1, v1, w1, p1 = oracle.project(us, vs, ws, phat, rho, rho0, s, dt, g)
    T = lambda a: _dev(torch, a)  # noqa: E731
    plan = _plan(g)
    out = plan.project(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt)
    torch.cuda.synchronize()
    for name, a, b in zip("uvwp", out, (u1, v1, w1, p1)):
        err = rel_l2(a.cpu().numpy(), b)
        print(f"outflow project {shape} {bc} {name}: {err:.3e}")
        assert err <= FP64_TOL, (name, err)
    d = oracle.div(*(a.cpu().numpy() for a in out[:3]), g)
    assert np.abs(d - s).max() <= 1e-11 * np.abs(oracle.div(us, vs, ws, g)).max()

    ref = oracle.extend(u1, v1, w1, s, g, q=q)
    ext = plan.extend(T(u1), T(v1), T(w1), T(s), q=tuple(T(a) for a in q),
                      phi=T(np.zeros(g.shape)))
    torch.cuda.synchronize()
    for name, a, b in zip(("ue", "ve", "we", "ug", "vg", "wg", "phi"), ext, ref):
        assert rel_l2(a.cpu().numpy(), b) <= FP64_TOL, name

    got = {}
    for tiled in (0, 8):
        plan.tune("epilogue_tiled", tiled)
        plan.tune("rhs_tiled", tiled)
        o = plan.step(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt, T(s),
                      q=tuple(T(a) for a in q), out=tuple(T(np.zeros(g.shape)) for _ in range(3)))
        torch.cuda.synchronize()
        got[tiled] = [a.cpu().numpy() for a in o]
    u, v, w, p, phi, ue, ve, we, ug, vg, wg = got[0]
    for name, a, b in [("u", u, u1), ("v", v, v1), ("w", w, w1), ("p", p, p1), ("phi", phi, ref[6]),
                       ("ue", ue, ref[0]), ("ve", ve, ref[1]), ("we", we, ref[2]),
                       ("ug", ug, ref[3]), ("vg", vg, ref[4]), ("wg", wg, ref[5])]:
        assert rel_l2(a, b) <= FP64_TOL, name
    for a, b in zip(got[0], got[8]):
        assert np.array_equal(a, b)  # plain and LDS-staged stencils: same bits


def test_static_extension_with_outflow_top(torch_dev):
    """u = G psi, s = L_h psi with outflow at the top: phi = psi, u_1^e = 0."""
    torch = torch_dev
    g = _grid(64, 64, 48, "NNNNND", 1.2)
    psi = vofsynth.gaussian_field(g.shape, 9)
    u = oracle.grad(psi, g)
    s = oracle.lap(psi, g)
    out = _plan(g).extend(*(_dev(torch, a) for a in u), _dev(torch, s),
                          phi=_dev(torch, np.zeros(g.shape)))
    torch.cuda.synchronize()
    scale = max(np.abs(a).max() for a in u)
    for a in out[:3]:
        assert np.abs(a.cpu().numpy()).max() <= 1e-10 * scale
    assert np.abs(out[6].cpu().numpy() - psi).max() <= 1e-10 * np.abs(psi).max()


def test_lower_outflow_face_stencils_refused(torch_dev):
    """An outflow face at a lower end has no stored velocity: the face-stencil
    entry points refuse the plan (the solve accepts it)."""
    torch = torch_dev
    from paper_1907_00890_amd import VofPoissonError
    g = _grid(32, 32, 16, "NNNNDN")
    plan = _plan(g)
    z = lambda: _dev(torch, np.zeros(g.shape))  # noqa: E731
    with pytest.raises(VofPoissonError) as e:
        plan.project(z(), z(), z(), z(), _dev(torch, np.ones(g.shape)), 1.0, None, 0.1)
    assert e.value.status == -2
    with pytest.raises(VofPoissonError) as e:
        plan.extend(z(), z(), z(), z(), phi=z())
    assert e.value.status == -2
    f = vofsynth.gaussian_field(g.shape, 3)
    assert rel_l2(plan.solve(_dev(torch, f)).cpu().numpy(), oracle.solve(f, g)) <= FP64_TOL
