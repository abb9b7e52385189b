"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Element-by-element relative L2 on seeded inputs at sizes the oracle finishes
in seconds (several FFT tiles, ragged z segments, every boundary
combination); at the full benchmark sizes, properties that hold at any size
(residual of the discrete equation and the gauge) evaluated with plain torch
ops, independent of the library's own stencils.

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
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _grid(nx, ny, nz, bc, beta=None, lx=1.0, ly=1.0, lz=1.0):
    dzf = vofsynth.uniform_dz(nz, lz) if beta is None else vofsynth.stretched_dz(nz, lz, beta)
    return oracle.Grid(nx, ny, nz, lx / nx, ly / ny, dzf, bc)


def _plan(g, precision="fp64", max_batch=1):
    from paper_1907_00890_amd import Plan
    return Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc, precision=precision,
                max_batch=max_batch)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


SOLVE_CASES = [
    # (nx, ny, nz, bc, beta)
    (32, 32, 32, "PPP", None),       # 32^3 triply periodic
    (128, 128, 128, "PPN", None),    # 128^3 periodic x/y, walls z
    (64, 32, 40, "NPN", 1.5),        # stretched, ragged segments
    (16, 8, 12, "PNN", 1.3),
    (8, 16, 3, "PPP", None),         # shortest periodic z
    (32, 64, 17, "NNP", None),       # odd periodic z (segments 9 + 8)
    (16, 16, 2, "NNN", None),
    (16, 32, 1, "PPN", None),        # one-cell slab
    (1024, 8, 5, "PNN", None),       # longest x line
    (8, 1024, 4, "NPN", None),       # longest y line
    (16, 8, 600, "PPN", 1.5),        # 32-row segments
    (8, 8, 1024, "PPP", None),       # longest z
    (256, 16, 33, "NNN", 1.1),
]


@pytest.mark.parametrize("case", SOLVE_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_solve_parity(torch_dev, case):
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 100 + nx + ny + nz)
    ref = oracle.solve(f, g)
    plan = _plan(g)
    p = plan.solve(_dev(torch, f))
    torch.cuda.synchronize()
    err = rel_l2(p.cpu().numpy(), ref)
    print(f"solve {case}: rel L2 {err:.3e}")
    assert err <= FP64_TOL, err
    # the weighted mean of the rhs is reported
    assert abs(plan.last_mean() - g.weighted_mean(f)) <= 1e-13 * np.abs(f).max()
    plan.close()


def test_solve_in_place_and_offset(torch_dev):
    torch = torch_dev
    g = _grid(64, 64, 48, "PPN", 1.5)
    f = vofsynth.gaussian_field(g.shape, 7) + 5.0
    ref = oracle.solve(f, g)
    plan = _plan(g)
    t = _dev(torch, f)
    plan.solve(t, out=t)
    torch.cuda.synchronize()
    assert rel_l2(t.cpu().numpy(), ref) <= FP64_TOL


def test_eigenfunction_closed_form(torch_dev):
    """sin(2 pi x) cos(4 pi y) sin(2 pi z), 32^3 periodic: p = f / Lambda."""
    torch = torch_dev
    n, h = 32, 1.0 / 32
    x = (np.arange(n) + 0.5) * h
    f = (np.sin(2 * np.pi * x)[None, None, :] * np.cos(4 * np.pi * x)[None, :, None]
         * np.sin(2 * np.pi * x)[:, None, None])
    lam = -(4.0 / h**2) * (2 * np.sin(np.pi / n) ** 2 + np.sin(2 * np.pi / n) ** 2)
    g = _grid(n, n, n, "PPP")
    p = _plan(g).solve(_dev(torch, f)).cpu().numpy()
    assert rel_l2(p, f / lam) <= FP64_TOL


def _project_inputs(g, seed=2):
    us, vs, ws = vofsynth.random_faces(g.shape, seed + 1, g.bc)
    phat = vofsynth.gaussian_field(g.shape, seed + 20)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=seed)
    rho = 1000.0 * C + 1.0 * (1 - C)
    mag, _ = vofsynth.grad_mag_central(C, g.dx, g.dy, g.dzf, g.bc)
    s = 1e-2 * mag
    return us, vs, ws, phat, rho, 1.0, s, 0.3


@pytest.mark.parametrize("shape,bc,beta", [((128, 128, 128), "PPN", None),
                                           ((64, 32, 48), "NPN", 1.5),
                                           ((32, 32, 32), "PPP", None)])
def test_project_parity(torch_dev, shape, bc, beta):
    torch = torch_dev
    g = _grid(*shape, bc, beta)
    us, vs, ws, phat, rho, rho0, s, dt = _project_inputs(g)
    u, v, w, p = oracle.project(us, vs, ws, phat, rho, rho0, s, dt, g)
    plan = _plan(g)
    du, dv, dw = _dev(torch, us), _dev(torch, vs), _dev(torch, ws)
    out = plan.project(du, dv, dw, _dev(torch, phat), _dev(torch, rho), rho0, _dev(torch, s), dt)
    torch.cuda.synchronize()
    for name, a, b in zip("uvwp", out, (u, v, w, p)):
        err = rel_l2(a.cpu().numpy(), b)
        print(f"project {shape} {bc} {name}: {err:.3e}")
        assert err <= FP64_TOL, (name, err)
    # invariant on the GPU result: D u^{n+1} = s - mean_W(s)
    d = oracle.div(out[0].cpu().numpy(), out[1].cpu().numpy(), out[2].cpu().numpy(), g)
    scale = np.abs(oracle.div(us, vs, ws, g)).max()
    assert np.abs(d - (s - g.weighted_mean(s))).max() <= 1e-11 * scale


@pytest.mark.parametrize("shape,bc,beta", [((64, 32, 40), "NPN", 1.5), ((128, 64, 24), "PPP", None),
                                           ((64, 16, 5), "NNN", None), ((256, 16, 9), "PNP", None)])
def test_rhs_tiled_bit_identical(torch_dev, shape, bc, beta):
    """The LDS-tiled right-hand side gives the plain kernel's projection bit for
    bit, for several planes per block, and the oracle's within tolerance."""
    torch = torch_dev
    g = _grid(*shape, bc, beta)
    us, vs, ws, phat, rho, rho0, s, dt, q = _step_inputs(g)
    T = lambda a: _dev(torch, a)  # noqa: E731
    plan = _plan(g)
    outs, nosrc = {}, {}
    for tiled in (0, 8, 16):
        for kc in (1, 2, 3, 4, 8):
            plan.tune("rhs_tiled", tiled)
            plan.tune("stencil_planes", min(kc, g.nz))
            u, v, w, p = plan.project(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt)
            outs[(tiled, kc)] = [a.cpu().numpy() for a in (u, v, w, p)]
            if kc in (1, 3):  # without a source term (s = 0)
                u, v, w, p = plan.project(T(us), T(vs), T(ws), T(phat), T(rho), rho0, None, dt)
                nosrc[(tiled, kc)] = [a.cpu().numpy() for a in (u, v, w, p)]
    for res in (outs, nosrc):
        base = res[(0, 1)]
        for key, val in res.items():
            for a, b in zip(val, base):
                assert np.array_equal(a, b), key
    base = outs[(0, 1)]
    ref = oracle.project(us, vs, ws, phat, rho, rho0, s, dt, g)
    for a, b in zip(base, ref):
        assert rel_l2(a, b) <= FP64_TOL


def test_project_without_source(torch_dev):
    torch = torch_dev
    g = _grid(32, 32, 32, "PPP")
    us, vs, ws = vofsynth.random_faces(g.shape, 1, g.bc)
    rho = np.ones(g.shape)
    z = np.zeros(g.shape)
    u, v, w, p = oracle.project(us, vs, ws, z, rho, 1.0, z, 1.0, g)
    plan = _plan(g)
    out = plan.project(_dev(torch, us), _dev(torch, vs), _dev(torch, ws), _dev(torch, z),
                       _dev(torch, rho), 1.0, None, 1.0)
    for a, b in zip(out, (u, v, w, p)):
        assert rel_l2(a.cpu().numpy(), b) <= FP64_TOL
    d = oracle.div(*(t.cpu().numpy() for t in out[:3]), g)
    assert np.abs(d).max() <= 1e-11 * np.abs(oracle.div(us, vs, ws, g)).max()


@pytest.mark.parametrize("shape,bc,beta", [((128, 128, 128), "PPN", None),
                                           ((64, 32, 48), "NPN", 1.5)])
def test_extend_parity(torch_dev, shape, bc, beta):
    torch = torch_dev
    g = _grid(*shape, bc, beta)
    usol = vofsynth.solenoidal_faces(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc, seed=3)
    psi = vofsynth.gaussian_field(g.shape, 4)
    u = [a + b for a, b in zip(usol, oracle.grad(psi, g))]
    s = oracle.lap(psi, g)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=2)
    q = vofsynth.interface_normal_faces(C, g.dx, g.dy, g.dzf, g.bc, 1.001e-2 / 1000.0)
    ref = oracle.extend(u[0], u[1], u[2], s, g, q=q)
    plan = _plan(g)
    out = plan.extend(*(_dev(torch, a) for a in u), _dev(torch, s),
                      q=tuple(_dev(torch, a) for a in q), phi=_dev(torch, np.zeros(g.shape)))
    torch.cuda.synchronize()
    for name, a, b in zip(("ue", "ve", "we", "ug", "vg", "wg", "phi"), out, ref):
        err = rel_l2(a.cpu().numpy(), b)
        print(f"extend {shape} {bc} {name}: {err:.3e}")
        assert err <= FP64_TOL, (name, err)
    # extension recovers the solenoidal part (invariant, GPU result)
    scale = max(np.abs(a).max() for a in u)
    for a, b in zip(out[:3], usol):
        assert np.abs(a.cpu().numpy() - b).max() <= 1e-10 * scale


def test_extend_static_droplet(torch_dev):
    """u = G psi only (pure Stefan flow): u_1^e = 0 and u_Gamma = -q."""
    torch = torch_dev
    g = _grid(64, 64, 64, "PPN")
    psi = vofsynth.gaussian_field(g.shape, 9)
    u = oracle.grad(psi, g)
    s = oracle.lap(psi, g)
    q = vofsynth.random_faces(g.shape, 10, g.bc)
    out = _plan(g).extend(*(_dev(torch, a) for a in u), _dev(torch, s),
                          q=tuple(_dev(torch, a) for a in q))
    scale = max(np.abs(a).max() for a in u)
    for a in out[:3]:
        assert np.abs(a.cpu().numpy()).max() <= 1e-10 * scale
    for a, b in zip(out[3:6], q):
        assert np.abs(a.cpu().numpy() + b).max() <= 1e-10 * scale


@pytest.mark.parametrize("case,dc", [((64, 64, 64, "PPP", None), 1),
                                     ((128, 128, 128, "PPN", None), 2),
                                     ((64, 32, 40, "NPN", 1.5), 2)])
def test_mixed_parity(torch_dev, case, dc):
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 4)
    f = vofsynth.remove_weighted_mean(f, g.dzf)
    ref = oracle.solve(f, g)
    plan = _plan(g, precision="mixed")
    plan.set_mixed(dc)
    p = plan.solve(_dev(torch, f))
    torch.cuda.synchronize()
    err = rel_l2(p.cpu().numpy(), ref)
    print(f"mixed {case} dc={dc}: rel L2 {err:.3e}")
    assert err <= MIXED_TOL, err
    # both radix schedules of the x passes (the correction's x forward forms
    # the defect itself)
    for xr in (8, 16):
        plan.tune("x_radix", xr)
        q = plan.solve(_dev(torch, f)).cpu().numpy()
        assert rel_l2(q, ref) <= MIXED_TOL, xr


RADIX8_CASES = [
    (256, 16, 33, "NNN", 1.1),
    (32, 32, 32, "PPP", None),
    (8, 1024, 4, "NPN", None),
    (1024, 8, 5, "PNN", None),
    (16, 512, 24, "PPN", 1.5),
]


@pytest.mark.parametrize("case", RADIX8_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_radix8_schedule_parity(torch_dev, case):
    """The radix-8 schedule of the x and y passes (a tuning knob) gives the
    oracle's result, and the radix-16 result up to rounding order."""
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 7 + nx)
    ref = oracle.solve(f, g)
    plan = _plan(g)
    p16 = plan.solve(_dev(torch, f)).cpu().numpy()
    plan.tune("x_radix", 8)
    plan.tune("y_radix", 8)
    assert plan.tuning()["x_radix"] == 8 and plan.tuning()["y_radix"] == 8
    p8 = plan.solve(_dev(torch, f)).cpu().numpy()
    assert rel_l2(p8, ref) <= FP64_TOL
    assert rel_l2(p8, p16) <= 1e-13
    # narrower y tiles move the same data through the same passes
    plan.tune("y_lines", 4)
    assert np.array_equal(plan.solve(_dev(torch, f)).cpu().numpy(), p8)
    plan.tune("y_lines", 0)
    mixed = _plan(g, precision="mixed")
    mixed.tune("x_radix", 8)
    mixed.tune("y_radix", 8)
    pm = mixed.solve(_dev(torch, f)).cpu().numpy()
    assert rel_l2(pm, ref) <= MIXED_TOL


@pytest.mark.parametrize("case", [(1024, 8, 5, "PNN", None), (8, 1024, 4, "NPN", None),
                                  (64, 64, 64, "PPP", None)],
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_mixed_stops_on_error_estimate(torch_dev, case):
    """The device-side stopping rule: its estimate bounds the error left after
    the steps it takes (one where that suffices), and after one fixed step."""
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 5 + nz)
    ref = oracle.solve(f, g)
    plan = _plan(g, precision="mixed")
    p = plan.solve(_dev(torch, f)).cpu().numpy()
    (steps, est), = plan.mixed_report()
    err = rel_l2(p, ref)
    print(f"mixed {case}: {steps} steps, estimate {est:.2e}, error {err:.2e}")
    assert err <= MIXED_TOL and 1 <= steps <= 3 and est <= 1e-11
    # the estimate bounds the error it predicts (above the FP64 parity floor)
    assert err <= est + FP64_TOL
    # fixed single step: the estimate exposes what one step leaves
    plan.set_mixed(1, tol=0.0)
    p1 = plan.solve(_dev(torch, f)).cpu().numpy()
    (s1, e1), = plan.mixed_report()
    assert s1 == 1
    err1 = rel_l2(p1, ref)
    print(f"mixed {case}, one step: estimate {e1:.2e}, error {err1:.2e}")
    assert err1 <= e1 + FP64_TOL


@pytest.mark.parametrize("case", [(32, 32, 32, "PPP", None), (128, 128, 128, "PPN", None),
                                  (16, 8, 16, "NNN", None), (8, 8, 1024, "PPP", None),
                                  (64, 16, 8, "NPP", None), (16, 64, 512, "PNN", None)],
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_z_spectral_matches_tridiagonal(torch_dev, case):
    """Uniform z: the spectral z pass (both radix schedules) and the tridiagonal
    pass agree to rounding, match the oracle, and remove the same mean."""
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 31 + nz)  # non-zero mean on purpose
    ref = oracle.solve(f, g)
    plan = _plan(g)
    assert plan.tuning()["z_spectral"] == 1
    got = {}
    for spec, radix, lines in ((0, 16, 0), (1, 16, 0), (1, 8, 0), (1, 8, 8), (1, 16, 4)):
        plan.tune("z_spectral", spec)
        plan.tune("z_radix", radix)
        plan.tune("z_spectral_lines", lines)
        got[(spec, radix, lines)] = (plan.solve(_dev(torch, f)).cpu().numpy(), plan.last_mean())
    tri, tri_mean = got[(0, 16, 0)]
    for key, (p, mean) in got.items():
        assert rel_l2(p, ref) <= FP64_TOL, key
        assert rel_l2(p, tri) <= 1e-13, key
        assert abs(mean - tri_mean) <= 1e-14 * max(1.0, abs(tri_mean)), key
    mixed = _plan(g, precision="mixed")
    pm = mixed.solve(_dev(torch, f)).cpu().numpy()
    assert rel_l2(pm, ref) <= MIXED_TOL


def test_z_spectral_refused_on_stretched_grid(torch_dev):
    from paper_1907_00890_amd import VofPoissonError
    g = _grid(32, 32, 32, "PPN", 1.5)
    plan = _plan(g)
    assert plan.tuning()["z_spectral"] == 0
    with pytest.raises(VofPoissonError):
        plan.tune("z_spectral", 1)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_autotune_keeps_parity(torch_dev, prec):
    torch = torch_dev
    g = _grid(64, 64, 48, "PPN", 1.5)
    plan = _plan(g, precision=prec, max_batch=2)
    chosen = plan.autotune(batch=2)
    assert chosen == {k: v for k, v in plan.tuning().items() if k in chosen}
    assert chosen["x_radix"] in (8, 16) and chosen["y_radix"] in (8, 16)
    assert chosen["z_lines"] in (8, 16, 32) and 1 <= chosen["stencil_planes"] <= g.nz
    f = vofsynth.gaussian_field(g.shape, 77)
    p = plan.solve(_dev(torch, f)).cpu().numpy()
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    assert rel_l2(p, oracle.solve(f, g)) <= tol


BATCH_CASES = [
    # (nx, ny, nz, bc, beta, precision, n)
    (64, 32, 24, "PPN", 1.5, "fp64", 3),
    (32, 32, 32, "PPP", None, "mixed", 4),
    (16, 8, 1, "NPN", None, "fp64", 16),      # slab, the largest batch
    (8, 16, 40, "NNP", None, "mixed", 2),
]


@pytest.mark.parametrize("case", BATCH_CASES,
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}-{c[5]}-b{c[6]}")
def test_batched_equals_single(torch_dev, case):
    """One launch per pass for the whole batch gives each member's single result
    bit for bit (the arithmetic of a member never depends on the others)."""
    torch = torch_dev
    nx, ny, nz, bc, beta, prec, n = case
    g = _grid(nx, ny, nz, bc, beta)
    fs = [vofsynth.gaussian_field(g.shape, 50 + i) for i in range(n)]
    plan = _plan(g, precision=prec, max_batch=n)
    singles = [plan.solve(_dev(torch, f)).cpu().numpy() for f in fs]
    outs = plan.solve_batched([_dev(torch, f) for f in fs])
    # in place: every member's output overwrites its own input
    ins = [_dev(torch, f) for f in fs]
    plan.solve_batched(ins, ins)
    # a smaller batch after a larger one on the same plan
    part = plan.solve_batched([_dev(torch, f) for f in fs[: max(1, n // 2)]])
    torch.cuda.synchronize()
    tol = FP64_TOL if prec == "fp64" else MIXED_TOL
    for k, (a, b, c, f) in enumerate(zip(outs, singles, ins, fs)):
        assert np.array_equal(a.cpu().numpy(), b), k
        assert np.array_equal(c.cpu().numpy(), b), k
        assert rel_l2(b, oracle.solve(f, g)) <= tol
    for a, b in zip(part, singles):
        assert np.array_equal(a.cpu().numpy(), b)


def test_extend_batched_equals_single(torch_dev):
    torch = torch_dev
    g = _grid(32, 16, 20, "PPN", 1.5)
    n = 3
    items, singles = [], []
    plan = _plan(g, max_batch=n)
    for k in range(n):
        u, v, w = vofsynth.random_faces(g.shape, 300 + k, g.bc)
        s = vofsynth.remove_weighted_mean(vofsynth.gaussian_field(g.shape, 310 + k), g.dzf)
        q = vofsynth.random_faces(g.shape, 320 + k, g.bc)
        d = [_dev(torch, a) for a in (u, v, w, s)]
        dq = tuple(_dev(torch, a) for a in q)
        items.append({"u": d[0], "v": d[1], "w": d[2], "src": d[3], "q": dq,
                      "phi": torch.empty_like(d[0])})
        out = plan.extend(*d, q=dq, phi=torch.empty_like(d[0]))
        singles.append([t.cpu().numpy() for t in out])
    res = plan.extend_batched(items)
    # phi left in the workspace slots (no caller buffer)
    res2 = plan.extend_batched([{k2: it[k2] for k2 in ("u", "v", "w", "src")} for it in items])
    torch.cuda.synchronize()
    for k in range(n):
        got = [t.cpu().numpy() for t in res[k]]
        for a, b in zip(got, singles[k]):
            assert np.array_equal(a, b), k
        for a, b in zip(res2[k][:3], singles[k][:3]):
            assert np.array_equal(a.cpu().numpy(), b), k
        ref = oracle.extend(items[k]["u"].cpu().numpy(), items[k]["v"].cpu().numpy(),
                            items[k]["w"].cpu().numpy(), items[k]["src"].cpu().numpy(), g)
        assert rel_l2(got[0], ref[0]) <= FP64_TOL


def test_footprint_matches_allocation(torch_dev):
    from paper_1907_00890_amd import footprint
    for prec, b in (("fp64", 1), ("fp64", 5), ("mixed", 3)):
        g = _grid(32, 16, 12, "PNN")
        plan = _plan(g, precision=prec, max_batch=b)
        assert plan.device_bytes() == footprint(32, 16, 12, prec, b)


# ----------------------------------------------------------------------------
# full benchmark sizes: properties computed with plain torch on the device
# ----------------------------------------------------------------------------
def torch_laplacian(torch, p, g):
    """L_h p with torch.roll / slicing (independent of the library)."""
    dzf = torch.as_tensor(g.dzf, device=p.device)
    dzc = torch.as_tensor(np.nan_to_num(g.dzc, nan=1.0), device=p.device)

    def fdiff(a, axis, h, letter):
        if letter == "P":
            return (torch.roll(a, -1, dims=axis) - a) / h
        out = torch.zeros_like(a)
        n = a.shape[axis]
        lo = a.narrow(axis, 0, n - 1)
        hi = a.narrow(axis, 1, n - 1)
        hh = h if not torch.is_tensor(h) else h.narrow(axis, 0, n - 1)
        out.narrow(axis, 0, n - 1).copy_((hi - lo) / hh)
        return out

    def bdiv(a, axis, h, letter):
        if letter == "P":
            return (a - torch.roll(a, 1, dims=axis)) / h
        prev = torch.zeros_like(a)
        n = a.shape[axis]
        prev.narrow(axis, 1, n - 1).copy_(a.narrow(axis, 0, n - 1))
        return (a - prev) / h

    gx = fdiff(p, 2, g.dx, g.bc[0])
    gy = fdiff(p, 1, g.dy, g.bc[1])
    gz = fdiff(p, 0, dzc[:, None, None], g.bc[2])
    return (bdiv(gx, 2, g.dx, g.bc[0]) + bdiv(gy, 1, g.dy, g.bc[1])
            + bdiv(gz, 0, dzf[:, None, None], g.bc[2]))


@pytest.mark.parametrize("name", ["ppn256", "ppn512s"])
def test_full_size_residual(torch_dev, name):
    torch = torch_dev
    cfg = vofsynth.config(name)
    g = oracle.Grid.from_config(cfg)
    f = vofsynth.remove_weighted_mean(vofsynth.gaussian_field(g.shape, 200), g.dzf)
    plan = _plan(g)
    fd = _dev(torch, f)
    p = plan.solve(fd)
    r = torch_laplacian(torch, p, g) - fd
    rel = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(fd)).item()
    dv = torch.as_tensor(g.dzf, device=p.device)[:, None, None]
    gauge = (p * dv).sum().abs().item() / (p.abs() * dv).sum().item()
    print(f"{name}: residual {rel:.3e} gauge {gauge:.3e}")
    assert rel <= 1e-10 and gauge <= 1e-12


def test_full_size_mixed_512(torch_dev):
    """512^3 triply periodic, seeded N(0,1) RHS (mean removed): the FP64 solve
    satisfies the discrete equation, and the mixed solve (FP32 chain, FP64
    defect correction with the device-side stopping rule) is within 1e-10 of it."""
    torch = torch_dev
    cfg = vofsynth.config("ppp512")
    g = oracle.Grid.from_config(cfg)
    f = vofsynth.remove_weighted_mean(vofsynth.gaussian_field(g.shape, 4), g.dzf)
    fd = _dev(torch, f)
    del f
    p64 = _plan(g).solve(fd)
    r = torch_laplacian(torch, p64, g) - fd
    rel = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(fd)).item()
    del r
    mixed = _plan(g, precision="mixed")
    pm = mixed.solve(fd)
    (steps, est), = mixed.mixed_report()
    err = (torch.linalg.vector_norm(pm - p64) / torch.linalg.vector_norm(p64)).item()
    print(f"ppp512: residual {rel:.3e}; mixed {steps} steps, estimate {est:.2e}, vs FP64 {err:.3e}")
    assert rel <= 1e-10
    assert err <= MIXED_TOL and 1 <= steps <= 3


def _step_inputs(g, seed=2):
    us, vs, ws, phat, rho, rho0, s, dt = _project_inputs(g, seed)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=seed)
    q = vofsynth.interface_normal_faces(C, g.dx, g.dy, g.dzf, g.bc, 1e-5)
    return us, vs, ws, phat, rho, rho0, s, dt, q


@pytest.mark.parametrize("shape,bc,beta", [((128, 128, 128), "PPN", None),
                                           ((64, 32, 48), "NPN", 1.5),
                                           ((32, 32, 32), "PPP", None)])
def test_fused_step_parity(torch_dev, shape, bc, beta):
    """vof_step == oracle project followed by oracle extend of the projected u."""
    torch = torch_dev
    g = _grid(*shape, bc, beta)
    us, vs, ws, phat, rho, rho0, s, dt, q = _step_inputs(g)
    u1, v1, w1, p1 = oracle.project(us, vs, ws, phat, rho, rho0, s, dt, g)
    ref = oracle.extend(u1, v1, w1, s, g, q=q)
    plan = _plan(g)
    T = lambda a: _dev(torch, a)  # noqa: E731
    out = plan.step(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt, T(s),
                    q=tuple(T(a) for a in q), out=tuple(T(np.zeros(g.shape)) for _ in range(3)))
    torch.cuda.synchronize()
    u, v, w, p, phi, ue, ve, we, ug, vg, wg = (a.cpu().numpy() for a in out)
    for name, a, b in [("u", u, u1), ("v", v, v1), ("w", w, w1), ("p", p, p1), ("phi", phi, ref[6]),
                       ("ue", ue, ref[0]), ("ve", ve, ref[1]), ("we", we, ref[2]),
                       ("ug", ug, ref[3]), ("vg", vg, ref[4]), ("wg", wg, ref[5])]:
        err = rel_l2(a, b)
        print(f"step {shape} {bc} {name}: {err:.3e}")
        assert err <= FP64_TOL, (name, err)
    # u_1^e is divergence-free (the Stefan source of both solves is the same s)
    dmax = np.abs(oracle.div(ue, ve, we, g)).max()
    assert dmax <= 1e-10 * np.abs(oracle.div(us, vs, ws, g)).max()
    # the epilogue's launch shapes (plain or LDS-staged tiles, planes per block)
    # change no bit of any result
    for tiled, planes in ((0, 1), (0, 3), (8, 1), (8, 5), (16, 2)):
        plan.tune("epilogue_tiled", tiled)
        plan.tune("epilogue_planes", min(planes, g.nz))
        out3 = plan.step(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt, T(s),
                         q=tuple(T(a) for a in q),
                         out=tuple(T(np.zeros(g.shape)) for _ in range(3)))
        torch.cuda.synchronize()
        for a, b in zip(out3, (u, v, w, p, phi, ue, ve, we, ug, vg, wg)):
            assert np.array_equal(a.cpu().numpy(), b), (tiled, planes)
    # project and extend alone: the correction and extension kernels on plain
    # or LDS-staged tiles, several planes per block, give the same bits, and
    # the oracle's projection and extension
    sep = {}
    for tiled, planes in ((0, 1), (8, 1), (8, 3), (16, 2), (0, 4)):
        plan.tune("stream_tiled", tiled)
        plan.tune("stream_planes", min(planes, g.nz))
        pu, pv, pw, pp_ = plan.project(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt)
        ext = plan.extend(pu, pv, pw, T(s), q=tuple(T(a) for a in q), phi=torch.empty_like(pu))
        torch.cuda.synchronize()
        sep[(tiled, planes)] = [a.cpu().numpy() for a in (pu, pv, pw, pp_, *ext)]
    base = sep[(0, 1)]
    for key, val in sep.items():
        for a, b in zip(val, base):
            assert np.array_equal(a, b), key
    for name, a, b in [("u", base[0], u1), ("w", base[2], w1), ("ue", base[4], ref[0]),
                       ("we", base[6], ref[2]), ("ug", base[7], ref[3]), ("wg", base[9], ref[5]),
                       ("phi", base[10], ref[6])]:
        assert rel_l2(a, b) <= FP64_TOL, ("separate", name)


def test_fused_step_graph_replay(torch_dev):
    """The step captured in a HIP graph, replayed three times with eager work and
    synchronisations in between; every replay equals the eager result."""
    torch = torch_dev
    g = _grid(64, 64, 48, "PPN", 1.5)
    us, vs, ws, phat, rho, rho0, s, dt, q = _step_inputs(g)
    T = lambda a: _dev(torch, a)  # noqa: E731
    plan = _plan(g)
    U0 = [T(us), T(vs), T(ws)]
    U = [a.clone() for a in U0]
    PH, RHO, S = T(phat), T(rho), T(s)
    Q = tuple(T(a) for a in q)
    P, PHI = T(np.zeros(g.shape)), T(np.zeros(g.shape))
    UG = tuple(T(np.zeros(g.shape)) for _ in range(3))
    stream = torch.cuda.Stream()

    def run():
        plan.step(U[0], U[1], U[2], PH, RHO, rho0, S, dt, S, p=P, phi=PHI, q=Q, gamma=UG,
                  stream=torch.cuda.current_stream())

    with torch.cuda.stream(stream):
        run()  # warm-up outside capture (one-time kernel attributes)
    torch.cuda.synchronize()
    eager = [a.clone() for a in (*U, P, PHI, *UG)]
    graph = torch.cuda.CUDAGraph()
    for a, b in zip(U, U0):
        a.copy_(b)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        run()
    for rep in range(3):
        for a, b in zip(U, U0):
            a.copy_(b)
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (*U, P, PHI, *UG)
        for a, b in zip(got, eager):
            assert torch.equal(a, b), f"replay {rep} differs"
        assert torch.isfinite(junk)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fused_step_batches_its_two_solves(torch_dev, prec):
    """A plan with room for two fields runs the step's pressure and Stefan
    solves as one batch: every output equals the one-field plan's, bit for bit."""
    torch = torch_dev
    g = _grid(64, 32, 24, "PPN", 1.3)
    us, vs, ws, phat, rho, rho0, s, dt, q = _step_inputs(g)
    T = lambda a: _dev(torch, a)  # noqa: E731
    outs = []
    for mb in (1, 2):
        plan = _plan(g, precision=prec, max_batch=mb)
        o = plan.step(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt, T(s),
                      q=tuple(T(a) for a in q), out=tuple(T(np.zeros(g.shape)) for _ in range(3)))
        torch.cuda.synchronize()
        outs.append([a.cpu().numpy() for a in o])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("case", [(32, 32, 256, "PPN", None), (16, 16, 300, "NNP", 1.5),
                                  (16, 8, 512, "PPN", 1.3), (8, 8, 40, "NNNNND", None),
                                  (16, 16, 256, "PPP", 1.5)],
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_z_segment_lengths(torch_dev, case):
    """Segments of 8 or 16 rows and 8, 16 or 32 lines per block in the
    partitioned z solve (tuning knobs): every shape matches the oracle.  With
    8-row segments and 32 lines a 256-long line takes a 1024-lane block; on a
    periodic z line that block keeps one LDS buffer for the reduced system."""
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 91 + nz)
    ref = oracle.solve(f, g)
    plan = _plan(g)
    plan.tune("z_spectral", 0) if plan.tuning()["z_spectral"] else None
    for seg in (8, 16):
        for lines in (8, 16, 32):
            plan.tune("z_segment", seg)
            plan.tune("z_lines", lines)
            assert plan.tuning()["z_segment"] == seg
            p = plan.solve(_dev(torch, f)).cpu().numpy()
            err = rel_l2(p, ref)
            print(f"z segments {case} seg {seg} lines {lines}: {err:.3e}", flush=True)
            assert err <= FP64_TOL, (seg, lines)
