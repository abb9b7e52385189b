"""GPU parity of the face stencils with outflow at lower ends (project_lf,
extend_liquid_velocity_lf, vof_step_lf, vof_advect with lower planes)
against the FP64 oracle, element by element, including the velocities on the
faces at -1/2, which travel as planes.  The boxes include the zero-pressure
outflow on every side of the cases of section 4 ('DDD').

Tolerance: FP64 relative L2 <= 1e-12 (the advection: <= 1e-12 too).
"""
import numpy as np
import pytest

import oracle
from oracle import advection as adv
import vofsynth

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1907_00890_amd  # noqa: F401  (fails loudly without the library)
    return torch


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def _dev(torch, a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _grid(nx, ny, nz, bc, beta=None):
    dzf = vofsynth.uniform_dz(nz) if beta is None else vofsynth.stretched_dz(nz, 1.0, beta)
    return oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, bc)


def _plan(g, max_batch=1):
    from paper_1907_00890_amd import Plan
    return Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc, max_batch=max_batch)


def _lower_planes(g, seed):
    r = np.random.default_rng(seed)
    shapes = ((g.nz, g.ny), (g.nz, g.nx), (g.ny, g.nx))
    return tuple(r.standard_normal(shp) if lo == "D" else None
                 for (lo, _), shp in zip(g.ends, shapes))


def _inputs(g, seed=2):
    us, vs, ws = vofsynth.random_faces(g.shape, seed + 1, g.bc)
    phat = vofsynth.gaussian_field(g.shape, seed + 20)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=seed)
    rho = 1000.0 * C + 1.0 * (1 - C)
    mag, _ = vofsynth.grad_mag_central(C, g.dx, g.dy, g.dzf, g.bc)
    q = vofsynth.interface_normal_faces(C, g.dx, g.dy, g.dzf, g.bc, 1e-5)
    return us, vs, ws, phat, rho, 1.0, 1e-2 * mag, 0.3, q


CASES = [
    # (nx, ny, nz, bc, z stretching): 64-wide x takes the LDS-tiled stencils
    (64, 32, 24, "DDD", 1.3),
    (24, 40, 20, "DDD", None),
    (64, 16, 12, "DNDNDN", None),
    (32, 64, 16, "DDPPND", 1.5),
    (40, 24, 12, "NNDNPP", None),
    (64, 8, 1, "DDDDNN", None),  # a slab: outflow on the four sides
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_project_lf_parity(torch_dev, case):
    torch = torch_dev
    nx, ny, nz, bc, zb = case
    g = _grid(nx, ny, nz, bc, zb)
    us, vs, ws, phat, rho, rho0, s, dt, _ = _inputs(g)
    lower = _lower_planes(g, 5)
    u, v, w, p, low = oracle.project(us, vs, ws, phat, rho, rho0, s, dt, g, lower=lower)
    plan = _plan(g)
    dl = tuple(_dev(torch, a) for a in lower)
    out = plan.project(_dev(torch, us), _dev(torch, vs), _dev(torch, ws), _dev(torch, phat),
                       _dev(torch, rho), rho0, _dev(torch, s), dt, lower=dl)
    torch.cuda.synchronize()
    for name, a, b in zip("uvwp", out, (u, v, w, p)):
        err = rel_l2(a.cpu().numpy(), b)
        print(f"project_lf {case} {name}: {err:.3e}", flush=True)
        assert err <= TOL, (name, err)
    for d, (a, b) in enumerate(zip(dl, low)):
        if b is not None:
            err = rel_l2(a.cpu().numpy(), b)
            print(f"project_lf {case} lower {'xyz'[d]}: {err:.3e}", flush=True)
            assert err <= TOL, (d, err)
    # the device result is exactly divergence-free up to the source
    gl = tuple(None if a is None else a.cpu().numpy() for a in dl)
    dv = oracle.div(*(t.cpu().numpy() for t in out[:3]), g, gl)
    scale = np.abs(oracle.div(us, vs, ws, g, lower)).max()
    assert np.abs(dv - s).max() <= 1e-11 * scale
    plan.close()


@pytest.mark.parametrize("case", CASES[:4], ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_extend_lf_parity(torch_dev, case):
    torch = torch_dev
    nx, ny, nz, bc, zb = case
    g = _grid(nx, ny, nz, bc, zb)
    u = vofsynth.random_faces(g.shape, 31, g.bc)
    lower = _lower_planes(g, 32)
    s = vofsynth.gaussian_field(g.shape, 33)
    q = vofsynth.random_faces(g.shape, 34, g.bc)
    ref = oracle.extend(*u, s, g, q=q, lower=lower)
    plan = _plan(g)
    dl = tuple(_dev(torch, a) for a in lower)
    dle = tuple(None if a is None else torch.empty_like(a) for a in dl)
    out = plan.extend(*(_dev(torch, a) for a in u), _dev(torch, s),
                      q=tuple(_dev(torch, a) for a in q), phi=_dev(torch, np.zeros(g.shape)),
                      lower=dl, lower_out=dle)
    torch.cuda.synchronize()
    for name, a, b in zip(("ue", "ve", "we", "ug", "vg", "wg", "phi"), out, ref[:7]):
        err = rel_l2(a.cpu().numpy(), b)
        assert err <= TOL, (name, err)
    for d, (a, b) in enumerate(zip(dle, ref[7])):
        if b is not None:
            err = rel_l2(a.cpu().numpy(), b)
            print(f"extend_lf {case} lower {'xyz'[d]}: {err:.3e}", flush=True)
            assert err <= TOL, (d, err)
    plan.close()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
@pytest.mark.parametrize("mb", [1, 2])
def test_step_lf_parity(torch_dev, case, mb):
    """vof_step_lf == oracle projection followed by the oracle's extension of
    the projected velocity (lower faces carried through both)."""
    torch = torch_dev
    nx, ny, nz, bc, zb = case
    g = _grid(nx, ny, nz, bc, zb)
    us, vs, ws, phat, rho, rho0, s, dt, q = _inputs(g)
    lower = _lower_planes(g, 6)
    u1, v1, w1, p1, low1 = oracle.project(us, vs, ws, phat, rho, rho0, s, dt, g, lower=lower)
    ref = oracle.extend(u1, v1, w1, s, g, q=q, lower=low1)
    plan = _plan(g, max_batch=mb)
    T = lambda a: _dev(torch, a)  # noqa: E731
    dl = tuple(T(a) for a in lower)
    dle = tuple(None if a is None else torch.empty_like(a) for a in dl)
    out = plan.step(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt, T(s),
                    q=tuple(T(a) for a in q), out=tuple(T(np.zeros(g.shape)) for _ in range(3)),
                    lower=dl, lower_e=dle)
    torch.cuda.synchronize()
    names = ("u", "v", "w", "p", "phi", "ue", "ve", "we", "ug", "vg", "wg")
    want = (u1, v1, w1, p1, ref[6], ref[0], ref[1], ref[2], ref[3], ref[4], ref[5])
    for name, a, b in zip(names, out, want):
        err = rel_l2(a.cpu().numpy(), b)
        assert err <= TOL, (name, err)
    for d in range(3):
        if lower[d] is not None:
            assert rel_l2(dl[d].cpu().numpy(), low1[d]) <= TOL, ("lower", d)
            assert rel_l2(dle[d].cpu().numpy(), ref[7][d]) <= TOL, ("lower_e", d)
    plan.close()


@pytest.mark.parametrize("case", [(32, 32, 24, "DDD", None), (64, 24, 16, "DNDNDN", 1.3)],
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_advect_lower_outflow(torch_dev, case):
    """The VoF advection with inflow and outflow through the lower outflow
    faces (their interface velocity from planes), against the oracle."""
    torch = torch_dev
    nx, ny, nz, bc, zb = case
    g = _grid(nx, ny, nz, bc, zb)
    C, _ = vofsynth.sphere_vof(nx, ny, nz, g.dx, g.dy, g.dzf, seed=8, radius=0.3)
    u, v, w = vofsynth.random_faces(g.shape, 9, g.bc)
    lower = _lower_planes(g, 10)
    h = min(g.dx, g.dy, float(g.dzf.min()))
    vmax = max(np.abs(a).max() for a in (u, v, w) + tuple(x for x in lower if x is not None))
    dt = 0.5 * h / vmax
    ref = adv.advect(C, u, v, w, dt, g, lower=lower)
    plan = _plan(g)
    got = plan.advect(*(_dev(torch, a) for a in (C, u, v, w)), dt,
                      lower=tuple(_dev(torch, a) for a in lower)).cpu().numpy()
    err = rel_l2(got, ref)
    print(f"advect lower {case}: {err:.3e}", flush=True)
    assert err <= TOL


def test_lower_faces_refusals(torch_dev):
    from paper_1907_00890_amd import VofPoissonError, _lib
    torch = torch_dev
    g = _grid(16, 16, 8, "DDD")
    plan = _plan(g)
    us, vs, ws, phat, rho, rho0, s, dt, q = _inputs(g)
    T = lambda a: _dev(torch, a)  # noqa: E731
    with pytest.raises(VofPoissonError) as e:
        plan.project(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt)
    assert e.value.status == _lib.VP_EUNSUPPORTED
    lower = tuple(T(a) for a in _lower_planes(g, 1))
    with pytest.raises(VofPoissonError) as e:  # a plane missing
        plan.project(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt,
                     lower=(lower[0], lower[1], None))
    assert e.value.status == _lib.VP_EINVAL
    g2 = _grid(16, 16, 8, "PPN")
    plan2 = _plan(g2)
    with pytest.raises(VofPoissonError) as e:  # a plane where there is no lower outflow
        plan2.project(T(us), T(vs), T(ws), T(phat), T(rho), rho0, T(s), dt,
                      lower=(lower[0], None, None))
    assert e.value.status == _lib.VP_EINVAL
