"""GPU parity of the interface terms (Youngs gradient of C, the Stefan source
s and the interface-velocity jump q on faces) through the C ABI against the
FP64 oracle, on every tile width (nx = 8 .. 1024), periodic / wall / outflow
ends, stretched z and nz = 1; the planes marched per block change no bit."""
import numpy as np
import pytest

import oracle
import oracle.interface as oi
import vofsynth

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1907_00890_amd  # noqa: F401  (fails loudly without the library)
    return torch


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [
    # (nx, ny, nz, bc, beta, field)
    (64, 64, 64, "PPN", None, "sphere"),
    (32, 16, 24, "NPN", 1.5, "sphere"),
    (16, 16, 16, "PPP", None, "random"),
    (8, 32, 12, "NNNNND", 1.2, "random"),
    (8, 8, 10, "PPP", None, "random"),      # tall tile wider than the grid in y
    (128, 32, 5, "DDN", None, "random"),
    (32, 32, 1, "PPN", None, "random"),     # one-cell slab
    (1024, 8, 3, "PNN", None, "random"),
    (256, 16, 40, "NNP", 1.0, "sphere"),
]


def _inputs(g, field, seed):
    rng = np.random.default_rng(seed)
    if field == "sphere":
        C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=seed)
    else:
        C = rng.uniform(0.0, 1.0, g.shape)
    mdot = 0.01 * rng.uniform(0.5, 1.5, g.shape)
    return C, mdot


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}-{c[5]}")
def test_interface_terms_parity(torch_dev, case):
    torch = torch_dev
    from paper_1907_00890_amd import Plan
    nx, ny, nz, bc, beta, field = case
    dzf = vofsynth.uniform_dz(nz, 1.0) if beta is None else vofsynth.stretched_dz(nz, 1.0, beta)
    g = oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, bc)
    C, mdot = _inputs(g, field, 7 + nz)
    rho1, rho2 = 1000.0, 1.0
    ref = oi.interface_terms(C, mdot, rho1, rho2, g)[:4]
    plan = Plan(nx, ny, nz, g.dx, g.dy, dzf, g.bc)
    dC, dm = _dev(torch, C), _dev(torch, mdot)
    out = plan.interface_terms(dC, dm, rho1, rho2)
    torch.cuda.synchronize()
    got = [a.cpu().numpy() for a in out]
    for name, a, b in zip(("s", "qx", "qy", "qz"), got, ref):
        if not np.any(b):
            assert not np.any(a), name  # e.g. qz of a one-cell slab
            continue
        err = rel_l2(a, b)
        print(f"interface {case} {name}: {err:.3e}")
        assert err <= FP64_TOL, (name, err)
    # boiling: the vapour extension's jump (mdot/rho2) n, same source
    vap = plan.interface_terms(dC, dm, rho1, rho2, phase=2)
    torch.cuda.synchronize()
    ref2 = oi.interface_terms(C, mdot, rho1, rho2, g, phase=2)[:4]
    assert np.array_equal(vap[0].cpu().numpy(), got[0])
    for a, b in zip(vap[1:], ref2[1:]):
        if np.any(b):
            assert rel_l2(a.cpu().numpy(), b) <= FP64_TOL
    # planes marched per block and tile widths: same bits
    txp = nx & -nx
    for planes, tile in sorted({(1, 8), (3, 16), (nz, 32), (min(16, nz), 64)}):
        if tile > txp:
            with pytest.raises(Exception):
                plan.tune("interface_tile", tile)
            continue
        plan.tune("interface_planes", min(planes, nz))
        plan.tune("interface_tile", tile)
        again = plan.interface_terms(dC, dm, rho1, rho2)
        torch.cuda.synchronize()
        for a, b in zip(again, got):
            assert np.array_equal(a.cpu().numpy(), b), (planes, tile)


def test_interface_terms_feed_the_step(torch_dev):
    """s and q from the kernel, used by the fused step, give the oracle's step
    with the oracle's interface terms."""
    torch = torch_dev
    from paper_1907_00890_amd import Plan
    g = oracle.Grid(64, 32, 48, 1 / 64, 1 / 32, vofsynth.stretched_dz(48, 1.0, 1.5), "PPN")
    C, mdot = _inputs(g, "sphere", 3)
    rho1, rho2 = 1000.0, 1.0
    s_ref, qx, qy, qz, _ = oi.interface_terms(C, mdot, rho1, rho2, g)
    us, vs, ws = vofsynth.random_faces(g.shape, 4, g.bc)
    phat = vofsynth.gaussian_field(g.shape, 5)
    rho = rho1 * C + rho2 * (1 - C)
    dt = 0.2
    u1, v1, w1, p1 = oracle.project(us, vs, ws, phat, rho, rho2, s_ref, dt, g)
    ref = oracle.extend(u1, v1, w1, s_ref, g, q=(qx, qy, qz))
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc)
    T = lambda a: _dev(torch, a)  # noqa: E731
    s, dqx, dqy, dqz = plan.interface_terms(T(C), T(mdot), rho1, rho2)
    out = plan.step(T(us), T(vs), T(ws), T(phat), T(rho), rho2, s, dt, s, q=(dqx, dqy, dqz),
                    out=tuple(T(np.zeros(g.shape)) for _ in range(3)))
    torch.cuda.synchronize()
    u, v, w, p, phi, ue, ve, we, ug, vg, wg = (a.cpu().numpy() for a in out)
    for name, a, b in [("u", u, u1), ("p", p, p1), ("phi", phi, ref[6]), ("we", we, ref[2]),
                       ("ug", ug, ref[3]), ("wg", wg, ref[5])]:
        assert rel_l2(a, b) <= FP64_TOL, name


STEP_IF_CASES = [
    # (nx, ny, nz, bc, beta, max_batch, precision)
    (64, 32, 48, "PPN", 1.5, 2, "fp64"),
    (32, 32, 24, "NNNNND", None, 2, "fp64"),   # the container: outflow top
    (8, 40, 12, "PNN", None, 1, "fp64"),       # tall tiles beyond ny, one field per solve
    (64, 16, 20, "NPP", 1.2, 2, "mixed"),
    (32, 16, 1, "PPN", None, 2, "fp64"),       # one-cell slab
]


@pytest.mark.parametrize("case", STEP_IF_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}-{c[6]}")
def test_step_interface_same_bits(torch_dev, case):
    """vof_step_interface (s in the right-hand-side pass, q in the epilogue)
    gives the bits of interface_terms followed by vof_step, and the oracle's
    step with the oracle's interface terms."""
    torch = torch_dev
    from paper_1907_00890_amd import Plan
    nx, ny, nz, bc, beta, mb, prec = case
    dzf = vofsynth.uniform_dz(nz, 1.0) if beta is None else vofsynth.stretched_dz(nz, 1.0, beta)
    g = oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, bc)
    C, mdot = _inputs(g, "sphere", 11 + nz)
    rho1, rho2 = 1000.0, 1.0
    us, vs, ws = vofsynth.random_faces(g.shape, 12, g.bc)
    phat = vofsynth.gaussian_field(g.shape, 13)
    rho = rho1 * C + rho2 * (1 - C)
    dt = 0.2
    plan = Plan(nx, ny, nz, g.dx, g.dy, dzf, g.bc, precision=prec, max_batch=mb)
    T = lambda a: _dev(torch, a)  # noqa: E731
    dC, dm = T(C), T(mdot)
    for phase in (1, 2):
        s, qx, qy, qz = plan.interface_terms(dC, dm, rho1, rho2, phase=phase)
        ref = plan.step(T(us), T(vs), T(ws), T(phat), T(rho), rho2, s, dt, s, q=(qx, qy, qz),
                        out=tuple(T(np.zeros(g.shape)) for _ in range(3)))
        got = plan.step_interface(T(us), T(vs), T(ws), T(phat), T(rho), rho2, dC, dm, rho1, rho2,
                                  dt, phase=phase,
                                  out=tuple(T(np.zeros(g.shape)) for _ in range(3)))
        torch.cuda.synchronize()
        names = ("u", "v", "w", "p", "phi", "ue", "ve", "we", "ug", "vg", "wg")
        want = dict(zip(names, (a.cpu().numpy() for a in ref)))
        have = dict(zip(names[:5], (a.cpu().numpy() for a in got[:5])))
        have.update(zip(names[5:], (a.cpu().numpy() for a in got[6:])))
        assert np.array_equal(got[5].cpu().numpy(), s.cpu().numpy()), (phase, "s")
        for name in names:
            assert np.array_equal(have[name], want[name]), (phase, name)
    # and the oracle's step with the oracle's terms (liquid phase)
    if prec == "fp64":
        s_ref, rqx, rqy, rqz, _ = oi.interface_terms(C, mdot, rho1, rho2, g)
        u1, v1, w1, p1 = oracle.project(us, vs, ws, phat, rho, rho2, s_ref, dt, g)
        ext = oracle.extend(u1, v1, w1, s_ref, g, q=(rqx, rqy, rqz))
        got = plan.step_interface(T(us), T(vs), T(ws), T(phat), T(rho), rho2, dC, dm, rho1, rho2,
                                  dt)
        torch.cuda.synchronize()
        for name, a, b in [("u", got[0], u1), ("p", got[3], p1), ("phi", got[4], ext[6]),
                           ("s", got[5], s_ref), ("ug", got[9], ext[3]), ("wg", got[11], ext[5])]:
            if not np.any(b):
                assert not np.any(a.cpu().numpy()), name
                continue
            err = rel_l2(a.cpu().numpy(), b)
            print(f"step_interface {case} {name}: {err:.3e}")
            assert err <= FP64_TOL, (name, err)
    plan.close()


def test_step_interface_refusals(torch_dev):
    torch = torch_dev
    from paper_1907_00890_amd import Plan, VofPoissonError, _lib
    g = oracle.Grid(16, 16, 8, 1 / 16, 1 / 16, vofsynth.uniform_dz(8, 1.0), "DNPPNN")
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc)
    z = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(VofPoissonError) as e:  # outflow at a lower end: the _lf calls
        plan.step_interface(z.clone(), z.clone(), z.clone(), z, z + 1, 1.0, z, z, 2.0, 1.0, 0.1)
    assert e.value.status == _lib.VP_EUNSUPPORTED
    g = oracle.Grid(16, 16, 8, 1 / 16, 1 / 16, vofsynth.uniform_dz(8, 1.0), "PPN")
    plan = Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc)
    with pytest.raises(VofPoissonError):
        plan.step_interface(z.clone(), z.clone(), z.clone(), z, z + 1, 1.0, z, z, 2.0, 1.0, 0.1,
                            phase=3)
