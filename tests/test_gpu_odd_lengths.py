"""GPU parity for transform lengths with an odd factor, 5 * 2^k (40 .. 640;
the 320 x 320 x 640 grid of the paper's three-dimensional droplet case) and
3 * 2^k (24 .. 768): a radix-5 or radix-3 Stockham pass, then radix 4 and 2,
in every transform (real DFT, cosine, sine and quarter-wave; x, y and the
spectral z pass), tile widths that divide such lengths in the stencils, and
the interface terms, against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import oracle.interface as oi
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
    (40, 40, 40, "PPP", None),       # spectral z of length 40
    (320, 16, 9, "PPN", None),       # x real DFT, 16 threads per line
    (16, 320, 7, "NNN", 1.3),        # y cosine transform
    (80, 160, 12, "DDN", 1.5),       # sine transforms
    (640, 8, 3, "PNN", None),        # longest x
    (8, 640, 3, "NPP", None),        # longest y
    (40, 8, 320, "PPN", None),       # spectral z cosine, 320
    (8, 8, 640, "PPP", None),        # spectral z real DFT, 640
    (160, 40, 10, "NDNNND", None),   # quarter-wave x (half length 80), y walls
    (40, 80, 20, "DNPPND", 1.2),     # quarter-wave x (half length 20)
    (320, 320, 4, "PPP", None),      # the droplet grid's x-y plane
    # 3 * 2^k: 12 values per thread, a radix-3 pass first
    (48, 48, 48, "PPP", None),       # spectral z of length 48
    (384, 16, 9, "PPN", None),       # x real DFT, 32 threads per line
    (16, 384, 7, "NNN", 1.3),        # y cosine transform
    (96, 192, 12, "DDN", 1.5),       # sine transforms
    (768, 8, 3, "PNN", None),        # longest x
    (8, 768, 3, "NPP", None),        # longest y
    (24, 8, 384, "PPN", None),       # spectral z cosine, 384
    (8, 8, 768, "PPP", None),        # spectral z real DFT, 768
    (24, 24, 24, "DDD", None),       # spectral z sine, shortest length
    (192, 24, 10, "NDNNND", None),   # quarter-wave x (half length 96)
    (24, 48, 20, "DNPPND", 1.2),     # quarter-wave x (half length 12)
    (16, 96, 8, "PPNDNN", None),     # quarter-wave y (half length 48)
    (384, 384, 4, "PPP", None),
    (40, 48, 24, "NNPPNN", None),    # radix 5 in x, radix 3 in y and spectral z
]


@pytest.mark.parametrize("case", SOLVE_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_solve_parity(torch_dev, case):
    torch = torch_dev
    nx, ny, nz, bc, beta = case
    g = _grid(nx, ny, nz, bc, beta)
    f = vofsynth.gaussian_field(g.shape, 500 + nx + ny + nz)
    ref = oracle.solve(f, g)
    plan = _plan(g)
    p = plan.solve(_dev(torch, f))
    torch.cuda.synchronize()
    err = rel_l2(p.cpu().numpy(), ref)
    print(f"odd-length solve {case}: rel L2 {err:.3e}")
    assert err <= FP64_TOL, err
    if plan.tuning()["z_spectral"]:
        plan.tune("z_spectral", 0)
        q = plan.solve(_dev(torch, f)).cpu().numpy()
        assert rel_l2(q, ref) <= FP64_TOL
    # the radix knob does not apply to these lengths: same bits
    plan2 = _plan(g)
    plan2.tune("x_radix", 8)
    plan2.tune("y_radix", 8)
    if plan.tuning()["z_spectral"]:
        plan2.tune("z_spectral", 0)
    r = plan2.solve(_dev(torch, f)).cpu().numpy()
    assert rel_l2(r, ref) <= FP64_TOL


@pytest.mark.parametrize("shape", [(80, 40, 40), (96, 48, 24)])
def test_mixed_and_batched(torch_dev, shape):
    torch = torch_dev
    g = _grid(*shape, "PPN", None)
    fs = [vofsynth.gaussian_field(g.shape, 70 + i) for i in range(3)]
    plan = _plan(g, precision="mixed", max_batch=3)
    singles = [plan.solve(_dev(torch, f)).cpu().numpy() for f in fs]
    outs = plan.solve_batched([_dev(torch, f) for f in fs])
    torch.cuda.synchronize()
    for a, b, f in zip(outs, singles, fs):
        assert np.array_equal(a.cpu().numpy(), b)
        assert rel_l2(b, oracle.solve(f, g)) <= MIXED_TOL


@pytest.mark.parametrize("shape,bc", [((320, 40, 16), "PPN"), ((40, 80, 12), "NPN"),
                                      ((160, 32, 8), "NNNNND"), ((384, 24, 16), "PPN"),
                                      ((48, 96, 12), "NNNNND")])
def test_step_parity(torch_dev, shape, bc):
    """Projection + extension with tile widths dividing 5 * 2^k and 3 * 2^k
    rows (LDS-staged and plain stencils), and the interface terms."""
    torch = torch_dev
    g = _grid(*shape, bc, 1.3)
    us, vs, ws = vofsynth.random_faces(g.shape, 1, g.bc)
    phat = vofsynth.gaussian_field(g.shape, 2)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, seed=3)
    rho1, rho2 = 1000.0, 1.0
    rho = rho1 * C + rho2 * (1 - C)
    mdot = 0.01 * np.random.default_rng(4).uniform(0.5, 1.5, g.shape)
    s, qx, qy, qz, _ = oi.interface_terms(C, mdot, rho1, rho2, g)
    u1, v1, w1, p1 = oracle.project(us, vs, ws, phat, rho, rho2, s, 0.3, g)
    ref = oracle.extend(u1, v1, w1, s, g, q=(qx, qy, qz))
    plan = _plan(g)
    T = lambda a: _dev(torch, a)  # noqa: E731
    terms = plan.interface_terms(T(C), T(mdot), rho1, rho2)
    torch.cuda.synchronize()
    for a, b in zip(terms, (s, qx, qy, qz)):
        if np.any(b):
            assert rel_l2(a.cpu().numpy(), b) <= FP64_TOL
    got = {}
    for tiled in (0, 8):
        plan.tune("rhs_tiled", tiled)
        plan.tune("epilogue_tiled", tiled)
        out = plan.step(T(us), T(vs), T(ws), T(phat), T(rho), rho2, terms[0], 0.3, terms[0],
                        q=terms[1:], out=tuple(T(np.zeros(g.shape)) for _ in range(3)))
        torch.cuda.synchronize()
        got[tiled] = [a.cpu().numpy() for a in out]
    u, v, w, p, phi, ue, ve, we, ug, vg, wg = got[0]
    for name, a, b in [("u", u, u1), ("v", v, v1), ("w", w, w1), ("p", p, p1), ("phi", phi, ref[6]),
                       ("ue", ue, ref[0]), ("ug", ug, ref[3]), ("wg", wg, ref[5])]:
        err = rel_l2(a, b)
        print(f"odd-length step {shape} {bc} {name}: {err:.3e}")
        assert err <= FP64_TOL, (name, err)
    for a, b in zip(got[0], got[8]):
        assert np.array_equal(a, b)
