"""poisson_solve_noalloc (through the C ABI): the FP64 solve with its spectrum
in the library's static device array gives poisson_solve's result bit for
bit, on consecutive calls whose second input is smaller than the first (the
array keeps the last call's contents), in place, and at the size limit; it
refuses mixed plans and grids above the limit."""
import numpy as np
import pytest

import oracle
import vofsynth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1907_00890_amd  # noqa: F401  (fails loudly without the library)
    return torch


def _grid(nx, ny, nz, bc, beta=None):
    dzf = vofsynth.uniform_dz(nz) if beta is None else vofsynth.stretched_dz(nz, 1.0, beta)
    return oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, bc)


def _plan(g, precision="fp64"):
    from paper_1907_00890_amd import Plan
    return Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc, precision=precision)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_noalloc_equals_solve_on_consecutive_calls(torch_dev):
    torch = torch_dev
    # a larger grid, then a smaller one with other ends, then the larger again
    cases = [(_grid(128, 64, 48, "PPN", 1.5), 11), (_grid(32, 16, 12, "NNP"), 12),
             (_grid(64, 32, 40, "NNPPND"), 13), (_grid(128, 64, 48, "PPN", 1.5), 14)]
    for g, seed in cases:
        f = vofsynth.gaussian_field(g.shape, seed)
        plan = _plan(g)
        fd = _dev(torch, f)
        ref = plan.solve(fd)
        got = plan.solve_noalloc(fd)
        torch.cuda.synchronize()
        print(f"noalloc {g.nx}x{g.ny}x{g.nz} {g.bc}", flush=True)
        assert torch.equal(got, ref)
        # in place, through the same static slot
        t = fd.clone()
        plan.solve_noalloc(t, out=t)
        assert torch.equal(t, ref)
        err = np.linalg.norm(got.cpu().numpy() - oracle.solve(f, g)) / np.linalg.norm(
            ref.cpu().numpy())
        assert err <= 1e-12
        plan.close()


def test_noalloc_at_the_size_limit(torch_dev):
    from paper_1907_00890_amd import _lib
    torch = torch_dev
    g = _grid(256, 256, 128, "PPN")
    assert g.nx * g.ny * g.nz == _lib.NOALLOC_MAX_POINTS
    f = vofsynth.gaussian_field(g.shape, 21)
    plan = _plan(g)
    fd = _dev(torch, f)
    ref = plan.solve(fd)
    got = plan.solve_noalloc(fd)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    plan.close()
    # a smaller call after the largest one
    g2 = _grid(16, 8, 8, "PPP")
    f2 = vofsynth.gaussian_field(g2.shape, 22)
    p2 = _plan(g2)
    d2 = _dev(torch, f2)
    assert torch.equal(p2.solve_noalloc(d2), p2.solve(d2))
    p2.close()


def test_noalloc_refuses_what_it_cannot_hold(torch_dev):
    from paper_1907_00890_amd import VofPoissonError, _lib
    torch = torch_dev
    g = _grid(256, 256, 160, "PPN")  # 10.5 M points, above the limit
    plan = _plan(g)
    fd = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(VofPoissonError) as e:
        plan.solve_noalloc(fd)
    assert e.value.status == _lib.VP_EUNSUPPORTED
    plan.close()
    g = _grid(16, 16, 16, "PPP")
    mixed = _plan(g, precision="mixed")
    fd = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(VofPoissonError) as e:
        mixed.solve_noalloc(fd)
    assert e.value.status == _lib.VP_EUNSUPPORTED
    mixed.close()
