"""GPU parity at the benchmark's own sizes and launch shapes, element by element
against the FP64 oracle.

The benchmark times the 256^3 step (periodic x/y, walls in z, uniform) on a
plan whose launch shapes the autotuner picks, and a 512 x 512 x 256 step with
tanh-stretched z (beta = 1.5).  These tests run exactly those inputs
(``bench.make_inputs``, the same seeds) through the same entry points, with
the autotuner's choice and with every other launch shape it can pick (radix-8
and radix-16 x / y / spectral-z schedules, y and spectral-z tile widths, the
tridiagonal z pass with 8- and 16-row segments and 8 / 16 / 32 lines per
block), and compare every output with the oracle's:

* FP64 relative L2 <= 1e-12 (the target tolerance);
* mixed precision (FP32 chain + FP64 defect correction) <= 1e-10.

Periodic x and y lines of length 256 and 512 (the benchmark's x / y passes
and the 512^3 comparison) are covered at both radices on small slabs.
"""
import numpy as np
import pytest

import bench
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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _plan(g, precision="fp64", max_batch=1):
    from paper_1907_00890_amd import Plan
    return Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dzf, g.bc, precision=precision,
                max_batch=max_batch)


def _apply(plan, tuning):
    for k, v in tuning.items():
        plan.tune(k, v)
    got = plan.tuning()
    assert all(got[k] == v for k, v in tuning.items()), (tuning, got)


def _bench_rhs(g):
    """The benchmark's bare-solve right-hand side (seed 200, weighted mean removed)."""
    return vofsynth.remove_weighted_mean(vofsynth.gaussian_field(g.shape, 200), g.dzf)


# every launch shape of the 256^3 uniform solve: the autotuner's pick on MI355X
# for the step plan first (x radix 8, y radix 16, spectral z at radix 8 on
# 8-pair tiles), then the other radices and tile widths and the tridiagonal z
# pass it is timed against
UNIFORM_SHAPES = [
    dict(x_radix=8, y_radix=16, z_spectral=1, z_radix=8, y_lines=8, z_spectral_lines=8),
    dict(x_radix=16, y_radix=8, z_spectral=1, z_radix=16, y_lines=0, z_spectral_lines=0),
    dict(x_radix=8, y_radix=8, z_spectral=1, z_radix=8, y_lines=4, z_spectral_lines=4),
    dict(x_radix=16, y_radix=16, z_spectral=1, z_radix=16, y_lines=8, z_spectral_lines=8),
    dict(x_radix=16, y_radix=16, z_spectral=0, z_segment=16, z_lines=16),
    dict(x_radix=8, y_radix=8, z_spectral=0, z_segment=8, z_lines=32),
]
# stretched z: the tridiagonal pass at both segment lengths and every width
STRETCHED_SHAPES = [
    dict(z_segment=8, z_lines=8), dict(z_segment=8, z_lines=16), dict(z_segment=8, z_lines=32),
    dict(z_segment=16, z_lines=8), dict(z_segment=16, z_lines=16),
    dict(x_radix=8, y_radix=8, z_segment=16, z_lines=32),
]


@pytest.fixture(scope="module")
def ppn256():
    cfg = vofsynth.config("ppn256")
    g = oracle.Grid.from_config(cfg)
    f = _bench_rhs(g)
    return cfg, g, f, oracle.solve(f, g)


def test_ppn256_solve_every_benchmarked_shape(torch_dev, ppn256):
    """The 256^3 FP64 solve the headline metric is quoted on: the autotuned
    two-field plan of the benchmark, every launch shape, and the two-member
    batch the step runs (pressure and Stefan potential in one launch per pass)."""
    torch = torch_dev
    cfg, g, f, ref = ppn256
    plan = _plan(g, max_batch=bench.STEP_BATCH)
    chosen = plan.autotune(batch=bench.STEP_BATCH)
    fd = _dev(torch, f)
    out = torch.empty_like(fd)
    plan.solve(fd, out)
    err = rel_l2(out.cpu().numpy(), ref)
    print(f"ppn256 autotuned {chosen}: rel L2 {err:.3e}", flush=True)
    assert err <= FP64_TOL
    for shape in UNIFORM_SHAPES:
        _apply(plan, shape)
        plan.solve(fd, out)
        err = rel_l2(out.cpu().numpy(), ref)
        print(f"ppn256 {shape}: rel L2 {err:.3e}", flush=True)
        assert err <= FP64_TOL, shape
        # two members per launch, the second with another right-hand side
        f2 = -0.5 * f
        a, b = plan.solve_batched([fd, _dev(torch, f2)])
        assert np.array_equal(a.cpu().numpy(), out.cpu().numpy())
        assert rel_l2(b.cpu().numpy(), -0.5 * ref) <= FP64_TOL
    plan.close()


def test_ppn256_mixed_as_benchmarked(torch_dev, ppn256):
    """The benchmark's mixed solve at 256^3 (autotuned one-field plan, device
    stopping rule at its default tolerance) against the oracle."""
    torch = torch_dev
    cfg, g, f, ref = ppn256
    plan = _plan(g, precision="mixed")
    chosen = plan.autotune(batch=1)
    p = plan.solve(_dev(torch, f)).cpu().numpy()
    (steps, est), = plan.mixed_report()
    err = rel_l2(p, ref)
    print(f"ppn256 mixed {chosen}: {steps} steps, estimate {est:.2e}, rel L2 {err:.3e}",
          flush=True)
    assert err <= MIXED_TOL and 1 <= steps <= 3
    for shape in UNIFORM_SHAPES[:3]:
        _apply(plan, shape)
        p = plan.solve(_dev(torch, f)).cpu().numpy()
        assert rel_l2(p, ref) <= MIXED_TOL, shape
    plan.close()


def _step_reference(X, g):
    """Oracle projection + extension of the benchmark's step inputs."""
    h = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in X.items()}
    u1, v1, w1, p1 = oracle.project(h["u"], h["v"], h["w"], h["phat"], h["rho"], h["rho0"],
                                    h["s"], h["dt"], g)
    ext = oracle.extend(u1, v1, w1, h["s"], g, q=(h["qx"], h["qy"], h["qz"]))
    return {"u": u1, "v": v1, "w": w1, "p": p1, "ue": ext[0], "ve": ext[1], "we": ext[2],
            "ug": ext[3], "vg": ext[4], "wg": ext[5], "phi": ext[6]}


def _run_step(torch, plan, X):
    u, v, w = X["u"].clone(), X["v"].clone(), X["w"].clone()
    e = lambda: torch.empty_like(u)  # noqa: E731
    out = plan.step(u, v, w, X["phat"], X["rho"], X["rho0"], X["s"], X["dt"], X["s"],
                    p=e(), phi=e(), q=(X["qx"], X["qy"], X["qz"]), out=(e(), e(), e()),
                    gamma=(e(), e(), e()))
    torch.cuda.synchronize()
    return dict(zip(("u", "v", "w", "p", "phi", "ue", "ve", "we", "ug", "vg", "wg"),
                    (a.cpu().numpy() for a in out)))


def _check_step(got, ref, label):
    for name, b in ref.items():
        err = rel_l2(got[name], b)
        print(f"{label} {name}: rel L2 {err:.3e}", flush=True)
        assert err <= FP64_TOL, (label, name, err)


def test_ppn256_step_as_benchmarked(torch_dev):
    """One benchmarked time step at 256^3 (vof_step on the benchmark's inputs and
    autotuned two-field plan) against the oracle's projection followed by its
    extension of the projected velocity, every output; then the same step with
    the tridiagonal z pass and the other epilogue / right-hand-side shapes."""
    torch = torch_dev
    cfg = vofsynth.config("ppn256")
    g = oracle.Grid.from_config(cfg)
    X = bench.make_inputs(cfg, torch, "cuda")
    ref = _step_reference(X, g)
    plan = _plan(g, max_batch=bench.STEP_BATCH)
    chosen = plan.autotune(batch=bench.STEP_BATCH)
    _check_step(_run_step(torch, plan, X), ref, f"ppn256 step {chosen}")
    for shape in (dict(UNIFORM_SHAPES[4], rhs_tiled=16, epilogue_tiled=16),
                  dict(UNIFORM_SHAPES[1], rhs_tiled=0, epilogue_tiled=0)):
        _apply(plan, shape)
        _check_step(_run_step(torch, plan, X), ref, f"ppn256 step {shape}")
    plan.close()


def test_stretched_256_solve_and_step(torch_dev):
    """256^3 with tanh-stretched z (beta = 1.5), periodic x/y, walls in z: the
    z path of the 512 x 512 x 256 workload at nz = 256, solve and step,
    every segment length and width of the tridiagonal pass."""
    torch = torch_dev
    cfg = vofsynth.Config("ppn256s", 256, 256, 256, "PPN", beta=1.5)
    g = oracle.Grid.from_config(cfg)
    f = _bench_rhs(g)
    ref = oracle.solve(f, g)
    plan = _plan(g, max_batch=bench.STEP_BATCH)
    chosen = plan.autotune(batch=bench.STEP_BATCH)
    fd = _dev(torch, f)
    err = rel_l2(plan.solve(fd).cpu().numpy(), ref)
    print(f"ppn256s autotuned {chosen}: rel L2 {err:.3e}", flush=True)
    assert err <= FP64_TOL
    for shape in STRETCHED_SHAPES:
        _apply(plan, shape)
        err = rel_l2(plan.solve(fd).cpu().numpy(), ref)
        print(f"ppn256s {shape}: rel L2 {err:.3e}", flush=True)
        assert err <= FP64_TOL, shape
    X = bench.make_inputs(cfg, torch, "cuda")
    sref = _step_reference(X, g)
    _check_step(_run_step(torch, plan, X), sref, "ppn256s step")
    plan.close()


def test_stretched_512x512x256_solve(torch_dev):
    """The full 512 x 512 x 256 stretched grid (beta = 1.5) of the paper-scale
    workload: the benchmark's seeded right-hand side through the autotuned
    plan and both segment lengths of the tridiagonal pass, against the oracle."""
    torch = torch_dev
    cfg = vofsynth.config("ppn512s")
    g = oracle.Grid.from_config(cfg)
    f = _bench_rhs(g)
    ref = oracle.solve(f, g)
    plan = _plan(g)
    chosen = plan.autotune(batch=1)
    fd = _dev(torch, f)
    out = torch.empty_like(fd)
    plan.solve(fd, out)
    err = rel_l2(out.cpu().numpy(), ref)
    print(f"ppn512s autotuned {chosen}: rel L2 {err:.3e}", flush=True)
    assert err <= FP64_TOL
    for shape in (dict(z_segment=8, z_lines=16), dict(z_segment=16, z_lines=32)):
        _apply(plan, shape)
        plan.solve(fd, out)
        err = rel_l2(out.cpu().numpy(), ref)
        print(f"ppn512s {shape}: rel L2 {err:.3e}", flush=True)
        assert err <= FP64_TOL, shape
    plan.close()


LONG_PERIODIC = [(256, 16, 8, "PPP"), (16, 256, 8, "PPP"), (512, 16, 8, "PPP"),
                 (16, 512, 8, "PPP"), (512, 512, 4, "PPN"), (256, 512, 6, "PPP")]


@pytest.mark.parametrize("case", LONG_PERIODIC, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}{c[3]}")
def test_long_periodic_lines(torch_dev, case):
    """Periodic x and y lines of length 256 and 512 (packed real DFT, the
    benchmark's x / y passes and the 512^3 comparison's) at both radix
    schedules and tile widths, FP64 and mixed, against the oracle."""
    torch = torch_dev
    nx, ny, nz, bc = case
    g = oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, vofsynth.uniform_dz(nz), bc)
    f = vofsynth.gaussian_field(g.shape, 17 + nx + 3 * ny)
    ref = oracle.solve(f, g)
    plan = _plan(g)
    fd = _dev(torch, f)
    for xr in (16, 8):
        for yr in (16, 8):
            for lines in (0, 8, 4):
                _apply(plan, dict(x_radix=xr, y_radix=yr, y_lines=lines))
                err = rel_l2(plan.solve(fd).cpu().numpy(), ref)
                assert err <= FP64_TOL, (xr, yr, lines, err)
    mixed = _plan(g, precision="mixed")
    for xr in (16, 8):
        _apply(mixed, dict(x_radix=xr, y_radix=xr))
        assert rel_l2(mixed.solve(fd).cpu().numpy(), ref) <= MIXED_TOL, xr


def test_mixed_512_cubed_against_oracle(torch_dev):
    """512^3 triply periodic, seeded N(0,1) right-hand side with its mean removed
    (the mixed-precision comparison of the benchmark): the FP64 solve within
    1e-12 and the mixed solve within 1e-10 of the oracle, element by element."""
    torch = torch_dev
    cfg = vofsynth.config("ppp512")
    g = oracle.Grid.from_config(cfg)
    f = vofsynth.remove_weighted_mean(vofsynth.gaussian_field(g.shape, 4), g.dzf)
    ref = oracle.solve(f, g)
    fd = _dev(torch, f)
    del f
    p64 = _plan(g)
    p64.autotune(batch=1)
    e64 = rel_l2(p64.solve(fd).cpu().numpy(), ref)
    p64.close()
    mixed = _plan(g, precision="mixed")
    mixed.autotune(batch=1)
    pm = mixed.solve(fd).cpu().numpy()
    (steps, est), = mixed.mixed_report()
    em = rel_l2(pm, ref)
    print(f"ppp512: FP64 {e64:.3e}; mixed {steps} steps, estimate {est:.2e}, {em:.3e}",
          flush=True)
    assert e64 <= FP64_TOL
    assert em <= MIXED_TOL and 1 <= steps <= 3
    mixed.close()
