#!/usr/bin/env python3
"""Benchmark of the Poisson / projection / extension hot path on one MI355X.

One step = one time step of the path: the pressure projection (right-hand
side assembly, Poisson solve, velocity correction) followed by the
liquid-velocity extension (Poisson solve of the Stefan source, extension and
interface velocity), on the 256^3 grid (periodic x/y, walls in z, uniform),
FP64, through the fused entry point vof_step (correction and extension in
one pass; every output written).  value = Poisson-solve throughput including the stencils around each
solve: 2 * nx*ny*nz / (time per step), in Mpts/s.

Also reported on the same line: the bare FP64 and mixed-precision solve
rates at the same size (mixed: FP32 chain plus FP64 defect correction, with
its relative L2 distance to the FP64 result), the per-kernel times measured
with HIP events over the timed steps, the roofline fraction of the dominant
kernel and the FP64 CPU oracle timed on the host on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--workload ppn256]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpts/s per Poisson solve at 256^3 (FP64 vs mixed) + %HBM peak; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X, FP64 vector (non-matrix) arithmetic

# Algorithmic HBM bytes per launch, in units of N = nx*ny*nz FP64 values of 8 B:
# every transform / z pass reads and writes one field once; the stencils read
# their inputs and write their outputs once each.
ALG_BYTES_PER_POINT = {
    "step_epilogue": 152,         # u*,v*,w*,p,p_hat,rho,phi,q(3) in; u,v,w,ue,ve,we,ug,vg,wg out
    "x_forward": 16, "y_forward": 16, "z_solve": 16, "y_inverse": 16, "x_inverse": 16,
    "x_forward_f32": 12, "y_forward_f32": 8, "z_solve_f32": 8, "y_inverse_f32": 8,
    "x_inverse_f32": 12,          # FP32 in, FP64 out (accumulate: +8)
    "x_forward_residual_f32": 20,  # f, p in (FP64); FP32 x spectrum of f - m - L_h p out
    "rhs_assembly": 56,           # u*, v*, w*, p_hat, rho, s in; b out
    "correction": 72,             # u*, v*, w*, p, p_hat, rho in; u, v, w out
    "extension": 104,             # u, v, w, phi, qx, qy, qz in; ue, ve, we, ug, vg, wg out
    "advect_x": 24,               # C, u_G in; C* out
    "advect_y": 24,               # C*, v_G in; C** out
    "advect_z": 48,               # C**, w_G, C*, u_G, v_G in; C^{n+1} out
}
# fields per launch of the solve passes inside the step (pressure and Stefan
# potential batched)
STEP_BATCH = 2
SOLVE_PASSES = ("x_forward", "y_forward", "z_solve", "y_inverse", "x_inverse")
KERNEL_SOURCES = {
    "x_forward": "transforms_x.hip", "y_forward": "transforms_y.hip",
    "y_inverse": "transforms_y.hip", "x_inverse": "transforms_x.hip",
    "z_solve": ("zsolve.hip", "transforms_z.hip"),
    "rhs_assembly": "stencils.hip",
    "correction": "stencils.hip", "extension": "stencils.hip", "step_epilogue": "stencils.hip",
}


EXTRAS = ("stretched", "mixed512", "interface", "droplet", "advect", "graphs", "hbm")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ppn256")
    ap.add_argument("--solve-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of autotuning the plans")
    ap.add_argument("--tune", default="",
                    help="launch shapes of the main workload's FP64 plan, 'key=value,...' "
                         "(poisson_plan_tune keys), applied instead of autotuning it")
    ap.add_argument("--tune-mixed", default="",
                    help="the same for the main workload's mixed plan")
    ap.add_argument("--cpu-sample", default="ppn256",
                    help="workload the CPU oracle is timed on (bounded sample)")
    ap.add_argument("--serve-rates", default="sweep",
                    help="comma-separated request rates (req/s) of the serving mix; "
                         "'sweep' for 50,100,200,500,1000,2000; 'none' to skip")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra workloads (same as --extra none)")
    ap.add_argument("--extra", default="all",
                    help="comma-separated extra workloads after the main line: stretched, "
                         "mixed512, interface, droplet, advect, graphs, hbm; 'all' (default) "
                         "or 'none'")
    ap.add_argument("--serve-lanes", type=int, default=4)
    ap.add_argument("--serve-batch", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three plain device copies of one field (a known byte "
                         "count for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def shape_plan(plan, batch, spec, no_autotune):
    """Apply `spec` ('key=value,...') to the plan, or autotune it for `batch`
    fields (unless no_autotune); returns the plan's launch shapes."""
    if spec:
        for item in spec.split(","):
            key, value = item.split("=")
            plan.tune(key.strip(), int(value))
        return plan.tuning()
    if no_autotune:
        return plan.tuning()
    return plan.autotune(batch=batch)


def source_sha(names):
    """First 16 hex digits of the SHA-256 of the kernel source file(s)."""
    h = hashlib.sha256()
    for name in (names,) if isinstance(names, str) else names:
        with open(os.path.join(ROOT, "paper_1907_00890_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch measured with rocprofv3 PMC counters (committed
    summary), or None if absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    with open(path) as fh:
        data = json.load(fh)
    rec = data.get(workload, {}).get(kernel)
    if not rec or rec.get("source_sha") != source_sha(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def load_alu_counts(workload):
    """FP64 operations per launch of the advection sweeps, from rocprofv3
    instruction counters (committed summary), for those taken on the current
    advect.hip; {} if absent."""
    path = os.path.join(ROOT, "profiles", "alu_counts.json")
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        data = json.load(fh).get(workload, {})
    sha = source_sha("advect.hip")
    return {k: v["fp64_flops_per_launch"] for k, v in data.items() if v.get("source_sha") == sha}


def make_inputs(cfg, torch, dev):
    import numpy as np

    import vofsynth
    g = cfg
    dzf = cfg.dzf()
    us, vs, ws = vofsynth.random_faces(cfg.shape, 100, cfg.bc)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, dzf, seed=2)
    rho1, rho2 = 1000.0, 1.0
    rho = rho1 * C + rho2 * (1.0 - C)
    mag, _ = vofsynth.grad_mag_central(C, g.dx, g.dy, dzf, cfg.bc)
    s = 1e-2 * mag
    mdot = 1e-2 / (1.0 / rho2 - 1.0 / rho1)
    q = vofsynth.interface_normal_faces(C, g.dx, g.dy, dzf, cfg.bc, mdot / rho1)
    phat = vofsynth.gaussian_field(cfg.shape, 101)
    f = vofsynth.remove_weighted_mean(vofsynth.gaussian_field(cfg.shape, 200), dzf)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    return dict(u=T(us), v=T(vs), w=T(ws), rho=T(rho), s=T(s), phat=T(phat),
                qx=T(q[0]), qy=T(q[1]), qz=T(q[2]), f=T(f), rho0=min(rho1, rho2), dt=1.0)


# ---------------------------------------------------------------------------
# serving mix: Poisson arrivals of solves and extensions of mixed grids
# ---------------------------------------------------------------------------
SERVE_CLASSES = [
    # name, nx, ny, nz, Lz, beta (tanh clustering of z; None = uniform)
    ("64^3", 64, 64, 64, 1.0, None),
    ("128^3", 128, 128, 128, 1.0, None),
    ("256^3", 256, 256, 256, 1.0, None),
    ("128x128x256s", 128, 128, 256, 1.0, 1.5),
    ("1024^2 slab", 1024, 1024, 1, 1.0 / 1024, None),
]


class ServeMix:
    """Device-resident inputs and output slots for the serving mix.

    Per class: a bank of two seeded zero-mean N(0,1) right-hand sides and
    velocity fields (inputs resident in HBM before timing), and `slots`
    output sets per request kind reused round-robin; a slot still in use by
    an unfinished request is waited for before reuse (client back-pressure,
    inside the measured latency).
    """

    def __init__(self, torch, dev, slots=32):
        import numpy as np

        import vofsynth
        from paper_1907_00890_amd.serve import Grid
        self.torch = torch
        self.cls = []
        for k, (name, nx, ny, nz, lz, beta) in enumerate(SERVE_CLASSES):
            dzf = vofsynth.uniform_dz(nz, lz) if beta is None else vofsynth.stretched_dz(nz, lz, beta)
            g = Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, "PPN")
            bank = []
            for b in range(2):
                f = vofsynth.remove_weighted_mean(
                    vofsynth.gaussian_field(g.shape, 1_000_000 + 10 * k + b), dzf)
                u = vofsynth.random_faces(g.shape, 2_000_000 + 10 * k + b, "PPN")
                T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
                bank.append({"f": T(f), "u": [T(a) for a in u]})
            e = lambda: torch.empty(g.shape, dtype=torch.float64, device=dev)  # noqa: E731
            outs = {"solve": [{"sol": e(), "ticket": None} for _ in range(slots)],
                    "extend": [{"out": (e(), e(), e()), "phi": e(), "ticket": None}
                               for _ in range(slots)]}
            self.cls.append({"name": name, "grid": g, "bank": bank, "outs": outs,
                             "next": {"solve": 0, "extend": 0}, "npts": nx * ny * nz})

    def submit(self, srv, ci, kind, precision, bank_i, early_results):
        c = self.cls[ci]
        pool = c["outs"][kind]
        slot = pool[c["next"][kind]]
        c["next"][kind] = (c["next"][kind] + 1) % len(pool)
        if slot["ticket"] is not None:  # back-pressure: the slot is still in use
            early_results[slot["ticket"]] = srv.wait(slot["ticket"], -1)
        b = c["bank"][bank_i]
        if kind == "solve":
            t = srv.submit_solve(c["grid"], b["f"], slot["sol"], precision=precision)
        else:
            u, v, w = b["u"]
            t = srv.submit_extend(c["grid"], u, v, w, b["f"], slot["out"], phi=slot["phi"],
                                  precision=precision)
        slot["ticket"] = t
        return t

    def release(self):
        for c in self.cls:
            for pool in c["outs"].values():
                for s in pool:
                    s["ticket"] = None


def serve_run(srv, mix, rate, n, seed):
    """Poisson arrivals at `rate` req/s; returns latency statistics (ms)."""
    import numpy as np

    from paper_1907_00890_amd.serve import now_us
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1e6 / rate, size=n)
    ci = rng.integers(0, len(mix.cls), size=n)
    kinds = np.where(rng.random(n) < 0.5, "solve", "extend")
    precs = np.where(rng.random(n) < 0.5, "fp64", "mixed")
    banks = rng.integers(0, 2, size=n)
    early = {}
    tickets, t_arr = [], []
    t0 = now_us() + 2000.0
    arrival = t0
    for i in range(n):
        arrival += gaps[i]
        while True:
            d = arrival - now_us()
            if d <= 0:
                break
            if d > 300:
                time.sleep((d - 200) * 1e-6)
        tickets.append(mix.submit(srv, int(ci[i]), kinds[i], precs[i], int(banks[i]), early))
        t_arr.append(arrival)
    res = []
    for t in tickets:
        r = early.pop(t, None) or srv.wait(t, -1)
        res.append(r)
    mix.release()
    ok = [r["status"] == 0 for r in res]
    lat = np.array([(r["t_done_us"] - a) * 1e-3 for r, a in zip(res, t_arr)])
    qwait = np.array([(r["t_dispatch_us"] - a) * 1e-3 for r, a in zip(res, t_arr)])
    t_end = max(r["t_done_us"] for r in res)
    pts = sum(mix.cls[int(c)]["npts"] for c in ci)
    per_class = {}
    for k, c in enumerate(mix.cls):
        m = ci == k
        if m.any():
            per_class[c["name"]] = {"n": int(m.sum()),
                                    "p50_ms": round(float(np.percentile(lat[m], 50)), 3),
                                    "p99_ms": round(float(np.percentile(lat[m], 99)), 3)}
    return {"rate_req_s": rate, "requests": n, "completed": int(sum(ok)),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3),
            "queue_wait_p99_ms": round(float(np.percentile(qwait, 99)), 3),
            "throughput_req_s": round(n / ((t_end - t0) * 1e-6), 1),
            "throughput_mpts_s": round(pts / ((t_end - t0) * 1e-6) / 1e6, 1),
            "mean_batch": round(float(np.mean([r["batch"] for r in res])), 2),
            "per_class": per_class}


def serve_bench(torch, dev, rates, n, lanes, max_batch):
    from paper_1907_00890_amd.serve import Server
    mix = ServeMix(torch, dev)
    out = []
    with Server(96 << 30, lanes=lanes, max_batch=max_batch, max_pending=1 << 20) as srv:
        # plans resident before timing: one instance per lane of every class and
        # precision, then one request of every class / kind / precision (first
        # launches of every kernel)
        for c in mix.cls:
            for prec in ("fp64", "mixed"):
                srv.prewarm(c["grid"], prec, instances=lanes)
        warm = []
        early = {}
        for k in range(len(mix.cls)):
            for kind in ("solve", "extend"):
                for prec in ("fp64", "mixed"):
                    warm.append(mix.submit(srv, k, kind, prec, 0, early))
        for t in warm:
            early.pop(t, None) or srv.wait(t, -1)
        mix.release()
        for rate in rates:
            # about 10 s of arrivals per rate, 500 to n requests
            r = serve_run(srv, mix, rate, int(min(n, max(500, 10 * rate))), seed=5)
            print(f"[serve] rate {rate} req/s: p50 {r['p50_ms']} ms, p99 {r['p99_ms']} ms, "
                  f"{r['throughput_req_s']} req/s, mean batch {r['mean_batch']}",
                  file=sys.stderr, flush=True)
            out.append(r)
        st = srv.stats()
    return out, {"lanes": lanes, "max_batch": max_batch, "hbm_budget_gib": 96,
                 "plans_resident": st["plans_resident"],
                 "bytes_resident_gib": round(st["bytes_resident"] / 2**30, 2),
                 "failed": st["failed"], "rejected": st["rejected"]}


def stretched_step_run(torch, dev, steps, no_autotune):
    """The 512x512x256 PPN tanh-stretched workload: `steps` time steps (two
    solves each, stencils in the loop) and a bare solve; the z pass is the
    partitioned tridiagonal solve (stretched z)."""
    import vofsynth
    from paper_1907_00890_amd import Plan
    cfg = vofsynth.config("ppn512s")
    X = make_inputs(cfg, torch, dev)
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dzf(), cfg.bc)
    tuned = plan.autotune(batch=1) if not no_autotune else plan.tuning()
    p = torch.empty(cfg.shape, dtype=torch.float64, device=dev)
    phi = torch.empty_like(p)
    ue = tuple(torch.empty_like(p) for _ in range(3))
    ug = tuple(torch.empty_like(p) for _ in range(3))
    q = (X["qx"], X["qy"], X["qz"])

    def step():
        plan.step(X["u"], X["v"], X["w"], X["phat"], X["rho"], X["rho0"], X["s"], X["dt"],
                  X["s"], p=p, phi=phi, q=q, out=ue, gamma=ug)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms_step = a.elapsed_time(b) / steps
    plan.kernel_times()
    plan.set_profiling(True)
    out = torch.empty_like(p)
    for _ in range(5):
        plan.solve(X["f"], out)
    torch.cuda.synchronize()
    kt = plan.kernel_times()
    plan.set_profiling(False)
    n = cfg.npts
    solve_ms = sum(ms for ms, _ in kt.values()) / 5
    z = kt.get("z_solve", (0.0, 1))
    res = {"workload": "ppn512s: 512x512x256 PPN, tanh beta=1.5 z, project + extend step",
           "steps": steps, "ms_per_step": round(ms_step, 4),
           "mpts_s": round(2 * n / (ms_step * 1e-3) / 1e6, 1),
           "solve_ms": round(solve_ms, 4), "solve_model_gbs_80N": round(80 * n / (solve_ms * 1e-3) / 1e9, 1),
           "z_tridiagonal_ms": round(z[0] / z[1], 4), "tuning": tuned}
    del X, plan
    torch.cuda.empty_cache()
    return res


def droplet_grid_run(torch, dev, steps, no_autotune):
    """The 320 x 320 x 640 triply periodic grid of the three-dimensional
    settling droplet (transform lengths 5 * 2^k, radix-5 passes): `steps`
    time steps (two solves each, stencils in the loop) and a bare solve."""
    import vofsynth
    from paper_1907_00890_amd import Plan
    cfg = vofsynth.config("ppp320x320x640")
    X = make_inputs(cfg, torch, dev)
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dzf(), cfg.bc)
    tuned = plan.autotune(batch=1) if not no_autotune else plan.tuning()
    p = torch.empty(cfg.shape, dtype=torch.float64, device=dev)
    phi = torch.empty_like(p)
    ue = tuple(torch.empty_like(p) for _ in range(3))
    ug = tuple(torch.empty_like(p) for _ in range(3))
    q = (X["qx"], X["qy"], X["qz"])

    def step():
        plan.step(X["u"], X["v"], X["w"], X["phat"], X["rho"], X["rho0"], X["s"], X["dt"],
                  X["s"], p=p, phi=phi, q=q, out=ue, gamma=ug)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms_step = a.elapsed_time(b) / steps
    out = torch.empty_like(p)
    a.record()
    for _ in range(steps):
        plan.solve(X["f"], out)
    b.record()
    torch.cuda.synchronize()
    solve_ms = a.elapsed_time(b) / steps
    plan.kernel_times()
    plan.set_profiling(True)
    for _ in range(3):
        plan.solve(X["f"], out)
    torch.cuda.synchronize()
    kt = {k: round(ms / c, 4) for k, (ms, c) in plan.kernel_times().items()}
    plan.set_profiling(False)
    n = cfg.npts
    res = {"solve_kernel_ms": kt,
           "workload": "ppp320x320x640: 320x320x640 triply periodic, cubic cells, project + "
                       "extend step", "steps": steps, "ms_per_step": round(ms_step, 4),
           "mpts_s": round(2 * n / (ms_step * 1e-3) / 1e6, 1), "solve_ms": round(solve_ms, 4),
           "solve_mpts_s": round(n / (solve_ms * 1e-3) / 1e6, 1),
           "solve_model_gbs_80N": round(80 * n / (solve_ms * 1e-3) / 1e9, 1), "tuning": tuned}
    del X, plan
    torch.cuda.empty_cache()
    return res


def interface_outflow_run(torch, dev, steps, no_autotune):
    """256^3 with walls and an outflow top (p = 0 on the top face, the
    container of section 4): the interface terms (Stefan source and
    interface-velocity jump from C and mdot, Youngs gradient) in one pass,
    the full step fed by them, and bare solves with outflow on every side
    and in the container against the periodic-x/y walls-z solve."""
    import numpy as np

    import vofsynth
    from paper_1907_00890_amd import Plan
    n = 256
    dz = vofsynth.uniform_dz(n, 1.0)
    C, _ = vofsynth.sphere_vof(n, n, n, 1.0 / n, 1.0 / n, dz, seed=2)
    rho1, rho2 = 1000.0, 1.0
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    dC = T(C)
    dm = torch.full_like(dC, 1e-2 / (1.0 / rho2 - 1.0 / rho1))
    rho = T(rho1 * C + rho2 * (1.0 - C))
    us, vs, ws = (T(a) for a in vofsynth.random_faces((n, n, n), 100, "NNNNND"))
    phat = T(vofsynth.gaussian_field((n, n, n), 101))
    f = T(vofsynth.gaussian_field((n, n, n), 200))
    del C
    plan = Plan(n, n, n, 1.0 / n, 1.0 / n, dz, "NNNNND")
    tuned = plan.autotune(batch=1) if not no_autotune else plan.tuning()
    terms = tuple(torch.empty_like(dC) for _ in range(4))
    p, phi = torch.empty_like(dC), torch.empty_like(dC)
    ue = tuple(torch.empty_like(dC) for _ in range(3))
    ug = tuple(torch.empty_like(dC) for _ in range(3))

    def step():
        sq = plan.interface_terms(dC, dm, rho1, rho2, out=terms)
        plan.step(us, vs, ws, phat, rho, rho2, sq[0], 1.0, sq[0], p=p, phi=phi, q=sq[1:],
                  out=ue, gamma=ug)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms_step = a.elapsed_time(b) / steps
    # the same step with the interface terms formed inside its first and last
    # passes (vof_step_interface: s in the right-hand side, q in the epilogue)
    sv = torch.empty_like(dC)

    def step_fused():
        plan.step_interface(us, vs, ws, phat, rho, rho2, dC, dm, rho1, rho2, 1.0, p=p, phi=phi,
                            s=sv, out=ue, gamma=ug)

    for _ in range(2):
        step_fused()
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        step_fused()
    b.record()
    torch.cuda.synchronize()
    ms_fused = a.elapsed_time(b) / steps
    plan.kernel_times()
    plan.set_profiling(True, classes=["rhs_assembly", "step_epilogue"])
    for _ in range(steps):
        step_fused()
    torch.cuda.synchronize()
    kf = plan.kernel_times()
    plan.set_profiling(False)
    plan.set_profiling(True, classes=["rhs_assembly", "step_epilogue"])
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ks = plan.kernel_times()
    plan.set_profiling(False)
    plan.set_profiling(True, classes=["interface_terms"])
    for _ in range(steps):
        plan.interface_terms(dC, dm, rho1, rho2, out=terms)
    torch.cuda.synchronize()
    ms_if, cnt = plan.kernel_times()["interface_terms"]
    plan.set_profiling(False)
    ms_if /= cnt
    knobs = plan.tuning()
    npts = n ** 3
    res = {"workload": "256x256x256, walls on the sides and the bottom, outflow top (NNNNND)",
           "interface_terms": {"ms": round(ms_if, 4), "alg_bytes": 48 * npts,
                               "gbs": round(48 * npts / (ms_if * 1e-3) / 1e9, 1),
                               "planes": knobs["interface_planes"], "tile": knobs["interface_tile"]},
           "step_with_interface_terms_ms": round(ms_step, 4),
           "step_interface_fused_ms": round(ms_fused, 4),
           "fused_vs_separate": {
               "separate": {"interface_terms_ms": round(ms_if, 4),
                            "rhs_ms": round(ks["rhs_assembly"][0] / ks["rhs_assembly"][1], 4),
                            "epilogue_ms": round(ks["step_epilogue"][0] / ks["step_epilogue"][1], 4),
                            "model_bytes_N": "48 + 56 + 152"},
               "fused": {"rhs_with_s_ms": round(kf["rhs_assembly"][0] / kf["rhs_assembly"][1], 4),
                         "epilogue_with_q_ms": round(kf["step_epilogue"][0] / kf["step_epilogue"][1], 4),
                         "model_bytes_N": "72 + 144"}},
           "tuning": tuned, "solve_ms": {}}
    out = torch.empty_like(f)
    for bc in ("NNNNND", "DDD", "PPN"):
        sp = Plan(n, n, n, 1.0 / n, 1.0 / n, dz, bc)
        if not no_autotune:
            sp.autotune(batch=1)
        for _ in range(2):
            sp.solve(f, out)
        torch.cuda.synchronize()
        a.record()
        for _ in range(10):
            sp.solve(f, out)
        b.record()
        torch.cuda.synchronize()
        res["solve_ms"][bc] = round(a.elapsed_time(b) / 10, 4)
        del sp
    del plan, terms, ue, ug
    torch.cuda.empty_cache()
    return res


def advect_run(torch, dev, steps):
    """VoF advection of section 3.1 on the 256^3 workload: the benchmark's
    sphere C advected by the interface velocity of one step (the extension of
    the projected velocity minus the jump), at CFL 0.4, `steps` consecutive
    advection steps; per-sweep kernel times and HBM rates on the algorithmic
    bytes (24 N + 24 N + 48 N per step)."""
    import numpy as np

    import vofsynth
    from paper_1907_00890_amd import Plan
    cfg = vofsynth.config("ppn256")
    X = make_inputs(cfg, torch, dev)
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dzf(), cfg.bc)
    e = lambda: torch.empty_like(X["u"])  # noqa: E731
    ug = (e(), e(), e())
    plan.step(X["u"].clone(), X["v"].clone(), X["w"].clone(), X["phat"], X["rho"], X["rho0"],
              X["s"], X["dt"], X["s"], q=(X["qx"], X["qy"], X["qz"]), gamma=ug)
    C, _ = vofsynth.sphere_vof(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dzf(), seed=2)
    dt = 0.4 * cfg.dx / max(a.abs().max().item() for a in ug)
    bufs = [torch.from_numpy(np.ascontiguousarray(C)).to(dev), e()]
    for _ in range(2):
        plan.advect(bufs[0], *ug, dt, out=bufs[1])
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for it in range(steps):
        plan.advect(bufs[it % 2], *ug, dt, out=bufs[(it + 1) % 2])
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    plan.kernel_times()
    plan.set_profiling(True, classes=["advect_x", "advect_y", "advect_z"])
    for it in range(steps):
        plan.advect(bufs[it % 2], *ug, dt, out=bufs[(it + 1) % 2])
    torch.cuda.synchronize()
    kt = plan.kernel_times()
    plan.set_profiling(False)
    n = cfg.npts
    kern = {}
    for name, (tot, cnt) in kt.items():
        per = tot / cnt
        alg = ALG_BYTES_PER_POINT[name] * n
        kern[name] = {"avg_ms": round(per, 5), "alg_bytes": alg,
                      "gbs": round(alg / (per * 1e-3) / 1e9, 1)}
    # FP64 operations per launch from rocprofv3 instruction counters of this same
    # sequence (committed, checked against the kernel source): the sweeps are
    # bound by FP64 arithmetic in the interface band, not by HBM
    flops = load_alu_counts("ppn256")
    for name, k in kern.items():
        fl = flops.get(name)
        if fl:
            k["fp64_flops_per_launch"] = fl
            k["tflops"] = round(fl / (k["avg_ms"] * 1e-3) / 1e12, 3)
    roof = None
    dom_k = max(kern, key=lambda k: kern[k]["avg_ms"]) if kern else None
    if dom_k and "tflops" in kern[dom_k]:
        roof = {"bound": "alu", "kernel": dom_k, "achieved": kern[dom_k]["tflops"],
                "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(kern[dom_k]["tflops"] / FP64_VECTOR_PEAK_TFLOPS, 4)}
    band = ((bufs[0] > 1e-8) & (bufs[0] < 1 - 1e-8)).sum().item()
    res = {"workload": "256x256x256 PPN: the sphere's C advected by the step's interface "
                       "velocity, CFL 0.4, MTHINC beta = 1, deflation on", "steps": steps,
           "ms_per_advect": round(ms, 4), "mpts_s": round(n / (ms * 1e-3) / 1e6, 1),
           "alg_bytes_96N": 96 * n, "gbs_96N": round(96 * n / (ms * 1e-3) / 1e9, 1),
           "band_cells": int(band), "roofline": roof, "kernels": kern}
    del X, plan, bufs, ug
    torch.cuda.empty_cache()
    return res


def mixed512_run(torch, dev, reps, no_autotune):
    """512^3 PPP, seeded N(0,1) RHS with its mean removed: FP64 against mixed
    (FP32 chain + FP64 defect correction with the device-side stopping rule)."""
    import numpy as np

    import vofsynth
    from paper_1907_00890_amd import Plan
    cfg = vofsynth.config("ppp512")
    f = torch.from_numpy(np.ascontiguousarray(vofsynth.remove_weighted_mean(
        vofsynth.gaussian_field(cfg.shape, 4), cfg.dzf()))).to(dev)
    out = {}
    res = {"workload": "ppp512: 512^3 triply periodic, uniform"}
    for prec in ("fp64", "mixed"):
        plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dzf(), cfg.bc, precision=prec)
        if not no_autotune:
            plan.autotune(batch=1)
        o = torch.empty_like(f)
        for _ in range(2):
            plan.solve(f, o)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            plan.solve(f, o)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        res[prec] = {"ms": round(ms, 4), "mpts_s": round(cfg.npts / (ms * 1e-3) / 1e6, 1)}
        if prec == "mixed":
            (steps, est), = plan.mixed_report()
            res[prec].update({"dc_steps": steps, "dc_error_estimate": est})
        out[prec] = o
        del plan
    res["mixed"]["rel_l2_vs_fp64"] = (torch.linalg.vector_norm(out["mixed"] - out["fp64"]) /
                                      torch.linalg.vector_norm(out["fp64"])).item()
    res["speedup_mixed_vs_fp64"] = round(res["fp64"]["ms"] / res["mixed"]["ms"], 3)
    del out, f
    torch.cuda.empty_cache()
    return res


def hbm_ceiling_run(torch, dev, reps=10):
    """Streaming rates of plain device kernels (torch's own) on 2 GiB FP64 tensors,
    far above the 256 MB Infinity Cache: read (a sum), write (a fill), copy.  The
    practical HBM ceiling of this device, beside the 8 TB/s peak that the roofline
    fractions are taken against."""
    n = (2 << 30) // 8
    a = torch.zeros(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    h = n // 2

    def rate(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        return {"ms": round(ms, 4), "tb_s": round(8 * n / (ms * 1e-3) / 1e12, 3)}

    out = {"bytes_moved": 8 * n,
           "read": rate(lambda: a.sum()),
           "write": rate(lambda: b.fill_(1.0)),
           "copy": rate(lambda: b[:h].copy_(a[:h]))}
    del a, b
    torch.cuda.empty_cache()
    return out


def graph_replay_run(torch, dev, reps=200):
    """Per-request latency of the serving mix's small classes (64^3, 128^3,
    1024^2 slab; solve and extension, FP64 and mixed): eager launches against
    the same call replayed from a captured HIP graph on fixed buffers, the
    caller synchronising after each call (median and 99th percentile, us)."""
    import vofsynth
    from paper_1907_00890_amd import Plan

    def lat(fn):
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        return {"p50_us": round(ts[len(ts) // 2] * 1e6, 1),
                "p99_us": round(ts[int(len(ts) * 0.99)] * 1e6, 1)}

    out = {}
    for name, (nx, ny, nz, lz) in {"64^3": (64, 64, 64, 1.0), "128^3": (128, 128, 128, 1.0),
                                   "1024^2 slab": (1024, 1024, 1, 1.0 / 1024)}.items():
        dz = vofsynth.uniform_dz(nz, lz)
        for prec in ("fp64", "mixed"):
            plan = Plan(nx, ny, nz, 1.0 / nx, 1.0 / ny, dz, "PPN", precision=prec)
            f = torch.randn((nz, ny, nx), dtype=torch.float64, device=dev)
            f -= f.mean()
            sol = torch.empty_like(f)
            u = [torch.randn_like(f) for _ in range(3)]
            eo = [torch.empty_like(f) for _ in range(3)]
            phi = torch.empty_like(f)
            st = torch.cuda.Stream()
            res = {}
            with torch.cuda.stream(st):
                for kind, fn in (("solve", lambda: plan.solve(f, out=sol, stream=st)),
                                 ("extend", lambda: plan.extend(*u, f, out=eo, phi=phi,
                                                                stream=st))):
                    res[kind] = {"eager": lat(fn)}
                    g = torch.cuda.CUDAGraph()
                    fn()
                    torch.cuda.synchronize()
                    with torch.cuda.graph(g, stream=st):
                        fn()
                    res[kind]["graph"] = lat(g.replay)
            out[f"{name} {prec}"] = res
            plan.close()
    return out


def cpu_baseline(sample_name, runs=3):
    """Time the FP64 oracle's project + extend step on a bounded sample: the
    median of `runs` runs with the host's BLAS threads, and of `runs` runs on
    one thread (the oracle's FFTs run on one thread either way)."""
    import numpy as np

    import oracle
    import vofsynth
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = 1
    cfg = vofsynth.config(sample_name)
    g = oracle.Grid.from_config(cfg)
    dzf = cfg.dzf()
    us, vs, ws = vofsynth.random_faces(cfg.shape, 100, cfg.bc)
    C, _ = vofsynth.sphere_vof(g.nx, g.ny, g.nz, g.dx, g.dy, dzf, seed=2)
    rho = 1000.0 * C + (1.0 - C)
    s = 1e-2 * vofsynth.grad_mag_central(C, g.dx, g.dy, dzf, cfg.bc)[0]
    q = vofsynth.interface_normal_faces(C, g.dx, g.dy, dzf, cfg.bc, 1e-5)
    phat = vofsynth.gaussian_field(cfg.shape, 101)

    def one():
        t0 = time.perf_counter()
        u, v, w, p = oracle.project(us, vs, ws, phat, rho, 1.0, s, 1.0, g)
        oracle.extend(u, v, w, s, g, q=q)
        return time.perf_counter() - t0

    t_all = sorted(one() for _ in range(runs))
    t_one = []
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t_one = sorted(one() for _ in range(runs))
    med = t_all[len(t_all) // 2]
    out = {"value": round(2 * cfg.npts / med / 1e6, 3), "unit": "Mpts/s", "cores": int(threads),
           "kind": "oracle",
           "sample": f"one project + extend step of the same recipe on {cfg.nx}x{cfg.ny}x{cfg.nz} "
                     f"{cfg.bc} (FP64 numpy/scipy oracle), median of {runs} runs "
                     f"({', '.join(f'{t:.1f}' for t in t_all)} s)",
           "host_cpus": os.cpu_count()}
    if t_one:
        med1 = t_one[len(t_one) // 2]
        out["one_thread"] = {"value": round(2 * cfg.npts / med1 / 1e6, 3), "cores": 1,
                             "runs_s": [round(t, 2) for t in t_one]}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import vofsynth
    from paper_1907_00890_amd import Plan

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = vofsynth.config(args.workload)
    n = cfg.npts
    X = make_inputs(cfg, torch, dev)
    # room for two fields: the step's pressure and Stefan-potential solves run
    # as one batch (one launch per pass for both)
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dzf(), cfg.bc, max_batch=STEP_BATCH)
    p = torch.empty(cfg.shape, dtype=torch.float64, device=dev)
    phi = torch.empty_like(p)
    ue, ve, we = torch.empty_like(p), torch.empty_like(p), torch.empty_like(p)
    ug, vg, wg = torch.empty_like(p), torch.empty_like(p), torch.empty_like(p)
    stream = torch.cuda.current_stream()

    q = (X["qx"], X["qy"], X["qz"])
    # launch shapes and radix schedules picked by the autotuner (before timing)
    tuned = shape_plan(plan, STEP_BATCH, args.tune, args.no_autotune)

    def step():
        # one time step through the fused entry point (all outputs written)
        plan.step(X["u"], X["v"], X["w"], X["phat"], X["rho"], X["rho0"], X["s"], X["dt"],
                  X["s"], p=p, phi=phi, q=q, out=(ue, ve, we), gamma=(ug, vg, wg))

    def step_separate():
        plan.project(X["u"], X["v"], X["w"], X["phat"], X["rho"], X["rho0"], X["s"], X["dt"], p)
        plan.extend(X["u"], X["v"], X["w"], X["s"], q=q, out=(ue, ve, we), gamma=(ug, vg, wg),
                    phi=phi)

    for _ in range(args.warmup):
        step()
        step_separate()
    torch.cuda.synchronize()
    # a short pass with every launch bracketed finds the dominant kernel and the
    # per-kernel breakdown; the timed region then brackets only that kernel
    plan.kernel_times()
    plan.set_profiling(True)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    kall = plan.kernel_times()
    dom = max(kall, key=lambda k: kall[k][0])
    plan.set_profiling(True, classes=[dom])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = e0.elapsed_time(e1)
    ktimes = plan.kernel_times()
    plan.set_profiling(False)
    ms_step = ms_total / args.steps
    value = 2 * n / (ms_step * 1e-3) / 1e6

    # the same step without event bracketing, eagerly and replayed from a HIP graph,
    # and as separate project + extend calls
    def time_steps(fn, k):
        a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a_.record(stream)
        for _ in range(k):
            fn()
        b_.record(stream)
        torch.cuda.synchronize()
        return a_.elapsed_time(b_) / k

    ms_eager = time_steps(step, args.steps)
    ms_separate = time_steps(step_separate, args.steps)
    gstream = torch.cuda.Stream()
    with torch.cuda.stream(gstream):
        step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gstream):
        step()
    ms_graph = time_steps(graph.replay, args.steps)

    # bare solves at the same size: FP64 and mixed (FP32 chain + FP64 defect corrections)
    f = X["f"]
    out64 = torch.empty_like(f)
    for _ in range(3):
        plan.solve(f, out64)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(args.solve_reps):
        plan.solve(f, out64)
    b.record(stream)
    torch.cuda.synchronize()
    ms64 = a.elapsed_time(b) / args.solve_reps
    # mixed: FP32 chain + FP64 defect correction, up to 3 steps, stopping on the
    # device once the estimated error is at most 1e-11 (the library default).
    # Its byte model: the first FP32 chain moves 48 N bytes (x forward 8 in +
    # 4 out, y / z / y 8 each, x inverse 4 in + 8 out); a correction 64 N (x
    # forward of the defect 16 in + 4 out, y / z / y 8 each, accumulating x
    # inverse 4 + 8 in + 8 out).
    mixed = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dzf(), cfg.bc, precision="mixed")
    tuned_mixed = shape_plan(mixed, 1, args.tune_mixed, args.no_autotune)
    out32 = torch.empty_like(f)
    for _ in range(3):
        mixed.solve(f, out32)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(args.solve_reps):
        mixed.solve(f, out32)
    b.record(stream)
    torch.cuda.synchronize()
    ms32 = a.elapsed_time(b) / args.solve_reps
    rel_mixed = (torch.linalg.vector_norm(out32 - out64) / torch.linalg.vector_norm(out64)).item()
    (dc_steps, dc_est), = mixed.mixed_report()
    mixed_bytes = (48 + 64 * dc_steps) * n
    mixed_gbs = mixed_bytes / (ms32 * 1e-3) / 1e9

    # roofline of the dominant kernel, timed over the timed steps; the other
    # kernels' times come from the fully bracketed pass
    kernels = {}
    for name, (ms, cnt) in {**kall, **ktimes}.items():
        per = ms / cnt
        alg = ALG_BYTES_PER_POINT.get(name, 0) * n * (STEP_BATCH if name in SOLVE_PASSES else 1)
        kernels[name] = {"launches": cnt, "avg_ms": round(per, 5),
                         "alg_bytes": alg, "gbs": round(alg / (per * 1e-3) / 1e9, 1)}
    dk = kernels[dom]
    traffic = load_traffic(dom, args.workload)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(dk["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_launch_ms": dk["avg_ms"]}
    kern_ms_step = sum(ms for ms, _ in kall.values()) / 3

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: project + extend step, {cfg.nx}x{cfg.ny}x{cfg.nz} "
                               f"{cfg.bc}, {'uniform' if cfg.beta is None else 'tanh beta=%g' % cfg.beta}"
                               " z, 2 Poisson solves per step",
                   "grid": [cfg.nx, cfg.ny, cfg.nz], "bc": cfg.bc, "parallelism": "single GPU"},
        "roofline": roofline,
        "solve_fp64": {"ms": round(ms64, 4), "mpts_s": round(n / (ms64 * 1e-3) / 1e6, 1),
                       "model_gbs_80N": round(80 * n / (ms64 * 1e-3) / 1e9, 1)},
        "solve_mixed": {"ms": round(ms32, 4), "mpts_s": round(n / (ms32 * 1e-3) / 1e6, 1),
                        "dc_steps": dc_steps, "dc_error_estimate": dc_est,
                        "rel_l2_vs_fp64": rel_mixed,
                        "roofline": {"bound": "hbm", "model_bytes": mixed_bytes,
                                     "model": f"{48 + 64 * dc_steps}N",
                                     "achieved": round(mixed_gbs, 1), "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": round(mixed_gbs / HBM_PEAK_GBS, 4)},
                        "speedup_vs_fp64": round(ms64 / ms32, 3)},
        "step_variants_ms": {"fused_timed_region": round(ms_step, 4), "fused": round(ms_eager, 4),
                             "fused_hip_graph": round(ms_graph, 4),
                             "separate_project_extend": round(ms_separate, 4)},
        "tuning": {"fp64": tuned, "mixed": tuned_mixed},
        "kernels": kernels,
        "kernel_ms_per_step": round(kern_ms_step, 4),
        "wall_s_timed": round(t_wall, 3),
    }
    extras = EXTRAS if args.extra == "all" else [e for e in args.extra.split(",") if e != "none"]
    if args.no_extra:
        extras = []
    for e in extras:
        if e not in EXTRAS:
            raise SystemExit(f"unknown extra workload {e!r} (one of {', '.join(EXTRAS)})")
    if "stretched" in extras:
        line["stretched_512x512x256"] = stretched_step_run(torch, dev, 20, args.no_autotune)
    if "mixed512" in extras:
        line["mixed_vs_fp64_512"] = mixed512_run(torch, dev, 5, args.no_autotune)
    if "interface" in extras:
        line["interface_outflow_256"] = interface_outflow_run(torch, dev, 10, args.no_autotune)
    if "droplet" in extras:
        line["droplet_320x320x640"] = droplet_grid_run(torch, dev, 10, args.no_autotune)
    if "advect" in extras:
        line["advect_256"] = advect_run(torch, dev, 10)
    if "graphs" in extras:
        line["graph_replay_small_classes"] = graph_replay_run(torch, dev)
    if "hbm" in extras:
        line["hbm_ceiling"] = hbm_ceiling_run(torch, dev)
    rates = {"none": [], "sweep": [50, 100, 200, 500, 1000, 2000]}.get(
        args.serve_rates, None)
    if rates is None:
        rates = [float(r) for r in args.serve_rates.split(",") if r]
    if rates:
        runs, setup = serve_bench(torch, dev, rates, args.serve_requests, args.serve_lanes,
                                  args.serve_batch)
        line["serving"] = {"mix": "Poisson arrivals (seed 5), classes uniform over "
                                  + ", ".join(c[0] for c in SERVE_CLASSES)
                                  + " (PPN; 128x128x256 tanh beta=1.5), solve/extend 50/50, "
                                  "FP64/mixed 50/50, device-resident seeded inputs",
                           "latency": "arrival to completion observed by the server",
                           "setup": setup, "runs": runs}
    if args.copy_calibration:
        src = torch.randn(cfg.shape, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = int(src.numel() * 8)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(line), flush=True)
    plan.close()
    mixed.close()


if __name__ == "__main__":
    main()
