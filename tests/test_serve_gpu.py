"""The serving loop on the device: every request's result is the same when it
is served alone and when it is served in a mix (other classes, kinds and
precisions in flight, batched with requests of its own class), bit for bit,
and matches the FP64 oracle within the parity tolerances."""
import numpy as np
import pytest

import oracle
import vofsynth

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-10

# (nx, ny, nz, bc, beta): small grids the oracle solves in well under a second
CLASSES = [
    (32, 32, 32, "PPN", None),
    (16, 16, 24, "PPN", 1.5),
    (64, 64, 1, "PPN", None),
    (32, 16, 20, "NPN", None),
]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1907_00890_amd  # noqa: F401
    return torch


def _oracle_grid(c):
    nx, ny, nz, bc, beta = c
    dzf = vofsynth.uniform_dz(nz, 1.0) if beta is None else vofsynth.stretched_dz(nz, 1.0, beta)
    return oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, dzf, bc)


def _requests(torch):
    """A seeded mix: every class x kind x precision, two requests each."""
    from paper_1907_00890_amd.serve import Grid
    reqs = []
    rid = 0
    for c in CLASSES:
        og = _oracle_grid(c)
        g = Grid(og.nx, og.ny, og.nz, og.dx, og.dy, og.dzf, og.bc)
        for kind in ("solve", "extend"):
            for prec in ("fp64", "mixed"):
                for _ in range(2):
                    rid += 1
                    f = vofsynth.remove_weighted_mean(
                        vofsynth.gaussian_field(og.shape, 1_000_000 + rid), og.dzf)
                    r = {"id": rid, "class": c, "grid": g, "og": og, "kind": kind,
                         "precision": prec, "f": f,
                         "rhs": torch.from_numpy(f).cuda()}
                    if kind == "extend":
                        u = vofsynth.random_faces(og.shape, 2_000_000 + rid, og.bc)
                        r["u"] = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in u]
                        r["u_np"] = u
                    reqs.append(r)
    return reqs


def _outputs(torch, r):
    sh = r["grid"].shape
    z = lambda: torch.full(sh, np.nan, dtype=torch.float64, device="cuda")  # noqa: E731
    if r["kind"] == "solve":
        return {"sol": z()}
    return {"out": (z(), z(), z()), "phi": z()}


def _submit(srv, r, outs):
    if r["kind"] == "solve":
        return srv.submit_solve(r["grid"], r["rhs"], outs["sol"], precision=r["precision"])
    u, v, w = r["u"]
    return srv.submit_extend(r["grid"], u, v, w, r["rhs"], outs["out"], phi=outs["phi"],
                             precision=r["precision"])


def _host(outs):
    if "sol" in outs:
        return [outs["sol"].cpu().numpy()]
    return [t.cpu().numpy() for t in (*outs["out"], outs["phi"])]


def test_results_same_alone_and_in_the_mix(torch_dev):
    torch = torch_dev
    from paper_1907_00890_amd.serve import Server
    reqs = _requests(torch)
    with Server(8 << 30, lanes=3, max_batch=4) as srv:
        # alone: one request in the server at a time
        alone = []
        for r in reqs:
            outs = _outputs(torch, r)
            res = srv.wait(_submit(srv, r, outs), 60000)
            assert res is not None and res["status"] == 0 and res["batch"] == 1
            alone.append(_host(outs))
        # in the mix: everything at once, in a shuffled order.  The scheduler
        # starts a batch whenever a lane has room, so requests share a batch
        # only when they arrive faster than the lanes drain: the outputs are
        # allocated before the burst and the burst is repeated (every
        # repetition checked bit for bit) until one of them has batched.
        rng = np.random.default_rng(7)
        batched_total = 0
        for rep in range(8):
            order = rng.permutation(len(reqs))
            outs = {i: _outputs(torch, reqs[i]) for i in order}
            torch.cuda.synchronize()
            tickets = {i: _submit(srv, reqs[i], outs[i]) for i in order}
            batched = 0
            for i in order:
                res = srv.wait(tickets[i], 60000)
                assert res is not None and res["status"] == 0, (rep, reqs[i]["id"])
                batched += res["batch"] > 1
            for i in order:
                for a, b in zip(_host(outs[i]), alone[i]):
                    assert np.array_equal(a, b), (rep, reqs[i]["id"], reqs[i]["kind"])
            batched_total += batched
            if rep >= 1 and batched_total > 0:
                break
        assert batched_total > 0  # some repetition did batch requests together
        st = srv.stats()
        assert st["failed"] == 0 and st["plans_resident"] >= len(CLASSES)
    # and the results are right
    for r, got in zip(reqs, alone):
        og = r["og"]
        tol = FP64_TOL if r["precision"] == "fp64" else MIXED_TOL
        if r["kind"] == "solve":
            ref = [oracle.solve(r["f"], og)]
        else:
            u, v, w = r["u_np"]
            e = oracle.extend(u, v, w, r["f"], og)
            ref = [e[0], e[1], e[2], e[6]]
        for a, b in zip(got, ref):
            err = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
            assert err <= tol, (r["id"], r["kind"], r["precision"], err)


def test_memory_budget_admission_on_device(torch_dev):
    """A budget that holds one plan at a time: requests of three classes still
    all complete (plans are evicted and rebuilt), with correct results."""
    torch = torch_dev
    from paper_1907_00890_amd import footprint
    from paper_1907_00890_amd.serve import Grid, Server
    cls = [(32, 32, 16, "PPN"), (32, 32, 16, "NNN"), (32, 16, 32, "PPP")]
    budget = max(footprint(nx, ny, nz, "fp64", 2) for nx, ny, nz, _ in cls) * 3 // 2
    with Server(budget, lanes=2, max_batch=2) as srv:
        jobs = []
        for k in range(9):
            nx, ny, nz, bc = cls[k % 3]
            og = oracle.Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, vofsynth.uniform_dz(nz, 1.0), bc)
            g = Grid(nx, ny, nz, og.dx, og.dy, og.dzf, bc)
            f = vofsynth.remove_weighted_mean(vofsynth.gaussian_field(og.shape, 40 + k), og.dzf)
            rhs = torch.from_numpy(f).cuda()
            sol = torch.empty_like(rhs)
            jobs.append((srv.submit_solve(g, rhs, sol), f, og, sol))
        for t, f, og, sol in jobs:
            res = srv.wait(t, 60000)
            assert res is not None and res["status"] == 0
            ref = oracle.solve(f, og)
            got = sol.cpu().numpy()
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= FP64_TOL
        st = srv.stats()
        assert st["bytes_peak"] <= budget and st["plans_evicted"] >= 1
