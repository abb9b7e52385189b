"""Host logic of the continuous-batching server, on the CPU (dry-run mode: the
scheduler, admission by plan footprint, batching, lanes, cancellation,
timeouts and host-forced faults run exactly as on a device; a batch takes a
fixed time instead of launching kernels, and the field addresses are never
dereferenced)."""
import time

import pytest

from paper_1907_00890_amd import footprint, serve
from paper_1907_00890_amd.serve import Grid, Server, ServeError

FAKE = 0x10000  # never dereferenced in a dry run


def grid(nx=32, ny=32, nz=32, bc="PPN"):
    return Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, [1.0 / nz] * nz, bc)


def solve(srv, g, precision="fp64", timeout_ms=0.0):
    return srv.submit_raw(serve.SOLVE, g, precision, rhs=FAKE, sol=FAKE + 8, timeout_ms=timeout_ms)


def extend(srv, g, precision="fp64"):
    ext = {n: FAKE for n in ("u", "v", "w", "src", "ue", "ve", "we", "phi")}
    return srv.submit_raw(serve.EXTEND, g, precision, ext=ext)


def wait_all(srv, tickets, timeout_ms=20000):
    out = []
    for t in tickets:
        r = srv.wait(t, timeout_ms)
        assert r is not None, f"ticket {t} did not end"
        out.append(r)
    return out


BIG = 1 << 40


def wait_running(srv, n, timeout=5.0):
    """Wait until n batches are in flight (the scheduler thread is asynchronous)."""
    t0 = time.perf_counter()
    while srv.stats()["running"] < n:
        assert time.perf_counter() - t0 < timeout
        time.sleep(0.0005)


def test_all_requests_complete_and_stats_add_up():
    with Server(BIG, lanes=2, max_batch=4, dry_run=True, dry_run_us=200) as srv:
        g1, g2 = grid(), grid(64, 64, 16, "NPN")
        ts = [solve(srv, g1) for _ in range(6)] + [extend(srv, g2) for _ in range(5)]
        res = wait_all(srv, ts)
        assert all(r["status"] == 0 for r in res)
        assert all(r["t_submit_us"] <= r["t_dispatch_us"] <= r["t_done_us"] for r in res)
        assert srv.drain(5000)
        st = srv.stats()
        assert st["submitted"] == 11 and st["completed"] == 11 and st["failed"] == 0
        assert st["batched_requests"] == 11 and 1 <= st["batches"] <= 11
        assert st["plans_resident"] == st["plans_created"] >= 2
        assert st["pending"] == 0 and st["running"] == 0


def test_requests_arriving_while_busy_join_one_batch():
    """One lane with two batches in flight: the next requests queue and leave
    together in one batch of up to max_batch members (continuous batching)."""
    with Server(BIG, lanes=1, max_batch=8, dry_run=True, dry_run_us=50000) as srv:
        g = grid()
        first = [solve(srv, g)]
        wait_running(srv, 1)
        second = [solve(srv, g)]
        wait_running(srv, 2)
        rest = [solve(srv, g) for _ in range(10)]
        res = wait_all(srv, first + second + rest)
        assert res[0]["batch"] == 1 and res[1]["batch"] == 1
        sizes = sorted({(r["t_dispatch_us"], r["batch"]) for r in res[2:]})
        assert [b for _, b in sizes] == [8, 2]
        # same class, one lane: first in, first out
        done = [r["t_done_us"] for r in res]
        assert done == sorted(done)


def test_kinds_and_precisions_are_batched_separately():
    with Server(BIG, lanes=1, max_batch=16, dry_run=True, dry_run_us=30000) as srv:
        g = grid()
        block = [solve(srv, g)]  # occupy the lane
        wait_running(srv, 1)
        block.append(solve(srv, g))
        wait_running(srv, 2)
        a = [solve(srv, g) for _ in range(3)]
        b = [extend(srv, g) for _ in range(3)]
        c = [solve(srv, g, "mixed") for _ in range(3)]
        res = wait_all(srv, block + a + b + c)
        for grp in (res[2:5], res[5:8], res[8:11]):
            assert {r["batch"] for r in grp} == {3}
            assert len({r["t_dispatch_us"] for r in grp}) == 1


def test_admission_by_plan_footprint_evicts_idle_plans():
    # three classes of (nearly) the same footprint
    g1, g2, g3 = grid(64, 64, 32), grid(64, 64, 32, "NNN"), grid(64, 32, 64, "PPP")
    mb = 2
    f = [footprint(g.nx, g.ny, g.nz, "fp64", mb) for g in (g1, g2, g3)]
    budget = max(f) + min(f) // 2  # room for one plan at a time
    with Server(budget, lanes=2, max_batch=mb, dry_run=True, dry_run_us=500) as srv:
        ts = []
        for k in range(12):
            ts.append(solve(srv, (g1, g2, g3)[k % 3]))
        res = wait_all(srv, ts)
        assert all(r["status"] == 0 for r in res)
        st = srv.stats()
        assert st["bytes_peak"] <= budget
        assert st["plans_resident"] <= 1
        assert st["plans_evicted"] >= 2


def test_too_big_and_unsupported_rejected_at_submit():
    g = grid(64, 64, 64)
    with Server(footprint(64, 64, 64, "fp64", 4) - 1, lanes=1, max_batch=4, dry_run=True) as srv:
        with pytest.raises(ServeError) as e:
            solve(srv, g)
        assert e.value.status == serve.VP_ETOOBIG
        with pytest.raises(ServeError) as e:
            solve(srv, grid(36, 32, 8))
        assert e.value.status == -2
        with pytest.raises(ServeError) as e:
            srv.submit_raw(serve.SOLVE, grid(), rhs=0, sol=FAKE)  # no rhs
        assert e.value.status == -1
        with pytest.raises(ServeError) as e:  # mixed extension needs a phi buffer
            ext = {n: FAKE for n in ("u", "v", "w", "src", "ue", "ve", "we")}
            srv.submit_raw(serve.EXTEND, grid(), "mixed", ext=ext)
        assert e.value.status == -1
        assert srv.stats()["rejected"] == 4
        # the loop still serves
        assert wait_all(srv, [solve(srv, grid())])[0]["status"] == 0


def test_queue_bound_returns_eagain():
    with Server(BIG, lanes=1, max_batch=1, max_pending=2, dry_run=True, dry_run_us=300000) as srv:
        g = grid()
        accepted, refused = [solve(srv, g)], 0
        wait_running(srv, 1)
        accepted.append(solve(srv, g))
        wait_running(srv, 2)
        for _ in range(8):
            try:
                accepted.append(solve(srv, g))
            except ServeError as e:
                assert e.status == serve.VP_EAGAIN
                refused += 1
        # two batches in flight on the lane plus two queued
        assert len(accepted) == 4 and refused == 6
        for t in accepted[2:]:
            srv.cancel(t)
        res = wait_all(srv, accepted)
        assert [r["status"] for r in res[2:]] == [serve.VP_ECANCELED] * 2


def test_cancel_and_queue_timeout():
    with Server(BIG, lanes=1, max_batch=1, dry_run=True, dry_run_us=100000) as srv:
        g = grid()
        busy = [solve(srv, g)]
        wait_running(srv, 1)
        busy.append(solve(srv, g))
        wait_running(srv, 2)
        c = solve(srv, g)
        t = solve(srv, g, timeout_ms=20)
        srv.cancel(c)
        rc, rt = srv.wait(c, 5000), srv.wait(t, 5000)
        assert rc["status"] == serve.VP_ECANCELED and rc["batch"] == 0 and rc["lane"] == -1
        assert rt["status"] == serve.VP_ETIMEDOUT
        assert rt["t_done_us"] - rt["t_submit_us"] >= 20000
        assert all(r["status"] == 0 for r in wait_all(srv, busy))
        st = srv.stats()
        assert st["cancelled"] == 1 and st["timed_out"] == 1
        with pytest.raises(ServeError):
            srv.cancel(c)  # released ticket


def test_injected_launch_fault_fails_one_batch_and_serving_continues():
    with Server(BIG, lanes=1, max_batch=4, dry_run=True, dry_run_us=1000) as srv:
        g = grid()
        srv.inject(serve.FAULT_LAUNCH, 1)
        bad = srv.wait(solve(srv, g), 5000)
        assert bad["status"] == -4
        good = wait_all(srv, [solve(srv, g) for _ in range(3)])
        assert all(r["status"] == 0 for r in good)
        assert srv.stats()["failed"] == 1


def test_injected_plan_fault():
    with Server(BIG, lanes=1, max_batch=2, dry_run=True, dry_run_us=1000) as srv:
        g1, g2 = grid(), grid(16, 16, 16)
        wait_all(srv, [solve(srv, g1)])
        # one failure: idle plans are evicted and the creation is retried
        srv.inject(serve.FAULT_PLAN, 1)
        r = srv.wait(solve(srv, g2), 5000)
        assert r["status"] == 0
        st = srv.stats()
        assert st["plans_evicted"] == 1 and st["plans_resident"] == 1
        # two failures in a row: the class's requests end with VP_ENOMEM
        srv.inject(serve.FAULT_PLAN, 2)
        r = srv.wait(solve(srv, g1), 5000)
        assert r["status"] == -3
        assert wait_all(srv, [solve(srv, g1)])[0]["status"] == 0


def test_destroy_drains_queued_work():
    srv = Server(BIG, lanes=1, max_batch=2, dry_run=True, dry_run_us=2000)
    for _ in range(6):
        solve(srv, grid())
    t0 = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t0 >= 0.004  # 3 batches of 2 at 2 ms


def test_bad_configurations():
    for kw in ({"hbm_budget": 0}, {"lanes": 0}, {"lanes": 9}, {"max_batch": 17},
               {"max_pending": 0}):
        args = {"hbm_budget": BIG, "lanes": 1, "max_batch": 1, "max_pending": 8}
        args.update(kw)
        with pytest.raises(ServeError):
            Server(args.pop("hbm_budget"), dry_run=True, **args)


def test_prewarm_makes_plans_resident():
    g = grid()
    with Server(BIG, lanes=3, max_batch=4, dry_run=True, dry_run_us=100) as srv:
        assert srv.prewarm(g, "fp64", instances=3) == 3
        assert srv.prewarm(g, "fp64", instances=2) == 0  # already there
        assert srv.prewarm(g, "mixed", instances=1) == 1
        st = srv.stats()
        assert st["plans_created"] == 4 and st["plans_resident"] == 4
        with pytest.raises(ServeError) as e:
            srv.prewarm(g, instances=4)  # more than lanes
        assert e.value.status == -1
        # traffic finds them: no plan is created while serving
        wait_all(srv, [solve(srv, g) for _ in range(12)])
        assert srv.stats()["plans_created"] == 4
    one = footprint(32, 32, 32, "fp64", 4)
    with Server(2 * one + one // 2, lanes=3, max_batch=4, dry_run=True) as srv:
        with pytest.raises(ServeError) as e:
            srv.prewarm(g, instances=3)
        assert e.value.status == serve.VP_ETOOBIG


def test_new_instance_only_for_a_backlog():
    """With the class's only plan busy on a full lane, one queued request waits
    for that lane; half a batch of them gets a second instance on a free lane."""
    g = grid()
    with Server(BIG, lanes=2, max_batch=4, dry_run=True, dry_run_us=100000) as srv:
        ts = [solve(srv, g)]
        wait_running(srv, 1)
        ts.append(solve(srv, g))
        wait_running(srv, 2)  # both on the plan's lane (depth 2)
        ts.append(solve(srv, g))
        time.sleep(0.02)
        st = srv.stats()
        assert st["plans_created"] == 1 and st["running"] == 2 and st["pending"] == 1
        ts.append(solve(srv, g))  # backlog of 2 = max_batch / 2
        wait_running(srv, 3)
        assert srv.stats()["plans_created"] == 2
        res = wait_all(srv, ts)
        assert sorted({r["lane"] for r in res}) == [0, 1]
