"""Host-side logic of the hologram server (cgh_server_*), run in its simulation mode: no device
work, each job occupies its slot for sim_ns_per_pixel * nx * ny.  Admission order, the memory
budget, timeouts, cancellation, release and shutdown are the same code as on the GPU."""
import threading
import time

import numpy as np
import pytest

import paper_1708_04233_amd as cgh

NS = 2.0  # simulated ns per pixel: a 1024^2 job runs ~2 ms


@pytest.fixture
def lib():
    return cgh.load()


def server(budget, slots=4, ns=NS):
    return cgh.Server(None, budget, max_slots=slots, simulate=True, sim_ns_per_pixel=ns)


def pts(n):
    return np.zeros((n, 4))


def result_bytes(side):
    return 8 * side * side


def work_bytes(n):
    """Arena bytes of a job without a LUT: device points + quantised points, 256-byte granules."""
    r = lambda b: (b + 255) // 256 * 256
    return r(32 * n) + r(16 * n)


def test_all_jobs_complete_with_ordered_times(lib):
    with server(1 << 40) as s:
        tickets = [s.submit(pts(10 * i), 256 * (1 + i % 3), 256) for i in range(12)]
        for t in tickets:
            r = s.wait(t, 5000)
            assert r["status"] == cgh.CGH_OK
            assert r["u"] is None
            assert 0 <= r["t_submit"] <= r["t_admit"] <= r["t_start"] <= r["t_done"]
            assert 0 <= r["slot"] < 4
            s.release(t)
        st = s.stats()
        assert st["submitted"] == 12 and st["completed"] == 12 and st["canceled"] == 0
        assert st["queued"] == 0 and st["running"] == 0
        assert st["bytes_in_use"] == st["arena_bytes"] > 0      # only the slots' arenas remain
        assert 1 <= st["max_running"] <= 4


def test_slots_bound_concurrency_and_jobs_overlap(lib):
    with server(1 << 40, slots=3) as s:
        tickets = [s.submit(None, 1024, 1024) for _ in range(9)]
        res = [s.wait(t, 5000) for t in tickets]
        st = s.stats()
        assert st["max_running"] == 3
        # continuous batching: a job is admitted while others still run
        overlaps = sum(1 for a in res for b in res if a is not b and b["t_admit"] < a["t_done"] and b["t_admit"] > a["t_admit"])
        assert overlaps > 0
        for t in tickets:
            s.release(t)


def test_budget_limits_admission_in_fifo_order(lib):
    side = 1024
    job = result_bytes(side) + work_bytes(100)
    budget = 2 * job + job // 2          # room for two jobs at once
    with server(budget, slots=8) as s:
        tickets = [s.submit(pts(100), side, side) for _ in range(6)]
        res = []
        for t in tickets:
            res.append(s.wait(t, 5000))
            s.release(t)                 # give the result back so the next jobs fit
        st = s.stats()
        assert st["max_running"] <= 2
        assert st["peak_bytes"] <= budget
        admits = [r["t_admit"] for r in res]
        assert admits == sorted(admits)  # strictly in submission order


def test_results_stay_charged_until_release(lib):
    side = 512
    with server(1 << 40) as s:
        t = s.submit(pts(7), side, side)
        s.wait(t, 5000)
        st = s.stats()
        assert st["arena_bytes"] == work_bytes(7)
        assert st["bytes_in_use"] == result_bytes(side) + work_bytes(7)
        s.release(t)
        assert s.stats()["bytes_in_use"] == work_bytes(7)      # the slot keeps its arena


def test_unreleased_results_block_admission(lib):
    side = 1024
    budget = result_bytes(side) + work_bytes(0) + 1000
    with server(budget, slots=2) as s:
        a = s.submit(None, side, side)
        b = s.submit(None, side, side)
        assert s.wait(a, 5000)["status"] == cgh.CGH_OK
        with pytest.raises(cgh.CghError) as e:   # b cannot start: a's result holds the budget
            s.wait(b, 100)
        assert e.value.code == cgh.CGH_ETIMEDOUT
        s.release(a)
        assert s.wait(b, 5000)["status"] == cgh.CGH_OK
        s.release(b)


def test_idle_arenas_give_way(lib):
    """A job that fits only if idle slots give back their arenas is admitted after they do."""
    big = work_bytes(400_000)                          # 19.2 MB arena
    budget = 2 * result_bytes(64) + big + 4096         # one arena of `big`, two results
    with server(budget, slots=2) as s:
        a = s.submit(pts(400_000), 64, 64)             # slot 0 grows to `big`
        s.wait(a, 5000)
        s.release(a)
        b = s.submit(pts(10), 64, 64)                  # reuses slot 0's arena
        s.wait(b, 5000)
        s.release(b)
        assert s.stats()["arena_bytes"] == big
        t1 = s.submit(pts(400_000), 64, 64)
        t2 = s.submit(pts(400_000), 64, 64)            # needs slot 0's arena: runs after t1
        r1, r2 = s.wait(t1, 5000), s.wait(t2, 5000)
        assert r2["t_admit"] >= r1["t_done"]
        assert s.stats()["peak_bytes"] <= budget
        s.release(t1)
        s.release(t2)


def test_idle_arena_dropped_to_admit(lib):
    """An idle slot gives its arena back when a larger job needs the room."""
    big, bigger = work_bytes(400_000), work_bytes(600_000)
    budget = 2 * big + 2 * result_bytes(64) + 4096
    with server(budget, slots=2, ns=10_000.0) as s:        # 64^2 -> ~40 ms: a and b overlap
        a, b = s.submit(pts(400_000), 64, 64), s.submit(pts(400_000), 64, 64)
        s.wait(a, 5000)
        s.wait(b, 5000)
        s.release(a)
        s.release(b)
        assert s.stats()["arena_bytes"] == 2 * big         # both slots grew
        c = s.submit(pts(600_000), 64, 64)                 # fits only without the other arena
        assert s.wait(c, 5000)["status"] == cgh.CGH_OK
        st = s.stats()
        assert st["arena_bytes"] == bigger and st["peak_bytes"] <= budget
        s.release(c)


def test_oversized_job_rejected(lib):
    with server(result_bytes(1024)) as s:
        with pytest.raises(cgh.CghError) as e:
            s.submit(pts(10), 1024, 1024)        # result + working memory > budget
        assert e.value.code == cgh.CGH_ENOMEM
        assert s.stats()["submitted"] == 0


@pytest.mark.parametrize("nx,ny", [(0, 64), (64, 0), (100, 64), (64, 65536 + 8), (-8, 64)])
def test_bad_sizes_rejected(lib, nx, ny):
    with server(1 << 40) as s:
        with pytest.raises(cgh.CghError) as e:
            s.submit(pts(1), nx, ny)
        assert e.value.code == cgh.CGH_EINVAL


def test_bad_config_rejected(lib):
    for kw in (dict(hbm_budget_bytes=0), dict(max_slots=0), dict(max_slots=65)):
        args = dict(hbm_budget_bytes=1 << 30, max_slots=2)
        args.update(kw)
        with pytest.raises(cgh.CghError) as e:
            cgh.Server(None, args["hbm_budget_bytes"], max_slots=args["max_slots"], simulate=True)
        assert e.value.code == cgh.CGH_EINVAL
    with pytest.raises(cgh.CghError) as e:      # a real server needs a LUT
        cgh.Server(None, 1 << 30)
    assert e.value.code == cgh.CGH_EINVAL


def test_wait_timeout_then_success(lib):
    with server(1 << 40, ns=200.0) as s:         # 1024^2 -> ~210 ms
        t = s.submit(None, 1024, 1024)
        with pytest.raises(cgh.CghError) as e:
            s.wait(t, 10)
        assert e.value.code == cgh.CGH_ETIMEDOUT
        with pytest.raises(cgh.CghError) as e:
            s.release(t)                          # not ended yet
        assert e.value.code == cgh.CGH_EAGAIN
        assert s.wait(t, 5000)["status"] == cgh.CGH_OK
        s.release(t)


def test_unknown_and_released_tickets(lib):
    with server(1 << 40) as s:
        for call in (lambda: s.wait(12345, 0), lambda: s.cancel(12345), lambda: s.release(12345)):
            with pytest.raises(cgh.CghError) as e:
                call()
            assert e.value.code == cgh.CGH_ENOTFOUND
        t = s.submit(None, 64, 64)
        s.wait(t, 5000)
        s.release(t)
        with pytest.raises(cgh.CghError) as e:
            s.release(t)
        assert e.value.code == cgh.CGH_ENOTFOUND


def test_cancel_queued_and_running(lib):
    with server(1 << 40, slots=1, ns=100.0) as s:    # one slot: the second job waits in the queue
        a = s.submit(None, 1024, 1024)
        b = s.submit(None, 1024, 1024)
        s.cancel(b)
        rb = s.wait(b, 0)
        assert rb["status"] == cgh.CGH_ECANCELED and rb["slot"] == -1
        s.cancel(a)                                   # running: ends when its work ends
        ra = s.wait(a, 5000)
        assert ra["status"] == cgh.CGH_ECANCELED
        with pytest.raises(cgh.CghError) as e:
            s.cancel(a)                               # already ended
        assert e.value.code == cgh.CGH_EINVAL
        st = s.stats()
        assert st["canceled"] == 2 and st["bytes_in_use"] == 0
        s.release(a)
        s.release(b)


def test_destroy_cancels_queue_and_wakes_waiters(lib):
    s = server(1 << 40, slots=1, ns=100.0)
    tickets = [s.submit(None, 1024, 1024) for _ in range(4)]
    out = {}

    def waiter():
        try:
            out["r"] = s.wait(tickets[-1], -1)
        except cgh.CghError as e:
            out["err"] = e.code

    th = threading.Thread(target=waiter)
    th.start()
    time.sleep(0.02)
    s.close()
    th.join(5)
    assert not th.is_alive()
    # the last job was still queued: it ends cancelled (seen either as its result or as a
    # cancelled wait, depending on which the waiter saw first)
    assert out.get("err") == cgh.CGH_ECANCELED or out["r"]["status"] == cgh.CGH_ECANCELED


def test_submit_from_many_threads(lib):
    with server(1 << 40, slots=4, ns=0.5) as s:
        tickets = []
        lock = threading.Lock()

        def producer(k):
            for i in range(25):
                t = s.submit(pts(i), 64 * (1 + (i + k) % 4), 64)
                with lock:
                    tickets.append(t)

        ths = [threading.Thread(target=producer, args=(k,)) for k in range(4)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        assert len(set(tickets)) == 100
        for t in tickets:
            assert s.wait(t, 10000)["status"] == cgh.CGH_OK
            s.release(t)
        st = s.stats()
        assert st["completed"] == 100 and st["bytes_in_use"] == st["arena_bytes"]


def test_forced_issue_failure_spares_other_jobs(lib):
    """A job whose issue fails (forced with fail_ticket) ends with CGH_EHIP holding no memory; the
    jobs queued before and after it complete, and every byte comes back once they are released."""
    with cgh.Server(None, 1 << 40, max_slots=2, simulate=True, sim_ns_per_pixel=NS, fail_ticket=3) as s:
        tickets = [s.submit(pts(100), 512, 512) for _ in range(6)]
        assert tickets[2] == 3
        res = [s.wait(t, 5000) for t in tickets]
        assert res[2]["status"] == cgh.CGH_EHIP and res[2]["u"] is None
        assert all(r["status"] == cgh.CGH_OK for i, r in enumerate(res) if i != 2)
        st = s.stats()
        assert st["failed"] == 1 and st["completed"] == 5 and st["running"] == 0
        # the failed job gave its result memory back at once; the others hold theirs until released
        assert st["bytes_in_use"] == st["arena_bytes"] + 5 * result_bytes(512)
        for t in tickets:
            s.release(t)
        st = s.stats()
        assert st["bytes_in_use"] == st["arena_bytes"]
