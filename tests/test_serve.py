"""Scheduling logic of the serving loop, exercised on the CPU with fake jobs."""
import threading
import time

import pytest

from paper_2509_10103_amd.serve import Server, estimate_footprint


class FakeRunner:
    log = []
    lock = threading.Lock()

    def __init__(self, cfg):
        self.cfg = cfg
        self.n = 0

    def iterate(self):
        if self.cfg.get("fail_at") == self.n:
            raise RuntimeError("injected failure")
        time.sleep(self.cfg.get("t", 0.01))
        self.n += 1
        with FakeRunner.lock:
            FakeRunner.log.append((self.cfg["name"], self.n))
        G = float("nan") if self.cfg.get("nan_at") == self.n else 1.0 + self.n
        return {"G_new": G}, self.cfg.get("t", 0.01), 100

    def state(self):
        return ("final", self.cfg["name"], self.n)

    def release(self):
        pass


def cfg(name, nr=32, nt=24, nz=96, n_ckpt=10, **kw):
    d = dict(name=name, nr=nr, nt=nt, nz=nz, nsteps=100, n_ckpt=n_ckpt)
    d.update(kw)
    return d


def run(server, cfgs, iters, gap=0.0):
    server.start()
    jobs = []
    for c in cfgs:
        jobs.append(server.submit(c, iters))
        time.sleep(gap)
    server.join()
    return jobs


def test_footprint_grows_with_grid_and_checkpoints():
    a = estimate_footprint(cfg("a"))
    assert estimate_footprint(cfg("b", nr=64)) > a
    assert estimate_footprint(cfg("c", n_ckpt=50)) > a


def test_all_jobs_complete_and_interleave():
    FakeRunner.log = []
    s = Server(hbm_budget=1e12, max_active=4, workers=2, factory=FakeRunner)
    jobs = run(s, [cfg(f"j{i}") for i in range(4)], iters=3)
    assert all(j.error is None and j.done_iters == 3 for j in jobs)
    assert all(j.result == ("final", j.cfg["name"], 3) for j in jobs)
    # iteration-granular round robin: no job runs all its iterations before the others start
    first_done = min(i for i, (n, k) in enumerate(FakeRunner.log) if k == 3)
    started = {n for n, k in FakeRunner.log[:first_done]}
    assert len(started) >= 2


def test_admission_respects_budget():
    fp = estimate_footprint(cfg("x"))
    s = Server(hbm_budget=2.5 * fp, max_active=8, workers=4, factory=FakeRunner)
    peak = [0]

    def watch():
        while not s.closed or s.active:
            with s.lock:
                peak[0] = max(peak[0], len(s.active))
                assert s.used <= s.budget
            time.sleep(0.002)
    w = threading.Thread(target=watch, daemon=True)
    w.start()
    jobs = run(s, [cfg(f"j{i}", t=0.02) for i in range(6)], iters=2)
    w.join(timeout=5)
    assert peak[0] <= 2
    assert all(j.error is None for j in jobs)


def test_oversized_job_is_refused_and_others_run():
    big = cfg("big", nr=64, nt=96, nz=1536, n_ckpt=100000)
    s = Server(hbm_budget=estimate_footprint(cfg("x")) * 4, factory=FakeRunner, workers=2)
    jobs = run(s, [big, cfg("ok")], iters=1)
    assert jobs[0].error and "exceeds" in jobs[0].error
    assert jobs[1].error is None and jobs[1].done_iters == 1


def test_failures_are_isolated():
    s = Server(hbm_budget=1e12, max_active=4, workers=2, factory=FakeRunner)
    jobs = run(s, [cfg("a", fail_at=1), cfg("b", nan_at=2), cfg("c")], iters=3)
    assert "injected" in jobs[0].error
    assert jobs[1].error == "non-finite gain"
    assert jobs[2].error is None and jobs[2].done_iters == 3
    rep = s.report(0.0, 1.0)
    assert rep["failed"] == 2


def test_late_arrivals_join_running_work():
    FakeRunner.log = []
    s = Server(hbm_budget=1e12, max_active=4, workers=2, factory=FakeRunner)
    jobs = run(s, [cfg("early", t=0.03), cfg("late", t=0.01)], iters=4, gap=0.05)
    e = [i for i, (n, k) in enumerate(FakeRunner.log) if n == "early"]
    l = [i for i, (n, k) in enumerate(FakeRunner.log) if n == "late"]
    assert l[0] < e[-1]       # the late job starts before the early one finishes


def test_wall_budget_halts_and_reports_unfinished_work():
    """replay(..., budget): arrivals after the budget are not submitted; at the
    budget the server stops at iteration boundaries, and the report separates
    finished jobs, admitted-but-unfinished ones and requests that never got in."""
    from paper_2509_10103_amd.serve import replay
    released = []

    class R(FakeRunner):
        def release(self):
            released.append(self.cfg["name"])

    s = Server(hbm_budget=1e15, max_active=2, workers=2, factory=R)
    cfgs = [cfg(f"b{i}", t=0.05) for i in range(8)]
    arrivals = [0.0, 0.0, 0.01, 0.02, 0.03, 0.04, 5.0, 6.0]      # the last two arrive after the budget
    t = time.perf_counter()
    jobs, rep = replay(s, cfgs, 100, arrivals, budget=0.6)
    assert time.perf_counter() - t < 2.0
    assert len(jobs) == 6
    assert rep["jobs"] == 0 and rep["unfinished_admitted"] == 2 and rep["never_admitted"] == 4
    assert rep["iterations"] > 0
    assert sorted(released) == sorted(j.cfg["name"] for j in jobs if j.admitted is not None)
