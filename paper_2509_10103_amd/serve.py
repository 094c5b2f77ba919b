"""Serving loop: continuous batching of optimisation jobs on one GPU.

Requests (a job configuration and a number of optimisation iterations)
arrive at any time.  A job is admitted when its HBM footprint (checkpoint
arena + workspace + operator caches + its fields) fits the free budget and a
slot is free; admitted jobs keep their state resident and are advanced one
iteration at a time by a pool of worker threads, each job on its own HIP
stream, so the work of jobs admitted at different times overlaps on the
device (a new job joins at the next iteration boundary, a finished job frees
its slot and memory at once).  Each iteration's wall latency and each job's
queue wait are recorded.  A job whose gain becomes non-finite or whose calls
fail is retired with an error; the others continue.

The job factory is pluggable so that the scheduling can be exercised without
a GPU.
"""
import heapq
import math
import threading
import time

import numpy as np


def estimate_workspace(cfg):
    """Upper bound of a plan's workspace bytes: about 23 state fields (stage
    iterates and their vorticity parts, nonlinear terms, adjoint temporaries,
    run state) plus 15 axially transformed scalar fields and 6 more per
    corrector pass, each rounded up to 256 bytes."""
    nr, nt, nz = cfg["nr"], cfg["nt"], cfg["nz"]
    M, K = (nt - 1) // 3, (nz - 1) // 3
    f = 3 * nr * (M + 1) * (2 * K + 1) * 16
    g = nr * (M + 1) * nz * 16
    return 24 * f + (15 + 6 * cfg.get("ncorr", 2)) * g + 64 * 256 + 64 * 1024


def estimate_footprint(cfg):
    """Device bytes of one job: arena + workspace + operator caches + 2 fields."""
    nr, nt, nz = cfg["nr"], cfg["nt"], cfg["nz"]
    M, K = (nt - 1) // 3, (nz - 1) // 3
    f = 3 * nr * (M + 1) * (2 * K + 1) * 16
    cache = (K + 1) * ((M + 2) + (M + 1)) * (nr - 1) * 9 * 8 + (K + 1) * (M + 1) * (3 * nr + 1) * 8
    n_ckpt = max(1, min(cfg.get("n_ckpt") or cfg["nsteps"], cfg["nsteps"]))
    return n_ckpt * f + estimate_workspace(cfg) + cache + 2 * f


class Job:
    def __init__(self, jid, cfg, iters, arrival):
        self.id = jid
        self.cfg = cfg
        self.iters = iters
        self.arrival = arrival
        self.admitted = None
        self.finished = None
        self.done_iters = 0
        self.latencies = []
        self.error = None
        self.result = None
        self.footprint = estimate_footprint(cfg)
        self.runner = None
        self.busy = False
        self.counted = 0


class Server:
    """Admission by footprint, iteration-granular continuous batching."""

    def __init__(self, hbm_budget, max_active=16, workers=8, factory=None, log=None):
        self.budget = hbm_budget
        self.max_active = max_active
        self.workers = workers
        self.factory = factory or gpu_factory
        self.log = log             # called with one line per admitted or finished job
        self.lock = threading.Condition()
        self.pending = []          # heap of (arrival, id, job)
        self.active = []
        self.done = []
        self.used = 0
        self.closed = False
        self.halted = False
        self.next_id = 0
        self.iters_done = 0
        self._threads = []

    # ------------------------------------------------------------ client side
    def submit(self, cfg, iters, arrival=None):
        with self.lock:
            j = Job(self.next_id, cfg, iters, time.perf_counter() if arrival is None else arrival)
            self.next_id += 1
            if j.footprint > self.budget:
                j.error = f"footprint {j.footprint / 1e9:.1f} GB exceeds the budget {self.budget / 1e9:.1f} GB"
                j.finished = j.arrival
                self.done.append(j)
            else:
                heapq.heappush(self.pending, (j.arrival, j.id, j))
            self.lock.notify_all()
            return j

    def close(self):
        with self.lock:
            self.closed = True
            self.lock.notify_all()

    def halt(self):
        """Stop at the next iteration boundary: nothing more is admitted, and
        active jobs are released after their current iteration (they stay
        unfinished in the report)."""
        with self.lock:
            self.closed = True
            self.halted = True
            self.lock.notify_all()

    # ------------------------------------------------------------ scheduling
    def _admit_locked(self):
        while self.pending and len(self.active) < self.max_active:
            _, _, j = self.pending[0]
            if self.used + j.footprint > self.budget:
                break                  # first-come first-served: do not overtake
            heapq.heappop(self.pending)
            self.used += j.footprint
            j.admitted = time.perf_counter()
            self.active.append(j)
            if self.log:
                self.log(f"[serve] job {j.id} admitted ({j.cfg['nr']}x{j.cfg['nt']}x{j.cfg['nz']}, "
                         f"{j.footprint / 1e9:.2f} GB), {len(self.active)} active")

    def _retire_locked(self, j):
        self.active.remove(j)
        self.used -= j.footprint
        j.finished = time.perf_counter()
        self.done.append(j)
        if self.log:
            self.log(f"[serve] job {j.id} {'failed: ' + j.error if j.error else 'done'} after {j.done_iters} "
                     f"iterations, {len(self.done)} finished, {len(self.active)} active, {len(self.pending)} queued")
        self._admit_locked()
        self.lock.notify_all()

    def _next_locked(self):
        """Least-advanced idle active job (round-robin at iteration granularity)."""
        cands = [j for j in self.active if not j.busy]
        if not cands:
            return None
        j = min(cands, key=lambda x: (x.done_iters, x.admitted, x.id))
        j.busy = True
        return j

    def _worker(self):
        while True:
            with self.lock:
                if self.halted:
                    self._release_idle_locked()
                    return
                self._admit_locked()
                j = self._next_locked()
                while j is None:
                    if self.closed and not self.pending and not self.active:
                        return
                    if self.halted:
                        self._release_idle_locked()
                        return
                    self.lock.wait(timeout=0.05)
                    self._admit_locked()
                    j = self._next_locked()
            try:
                if j.runner is None:
                    j.runner = self.factory(j.cfg)
                st, dt, counted = j.runner.iterate()
                ok = st is None or math.isfinite(st.get("G_new", 0.0))
                with self.lock:
                    j.latencies.append(dt)
                    j.counted += counted
                    j.done_iters += 1
                    self.iters_done += 1
                    if self.log and self.iters_done % 20 == 0:
                        self.log(f"[serve] {self.iters_done} iterations done, {len(self.done)} jobs finished")
                    if not ok:
                        j.error = "non-finite gain"
                    finished = j.done_iters >= j.iters or j.error is not None
                    if finished:
                        j.result = j.runner.state() if j.error is None else None
                        j.runner.release()
                        j.runner = None
                    j.busy = False
                    if finished:
                        self._retire_locked(j)
            except Exception as e:       # isolate the failing job
                with self.lock:
                    j.error = repr(e)
                    try:
                        if j.runner is not None:
                            j.runner.release()
                    except Exception:
                        pass
                    j.runner = None
                    j.busy = False
                    self._retire_locked(j)

    def _release_idle_locked(self):
        for j in list(self.active):
            if not j.busy and j.runner is not None:
                j.runner.release()
                j.runner = None

    def start(self):
        for _ in range(self.workers):
            t = threading.Thread(target=self._worker, daemon=True)
            t.start()
            self._threads.append(t)

    def join(self):
        self.close()
        for t in self._threads:
            t.join()

    # ------------------------------------------------------------ reporting
    def report(self, t_start, t_end):
        jobs = self.done + self.active
        lat = [x for j in jobs for x in j.latencies]
        waits = [j.admitted - j.arrival for j in jobs if j.admitted is not None]
        counted = sum(j.counted for j in jobs)
        a = np.asarray(lat) if lat else np.zeros(1)
        w = np.asarray(waits) if waits else np.zeros(1)
        still = [t_end - j.arrival for _, _, j in self.pending]
        return {
            "jobs": len(self.done), "failed": sum(1 for j in self.done if j.error),
            "unfinished_admitted": len(self.active), "never_admitted": len(self.pending),
            "iterations": len(lat),
            "iteration_latency_s": {"p50": float(np.percentile(a, 50)), "p99": float(np.percentile(a, 99))},
            "queue_wait_s": {"p50": float(np.percentile(w, 50)), "p99": float(np.percentile(w, 99))},
            "wait_of_never_admitted_s": {"p50": float(np.percentile(still, 50)) if still else 0.0,
                                         "max": float(max(still)) if still else 0.0},
            "gp_steps_per_s": counted / max(t_end - t_start, 1e-9),
            "wall_s": t_end - t_start,
        }


def gpu_factory(cfg):
    from .batch import Instance
    return Instance(cfg)


def poisson_arrivals(n, rate, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def replay(server, cfgs, iters, arrivals, budget=None):
    """Submit cfgs at the given arrival offsets (seconds) and wait for all, or
    halt the server after `budget` seconds (then the report counts what was
    done, what is unfinished and what never got in)."""
    t0 = time.perf_counter()
    server.start()
    jobs = []
    for c, a in zip(cfgs, arrivals):
        now = time.perf_counter() - t0
        if budget is not None and a > budget:
            break
        if a > now:
            time.sleep(a - now)
        jobs.append(server.submit(c, iters, arrival=time.perf_counter()))
    if budget is not None:
        left = budget - (time.perf_counter() - t0)
        done = threading.Event()

        def waiter():
            server.join()
            done.set()
        th = threading.Thread(target=waiter, daemon=True)
        th.start()
        if not done.wait(timeout=max(left, 0.0)):
            server.halt()
            th.join()
    else:
        server.join()
    return jobs, server.report(t0, time.perf_counter())
