"""Batched optimisation instances of uneven size on one GPU.

Two ways of running many instances:

* ``LockstepBatch``: the instances' checkpointed sweeps advance in lockstep
  through the library's batched launches (npo_batch_*): every kernel of a
  step is launched once per shape class for all of its instances, each block
  reading its instance's constants, buffers and evaluation time from a device
  work-descriptor table, and each batched step is one replay of a captured
  graph.  The instances share the horizon and the number of checkpoint slots
  (one schedule).
* ``Batch``: each instance owns a plan, workspace, arena and HIP stream and
  runs whole optimisation iterations (Sec. 2.1-2.2) on its own host thread
  (the library calls release the GIL), its sweeps replaying captured step
  graphs, so the kernels of small instances overlap on the device.

Launch shapes come from the autotuner, cached per grid shape.  Results are
bitwise those of the same instance run alone: each instance's arithmetic and
launch order are fixed.
"""
import threading
import time

import numpy as np

from . import npo, synth, tune as tuner


class Instance:
    def __init__(self, cfg, device="cuda", autotune=True, graphs=True):
        import torch
        self.cfg = cfg
        self.stream = torch.cuda.Stream(device=device)
        with torch.cuda.stream(self.stream):
            self.plan = npo.Plan(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"],
                                 cfg["dt"], cfg["t0"], cfg["nsteps"], cfg.get("ncorr", 2), device=device)
            if autotune:
                tuner.tune(self.plan, cfg["nr"], cfg["nt"], cfg["nz"])
            # sweeps replay captured step graphs: one launch per step instead
            # of one per kernel (small instances are launch-bound)
            npo.npo_plan_set_graphs(self.plan.handle, int(graphs))
            self.n_ckpt = int(max(1, min(cfg["n_ckpt"] or cfg["nsteps"], cfg["nsteps"])))
            self.arena = self.plan.arena(self.n_ckpt)
            r = npo.npo_plan_tables(self.plan.handle, cfg["nr"])[0]
            raw = synth.solenoidal_modes(r, self.plan.M, self.plan.K, cfg["lz"], cfg["seed"])
            self.u0 = torch.from_numpy(np.ascontiguousarray(raw)).to(device)
            npo.npo_project(self.plan.handle, self.plan.ws, self.u0, self.u0, stream=self.stream.cuda_stream)
            npo.npo_normalize(self.plan.handle, self.plan.ws, self.u0, cfg["e0"], stream=self.stream.cuda_stream)
            self.uN = self.plan.field()
        self.swept = False
        self.history = []
        self.points = cfg["nr"] * cfg["nt"] * cfg["nz"]

    def footprint(self):
        """Device bytes held by this instance (arena, workspace, u0, uN)."""
        return self.arena.numel() * 16 + self.plan.ws.numel() + 2 * self.u0.numel() * 16

    def release(self):
        self.stream.synchronize()
        self.plan.close()
        self.arena = self.u0 = self.uN = None

    def forward(self):
        npo.npo_forward_run(self.plan.handle, self.plan.ws, self.arena, self.n_ckpt, self.u0, self.uN,
                            stream=self.stream.cuda_stream)
        self.swept = True

    def iterate(self):
        """One optimisation iteration; returns (stats, seconds, counted grid-point-steps)."""
        t = time.perf_counter()
        if not self.swept:
            self.forward()
        st = npo.npo_iterate(self.plan.handle, self.plan.ws, self.arena, self.n_ckpt, self.u0, self.uN,
                             self.cfg["e0"], stream=self.stream.cuda_stream)
        if not st["accepted"]:
            self.swept = False
        self.stream.synchronize()
        dt = time.perf_counter() - t
        self.history.append((st, dt))
        return st, dt, 2 * self.cfg["nsteps"] * self.points

    def state(self):
        self.stream.synchronize()
        return self.u0.detach().clone(), self.uN.detach().clone()


class Batch:
    def __init__(self, cfgs, device="cuda", autotune=True, graphs=True):
        self.instances = [Instance(c, device, autotune, graphs) for c in cfgs]

    def run(self, iters=1, workers=None):
        """Advance every instance by ``iters`` iterations concurrently.

        Returns (wall seconds, counted grid-point-steps, per-iteration latencies)."""
        import torch
        n = len(self.instances)
        workers = workers or min(n, 16)
        groups = [self.instances[i::workers] for i in range(workers)]
        lat = []
        counted = [0]
        lock = threading.Lock()
        errors = []

        def work(group):
            try:
                for _ in range(iters):
                    for inst in group:
                        _, dt, c = inst.iterate()
                        with lock:
                            lat.append(dt)
                            counted[0] += c
            except Exception as e:      # surfaced to the caller below
                errors.append(e)

        torch.cuda.synchronize()
        t = time.perf_counter()
        threads = [threading.Thread(target=work, args=(g,)) for g in groups]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        if errors:
            raise errors[0]
        return wall, counted[0], lat

    def run_sequential(self, iters=1):
        """The plain single-instance solver on the same instances, one after another."""
        import torch
        torch.cuda.synchronize()
        t = time.perf_counter()
        counted = 0
        for inst in self.instances:
            for _ in range(iters):
                _, _, c = inst.iterate()
                counted += c
        torch.cuda.synchronize()
        return time.perf_counter() - t, counted


def percentiles(lat):
    a = np.asarray(lat) if len(lat) else np.zeros(1)
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


class LockstepBatch:
    """Forward and adjoint sweeps of many instances through batched launches."""

    def __init__(self, cfgs, device="cuda", autotune=True):
        import torch
        self.cfgs = cfgs
        self.nsteps = cfgs[0]["nsteps"]
        if any(c["nsteps"] != self.nsteps for c in cfgs):
            raise ValueError("lockstep instances share the horizon")
        self.n_ckpt = int(max(1, min(min(c["n_ckpt"] or c["nsteps"] for c in cfgs), self.nsteps)))
        self.plans, self.u0, self.uN, self.lam, self.arena = [], [], [], [], []
        for c in cfgs:
            G = npo.Plan(c["nr"], c["nt"], c["nz"], c["lz"], c["re"], c["wo"], c["amp"], c["dt"], c["t0"],
                         c["nsteps"], c.get("ncorr", 2), device=device)
            if autotune:
                tuner.tune(G, c["nr"], c["nt"], c["nz"], batched=True)
            r = npo.npo_plan_tables(G.handle, c["nr"])[0]
            raw = synth.solenoidal_modes(r, G.M, G.K, c["lz"], c["seed"])
            u0 = torch.from_numpy(np.ascontiguousarray(raw)).to(device)
            npo.npo_project(G.handle, G.ws, u0, u0)
            npo.npo_normalize(G.handle, G.ws, u0, c["e0"])
            self.plans.append(G)
            self.u0.append(u0)
            self.uN.append(G.field())
            self.lam.append(G.field())
            self.arena.append(G.arena(self.n_ckpt))
        self.handles = [G.handle for G in self.plans]
        self.ws = [G.ws for G in self.plans]
        self.batch = npo.npo_batch_create(self.handles)
        self.points = [c["nr"] * c["nt"] * c["nz"] for c in cfgs]

    def gradients(self):
        """One forward and one adjoint sweep of every instance (lockstep)."""
        npo.npo_batch_forward_run(self.batch, self.handles, self.ws, self.arena, self.n_ckpt, self.u0, self.uN)
        return npo.npo_batch_adjoint_run(self.batch, self.handles, self.ws, self.arena, self.n_ckpt, self.uN,
                                         self.lam)

    def gradients_sequential(self):
        """The same sweeps with the plain single-instance calls, one instance after another."""
        for G, a, u0, uN, lam in zip(self.plans, self.arena, self.u0, self.uN, self.lam):
            npo.npo_forward_run(G.handle, G.ws, a, self.n_ckpt, u0, uN)
            npo.npo_adjoint_run(G.handle, G.ws, a, self.n_ckpt, uN, lam)

    def counted(self):
        """Grid-point-steps of one gradient of every instance (a forward and an adjoint step per point)."""
        return 2 * self.nsteps * sum(self.points)

    def info(self):
        return npo.npo_batch_info(self.batch)

    def close(self):
        npo.npo_batch_destroy(self.batch)
        for G in self.plans:
            G.close()
