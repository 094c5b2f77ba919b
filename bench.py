"""Benchmark: adjoint-looping iterations of the NLOP hot path on one MI355X.

One benchmark step is one optimisation iteration of the paper's method
(Sec. 2.1-2.2) on the paper-like workload: adjoint sweep over one pulsation
period with binomial checkpoints (Sec. 2.4), solenoidal projection of the
gradient, and the backtracking line search whose trial forward sweeps leave
the next iterate's checkpoints in place.  The initial forward sweep is done
before the timed region.  Metric: forward + adjoint grid-point-steps per
second, counting one forward and one adjoint sweep of N_r*N_theta*N_z points
per step per iteration; recomputation and extra trial sweeps are not counted.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2509_10103_amd import configs, synth  # noqa: E402

PEAK_HBM_GBS = 8000.0
HBM_RESERVE = 6 << 30


def alg_bytes(cfg):
    """Algorithmic HBM bytes per launch of each kernel family."""
    nr, nz = cfg["nr"], cfg["nz"]
    M, K = (cfg["nt"] - 1) // 3, (cfg["nz"] - 1) // 3
    f1 = nr * (M + 1) * (2 * K + 1) * 16        # one scalar spectral field
    g1 = nr * (M + 1) * nz * 16                 # one axially transformed scalar field
    return {
        "curl": 5 * f1, "zinv_fwd": 5 * f1 + 6 * g1, "theta_fwd": 9 * g1, "zfwd_fwd": 3 * g1 + 3 * f1,
        "zinv_adj": 8 * f1 + 9 * g1, "theta_adj": 15 * g1, "zfwd_adj": 6 * g1 + 6 * f1,
        "solve_pred": 14 * f1, "solve_corr": 11 * f1, "solve_raw": 6 * f1, "solve_adj": 6 * f1,
        "solve_adj2": 15 * f1, "adj_combine": 12 * f1, "wdot": 6 * f1, "project": 6 * f1, "axpby": 9 * f1,
        "zinv_adjy": 3 * f1 + 3 * g1,
    }


def cpu_baseline(cfg, seed):
    """Time the CPU oracle on a bounded sample of the same workload: one
    forward step (predictor and corrector passes) at full size, one BLAS
    thread.  The oracle's adjoint step costs about five forward steps, so the
    sample is forward-only; one forward step counts as one grid-point-step
    per point in the metric's unit, which overstates the oracle's forward +
    adjoint rate (conservative for the GPU comparison)."""
    from threadpoolctl import threadpool_limits
    from oracle.pipe import Pipe
    with threadpool_limits(limits=1):
        P = Pipe(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"], cfg["dt"], cfg["t0"])
        P.cache_limit = 0
        u = make_raw(cfg, P.r, P.M, P.K, seed)
        u *= math.sqrt(cfg["e0"] / P.energy(u))            # the cost does not depend on the values
        t = time.perf_counter()
        P.step(u, 0)
        tf = time.perf_counter() - t
    pts = cfg["nr"] * cfg["nt"] * cfg["nz"]
    return {"value": pts / tf, "unit": "grid-point-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 forward step of the same workload at full size ({tf:.1f} s, NumPy/SciPy oracle, "
                      f"1 BLAS thread); the oracle's adjoint step (about 5x the forward step) is not in the sample"}


def start_cpu_leg(workload):
    """Run the oracle timing in a child process so that it overlaps the GPU run
    (it uses one host core; the GPU path needs one more to launch)."""
    import subprocess
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-leg", "--workload", workload],
                            stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True, cwd=ROOT)


def finish_cpu_leg(proc):
    out, _ = proc.communicate()
    if proc.returncode != 0:
        raise RuntimeError(f"CPU oracle leg failed with status {proc.returncode}")
    return json.loads(out.strip().splitlines()[-1])


def make_raw(cfg, r, M, K, seed):
    if cfg["gen"] == "oblique":
        return synth.localized_oblique(r, M, K, cfg["lz"], cfg["nz"], seed)
    return synth.solenoidal_modes(r, M, K, cfg["lz"], seed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed optimisation iterations")
    ap.add_argument("--warmup", type=int, default=0, help="untimed optimisation iterations")
    ap.add_argument("--workload", default="c2", choices=sorted(configs.WORKLOADS))
    ap.add_argument("--nsteps", type=int, default=0, help="shorter horizon (development only)")
    ap.add_argument("--ckpt", type=int, default=0, help="checkpoint slots (default: the workload's)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--stride", type=int, default=8, help="profiler sampling stride")
    ap.add_argument("--mode", default="plain", choices=["plain", "batch", "serve"],
                    help="plain: one instance (the metric); batch / serve: the systems layers")
    ap.add_argument("--batch-n", type=int, default=16, help="instances of the batched workload")
    ap.add_argument("--serve-n", type=int, default=24, help="requests of the served workload")
    ap.add_argument("--serve-iters", type=int, default=2, help="iterations per served request")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sharded design is described "
              f"in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    if args.cpu_leg:
        print(json.dumps(cpu_baseline(configs.WORKLOADS[args.workload], configs.WORKLOADS[args.workload]["seed"])))
        return
    cpu_proc = None
    if args.mode == "plain" and not args.no_cpu:
        cpu_proc = start_cpu_leg(args.workload)

    import torch
    from paper_2509_10103_amd import npo

    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "serve":
        return bench_serve(args)
    cfg = dict(configs.WORKLOADS[args.workload])
    if args.nsteps:
        cfg["nsteps"] = args.nsteps
    torch.cuda.set_device(0)
    G = npo.Plan(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"], cfg["dt"],
                 cfg["t0"], cfg["nsteps"])
    if args.ckpt:
        nck = args.ckpt
    elif cfg["n_ckpt"]:
        nck = min(cfg["n_ckpt"], cfg["nsteps"])
    else:
        # checkpoint arena sized to the free HBM after the plan and workspace,
        # keeping HBM_RESERVE for fields, tuning and the runtime
        fb = 3 * cfg["nr"] * G.shape[2] * G.shape[3] * 16
        free = torch.cuda.mem_get_info()[0]
        nck = int(max(1, min(cfg["nsteps"], (free - HBM_RESERVE) // fb)))
    from paper_2509_10103_amd import tune
    shapes, _ = tune.tune(G, cfg["nr"], cfg["nt"], cfg["nz"], use_cache=False, save=False)
    shapes = list(shapes)
    r = npo.npo_plan_tables(G.handle, cfg["nr"])[0]
    raw = make_raw(cfg, r, G.M, G.K, cfg["seed"])
    u0 = torch.from_numpy(raw).to("cuda")
    npo.npo_project(G.handle, G.ws, u0, u0)
    npo.npo_normalize(G.handle, G.ws, u0, cfg["e0"])
    arena = G.arena(nck)
    uN = G.field()
    print(f"[bench] {cfg['name']} nsteps={cfg['nsteps']} n_ckpt={nck} arena={arena.numel() * 16 / 2**30:.1f} GiB "
          f"launch shapes {shapes}",
          file=sys.stderr, flush=True)
    t = time.perf_counter()
    npo.npo_forward_run(G.handle, G.ws, arena, nck, u0, uN)
    torch.cuda.synchronize()
    print(f"[bench] initial forward sweep {time.perf_counter() - t:.2f} s", file=sys.stderr, flush=True)

    def one_iter():
        st = npo.npo_iterate(G.handle, G.ws, arena, nck, u0, uN, cfg["e0"])
        if not st["accepted"]:
            npo.npo_forward_run(G.handle, G.ws, arena, nck, u0, uN)
        return st

    for _ in range(args.warmup):
        one_iter()
    torch.cuda.synchronize()
    npo.npo_profile_begin(G.handle, args.stride)
    lat = []
    hist = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ti = time.perf_counter()
        st = one_iter()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ti)
        hist.append(st)
        print(f"[bench] iteration {i}: G {st['G_old']:.6g} -> {st['G_new']:.6g} accepted={int(st['accepted'])} "
              f"sweeps={int(st['forward_sweeps'])} {lat[-1]:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = npo.npo_profile_read(G.handle)
    pts = cfg["nr"] * cfg["nt"] * cfg["nz"]
    counted = args.steps * 2 * cfg["nsteps"] * pts
    value = counted / elapsed
    ab = alg_bytes(cfg)
    tot = {k: v["launches"] * v["avg_ms"] for k, v in prof.items()}
    dom = max(tot, key=tot.get)
    avg_s = prof[dom]["avg_ms"] * 1e-3
    achieved = ab[dom] / avg_s / 1e9 if avg_s > 0 else 0.0
    # HBM traffic of the dominant kernel from the committed counter summary
    # (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated), only while it was
    # taken on these kernel sources
    from paper_2509_10103_amd import profsum
    tr = profsum.load_traffic(os.path.join(ROOT, "profiles", f"{cfg['name']}_hbm_bytes.md"), cfg["nt"], cfg["nz"])
    traffic = tr[dom]["fetch"] + tr[dom]["write"] if tr and dom in tr else None
    kern = {k: {"launches": v["launches"], "avg_us": round(v["avg_ms"] * 1e3, 2),
                "share": round(tot[k] / max(sum(tot.values()), 1e-30), 4),
                "GBps_alg": round(ab[k] / (v["avg_ms"] * 1e-3) / 1e9, 1) if v["avg_ms"] > 0 else None}
            for k, v in prof.items() if v["launches"]}
    out = {
        "metric": "fwd+adjoint grid-point-steps/s",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": [cfg["nr"], cfg["nt"], cfg["nz"]], "lz_radii": cfg["lz"],
                   "re": cfg["re"], "wo": cfg["wo"], "amp": cfg["amp"], "dt": cfg["dt"], "t0": cfg["t0"],
                   "nsteps": cfg["nsteps"], "n_ckpt": nck, "launch_shapes": shapes, "e0": cfg["e0"], "seed": cfg["seed"],
                   "iteration_latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                   "gains": [[h["G_old"], h["G_new"], int(h["accepted"]), int(h["forward_sweeps"])] for h in hist]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": ab[dom], "avg_launch_us": avg_s * 1e6},
        "kernels": kern,
    }
    out["cpu_baseline"] = finish_cpu_leg(cpu_proc) if cpu_proc is not None else None
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Uneven instances advanced concurrently vs the plain solver run on the same
    instances one after another (iterations are the same work either way)."""
    import torch
    from paper_2509_10103_amd.batch import Batch, percentiles
    cfgs = configs.batch_instances(64)[:args.batch_n]
    if args.nsteps:
        for c in cfgs:
            c["nsteps"] = args.nsteps
            c["n_ckpt"] = min(c["n_ckpt"], args.nsteps)
    torch.cuda.set_device(0)
    b = Batch(cfgs)
    for inst in b.instances:          # initial forward sweeps (untimed, as in the plain mode)
        inst.forward()
    torch.cuda.synchronize()
    wall, counted, lat = b.run(iters=args.steps)
    print(f"[bench] batched {len(cfgs)} instances: {wall:.2f} s", file=sys.stderr, flush=True)
    for inst in b.instances:
        inst.swept = False
    seq, counted_seq = b.run_sequential(iters=args.steps)
    print(f"[bench] sequential: {seq:.2f} s", file=sys.stderr, flush=True)
    p50, p99 = percentiles(lat)
    out = {"metric": "fwd+adjoint grid-point-steps/s (batched)", "value": counted / wall,
           "unit": "grid-point-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
           "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"batch-{len(cfgs)}-uneven", "instances": len(cfgs),
                      "plain_sequential_value": counted_seq / seq, "speedup_vs_plain": (counted / wall) /
                      (counted_seq / seq), "iteration_latency_s": {"p50": p50, "p99": p99}}}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Poisson arrivals of uneven optimisation jobs; continuous batching."""
    import torch
    from paper_2509_10103_amd import serve
    from paper_2509_10103_amd.batch import Instance
    pool = configs.batch_instances(64)
    rng = np.random.default_rng(7)
    cfgs = []
    for i in range(args.serve_n):
        c = dict(pool[int(rng.integers(0, len(pool)))])
        if args.nsteps:
            c["nsteps"] = args.nsteps
            c["n_ckpt"] = min(c["n_ckpt"], args.nsteps)
        cfgs.append(c)
    torch.cuda.set_device(0)
    # offered load ~0.8 of the measured capacity: time one job alone first
    probe = Instance(cfgs[0])
    t = time.perf_counter()
    for _ in range(args.serve_iters):
        probe.iterate()
    t1 = (time.perf_counter() - t)
    probe.release()
    mean_job = t1 * np.mean([c["nr"] * c["nt"] * c["nz"] for c in cfgs]) / (cfgs[0]["nr"] * cfgs[0]["nt"] * cfgs[0]["nz"])
    rate = 0.8 / max(mean_job, 1e-3)
    arrivals = serve.poisson_arrivals(len(cfgs), rate, seed=7)
    s = serve.Server(hbm_budget=250e9, max_active=16, workers=8)
    jobs, rep = serve.replay(s, cfgs, args.serve_iters, arrivals)
    out = {"metric": "fwd+adjoint grid-point-steps/s (served)", "value": rep["gp_steps_per_s"],
           "unit": "grid-point-steps/s", "n_gpus": 1, "steps": rep["iterations"], "warmup": 0,
           "ms_per_step": rep["wall_s"] / max(rep["iterations"], 1) * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"serve-{len(cfgs)}-poisson", "arrival_rate_per_s": rate,
                      "iterations_per_job": args.serve_iters, **rep}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
