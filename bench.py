"""Benchmark: adjoint-looping iterations of the NLOP hot path on one MI355X.

One benchmark step is one optimisation iteration of the paper's method
(Sec. 2.1-2.2) on the paper-like workload: adjoint sweep over one pulsation
period with binomial checkpoints (Sec. 2.4), solenoidal projection of the
gradient, and the backtracking line search whose trial forward sweeps leave
the next iterate's checkpoints in place.  The initial forward sweep is done
before the timed region.  Metric: forward + adjoint grid-point-steps per
second, counting one forward and one adjoint sweep of N_r*N_theta*N_z points
per step per iteration; recomputation and the line search's extra trial
sweeps are not counted, so their cost shows as lower throughput.  The JSON
line also gives the rate with every trial sweep counted, and the
per-iteration latency.

The run keeps to a wall-clock budget (``--budget``, measured from process
start, covering imports, plan set-up, the initial sweep, warm-up and timing):
at most one warm-up iteration is run, and timed iterations stop at
``--steps`` or when the next one would not fit the budget; ``steps`` in the
JSON line is the number actually timed.
"""
import argparse
import json
import math
import os
import sys
import time

T_START = time.perf_counter()

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2509_10103_amd import configs, synth  # noqa: E402

PEAK_HBM_GBS = 8000.0
HBM_RESERVE = 6 << 30
BUDGET_S = 420.0          # the whole run, from process start
TAIL_S = 20.0             # kept free for the profiler read, the CPU leg and the JSON line


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


# Families making up one evaluation of the nonlinear term (forward, adjoint)
EVAL_FAMILIES = {"theta_fwd": ("zinv_fwd", "theta_fwd", "zfwd_fwd"),
                 "theta_adj": ("zinv_adj", "theta_adj", "zfwd_adj")}


def op_bytes(cfg):
    """Compulsory bytes of the operation each kernel family performs, in the
    accounting of the two-exchange design (one spectral scalar field f per
    unit): a forward nonlinear evaluation moves u in and N out (6f), shared by
    its axial-inverse, azimuthal and axial-forward kernels; an adjoint one the
    state and the adjoint field in and the result out (9f); the solves their
    own spectral inputs and outputs.  The roofline of the dominant kernel
    divides the bytes of its operation by that kernel's launch time, the
    roofline of the evaluation by the time of all its kernels."""
    f1 = path_field_bytes(cfg)
    ev_f, ev_a = 6 * f1, 9 * f1
    return {"curl": 5 * f1, "zinv_fwd": ev_f, "theta_fwd": ev_f, "zfwd_fwd": ev_f, "zinv_adj": ev_a,
            "theta_adj": ev_a, "zfwd_adj": ev_a, "zinv_adjy": ev_a, "solve_pred": 9 * f1, "solve_corr": 12 * f1,
            "solve_raw": 6 * f1, "solve_adj": 6 * f1, "solve_adj2": 15 * f1, "adj_combine": 12 * f1, "wdot": 6 * f1,
            "project": 6 * f1, "axpby": 9 * f1}


def path_field_bytes(cfg):
    """f: bytes of one complex128 spectral scalar field."""
    M, K = (cfg["nt"] - 1) // 3, (cfg["nz"] - 1) // 3
    return cfg["nr"] * (M + 1) * (2 * K + 1) * 16


def path_step_bytes(cfg, ncorr):
    """Compulsory HBM bytes of one forward and one adjoint step of the
    two-exchange design with `ncorr` corrector passes, in units of f.

    One corrector pass: a forward step moves 33f (nonlinear term: u in, N out,
    6f per evaluation; predictor solve: u^n, N^n in, state out, 9f; corrector
    solve: u^n, N^n, N* in, state out, 12f, plus its evaluation 6f), an adjoint
    step about 60f including the recompute of its stage.  Each further corrector
    pass adds one evaluation and one corrector solve to the forward step (18f),
    and to the adjoint step the recompute of that stage (18f), the adjoint of its
    nonlinear term (state and adjoint field in, result out: 9f), its transposed
    solve (6f) and the accumulator update (6f): 39f."""
    return 15 + 18 * ncorr, 60 + 39 * (ncorr - 1)


def host_cores():
    """Host cores this process may use (the GPU machine grants 16 per GPU whatever
    the machine has)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, seed):
    """Time the CPU oracle on a bounded sample of the same workload at full
    size: one forward step (it also fills the oracle's operator-factor cache)
    and then one adjoint step, which recomputes the step's stages and applies
    their transposes, i.e. the work of one forward and one adjoint step of the
    sweep pair the metric counts (2 grid-point-steps per point).  BLAS may use
    every host core but two (those are left to the GPU leg running beside it);
    the reported `cores` is the CPU time over the wall time of the sample."""
    from threadpoolctl import threadpool_limits
    from oracle.pipe import Pipe
    threads = max(1, host_cores() - 2)
    with threadpool_limits(limits=threads):
        P = Pipe(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"], cfg["dt"], cfg["t0"])
        P.cache_limit = 0
        u = make_raw(cfg, P.r, P.M, P.K, seed)
        u *= math.sqrt(cfg["e0"] / P.energy(u))            # the cost does not depend on the values
        t = time.perf_counter()
        un = P.step(u, 0)
        tf = time.perf_counter() - t
        c0, t = os.times(), time.perf_counter()
        P.step_adj(u, 0, un)
        ta = time.perf_counter() - t
        c1 = os.times()
    used = (c1.user + c1.system - c0.user - c0.system) / ta
    pts = cfg["nr"] * cfg["nt"] * cfg["nz"]
    return {"value": 2 * pts / ta, "unit": "grid-point-steps/s", "cores": round(used, 2), "kind": "oracle",
            "threads_allowed": threads, "host_cores": host_cores(), "cpu_model": cpu_model(),
            "sample": f"one adjoint step of the same workload at full size ({ta:.1f} s; it recomputes the "
                      f"step's stages, so it is the work of one forward and one adjoint step = 2 grid-point-"
                      f"steps per point), after one forward step ({tf:.1f} s, fills the operator-factor cache); "
                      f"NumPy/SciPy oracle, BLAS limited to {threads} threads, {used:.2f} cores busy on average"}


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


def elapsed():
    return time.perf_counter() - T_START


def copy_calibration():
    """Counter calibration workload: one plain device-to-device copy of 1 GiB
    (FETCH_SIZE / WRITE_SIZE of this dispatch give the scale factors of the
    hardware byte counters)."""
    import torch
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"[bench] copied {b.numel()} bytes", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4, help="timed optimisation iterations (at most; see --budget)")
    ap.add_argument("--warmup", type=int, default=1, help="untimed optimisation iterations (at most one is run)")
    ap.add_argument("--budget", type=float, default=BUDGET_S,
                    help="wall-clock seconds for the whole run, from process start")
    ap.add_argument("--workload", default="c2", choices=sorted(configs.WORKLOADS))
    ap.add_argument("--nsteps", type=int, default=0, help="shorter horizon (development only)")
    ap.add_argument("--ckpt", type=int, default=0, help="checkpoint slots (default: the workload's)")
    ap.add_argument("--shapes", default="", help="launch shapes zgroup,zb_fwd,zb_adj (default: tuned)")
    ap.add_argument("--retune", action="store_true", help="time every launch shape instead of the tuning table")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--stride", type=int, default=8, help="profiler sampling stride")
    ap.add_argument("--adjoint", default="discrete", choices=["discrete", "continuous"],
                    help="adjoint of the validation run: the exact discrete one or the paper's continuous "
                         "adjoint equations (--mode validate)")
    ap.add_argument("--mode", default="plain", choices=["plain", "batch", "serve", "copy", "validate", "grad"],
                    help="plain: one instance (the metric); batch / serve: the systems layers; "
                         "copy: the 1 GiB copy that calibrates the byte counters; validate: the steady-pipe "
                         "validation setting (Re 1750, L_z = pi, tau = 80) run to convergence")
    ap.add_argument("--batch-n", type=int, default=16, help="instances of the batched workload")
    ap.add_argument("--serve-n", type=int, default=24, help="requests of the served workload")
    ap.add_argument("--serve-iters", type=int, default=2, help="iterations per served request")
    ap.add_argument("--c5", action="store_true",
                    help="the served workload as specified: 128 requests arriving at 4/s (seed 7), 10%% large "
                         "64x96x1536 jobs, 20 iterations each, within --serve-budget seconds; then the same job "
                         "mix offered at about 0.8 of the measured capacity")
    ap.add_argument("--serve-budget", type=float, default=240.0, help="wall seconds per served run (--c5)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this build measures one GPU's "
              f"share; how the path would shard over several GPUs is a design note, not a run", file=sys.stderr)
        sys.exit(2)
    if args.cpu_leg:
        print(json.dumps(cpu_baseline(configs.WORKLOADS[args.workload], configs.WORKLOADS[args.workload]["seed"])))
        return
    cpu_proc = None
    if args.mode == "plain" and not args.no_cpu:
        cpu_proc = start_cpu_leg(args.workload)

    import torch
    from paper_2509_10103_amd import npo

    if args.mode == "copy":
        return copy_calibration()
    if args.mode == "grad":
        return bench_grad(args)
    if args.mode == "validate":
        return bench_validate(args)
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
    ncorr = 2
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
    tuning = None
    if args.shapes:
        shapes = [int(x) for x in args.shapes.split(",")]
        npo.npo_plan_set_tuning(G.handle, *shapes)
    else:
        # the committed tuning table holds the shapes measured for this grid;
        # --retune measures them again
        best, tuning = tune.tune(G, cfg["nr"], cfg["nt"], cfg["nz"], use_cache=not args.retune, save=False)
        shapes = list(best)
    r = npo.npo_plan_tables(G.handle, cfg["nr"])[0]
    raw = make_raw(cfg, r, G.M, G.K, cfg["seed"])
    u0 = torch.from_numpy(np.ascontiguousarray(raw)).to("cuda")
    npo.npo_project(G.handle, G.ws, u0, u0)
    npo.npo_normalize(G.handle, G.ws, u0, cfg["e0"])
    arena = G.arena(nck)
    uN = G.field()
    n_rec = npo.npo_ckpt_count(cfg["nsteps"], nck)
    print(f"[bench] {cfg['name']} nsteps={cfg['nsteps']} n_ckpt={nck} arena={arena.numel() * 16 / 2**30:.1f} GiB "
          f"recompute/sweep={n_rec} launch shapes {shapes} (t={elapsed():.1f} s)", file=sys.stderr, flush=True)
    # the untimed initial sweep also records the largest CFL number of the
    # trajectory (the monitor is off in the timed iterations)
    cfl = torch.zeros(1, dtype=torch.float64, device="cuda")
    npo.npo_plan_set_cfl_monitor(G.handle, 1)
    npo.npo_cfl_read(G.handle, G.ws, cfl, reset=True)
    t = time.perf_counter()
    npo.npo_forward_run(G.handle, G.ws, arena, nck, u0, uN)
    torch.cuda.synchronize()
    t_sweep = time.perf_counter() - t
    npo.npo_cfl_read(G.handle, G.ws, cfl, reset=True)
    npo.npo_plan_set_cfl_monitor(G.handle, 0)
    cfl_max = float(cfl.item())
    print(f"[bench] initial forward sweep {t_sweep:.2f} s, CFL max {cfl_max:.3f} (t={elapsed():.1f} s)",
          file=sys.stderr, flush=True)

    def one_iter():
        st = npo.npo_iterate(G.handle, G.ws, arena, nck, u0, uN, cfg["e0"])
        if not st["accepted"]:
            npo.npo_forward_run(G.handle, G.ws, arena, nck, u0, uN)
            st["forward_sweeps"] += 1
        return st

    # an iteration is one adjoint sweep (about 1.8 forward sweeps of work plus
    # the recompute) and at least one trial sweep: estimate it before warm-up
    t_est = t_sweep * (3.0 + n_rec / max(cfg["nsteps"], 1))
    warm = 0
    for _ in range(min(args.warmup, 1)):
        if elapsed() + 2 * t_est + TAIL_S > args.budget:
            break
        t = time.perf_counter()
        one_iter()
        torch.cuda.synchronize()
        t_est = time.perf_counter() - t
        warm += 1
        print(f"[bench] warm-up iteration {t_est:.2f} s (t={elapsed():.1f} s)", file=sys.stderr, flush=True)
    npo.npo_profile_begin(G.handle, args.stride)
    lat = []
    hist = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        # the next iteration must fit the budget (the first timed one always runs)
        if i > 0 and elapsed() + 1.15 * max(t_est, max(lat)) + TAIL_S > args.budget:
            break
        ti = time.perf_counter()
        st = one_iter()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ti)
        hist.append(st)
        print(f"[bench] iteration {i}: G {st['G_old']:.6g} -> {st['G_new']:.6g} accepted={int(st['accepted'])} "
              f"sweeps={int(st['forward_sweeps'])} {lat[-1]:.2f} s (t={elapsed():.1f} s)", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed = len(lat)
    prof = npo.npo_profile_read(G.handle)
    pts = cfg["nr"] * cfg["nt"] * cfg["nz"]
    fwd_sweeps = sum(int(h["forward_sweeps"]) for h in hist)
    counted = timed * 2 * cfg["nsteps"] * pts
    value = counted / wall
    value_all = (fwd_sweeps + timed) * cfg["nsteps"] * pts / wall
    ab = alg_bytes(cfg)
    ob = op_bytes(cfg)
    tot = {k: v["launches"] * v["avg_ms"] for k, v in prof.items()}
    dom = max(tot, key=tot.get)
    avg_s = prof[dom]["avg_ms"] * 1e-3
    achieved = ob[dom] / avg_s / 1e9 if avg_s > 0 else 0.0
    own_io = ab[dom] / avg_s / 1e9 if avg_s > 0 else 0.0
    evaluation = None
    if dom in EVAL_FAMILIES and all(prof.get(k, {}).get("avg_ms", 0) > 0 for k in EVAL_FAMILIES[dom]):
        ev_s = sum(prof[k]["avg_ms"] for k in EVAL_FAMILIES[dom]) * 1e-3
        evaluation = {"kernels": list(EVAL_FAMILIES[dom]), "avg_us": ev_s * 1e6, "bytes": ob[dom],
                      "achieved": ob[dom] / ev_s / 1e9, "frac": ob[dom] / ev_s / 1e9 / PEAK_HBM_GBS}
    # HBM traffic per launch from the committed counter summary (rocprofv3
    # FETCH_SIZE / WRITE_SIZE, copy-calibrated), only while it was taken on
    # these kernel sources
    from paper_2509_10103_amd import profsum
    tr = profsum.load_traffic(os.path.join(ROOT, "profiles", f"{cfg['name']}_hbm_bytes.md"), cfg["nt"], cfg["nz"])
    traffic = tr[dom]["fetch"] + tr[dom]["write"] if tr and dom in tr else None
    # the whole path against the compulsory bytes of the two-exchange design:
    # every forward advance (trial sweeps and recompute) and adjoint step run
    f1 = path_field_bytes(cfg)
    bf, ba = path_step_bytes(cfg, ncorr)
    n_fwd = sum(h["forward_sweeps"] for h in hist) * cfg["nsteps"] + timed * n_rec
    n_adj = timed * cfg["nsteps"]
    b_alg = (n_fwd * bf + n_adj * ba) * f1
    measured = None
    if tr:
        measured = sum(v["launches"] * (tr[k]["fetch"] + tr[k]["write"]) for k, v in prof.items() if k in tr)
    path = {"alg_bytes": b_alg, "achieved": b_alg / wall / 1e9, "frac": b_alg / wall / 1e9 / PEAK_HBM_GBS,
            "measured_frac": (measured / wall / 1e9 / PEAK_HBM_GBS) if measured else None,
            "unit": "GB/s", "forward_advances": n_fwd, "adjoint_steps": n_adj,
            "bytes_per_forward_step_f": bf, "bytes_per_adjoint_step_f": ba, "f_bytes": f1,
            "measured_bytes": measured, "alg_over_measured": (b_alg / measured) if measured else None}
    kern = {k: {"launches": v["launches"], "avg_us": round(v["avg_ms"] * 1e3, 2),
                "share": round(tot[k] / max(sum(tot.values()), 1e-30), 4),
                "GBps_alg": round(ab[k] / (v["avg_ms"] * 1e-3) / 1e9, 1) if v["avg_ms"] > 0 else None}
            for k, v in prof.items() if v["launches"]}
    out = {
        "metric": "fwd+adjoint grid-point-steps/s",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": timed,
        "warmup": warm,
        "ms_per_step": wall / timed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": [cfg["nr"], cfg["nt"], cfg["nz"]], "lz_radii": cfg["lz"],
                   "re": cfg["re"], "wo": cfg["wo"], "amp": cfg["amp"], "dt": cfg["dt"], "t0": cfg["t0"],
                   "nsteps": cfg["nsteps"], "ncorr": ncorr, "n_ckpt": nck, "recompute_per_sweep": n_rec,
                   "launch_shapes": shapes, "radial_block": npo.npo_plan_get_radial_block(G.handle),
                   "tuning": tuning, "e0": cfg["e0"], "seed": cfg["seed"],
                   "steps_requested": args.steps, "warmup_requested": args.warmup, "budget_s": args.budget,
                   "run_s": round(elapsed(), 1),
                   "counted": "one forward and one adjoint sweep per iteration; recomputation and extra "
                              "line-search trial sweeps not counted",
                   "forward_sweeps_timed": fwd_sweeps,
                   "cfl_max_initial_sweep": cfl_max,
                   "value_counting_every_trial_sweep": value_all,
                   "iteration_latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                   "gains": [[h["G_old"], h["G_new"], int(h["accepted"]), int(h["forward_sweeps"])] for h in hist]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": ob[dom],
                     "alg_unit": "compulsory bytes of the operation the kernel performs (a nonlinear evaluation: "
                                 "u in, N out)",
                     "avg_launch_us": avg_s * 1e6,
                     "own_io_bytes_per_launch": ab[dom], "own_io_achieved": own_io,
                     "own_io_frac": own_io / PEAK_HBM_GBS, "evaluation": evaluation, "path": path},
        "kernels": kern,
    }
    out["cpu_baseline"] = finish_cpu_leg(cpu_proc) if cpu_proc is not None else None
    out["config"]["run_s"] = round(elapsed(), 1)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Uneven instances: their gradients (one forward and one checkpointed
    adjoint sweep each) through the batched launches in lockstep, against the
    plain single-instance calls on the same instances one after another (the
    same work); and whole optimisation iterations run concurrently on host
    threads (each instance's own launches) against the same run sequentially."""
    import torch
    from paper_2509_10103_amd.batch import Batch, LockstepBatch, percentiles
    cfgs = configs.batch_instances(64)[:args.batch_n]
    if args.nsteps:
        for c in cfgs:
            c["nsteps"] = args.nsteps
            c["n_ckpt"] = min(c["n_ckpt"], args.nsteps)
    torch.cuda.set_device(0)
    lk = LockstepBatch(cfgs)
    lk.gradients()                    # builds the descriptor tables and captures the step graphs
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        lk.gradients()
    torch.cuda.synchronize()
    wall_l = time.perf_counter() - t
    t = time.perf_counter()
    for _ in range(args.steps):
        lk.gradients_sequential()
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t
    counted_l = args.steps * lk.counted()
    info = lk.info()
    print(f"[bench] lockstep gradients of {len(cfgs)} instances: {wall_l:.2f} s, sequential {wall_s:.2f} s, "
          f"{info}", file=sys.stderr, flush=True)
    lk.close()
    del lk
    torch.cuda.empty_cache()
    b = Batch(cfgs)
    for inst in b.instances:          # initial forward sweeps (untimed, as in the plain mode)
        inst.forward()
    torch.cuda.synchronize()
    wall, counted, lat = b.run(iters=args.steps)
    print(f"[bench] concurrent iterations of {len(cfgs)} instances: {wall:.2f} s", file=sys.stderr, flush=True)
    for inst in b.instances:
        inst.swept = False
    seq, counted_seq = b.run_sequential(iters=args.steps)
    print(f"[bench] sequential iterations: {seq:.2f} s", file=sys.stderr, flush=True)
    p50, p99 = percentiles(lat)
    out = {"metric": "fwd+adjoint grid-point-steps/s (batched)", "value": counted_l / wall_l,
           "unit": "grid-point-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": wall_l / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"batch-{len(cfgs)}-uneven", "instances": len(cfgs),
                      "lockstep": {"value": counted_l / wall_l, "plain_sequential_value": counted_l / wall_s,
                                   "speedup_vs_plain": wall_s / wall_l, "shape_classes": info["classes"],
                                   "instances_batched": info["batched"],
                                   "launches_per_batched_step": info["launches"]},
                      "concurrent_iterations": {"value": counted / wall, "plain_sequential_value": counted_seq / seq,
                                                "speedup_vs_plain": (counted / wall) / (counted_seq / seq),
                                                "iteration_latency_s": {"p50": p50, "p99": p99}}}}
    print(json.dumps(out), flush=True)


def bench_validate(args):
    """The steady-pipe validation setting of the paper's appendix: Hagen-
    Poiseuille flow at Re = 1750 in a pipe of L_z = pi radii, resolution
    (N_r, M, K) = (38, >= 16, 21) (here N_theta = 54, N_z = 64: M = 17, K = 21),
    dt = 0.01, tau = 80, E0 = 1e-5, from a smooth seeded field (the paper starts
    from a turbulent one).  The loop runs until |dG/G| < 1e-8 or the budget; the
    G(t) history of the last iterate (npo_forward_run_diag) gives its maximum
    growth and the time of that maximum, beside the paper's G_max ~ 219 at
    t = 85.05 for this setting (context, not a pin)."""
    import torch
    from paper_2509_10103_amd import npo
    torch.cuda.set_device(0)
    nr, nt, nz, lz, re, dt, e0 = 38, 54, 64, math.pi, 1750.0, 0.01, 1e-5
    tau, extra = 80.0, 1200                      # the history runs on to t = 92
    nsteps = int(round(tau / dt))
    G = npo.Plan(nr, nt, nz, lz, re, 1.0, 0.0, dt, 0.0, nsteps)
    npo.npo_plan_set_graphs(G.handle, 1)
    npo.npo_plan_set_adjoint(G.handle, 1 if args.adjoint == "continuous" else 0)
    r = npo.npo_plan_tables(G.handle, nr)[0]
    u0 = torch.from_numpy(np.ascontiguousarray(synth.solenoidal_modes(r, G.M, G.K, lz, 11))).to("cuda")
    npo.npo_project(G.handle, G.ws, u0, u0)
    npo.npo_normalize(G.handle, G.ws, u0, e0)
    arena = G.arena(nsteps)
    uN = G.field()
    npo.npo_forward_run(G.handle, G.ws, arena, nsteps, u0, uN)
    hist = []
    t = time.perf_counter()
    while elapsed() + 30.0 < args.budget and len(hist) < 100:
        st = npo.npo_iterate(G.handle, G.ws, arena, nsteps, u0, uN, e0)
        hist.append([st["G_old"], st["G_new"], int(st["accepted"]), int(st["forward_sweeps"])])
        print(f"[validate] iteration {len(hist)}: G {st['G_new']:.9g} accepted={int(st['accepted'])} "
              f"(t={elapsed():.0f} s)", file=sys.stderr, flush=True)
        if not st["accepted"]:
            break
    wall = time.perf_counter() - t
    # G(t) of the final iterate over the horizon and beyond
    H = npo.Plan(nr, nt, nz, lz, re, 1.0, 0.0, dt, 0.0, nsteps + extra)
    rows = npo.diag_rows(nsteps + extra, 10)
    h = torch.zeros((rows, 5), dtype=torch.float64, device="cuda")
    a2 = H.arena(1)
    u1 = H.field()
    cfl = torch.zeros(1, dtype=torch.float64, device="cuda")
    npo.npo_plan_set_cfl_monitor(H.handle, 1)
    npo.npo_cfl_read(H.handle, H.ws, cfl, reset=True)
    npo.npo_forward_run_diag(H.handle, H.ws, a2, 1, u0, u1, h, 10)
    npo.npo_cfl_read(H.handle, H.ws, cfl, reset=True)
    e = h.cpu().numpy()
    g = e[:, :3].sum(axis=1) / e0
    ts = np.array([min(10 * i, nsteps + extra) for i in range(rows)]) * dt
    k = int(np.argmax(g))
    out = {"metric": "gain G(tau) of the converged optimum (validation setting)", "value": hist[-1][1] if hist else None,
           "unit": "E(tau)/E0", "n_gpus": 1, "steps": len(hist), "warmup": 0,
           "ms_per_step": wall / max(len(hist), 1) * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "steady-38x54x64-Re1750-Lz-pi-tau80", "e0": e0, "adjoint": args.adjoint,
                      "converged": bool(hist) and not hist[-1][2], "gains": hist,
                      "G_max": float(g[k]), "t_of_G_max": float(ts[k]), "cfl_max_of_history": float(cfl.item()),
                      "G_z_at_max": float(e[k, 2] / e0), "G_rtheta_at_max": float((e[k, 0] + e[k, 1]) / e0),
                      "energy_fraction_m_M_at_max": float(e[k, 3] / e[k, :3].sum()),
                      "energy_fraction_k_K_at_max": float(e[k, 4] / e[k, :3].sum()),
                      "paper_context": "G_max ~ 219 at t = 85.05 (E0 = 1e-5, (N_r, M, K) = (38, 16, 21))"}}
    print(json.dumps(out), flush=True)


def _log(line):
    print(line, file=sys.stderr, flush=True)


def bench_grad(args):
    """The differentiation workload at its full horizon: the gradient (one
    forward sweep and one checkpointed adjoint sweep) at checkpoint budgets
    {8, 32, 128, all} stored states, recomputation against memory, with the
    gradients of all budgets compared bitwise; then the gradient against
    central differences (eps = 1e-6) along 16 seeded solenoidal directions,
    every product and norm taken on the device."""
    import torch
    from paper_2509_10103_amd import npo
    torch.cuda.set_device(0)
    cfg = dict(configs.C3)
    N = cfg["nsteps"]
    G = npo.Plan(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"], cfg["dt"], cfg["t0"], N)
    npo.npo_plan_set_graphs(G.handle, 1)
    from paper_2509_10103_amd import tune
    best, _ = tune.tune(G, cfg["nr"], cfg["nt"], cfg["nz"], use_cache=not args.retune, save=False)
    tuning = list(best)
    r = npo.npo_plan_tables(G.handle, cfg["nr"])[0]
    u0 = torch.from_numpy(np.ascontiguousarray(synth.solenoidal_modes(r, G.M, G.K, cfg["lz"], cfg["seed"]))).to("cuda")
    npo.npo_project(G.handle, G.ws, u0, u0)
    npo.npo_normalize(G.handle, G.ws, u0, cfg["e0"])
    pts = cfg["nr"] * cfg["nt"] * cfg["nz"]
    runs, grads = [], {}
    for nck in (8, 32, 128, N):
        ck = G.arena(nck)
        uN, lam = G.field(), G.field()
        npo.npo_forward_run(G.handle, G.ws, ck, nck, u0, uN)            # warm-up (graph capture)
        torch.cuda.synchronize()
        t = time.perf_counter()
        npo.npo_forward_run(G.handle, G.ws, ck, nck, u0, uN)
        nrec = npo.npo_adjoint_run(G.handle, G.ws, ck, nck, uN, lam)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        grads[nck] = lam
        runs.append({"n_ckpt": nck, "arena_gb": nck * G.info["field_bytes"] / 1e9, "recompute_steps": nrec,
                     "gradient_s": wall, "gp_steps_per_s": 2 * N * pts / wall})
        print(f"[bench] gradient with {nck} slots: {wall:.2f} s, {nrec} recomputed steps (t={elapsed():.0f} s)",
              file=sys.stderr, flush=True)
        del ck
        torch.cuda.empty_cache()
    lam = grads[N]
    same = all(torch.equal(grads[k], lam) for k in grads)
    # central differences along seeded solenoidal directions
    ck1 = G.arena(1)
    tmp = G.field()
    nl = math.sqrt(G.inner(lam, lam))
    nu = math.sqrt(G.inner(u0, u0))
    eps, worst = 1e-6, 0.0

    def J(u):
        npo.npo_forward_run(G.handle, G.ws, ck1, 1, u, tmp)
        return G.energy(tmp)
    for s in range(100, 116):
        d = torch.from_numpy(np.ascontiguousarray(synth.solenoidal_modes(r, G.M, G.K, cfg["lz"], s))).to("cuda")
        npo.npo_project(G.handle, G.ws, d, d)
        d *= nu / math.sqrt(G.inner(d, d))
        fd = (J(u0 + eps * d) - J(u0 - eps * d)) / (2 * eps)
        worst = max(worst, abs(fd - G.inner(lam, d)) / (nl * nu))
    print(f"[bench] central differences along 16 directions: worst relative error {worst:.2e} "
          f"(t={elapsed():.0f} s)", file=sys.stderr, flush=True)
    best = max(runs, key=lambda x: x["gp_steps_per_s"])
    out = {"metric": "fwd+adjoint grid-point-steps/s (gradient)", "value": runs[-1]["gp_steps_per_s"],
           "unit": "grid-point-steps/s", "n_gpus": 1, "steps": len(runs), "warmup": 1,
           "ms_per_step": runs[-1]["gradient_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": cfg["name"], "grid": [cfg["nr"], cfg["nt"], cfg["nz"]], "nsteps": N,
                      "dt": cfg["dt"], "e0": cfg["e0"], "launch_shapes": tuning, "budgets": runs,
                      "gradients_bitwise_equal_across_budgets": same, "fd_worst_relative_error": worst,
                      "fd_directions": 16, "fd_eps": eps, "fastest_budget": best["n_ckpt"]}}
    print(json.dumps(out), flush=True)


def c5_jobs(n=128, seed=7):
    """The served job mix: 90% drawn from the batched workload's instances, 10%
    large 64 x 96 x 1536 jobs with L = 50 D (100 radii); parameters of the
    large jobs drawn as in the batched workload; seed 7."""
    pool = configs.batch_instances(64)
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        if rng.random() < 0.1:
            re, wo, amp = float(rng.uniform(1000, 3000)), float(rng.uniform(4, 18)), float(rng.uniform(0.25, 1.5))
            e0 = float(10 ** rng.uniform(-7, -3))
            T = configs.period(re, wo)
            t0 = float(rng.choice([0.0, 0.25, 0.5, 0.75])) * T
            c = dict(name=f"large-{i}-64x96x1536", nr=64, nt=96, nz=1536, lz=100.0, re=re, wo=wo, amp=amp, dt=0.02,
                     t0=t0, nsteps=2000, e0=e0, seed=2000 + i, n_ckpt=64, iters=20, gen="smooth")
        else:
            c = dict(pool[int(rng.integers(0, len(pool)))])
        out.append(c)
    return out


def bench_serve_c5(args):
    """The served workload as specified, within a wall budget per run."""
    import torch
    from paper_2509_10103_amd import serve
    from paper_2509_10103_amd.batch import Instance
    torch.cuda.set_device(0)
    cfgs = c5_jobs()
    iters = 20
    arrivals = serve.poisson_arrivals(len(cfgs), 4.0, seed=7)
    runs = {}
    s = serve.Server(hbm_budget=250e9, max_active=16, workers=8, log=_log)
    _, runs["offered_4_per_s"] = serve.replay(s, cfgs, iters, arrivals, budget=args.serve_budget)
    print(f"[bench] c5 at 4/s: {runs['offered_4_per_s']}", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    # capacity: one job of the mix's mean size, timed alone for two iterations
    probe = Instance(cfgs[1])
    t = time.perf_counter()
    for _ in range(2):
        probe.iterate()
    per_iter = (time.perf_counter() - t) / 2
    probe.release()
    size = lambda c: c["nr"] * c["nt"] * c["nz"]
    mean_job = per_iter * iters * np.mean([size(c) for c in cfgs]) / size(cfgs[1])
    rate = 0.8 / mean_job
    arrivals = serve.poisson_arrivals(len(cfgs), rate, seed=7)
    s = serve.Server(hbm_budget=250e9, max_active=16, workers=8, log=_log)
    _, runs["utilisation_0.8"] = serve.replay(s, cfgs, iters, arrivals, budget=args.serve_budget)
    runs["utilisation_0.8"]["arrival_rate_per_s"] = rate
    print(f"[bench] c5 at 0.8 utilisation: {runs['utilisation_0.8']}", file=sys.stderr, flush=True)
    r = runs["offered_4_per_s"]
    out = {"metric": "fwd+adjoint grid-point-steps/s (served)", "value": r["gp_steps_per_s"],
           "unit": "grid-point-steps/s", "n_gpus": 1, "steps": r["iterations"], "warmup": 0,
           "ms_per_step": r["wall_s"] / max(r["iterations"], 1) * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "serve-c5-poisson-4-per-s", "requests": len(cfgs), "iterations_per_job": iters,
                      "large_jobs": sum(1 for c in cfgs if c["nz"] == 1536), "budget_s": args.serve_budget,
                      **runs}}
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Poisson arrivals of uneven optimisation jobs; continuous batching."""
    import torch
    from paper_2509_10103_amd import serve
    from paper_2509_10103_amd.batch import Instance
    if args.c5:
        return bench_serve_c5(args)
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
    s = serve.Server(hbm_budget=250e9, max_active=16, workers=8, log=_log)
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
