"""Autotuner of the launch shapes.

For one grid shape it times the forward and the adjoint step of a plan under
every admissible transform shape (zgroup, zb_fwd, zb_adj), with HIP events on
the stream the kernels run on, keeps the fastest, and then times the radial
kernels' block size rg (|k| per block: 4, 8 or 16) under that shape.
Results are cached per shape class (nr, ntheta, nz) in a JSON file so that
batched and served runs tune once; an entry without rg keeps the default 16.
Shapes never change results (the tests run under several of them).
"""

RADIAL_BLOCKS = (4, 8, 16)
import itertools
import json
import os

from . import npo

CACHE = os.environ.get("NPO_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))


def candidates(plan):
    """Launch shapes the library accepts for this plan (it checks LDS fit and
    divisibility itself)."""
    out = []
    for c in itertools.product((1, 2, 3), (-16, -8, 2, 4, 8), (-16, -8, 2, 4, 8)):
        try:
            npo.npo_plan_set_tuning(plan.handle, *c)
        except npo.NpoError:
            continue
        out.append(c)
    return out


def _time_steps(plan, u, lam, reps):
    import torch
    st = torch.cuda.current_stream()
    out = plan.field()
    npo.npo_forward_step(plan.handle, plan.ws, u, out, 0)
    npo.npo_adjoint_step(plan.handle, plan.ws, u, lam, out, 0)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        npo.npo_forward_step(plan.handle, plan.ws, u, out, 0)
        npo.npo_adjoint_step(plan.handle, plan.ws, u, lam, out, 0)
    b.record(st)
    b.synchronize()
    return a.elapsed_time(b) / reps


def load_cache():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(plan, nr, nt, nz, reps=3, use_cache=True, save=True, batched=False):
    """Pick and set the fastest launch shapes for this plan; returns them.

    batched: only shapes whose kernels have batched forms (the LDS-staged
    azimuthal kernels, not the wave-resident ones), for npo_batch_* runs."""
    import torch
    key = f"{nr}x{nt}x{nz}"
    cache = load_cache() if use_cache else {}
    if key in cache:
        rec = cache[key]
        best = tuple(rec["shape"])
        if batched and min(best) < 0:
            ok = {k: v for k, v in rec.get("all", {}).items() if min(int(x) for x in k.split(",")) > 0}
            if ok:
                best = tuple(int(x) for x in min(ok, key=ok.get).split(","))
            else:
                best = npo.npo_plan_get_tuning(plan.handle)
                best = tuple(max(b, 2) if b < 0 else b for b in best)
        npo.npo_plan_set_tuning(plan.handle, *best)
        npo.npo_plan_set_radial_block(plan.handle, int(rec.get("rg", 16)))
        return best, rec
    u = torch.randn(plan.shape, dtype=torch.complex128, device=plan.device) * 1e-3
    lam = torch.randn(plan.shape, dtype=torch.complex128, device=plan.device)
    timings = {}
    for c in candidates(plan):
        if batched and min(c) < 0:
            continue
        npo.npo_plan_set_tuning(plan.handle, *c)
        timings[c] = _time_steps(plan, u, lam, reps)
    best = min(timings, key=timings.get)
    npo.npo_plan_set_tuning(plan.handle, *best)
    rg_ms = {}
    for rg in RADIAL_BLOCKS:
        npo.npo_plan_set_radial_block(plan.handle, rg)
        rg_ms[rg] = _time_steps(plan, u, lam, reps)
    rg = min(rg_ms, key=rg_ms.get)
    npo.npo_plan_set_radial_block(plan.handle, rg)
    rec = {"shape": list(best), "rg": rg, "ms_fwd_plus_adj": min(timings[best], rg_ms[rg]),
           "all": {",".join(map(str, c)): v for c, v in timings.items()},
           "rg_ms": {str(k): v for k, v in rg_ms.items()}}
    if save:
        cache = load_cache()
        cache[key] = rec
        try:
            with open(CACHE, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return best, rec
