"""Batched and served optimisation instances: each result equals the same
instance run alone (bitwise), whatever else shares the GPU."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def small_cfgs(n, nsteps=24):
    import math
    from paper_2509_10103_amd import configs
    shapes = [(16, 12, 24), (24, 24, 48), (16, 24, 12), (32, 12, 48), (24, 12, 24), (16, 12, 48)]
    out = []
    for i in range(n):
        nr, nt, nz = shapes[i % len(shapes)]
        rng = np.random.default_rng(500 + i)
        re, wo, amp = float(rng.uniform(1000, 3000)), float(rng.uniform(4, 18)), float(rng.uniform(0.25, 1.5))
        T = configs.period(re, wo)
        out.append(dict(name=f"t{i}", nr=nr, nt=nt, nz=nz, lz=50.0 * nz / 768.0 * 4, re=re, wo=wo, amp=amp,
                        dt=0.02, t0=float(rng.choice([0, 0.25, 0.5])) * T, nsteps=nsteps,
                        e0=float(10 ** rng.uniform(-5, -3)), seed=500 + i, n_ckpt=int(rng.choice([3, 8, nsteps])),
                        iters=1, gen="smooth"))
    return out


def alone(cfg, iters):
    """The instance alone, launching every kernel itself (no step graphs), so
    that the batched runs, which replay graphs, are checked against it too."""
    from paper_2509_10103_amd.batch import Instance
    inst = Instance(cfg, autotune=False, graphs=False)
    for _ in range(iters):
        inst.iterate()
    u0, uN = inst.state()
    return u0.cpu().numpy(), uN.cpu().numpy(), [h[0]["G_new"] for h in inst.history]


def test_batch_equals_alone():
    from paper_2509_10103_amd.batch import Batch
    cfgs = small_cfgs(6)
    b = Batch(cfgs, autotune=False)
    wall, counted, lat = b.run(iters=2, workers=3)
    assert counted == sum(2 * 2 * c["nsteps"] * c["nr"] * c["nt"] * c["nz"] for c in cfgs)
    for inst, c in zip(b.instances, cfgs):
        u0, uN = inst.state()
        a0, aN, G = alone(c, 2)
        assert np.array_equal(u0.cpu().numpy(), a0)
        assert np.array_equal(uN.cpu().numpy(), aN)
        assert [h[0]["G_new"] for h in inst.history] == G


def test_served_jobs_equal_alone_under_staggered_arrivals():
    from paper_2509_10103_amd import serve
    from paper_2509_10103_amd.batch import Instance
    cfgs = small_cfgs(5, nsteps=20)
    budget = 2.2 * max(serve.estimate_footprint(c) for c in cfgs)   # forces queueing
    s = serve.Server(hbm_budget=budget, max_active=3, workers=3,
                     factory=lambda c: Instance(c, autotune=False))
    jobs, rep = serve.replay(s, cfgs, 2, arrivals=[0.0, 0.05, 0.1, 0.3, 0.35])
    assert rep["failed"] == 0 and rep["iterations"] == 10
    for j in jobs:
        a0, aN, G = alone(j.cfg, 2)
        u0, uN = j.result
        assert np.array_equal(u0.cpu().numpy(), a0)
        assert np.array_equal(uN.cpu().numpy(), aN)


@pytest.mark.parametrize("ncorr", [1, 2, 3])
def test_footprint_estimate_bounds_the_workspace(ncorr):
    """The serving loop admits jobs by estimate_workspace: it must bound what
    a plan of that configuration asks for."""
    from paper_2509_10103_amd import npo, serve
    big = [dict(small_cfgs(1)[0], nr=64, nt=96, nz=768)] if ncorr == 2 else []
    for c in small_cfgs(4) + big:
        c = dict(c, ncorr=ncorr)
        G = npo.Plan(c["nr"], c["nt"], c["nz"], c["lz"], c["re"], c["wo"], c["amp"], c["dt"], c["t0"],
                     c["nsteps"], ncorr)
        assert serve.estimate_workspace(c) >= G.info["workspace_bytes"], (c["nr"], c["nt"], c["nz"], ncorr)
        del G


def test_autotuner_times_the_radial_block_sizes(tmp_path, monkeypatch):
    """The tuner times every transform shape, then the radial block sizes
    under the winner, leaves the plan on the fastest of each, and a cached
    entry restores both."""
    from paper_2509_10103_amd import npo, tune
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "tune.json"))
    G = npo.Plan(16, 12, 24, 2 * np.pi, 1500.0, 8.0, 1.0, 0.02, 0.3, 1)
    print("[tune] 16x12x24", flush=True)
    best, rec = tune.tune(G, 16, 12, 24, reps=1)
    assert sorted(rec["rg_ms"]) == ["16", "4", "8"]
    assert str(rec["rg"]) == min(rec["rg_ms"], key=lambda k: rec["rg_ms"][k]) and isinstance(rec["rg"], int)
    assert tuple(npo.npo_plan_get_tuning(G.handle)) == tuple(best)
    assert npo.npo_plan_get_radial_block(G.handle) == rec["rg"]
    npo.npo_plan_set_radial_block(G.handle, 16 if rec["rg"] != 16 else 4)
    best2, rec2 = tune.tune(G, 16, 12, 24)
    assert tuple(best2) == tuple(best) and npo.npo_plan_get_radial_block(G.handle) == rec["rg"]
    G.close()
