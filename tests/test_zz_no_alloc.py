"""The no-allocation forward step (fixed device scratch instead of a caller
workspace) gives bitwise the results of npo_forward_step, allocates no device
memory, and rejects grids whose workspace exceeds the fixed scratch."""
import math

import numpy as np
import pytest

from paper_2509_10103_amd import synth

pytestmark = pytest.mark.gpu

# two calls in a row, the second on a smaller grid (the scratch keeps the
# first call's contents)
GRIDS = [
    dict(nr=24, nt=24, nz=48, lz=4 * math.pi, re=2000.0, wo=8.0, amp=0.5, dt=0.04, t0=0.0, n=3, seed=21),
    dict(nr=16, nt=12, nz=24, lz=2 * math.pi, re=1500.0, wo=8.0, amp=1.0, dt=0.02, t0=0.3, n=0, seed=22),
]


def _plan(cfg):
    from paper_2509_10103_amd import npo
    return npo.Plan(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"], cfg["dt"],
                    cfg["t0"], 8)


def test_noalloc_step_equals_workspace_step_on_two_calls():
    import torch
    from paper_2509_10103_amd import npo
    torch.cuda.set_device(0)
    plans = [_plan(c) for c in GRIDS]           # set-up (may allocate) before the calls under test
    for cfg, G in zip(GRIDS, plans):
        print(f"[no-alloc] grid {cfg['nr']}x{cfg['nt']}x{cfg['nz']} step {cfg['n']}", flush=True)
        assert G.info["workspace_bytes"] <= npo.SCRATCH_BYTES
        r = npo.npo_plan_tables(G.handle, cfg["nr"])[0]
        u = torch.from_numpy(synth.solenoidal_modes(r, G.M, G.K, cfg["lz"], cfg["seed"])).to("cuda")
        npo.npo_project(G.handle, G.ws, u, u)
        npo.npo_normalize(G.handle, G.ws, u, 1e-3)
        ref, out = G.field(), G.field()
        npo.npo_forward_step(G.handle, G.ws, u, ref, cfg["n"])
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        alloc0 = torch.cuda.memory_allocated()
        npo.npo_forward_step_noalloc(G.handle, u, out, cfg["n"])
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        assert torch.cuda.memory_allocated() == alloc0
        assert torch.isfinite(torch.view_as_real(out)).all()
        assert torch.equal(out, ref)
        # in place (u_n aliasing u_np1) as well
        v = u.clone()
        npo.npo_forward_step_noalloc(G.handle, v, v, cfg["n"])
        torch.cuda.synchronize()
        assert torch.equal(v, ref)
    for G in plans:
        G.close()


def test_noalloc_step_rejects_grid_beyond_the_scratch():
    import torch
    from paper_2509_10103_amd import npo
    torch.cuda.set_device(0)
    G = npo.Plan(48, 64, 384, 24.0, 1500.0, 10.0, 1.0, 0.02, 0.0, 8)
    assert G.info["workspace_bytes"] > npo.SCRATCH_BYTES
    u, out = G.field(), G.field()
    with pytest.raises(npo.NpoError) as e:
        npo.npo_forward_step_noalloc(G.handle, u, out, 0)
    assert "npo error -1" in str(e.value) and "fixed scratch" in str(e.value)
    G.close()
