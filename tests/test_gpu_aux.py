"""Auxiliaries of the step driver: the CFL monitor folded into the forward
azimuthal pass, and injected failures of the step drivers (error paths of the
sweeps and of the serving loop, forced from the host: no device fault)."""
import numpy as np
import pytest

from tests.gpu_common import make, to_dev, seed_field

pytestmark = pytest.mark.gpu

CFG = dict(nr=10, nt=24, nz=24, lz=2 * np.pi, re=1500.0, wo=8.0, amp=1.0, dt=0.02, t0=0.3)


def cfl_of(P, u, t):
    """max over the physical points of dt (|u_z + U| / dz + |u_theta| / (r dtheta)
    + |u_r| / dr_j), dr_j the smaller gap to a neighbouring node (2 r_0 at the first)."""
    U, _ = P.base(t)
    f = P.to_phys(u)                                     # (3, nr, nz, ntheta)
    r = P.r
    gl = np.concatenate([[2 * r[0]], np.diff(r)])
    gr = np.concatenate([np.diff(r), [gl[-1]]])
    dr = np.minimum(gl, gr)
    c = (np.abs(f[2] + U[:, None, None]) * P.nz / P.lz
         + np.abs(f[1]) * P.ntheta / (2 * np.pi * r[:, None, None])
         + np.abs(f[0]) / dr[:, None, None])
    return P.dt * c.max()


def _read(G, reset=False):
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    from paper_2509_10103_amd import npo
    npo.npo_cfl_read(G.handle, G.ws, out, reset)
    torch.cuda.synchronize()
    return float(out.item())


# the pruned azimuthal kernel (N_theta = 24), the compiled-length one (64) and
# the generic one (54)
CFL_GRIDS = [CFG, dict(CFG, nt=64, nz=48, lz=5.0), dict(CFG, nt=54, nz=36, lz=4.0)]


@pytest.mark.parametrize("grid", CFL_GRIDS, ids=["pruned", "compiled", "generic"])
def test_cfl_monitor_matches_the_physical_maximum(grid):
    from paper_2509_10103_amd import npo
    P, G = make(dict(grid, nsteps=3))
    print(f"[aux] cfl monitor {grid['nr']}x{grid['nt']}x{grid['nz']}", flush=True)
    zg, _, zba = npo.npo_plan_get_tuning(G.handle)
    npo.npo_plan_set_tuning(G.handle, zg, 2, zba)          # pruned forward azimuthal kernel
    u = seed_field(P, 11, 3e-2)
    # the unperturbed flow: the axial base velocity alone
    npo.npo_plan_set_cfl_monitor(G.handle, 1)
    _read(G, reset=True)
    z = G.field()
    out = G.field()
    npo.npo_forward_step(G.handle, G.ws, z, out, 0)
    assert abs(_read(G) / cfl_of(P, P.zeros(), P.tau0) - 1) < 1e-13
    # three steps: the maximum over the states u^0, u^1, u^2 that start them
    _read(G, reset=True)
    assert _read(G) == 0.0
    _, hist = P.forward(u, 3, keep=True)
    ref = max(cfl_of(P, h, P.tau0 + n * P.dt) for n, h in enumerate(hist))
    ck = G.arena(3)
    npo.npo_forward_run(G.handle, G.ws, ck, 3, to_dev(u), out)
    got = _read(G, reset=True)
    assert ref > cfl_of(P, P.zeros(), P.tau0)               # the perturbation moves the maximum
    assert abs(got / ref - 1) < 1e-12, (got, ref)
    # switched off: nothing is folded in
    npo.npo_plan_set_cfl_monitor(G.handle, 0)
    npo.npo_forward_run(G.handle, G.ws, ck, 3, to_dev(u), out)
    assert _read(G) == 0.0
    assert npo.lib().npo_plan_set_cfl_monitor(G.handle, 2) == -1      # NPO_EINVAL
    G.close()


@pytest.mark.parametrize("site", [1, 2])
def test_injected_step_failure_is_reported_and_clears(site):
    import torch
    from paper_2509_10103_amd import npo
    P, G = make(dict(CFG, nsteps=6))
    print(f"[aux] injected failure at site {site}", flush=True)
    npo.npo_plan_set_graphs(G.handle, 0)
    u0 = to_dev(seed_field(P, 4, 1e-3))
    ck = G.arena(2)
    uN, lam0 = G.field(), G.field()
    npo.npo_forward_run(G.handle, G.ws, ck, 2, u0, uN)
    npo.npo_adjoint_run(G.handle, G.ws, ck, 2, uN, lam0)
    torch.cuda.synchronize()
    ref_N, ref_l = uN.clone(), lam0.clone()
    npo.npo_plan_inject_fault(G.handle, site, 3)
    with pytest.raises(npo.NpoError, match="-3"):
        npo.npo_forward_run(G.handle, G.ws, ck, 2, u0, uN)
        npo.npo_adjoint_run(G.handle, G.ws, ck, 2, uN, lam0)
    # the failure was one call's: with injection off the same sweeps agree bitwise
    npo.npo_plan_inject_fault(G.handle, 0, 0)
    npo.npo_forward_run(G.handle, G.ws, ck, 2, u0, uN)
    npo.npo_adjoint_run(G.handle, G.ws, ck, 2, uN, lam0)
    torch.cuda.synchronize()
    assert torch.equal(uN, ref_N) and torch.equal(lam0, ref_l)
    with pytest.raises(npo.NpoError):
        npo.npo_plan_inject_fault(G.handle, 3, 0)
    G.close()


def test_serving_loop_retires_a_failing_job():
    """One job's step driver fails in its first iteration: the server retires
    it with the error, and the other jobs finish with the results they have
    alone."""
    from paper_2509_10103_amd import npo, serve
    from paper_2509_10103_amd.batch import Instance
    from tests.test_gpu_batch_serve import small_cfgs, alone
    cfgs = small_cfgs(3, nsteps=12)
    bad = cfgs[1]["name"]

    def factory(c):
        inst = Instance(c, autotune=False, graphs=False)
        if c["name"] == bad:
            npo.npo_plan_inject_fault(inst.plan.handle, 2, 5)
        return inst
    print("[aux] serving with one failing job", flush=True)
    s = serve.Server(hbm_budget=1e12, max_active=3, workers=3, factory=factory)
    jobs, rep = serve.replay(s, cfgs, 2, arrivals=[0.0, 0.0, 0.0])
    assert rep["failed"] == 1
    for j in jobs:
        if j.cfg["name"] == bad:
            assert j.error and "-3" in j.error and j.result is None
            continue
        assert j.error is None
        a0, aN, _ = alone(j.cfg, 2)
        u0, uN = j.result
        assert np.array_equal(u0.cpu().numpy(), a0) and np.array_equal(uN.cpu().numpy(), aN)


def test_serving_loop_retires_a_job_with_a_non_finite_state():
    """A job whose initial field holds a NaN (poisoned from the host) is
    retired with an error at its first iteration; the others are unaffected."""
    import math
    import torch
    from paper_2509_10103_amd import serve
    from paper_2509_10103_amd.batch import Instance
    from tests.test_gpu_batch_serve import small_cfgs, alone
    cfgs = small_cfgs(3, nsteps=12)
    bad = cfgs[2]["name"]

    def factory(c):
        inst = Instance(c, autotune=False, graphs=False)
        if c["name"] == bad:
            inst.stream.synchronize()
            inst.u0[0, 1, 1, 1] = complex(math.nan, 0.0)
            torch.cuda.synchronize()
        return inst
    print("[aux] serving with one poisoned job", flush=True)
    s = serve.Server(hbm_budget=1e12, max_active=3, workers=3, factory=factory)
    jobs, rep = serve.replay(s, cfgs, 2, arrivals=[0.0, 0.0, 0.0])
    assert rep["failed"] == 1
    for j in jobs:
        if j.cfg["name"] == bad:
            assert j.error and j.result is None and j.done_iters <= 1, (j.error, j.done_iters)
            continue
        assert j.error is None
        a0, aN, _ = alone(j.cfg, 2)
        u0, uN = j.result
        assert np.array_equal(u0.cpu().numpy(), a0) and np.array_equal(uN.cpu().numpy(), aN)
