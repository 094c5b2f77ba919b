"""Batched instances through the descriptor-table launches: every instance
of a shape class advanced by one launch per kernel, bitwise equal to the
instance's own calls; a class without batched kernels falls back."""
import numpy as np
import pytest

from tests.gpu_common import to_dev, to_host
from oracle.pipe import Pipe
from oracle import optimize as opt
from paper_2509_10103_amd import synth

pytestmark = pytest.mark.gpu

NSTEPS = 12
INSTANCES = [
    # two shape classes with batched kernels, uneven parameters within a class
    dict(nr=16, nt=12, nz=24, lz=2 * np.pi, re=1500.0, wo=8.0, amp=1.0, dt=0.02, t0=0.3, seed=1),
    dict(nr=16, nt=12, nz=24, lz=5.0, re=2600.0, wo=5.0, amp=0.4, dt=0.015, t0=7.0, seed=2),
    dict(nr=16, nt=12, nz=24, lz=3.3, re=1100.0, wo=12.0, amp=1.3, dt=0.02, t0=0.0, seed=3),
    dict(nr=24, nt=24, nz=48, lz=4.0, re=2000.0, wo=8.0, amp=0.5, dt=0.02, t0=1.0, seed=4),
    dict(nr=24, nt=24, nz=48, lz=9.0, re=1800.0, wo=6.0, amp=1.1, dt=0.01, t0=3.0, seed=5),
    # a class without batched kernels (azimuthal length 6): per-instance fallback
    dict(nr=9, nt=6, nz=18, lz=3.0, re=1000.0, wo=5.0, amp=0.5, dt=0.01, t0=1.0, seed=6),
]


def _setup():
    from paper_2509_10103_amd import npo
    plans, u0s = [], []
    for c in INSTANCES:
        G = npo.Plan(c["nr"], c["nt"], c["nz"], c["lz"], c["re"], c["wo"], c["amp"], c["dt"], c["t0"], NSTEPS)
        P = Pipe(c["nr"], c["nt"], c["nz"], c["lz"], c["re"], c["wo"], c["amp"], c["dt"], c["t0"])
        u0s.append(to_dev(opt.normalise(P, synth.solenoidal_modes(P.r, P.M, P.K, P.lz, c["seed"]), 1e-3)))
        plans.append(G)
    return plans, u0s


def test_batched_sweeps_equal_alone_bitwise():
    from paper_2509_10103_amd import npo
    plans, u0s = _setup()
    nck = 4
    ref = []
    for G, u0 in zip(plans, u0s):
        ck = G.arena(nck)
        uN, lam = G.field(), G.field()
        npo.npo_forward_run(G.handle, G.ws, ck, nck, u0, uN)
        rec = npo.npo_adjoint_run(G.handle, G.ws, ck, nck, uN, lam)
        ref.append((to_host(uN), to_host(lam), rec))
    handles = [G.handle for G in plans]
    b = npo.npo_batch_create(handles)
    ws = [G.ws for G in plans]
    cks = [G.arena(nck) for G in plans]
    uNs = [G.field() for G in plans]
    lams = [G.field() for G in plans]
    for rep in range(2):                       # the second pass replays the captured step graphs
        print(f"[batch] lockstep sweeps pass {rep}", flush=True)
        npo.npo_batch_forward_run(b, handles, ws, cks, nck, u0s, uNs)
        rec = npo.npo_batch_adjoint_run(b, handles, ws, cks, nck, uNs, lams)
        for i, (ru, rl, rr) in enumerate(ref):
            assert np.array_equal(to_host(uNs[i]), ru), (rep, i)
            assert np.array_equal(to_host(lams[i]), rl), (rep, i)
            assert rec == rr
    info = npo.npo_batch_info(b)
    assert info["classes"] == 3 and info["batched"] == 5
    npo.npo_batch_destroy(b)
    for G in plans:
        G.close()


def test_radial_block_sizes_split_classes_and_keep_results():
    """Instances of one grid with different radial block sizes fall into
    classes of their own; every instance still equals its own calls bitwise."""
    from paper_2509_10103_amd import npo
    plans, u0s = _setup()
    npo.npo_plan_set_radial_block(plans[1].handle, 4)
    npo.npo_plan_set_radial_block(plans[3].handle, 8)
    nck = 4
    ref = []
    for G, u0 in zip(plans, u0s):
        ck = G.arena(nck)
        uN, lam = G.field(), G.field()
        npo.npo_forward_run(G.handle, G.ws, ck, nck, u0, uN)
        npo.npo_adjoint_run(G.handle, G.ws, ck, nck, uN, lam)
        ref.append((to_host(uN), to_host(lam)))
    handles = [G.handle for G in plans]
    b = npo.npo_batch_create(handles)
    ws = [G.ws for G in plans]
    cks = [G.arena(nck) for G in plans]
    uNs = [G.field() for G in plans]
    lams = [G.field() for G in plans]
    print("[batch] lockstep sweeps with mixed radial blocks", flush=True)
    npo.npo_batch_forward_run(b, handles, ws, cks, nck, u0s, uNs)
    npo.npo_batch_adjoint_run(b, handles, ws, cks, nck, uNs, lams)
    for i, (ru, rl) in enumerate(ref):
        assert np.array_equal(to_host(uNs[i]), ru), i
        assert np.array_equal(to_host(lams[i]), rl), i
    info = npo.npo_batch_info(b)
    assert info["classes"] == 5 and info["batched"] == 5
    npo.npo_batch_destroy(b)
    for G in plans:
        G.close()


def test_batched_step_launches_do_not_grow_with_instances():
    """One batched step: bitwise equal to each instance's npo_forward_step /
    npo_adjoint_step at its step index, and the launch count of a batched class
    is the same for one instance as for three."""
    from paper_2509_10103_amd import npo
    plans, u0s = _setup()
    plans, u0s = plans[:3], u0s[:3]            # one class
    handles = [G.handle for G in plans]
    ws = [G.ws for G in plans]
    launches = []
    for sub in (1, 3):
        b = npo.npo_batch_create(handles[:sub])
        npo.npo_batch_set_steps(b, handles[:sub], ws[:sub], 5)
        outs = [u.clone() for u in u0s[:sub]]
        npo.npo_batch_step(b, handles[:sub], ws[:sub], outs, 0)
        launches.append(npo.npo_batch_info(b)["launches"])
        for G, u, o in zip(plans, u0s, outs):
            ref = G.field()
            npo.npo_forward_step(G.handle, G.ws, u, ref, 5)
            assert np.array_equal(to_host(o), to_host(ref))
        # adjoint step at the step index (now 6)
        ys = [G.field() + 1e-3 for G in plans[:sub]]
        st = []
        for u, y in zip(u0s[:sub], ys):
            st += [u, y.clone()]
        npo.npo_batch_step(b, handles[:sub], ws[:sub], st, 1)
        for k, (G, u, y) in enumerate(zip(plans, u0s, ys)):
            ref = G.field()
            npo.npo_adjoint_step(G.handle, G.ws, u, y, ref, 6)
            assert np.array_equal(to_host(st[2 * k + 1]), to_host(ref))
        npo.npo_batch_destroy(b)
    assert launches[0] == launches[1]
    for G in plans:
        G.close()
