"""The continuous adjoint (the paper's adjoint equations integrated backwards
with the direct stepper) on the HIP path against the oracle: its convective
term, one backward step, and the checkpointed sweep through the plan's
adjoint kind; the iteration with it; batches refuse it."""
import numpy as np
import pytest

from tests.gpu_common import make, to_dev, to_host, seed_field, relerr, maxrel
from paper_2509_10103_amd import synth
from oracle import optimize as opt

pytestmark = pytest.mark.gpu

SMALL = dict(nr=16, nt=12, nz=24, lz=2 * np.pi, re=1500.0, wo=8.0, amp=1.0, dt=0.02, t0=0.3)
RAGGED = dict(nr=9, nt=6, nz=18, lz=3.0, re=1000.0, wo=5.0, amp=0.5, dt=0.01, t0=1.0)
TALL = dict(nr=64, nt=12, nz=24, lz=50.0, re=2000.0, wo=8.0, amp=1.0, dt=0.02, t0=98.17)


@pytest.fixture(scope="module", params=[SMALL, RAGGED, TALL], ids=["small", "ragged", "nr64"])
def prob(request):
    P, G = make(dict(request.param, nsteps=6))
    print(f"[adjoint-cont] grid {request.param['nr']}x{request.param['nt']}x{request.param['nz']}", flush=True)
    u = seed_field(P, 1, 1e-2)
    y = synth.random_field(P.shape, 3)
    tol = 10.0 if request.param["nr"] == 64 else 1.0     # the 64-node solves (see the parity tests)
    yield P, G, u, y, tol
    G.close()


def test_convective_term(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_nonlinear_adj_cont(G.handle, G.ws, to_dev(u), 0.9, to_dev(y), out)
    assert maxrel(to_host(out), P.N_adj_cont(u, 0.9, y)) < 1e-11 * f


def test_backward_step(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    u1 = P.step(u, 3)
    out = G.field()
    npo.npo_adjoint_step_cont(G.handle, G.ws, to_dev(u), to_dev(u1), to_dev(y), out, 3)
    assert relerr(P, to_host(out), P.step_adj_cont(u, u1, 3, y)) < 1e-11 * f
    # in place
    lam = to_dev(y)
    npo.npo_adjoint_step_cont(G.handle, G.ws, to_dev(u), to_dev(u1), lam, lam, 3)
    assert np.array_equal(to_host(lam), to_host(out))


@pytest.mark.parametrize("n_ckpt", [6, 2])
def test_checkpointed_sweep_matches_oracle(prob, n_ckpt):
    """The plan's continuous adjoint kind through npo_adjoint_run, with every
    state stored and with two slots (states re-advanced), against the oracle's
    gradient_cont; the discrete kind is unchanged afterwards."""
    P, G, u, _, f = prob
    from paper_2509_10103_amd import npo
    _, uN_ref, g_ref = P.gradient_cont(u, 6)
    ck = G.arena(n_ckpt)
    uN, lam0 = G.field(), G.field()
    npo.npo_plan_set_adjoint(G.handle, 1)
    try:
        npo.npo_forward_run(G.handle, G.ws, ck, n_ckpt, to_dev(u), uN)
        nrec = npo.npo_adjoint_run(G.handle, G.ws, ck, n_ckpt, uN, lam0)
    finally:
        npo.npo_plan_set_adjoint(G.handle, 0)
    assert (nrec > 0) == (n_ckpt < 6)
    assert relerr(P, to_host(lam0), g_ref) < 1e-10 * f
    npo.npo_forward_run(G.handle, G.ws, ck, n_ckpt, to_dev(u), uN)
    npo.npo_adjoint_run(G.handle, G.ws, ck, n_ckpt, uN, lam0)
    _, _, gd = P.gradient(u, 6)
    assert relerr(P, to_host(lam0), gd) < 1e-9 * f


def test_iteration_with_the_continuous_adjoint_raises_the_gain():
    from paper_2509_10103_amd import npo
    cfg = dict(SMALL, nsteps=10)
    P, G = make(cfg)
    u0 = to_dev(seed_field(P, 2, 1e-4))
    ck = G.arena(10)
    uN = G.field()
    npo.npo_plan_set_adjoint(G.handle, 1)
    npo.npo_forward_run(G.handle, G.ws, ck, 10, u0, uN)
    st = npo.npo_iterate(G.handle, G.ws, ck, 10, u0, uN, 1e-4)
    assert st["accepted"] and st["G_new"] > st["G_old"]
    assert abs(G.energy(u0) / 1e-4 - 1) < 1e-12
    G.close()


def test_batches_refuse_the_continuous_adjoint():
    from paper_2509_10103_amd import npo
    P, G = make(dict(SMALL, nsteps=4))
    npo.npo_plan_set_adjoint(G.handle, 1)
    b = npo.npo_batch_create([G.handle])
    ck = G.arena(4)
    with pytest.raises(npo.NpoError, match="-4"):       # NPO_EUNSUPPORTED, before anything is enqueued
        npo.npo_batch_adjoint_run(b, [G.handle], [G.ws], [ck], 4, [G.field()], [G.field()])
    npo.npo_batch_destroy(b)
    assert npo.lib().npo_plan_set_adjoint(G.handle, 2) == -1
    G.close()


@pytest.mark.parametrize("graphs", [0, 1])
def test_continuous_sweep_with_graphs_and_host_tier_is_bitwise_the_same(graphs):
    """Forward advances replayed from captured graphs and the two-level
    checkpoints (each interval makes its own u^{n+1} for its last step) leave
    the continuous gradient bitwise unchanged."""
    import torch
    from paper_2509_10103_amd import npo
    P, G = make(dict(SMALL, nsteps=24))
    print(f"[adjoint-cont] host tier, graphs {graphs}", flush=True)
    N, nck = 24, 4
    u0 = to_dev(seed_field(P, 3, 1e-2))
    ck = G.arena(nck)
    uN, lam = G.field(), G.field()
    npo.npo_plan_set_adjoint(G.handle, 1)
    npo.npo_forward_run(G.handle, G.ws, ck, nck, u0, uN)
    npo.npo_adjoint_run(G.handle, G.ws, ck, nck, uN, lam)
    ref = to_host(lam)
    _, _, g = P.gradient_cont(to_host(u0), N)
    assert relerr(P, ref, g) < 1e-10
    npo.npo_plan_set_graphs(G.handle, graphs)
    for nf in (0, 2, 5):
        host = torch.empty(max(nf, 1) * G.info["field_bytes"], dtype=torch.uint8, pin_memory=True)
        u2, l2 = G.field(), G.field()
        npo.npo_forward_run_hybrid(G.handle, G.ws, ck, nck, host, nf, u0, u2)
        npo.npo_adjoint_run_hybrid(G.handle, G.ws, ck, nck, host, nf, u2, l2)
        assert np.array_equal(to_host(l2), ref), nf
    npo.npo_plan_set_graphs(G.handle, 0)
    G.close()
