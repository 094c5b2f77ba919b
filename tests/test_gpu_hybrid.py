"""Two-level checkpointing with a pinned-host tier (Sec. 2.4): the gradient
equals the device-only one bitwise, and the sweep re-advances the counted
number of steps."""
import numpy as np
import pytest

from tests.gpu_common import make, to_dev, to_host, seed_field

pytestmark = pytest.mark.gpu

CFG = dict(nr=16, nt=12, nz=24, lz=2 * np.pi, re=1500.0, wo=8.0, amp=1.0, dt=0.02, t0=0.3, nsteps=40)


@pytest.mark.parametrize("graphs", [0, 1])
def test_hybrid_gradient_equals_device_only(graphs):
    import torch
    from paper_2509_10103_amd import npo
    P, G = make(CFG)
    npo.npo_plan_set_graphs(G.handle, graphs)
    N, nck = CFG["nsteps"], 4
    u0 = to_dev(seed_field(P, 3, 1e-2))
    ck = G.arena(nck)
    uN, lam = G.field(), G.field()
    npo.npo_forward_run(G.handle, G.ws, ck, nck, u0, uN)
    npo.npo_adjoint_run(G.handle, G.ws, ck, nck, uN, lam)
    ref_u, ref_l = to_host(uN), to_host(lam)
    for nf in (0, 1, 3, 7):
        print(f"[hybrid] n_file {nf} graphs {graphs}", flush=True)
        host = torch.empty(max(nf, 1) * G.info["field_bytes"], dtype=torch.uint8, pin_memory=True)
        u2, l2 = G.field(), G.field()
        npo.npo_forward_run_hybrid(G.handle, G.ws, ck, nck, host, nf, u0, u2)
        rec = npo.npo_adjoint_run_hybrid(G.handle, G.ws, ck, nck, host, nf, u2, l2)
        assert rec == npo.npo_hybrid_count(N, nck, nf)
        assert np.array_equal(to_host(u2), ref_u), nf
        assert np.array_equal(to_host(l2), ref_l), nf
    npo.npo_plan_set_graphs(G.handle, 0)
    G.close()
