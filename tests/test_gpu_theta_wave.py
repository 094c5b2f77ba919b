"""The wave-resident forward azimuthal kernel (tuning value zb_fwd = -L: the
packed sequences of a column spread over L lanes, radix-2 stages across the
lanes through cross-lane moves) against the oracle's nonlinear term, and
against the LDS-staged kernel, at every azimuthal length it supports."""
import numpy as np
import pytest

from tests.gpu_common import make, to_dev, to_host, seed_field, maxrel, relerr
from paper_2509_10103_amd import synth

pytestmark = pytest.mark.gpu

GRIDS = [
    dict(nr=12, nt=24, nz=48, lz=2 * np.pi, re=1500.0, wo=8.0, amp=1.0, dt=0.02, t0=0.3),
    dict(nr=10, nt=48, nz=96, lz=7.0, re=2000.0, wo=6.0, amp=0.8, dt=0.02, t0=1.1),
    dict(nr=8, nt=96, nz=192, lz=12.5, re=2000.0, wo=8.0, amp=1.0, dt=0.02, t0=98.17),
    dict(nr=9, nt=96, nz=36, lz=3.0, re=1000.0, wo=5.0, amp=0.5, dt=0.01, t0=2.0),   # nz = 36: partial blocks
]


@pytest.mark.parametrize("cfg", GRIDS, ids=lambda c: f"{c['nt']}x{c['nz']}")
def test_wave_kernel_matches_oracle_and_lds_kernel(cfg):
    from paper_2509_10103_amd import npo
    P, G = make(cfg)
    print(f"[theta-wave] grid {cfg['nr']}x{cfg['nt']}x{cfg['nz']}", flush=True)
    u = seed_field(P, 5, 1e-2)
    ref = P.N(u, 0.7)
    zg, zbf, zba = npo.npo_plan_get_tuning(G.handle)
    outs = {}
    for L in (8, 16):
        try:
            npo.npo_plan_set_tuning(G.handle, zg, -L, zba)
        except npo.NpoError:
            assert L == 16 and cfg["nt"] == 24 or cfg["nz"] % (64 // L)
            continue
        out = G.field()
        npo.npo_nonlinear(G.handle, G.ws, to_dev(u), 0.7, out)
        outs[L] = to_host(out)
        assert maxrel(outs[L], ref) < 1e-12, L
    assert outs
    npo.npo_plan_set_tuning(G.handle, zg, 2, zba)
    out = G.field()
    npo.npo_nonlinear(G.handle, G.ws, to_dev(u), 0.7, out)
    lds = to_host(out)
    for L, o in outs.items():
        assert maxrel(o, lds) < 1e-13, L
    # a whole step, and the adjoint term and step, with the wave kernels
    L = min(outs)
    npo.npo_plan_set_tuning(G.handle, zg, -L, -L)
    st = G.field()
    npo.npo_forward_step(G.handle, G.ws, to_dev(u), st, 2)
    assert relerr(P, to_host(st), P.step(u, 2)) < 1e-13
    y = synth.random_field(P.shape, 9)
    ad = G.field()
    npo.npo_nonlinear_adj(G.handle, G.ws, to_dev(u), 0.7, to_dev(y), ad)
    assert maxrel(to_host(ad), P.N_adj(u, 0.7, y)) < 1e-11
    npo.npo_adjoint_step(G.handle, G.ws, to_dev(u), to_dev(y), ad, 2)
    assert relerr(P, to_host(ad), P.step_adj(u, 2, y)) < 1e-11
    G.close()
