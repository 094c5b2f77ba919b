"""Energy diagnostics on the device (npo_energy_diag, npo_forward_run_diag)
against the oracle's component, band and mode energies."""
import numpy as np
import pytest

from tests.gpu_common import make, to_dev, to_host, seed_field
from paper_2509_10103_amd import synth

pytestmark = pytest.mark.gpu

CFG = dict(nr=16, nt=12, nz=24, lz=2 * np.pi, re=1500.0, wo=8.0, amp=1.0, dt=0.02, t0=0.3, nsteps=10)


def test_energy_diag_matches_oracle():
    import torch
    from paper_2509_10103_amd import npo
    P, G = make(CFG)
    u = synth.random_field(P.shape, 6)
    out = torch.full((5,), np.nan, dtype=torch.float64, device="cuda")
    spec = torch.full(((P.M + 1) * P.nk,), np.nan, dtype=torch.float64, device="cuda")
    npo.npo_energy_diag(G.handle, G.ws, to_dev(u), out, spec)
    d = to_host(out)
    E = P.energy(u)
    assert np.max(np.abs(d[:3] - P.component_energies(u))) < 1e-13 * E
    eM, eK = P.band_energies(u)
    assert abs(d[3] - eM) < 1e-13 * E and abs(d[4] - eK) < 1e-13 * E
    assert np.max(np.abs(to_host(spec).reshape(P.M + 1, P.nk) - P.mode_energies(u))) < 1e-13 * E
    G.close()


@pytest.mark.parametrize("stride", [1, 3, 10])
def test_forward_run_history_matches_oracle(stride):
    import torch
    from paper_2509_10103_amd import npo
    P, G = make(CFG)
    N = CFG["nsteps"]
    u0 = seed_field(P, 2, 1e-2)
    _, hist = P.forward(u0, N, keep=True)
    states = hist + [P.forward(u0, N)]
    rows = npo.diag_rows(N, stride)
    H = torch.full((rows, 5), np.nan, dtype=torch.float64, device="cuda")
    ck = G.arena(4)
    uN = G.field()
    npo.npo_forward_run_diag(G.handle, G.ws, ck, 4, to_dev(u0), uN, H, stride)
    h = to_host(H)
    ns = list(range(0, N, stride)) + [N]
    assert len(ns) == rows
    for row, n in enumerate(ns):
        u = states[n]
        E = P.energy(u)
        assert np.max(np.abs(h[row, :3] - P.component_energies(u))) < 1e-12 * E, (row, n)
        eM, eK = P.band_energies(u)
        assert abs(h[row, 3] - eM) < 1e-12 * E and abs(h[row, 4] - eK) < 1e-12 * E
    G.close()
