"""Full-size parity over a prefix of the horizon: the paper-like workload
(64 x 96 x 768, 8 steps) and the differentiation workload (48 x 64 x 384,
6 steps), forward sweep and checkpointed adjoint sweep (three checkpoint
slots, so the adjoint sweep re-advances from stored states), against the
oracle's values on a fixed set of modes (every radial node and component)
and whole-field scalars, written by tests/golden/make_fullsize_fixtures.py.

Bars: fields within 1e-10 (W-norm over the sampled modes and max element),
the gradient lambda^0 within 1e-8 (the targets the method is held to)."""
import ast
import importlib.util
import os

import numpy as np
import pytest

from tests.gpu_common import to_host
from oracle.radial import Radial

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _script():
    spec = importlib.util.spec_from_file_location("make_fullsize_fixtures",
                                                  os.path.join(GOLD, "make_fullsize_fixtures.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _pick(f, modes):
    return np.stack([f[:, :, m, k] for m, k in modes], axis=-1)


def _werr(a, b, w, modes):
    """W-weighted relative error over the sampled modes, and the max-element one."""
    cm = np.where(modes[:, 0] == 0, 1.0, 2.0)
    wt = w[None, :, None] * cm[None, None, :]
    num = np.sqrt(np.sum(wt * np.abs(a - b) ** 2))
    den = np.sqrt(np.sum(wt * np.abs(b) ** 2))
    return num / den, np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.fixture(scope="module", params=["c2", "c3"])
def case(request):
    path = os.path.join(GOLD, f"{request.param}_prefix_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("oracle fixture not generated")
    import torch
    from paper_2509_10103_amd import npo
    d = np.load(path)
    c = ast.literal_eval(str(d["config"]))
    print(f"[prefix] {request.param} {c['nr']}x{c['nt']}x{c['nz']} nsteps={c['nsteps']}", flush=True)
    torch.cuda.set_device(0)
    G = npo.Plan(c["nr"], c["nt"], c["nz"], c["lz"], c["re"], c["wo"], c["amp"], c["dt"], c["t0"], c["nsteps"])
    raw = torch.from_numpy(np.ascontiguousarray(_script().raw_seed(c))).to("cuda")
    u0 = G.field()
    npo.npo_project(G.handle, G.ws, raw, u0)
    npo.npo_normalize(G.handle, G.ws, u0, c["e0"])
    nck = 3
    ck = G.arena(nck)
    uN, lam0 = G.field(), G.field()
    npo.npo_forward_run(G.handle, G.ws, ck, nck, u0, uN)
    nrec = npo.npo_adjoint_run(G.handle, G.ws, ck, nck, uN, lam0)
    out = dict(c=c, d=d, G=G, u0=u0, uN=uN, lam0=lam0, nrec=nrec, w=Radial(c["nr"]).w, modes=d["modes"])
    yield out
    G.close()


def test_initial_state_matches(case):
    rel, mx = _werr(_pick(to_host(case["u0"]), case["modes"]), case["d"]["u0"], case["w"], case["modes"])
    assert rel < 1e-12 and mx < 1e-12


def test_forward_prefix_fields(case):
    d = case["d"]
    rel, mx = _werr(_pick(to_host(case["uN"]), case["modes"]), d["uN"], case["w"], case["modes"])
    assert rel < 1e-10 and mx < 1e-10, (rel, mx)
    J = case["G"].energy(case["uN"])
    assert abs(J / float(d["J"]) - 1.0) < 1e-10


def test_checkpointed_adjoint_prefix_gradient(case):
    d, G = case["d"], case["G"]
    assert case["nrec"] > 0                      # three slots over the prefix: states are re-advanced
    rel, mx = _werr(_pick(to_host(case["lam0"]), case["modes"]), d["lam0"], case["w"], case["modes"])
    assert rel < 1e-8 and mx < 1e-8, (rel, mx)
    assert abs(G.inner(case["lam0"], case["lam0"]) / float(d["lam_norm2"]) - 1.0) < 1e-8
    assert abs(G.inner(case["lam0"], case["u0"]) - float(d["lam_u0"])) < 1e-8 * np.sqrt(
        float(d["lam_norm2"]) * 2 * float(d["E0"]))


def test_autograd_gradient_matches_oracle(case):
    """The torch.autograd.Function's Euclidean gradient (q (.) lambda^0 with
    q = 2 pi L_z c_m w_j) against the oracle's adjoint on the sampled modes."""
    import math
    import torch
    from paper_2509_10103_amd.autograd import Solver, gain_energy
    c, d = case["c"], case["d"]
    S = Solver(c["nr"], c["nt"], c["nz"], c["lz"], c["re"], c["wo"], c["amp"], c["dt"], c["t0"], c["nsteps"], 2)
    u0 = case["u0"].detach().clone().requires_grad_(True)
    J = gain_energy(u0, S)
    J.backward()
    g = _pick(to_host(u0.grad), case["modes"])
    cm = np.where(case["modes"][:, 0] == 0, 1.0, 2.0)
    q = 2.0 * math.pi * c["lz"] * case["w"][None, :, None] * cm[None, None, :]
    ref = q * d["lam0"]
    rel = np.sqrt(np.sum(np.abs(g - ref) ** 2) / np.sum(np.abs(ref) ** 2))
    assert rel < 1e-8, rel
    assert abs(float(J) / float(d["J"]) - 1.0) < 1e-10
    del S
    torch.cuda.synchronize()
