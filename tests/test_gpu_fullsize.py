"""Parity at the paper-like workload's full size (64 x 96 x 768), in the
launch shapes the benchmark uses (autotuned): full-field comparison where the
oracle finishes in seconds, sampled modes for the radial adjoint, and the
adjoint step through the dot-product identity with central differences of the
forward step."""
import math

import numpy as np
import pytest

from tests.gpu_common import to_dev, to_host, maxrel
from oracle.pipe import Pipe
from paper_2509_10103_amd import configs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    from paper_2509_10103_amd import npo, tune
    c = configs.C2
    P = Pipe(c["nr"], c["nt"], c["nz"], c["lz"], c["re"], c["wo"], c["amp"], c["dt"], c["t0"])
    P.cache_limit = 0
    G = npo.Plan(c["nr"], c["nt"], c["nz"], c["lz"], c["re"], c["wo"], c["amp"], c["dt"], c["t0"], 4)
    tune.tune(G, c["nr"], c["nt"], c["nz"])
    raw = synth.localized_oblique(P.r, P.M, P.K, P.lz, P.nz, c["seed"])
    u = raw * (1e-3 / np.max(np.abs(raw)))          # a smooth perturbation of the workload's shape
    y = synth.random_field(P.shape, 21)
    rng = np.random.default_rng(5)
    modes = [(0, 0)] + [(int(rng.integers(0, P.M + 1)), int(rng.integers(0, P.nk))) for _ in range(40)]
    return c, P, G, u, y, modes


def test_nonlinear_term_full(full):
    c, P, G, u, y, modes = full
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_nonlinear(G.handle, G.ws, to_dev(u), c["t0"] + 1.0, out)
    assert maxrel(to_host(out), P.N(u, c["t0"] + 1.0)) < 1e-12


def test_solve_sampled_modes(full):
    c, P, G, u, y, modes = full
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_solve(G.handle, G.ws, to_dev(y), out)
    o = to_host(out)
    for m, kk in modes:
        ref = P.S_mode(m, P.alpha[kk], y[:, :, m, kk:kk + 1])[:, :, 0]
        assert np.max(np.abs(o[:, :, m, kk] - ref)) < 1e-10 * np.max(np.abs(ref)), (m, kk)


def test_solve_adjoint_sampled_modes(full):
    c, P, G, u, y, modes = full
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_solve_adj(G.handle, G.ws, to_dev(y), out)
    o = to_host(out)
    for m, kk in modes:
        ref = P.S_adj_mode(m, P.alpha[kk], y[:, :, m, kk:kk + 1])[:, :, 0]
        assert np.max(np.abs(o[:, :, m, kk] - ref)) < 1e-10 * np.max(np.abs(ref)), (m, kk)


def test_nonlinear_adjoint_sampled_modes(full):
    c, P, G, u, y, modes = full
    from paper_2509_10103_amd import npo
    t = c["t0"] + 0.5
    out = G.field()
    npo.npo_nonlinear_adj(G.handle, G.ws, to_dev(u), t, to_dev(y), out)
    o = to_host(out)
    # oracle pieces: full transforms, curl^dag only on the sampled modes
    U, Om = P.base(t)
    Y = P.to_phys(y)
    a = P.to_spec(P.cross(P.to_phys(P.curl(u)), Y))
    b = P.to_spec(P.cross(Y, P.to_phys(u)))
    Uc, Oc = U[:, None, None], Om[:, None, None]
    a = a + np.stack([Oc * y[2], np.zeros_like(y[1]), -Oc * y[0]])
    b = b + np.stack([Uc * y[1], -Uc * y[0], np.zeros_like(y[2])])
    for m, kk in modes:
        C = P.adjoint_matrix('C', m, P.alpha[kk])
        ref = a[:, :, m, kk] + (C @ b[:, :, m, kk].reshape(-1)).reshape(3, P.nr)
        assert np.max(np.abs(o[:, :, m, kk] - ref)) < 1e-11 * np.max(np.abs(ref)), (m, kk)


def test_forward_step_full(full):
    c, P, G, u, y, modes = full
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_forward_step(G.handle, G.ws, to_dev(u), out, 0)
    ref = P.step(u, 0)
    d = to_host(out) - ref
    assert math.sqrt(P.wdot(d, d) / P.wdot(ref, ref)) < 1e-12


def test_adjoint_step_dot_product_full(full):
    """<y, Phi'(u) v> from central differences of the forward step (Richardson-
    extrapolated over eps and eps/2 to remove the O(eps^2) term) equals
    <Phi'(u)^+ y, v> from the adjoint step."""
    c, P, G, u, y, modes = full
    from paper_2509_10103_amd import npo
    v = synth.random_field(P.shape, 22) * 1e-3
    lam = G.field()
    npo.npo_adjoint_step(G.handle, G.ws, to_dev(u), to_dev(y), lam, 1)
    rhs = G.inner(lam, to_dev(v))

    def fd(eps):
        fp, fm = G.field(), G.field()
        npo.npo_forward_step(G.handle, G.ws, to_dev(u + eps * v), fp, 1)
        npo.npo_forward_step(G.handle, G.ws, to_dev(u - eps * v), fm, 1)
        return G.inner(to_dev(y), (fp - fm) / (2 * eps))
    d1, d2 = fd(2e-3), fd(1e-3)
    extrap = (4 * d2 - d1) / 3
    assert abs(d1 - rhs) > 3 * abs(d2 - rhs)           # the raw error is the eps^2 truncation
    assert abs(extrap - rhs) < 1e-8 * abs(rhs)
