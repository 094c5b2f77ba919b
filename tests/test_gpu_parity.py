"""GPU (HIP, through the C ABI) versus CPU oracle, element by element."""
import numpy as np
import pytest

from tests.gpu_common import make, to_dev, to_host, seed_field, relerr, maxrel
from paper_2509_10103_amd import synth

pytestmark = pytest.mark.gpu

SMALL = dict(nr=16, nt=12, nz=24, lz=2 * np.pi, re=1500.0, wo=8.0, amp=1.0, dt=0.02, t0=0.3)
RAGGED = dict(nr=9, nt=6, nz=18, lz=3.0, re=1000.0, wo=5.0, amp=0.5, dt=0.01, t0=1.0)
TALL = dict(nr=64, nt=12, nz=24, lz=50.0, re=2000.0, wo=8.0, amp=1.0, dt=0.02, t0=98.17)


# At 64 radial nodes the near-wall Poisson operators are ill-conditioned enough
# that a pivoted LAPACK solve and the unpivoted banded factorisation differ by
# a few 1e-11 relative; the solve-level bounds are loosened to 1e-10 there.
@pytest.fixture(scope="module", params=[SMALL, RAGGED, TALL], ids=["small", "ragged", "nr64"])
def prob(request):
    P, G = make(request.param)
    u = seed_field(P, 1, 1e-2)
    y = synth.random_field(P.shape, 3)
    tol = 10.0 if request.param["nr"] == 64 else 1.0
    return P, G, u, y, tol


def test_tables_match_oracle(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    r, w, D1, D2, col0 = npo.npo_plan_tables(G.handle, P.nr)
    assert np.max(np.abs(r - P.r)) < 1e-15
    assert np.max(np.abs(w - P.w)) < 1e-15
    for pi, par in ((0, 1), (1, -1)):
        for j in range(P.nr):
            full1 = np.zeros(P.nr)
            full2 = np.zeros(P.nr)
            full1[col0[j]:col0[j] + 7] = D1[pi, j]
            full2[col0[j]:col0[j] + 7] = D2[pi, j]
            s1 = np.max(np.abs(P.rad.D1[par][j])) + 1
            s2 = np.max(np.abs(P.rad.D2[par][j])) + 1
            assert np.max(np.abs(full1 - P.rad.D1[par][j])) < 1e-11 * s1
            assert np.max(np.abs(full2 - P.rad.D2[par][j])) < 1e-10 * s2


def test_base_flow_matches_oracle(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    for t in (0.0, 3.7, 50.0):
        U, Om = npo.npo_base_flow(G.handle, t, P.nr)
        Uo, Oo = P.base(t)
        assert np.max(np.abs(U - Uo)) < 1e-13
        assert np.max(np.abs(Om - Oo)) < 1e-12


def test_inner_product(prob):
    P, G, u, y, f = prob
    a = G.inner(to_dev(u), to_dev(y))
    assert abs(a - P.wdot(u, y)) < 1e-13 * np.sqrt(P.wdot(u, u) * P.wdot(y, y))


def test_nonlinear_term(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_nonlinear(G.handle, G.ws, to_dev(u), 0.9, out)
    ref = P.N(u, 0.9)
    assert maxrel(to_host(out), ref) < 1e-12


def test_nonlinear_adjoint(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_nonlinear_adj(G.handle, G.ws, to_dev(u), 0.9, to_dev(y), out)
    ref = P.N_adj(u, 0.9, y)
    assert maxrel(to_host(out), ref) < 1e-11 * f


def test_solve(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_solve(G.handle, G.ws, to_dev(y), out)
    ref = P.S_direct(y)
    assert maxrel(to_host(out), ref) < 1e-11 * f


def test_solve_adjoint(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_solve_adj(G.handle, G.ws, to_dev(y), out)
    ref = P.apply_modes(y, 'S', adjoint=True)
    assert maxrel(to_host(out), ref) < 1e-10 * f


def test_projection(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    from oracle import optimize as opt
    out = G.field()
    npo.npo_project(G.handle, G.ws, to_dev(y), out)
    ref = opt.project(P, y)
    assert relerr(P, to_host(out), ref) < 1e-12


def test_forward_step(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_forward_step(G.handle, G.ws, to_dev(u), out, 3)
    ref = P.step(u, 3)
    assert relerr(P, to_host(out), ref) < 1e-13


def test_adjoint_step(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo
    out = G.field()
    npo.npo_adjoint_step(G.handle, G.ws, to_dev(u), to_dev(y), out, 3)
    ref = P.step_adj(u, 3, y)
    assert relerr(P, to_host(out), ref) < 1e-11 * f


def test_launch_shapes_do_not_change_results(prob):
    P, G, u, y, f = prob
    from paper_2509_10103_amd import npo, tune
    base = npo.npo_plan_get_tuning(G.handle)
    outs = []
    shapes = tune.candidates(G)
    for shape in shapes[::max(1, len(shapes) // 4)]:
        npo.npo_plan_set_tuning(G.handle, *shape)
        a, b = G.field(), G.field()
        npo.npo_forward_step(G.handle, G.ws, to_dev(u), a, 2)
        npo.npo_adjoint_step(G.handle, G.ws, to_dev(u), to_dev(y), b, 2)
        outs.append((to_host(a), to_host(b)))
    npo.npo_plan_set_tuning(G.handle, *base)
    for a, b in outs[1:]:
        assert maxrel(a, outs[0][0]) < 1e-13
        assert maxrel(b, outs[0][1]) < 1e-12
