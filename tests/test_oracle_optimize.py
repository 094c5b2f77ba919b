"""Pins of the oracle's projection, update, gradient and checkpoint counts."""
import json
import math
import os

import numpy as np
import pytest

from oracle.pipe import Pipe
from oracle import optimize as opt
from oracle import checkpoint as ck
from paper_2509_10103_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def prob():
    return Pipe(16, 12, 12, 2 * np.pi, 1500, 8, 1.0, 0.02, 0.3)


def test_projection_is_w_orthogonal_and_idempotent(prob):
    P = prob
    x = synth.random_field(P.shape, 7)
    y = synth.random_field(P.shape, 8)
    px = opt.project(P, x)
    py = opt.project(P, y)
    assert np.max(np.abs(opt.project(P, px) - px)) < 1e-12 * np.max(np.abs(px))
    # self-adjoint in W: <Px, y> = <x, Py>
    a, b = P.wdot(px, y), P.wdot(x, py)
    assert abs(a - b) < 1e-12 * abs(a)
    # constraints hold: wall zero, discrete divergence zero, mean mode u_r = 0 and zero flux
    for m, kk, al in P.modes():
        G = opt.constraint_rows(P, m, al)
        v = px[:, :, m, kk].reshape(-1)
        assert np.max(np.abs(G @ v)) < 1e-9 * max(1.0, np.max(np.abs(v))) * P.nr ** 2


def test_update_preserves_energy_and_lambda_solves_quadratic(prob):
    P = prob
    E0 = 1e-3
    u0 = opt.normalise(P, opt.project(P, synth.solenoidal_modes(P.r, P.M, P.K, P.lz, 1)), E0)
    ud = opt.project(P, synth.random_field(P.shape, 9)) * 1e-2
    E0d = 0.5 * P.wdot(ud, ud)
    C0 = P.wdot(u0, ud)
    amax = opt.alpha_max(E0, E0d, C0)
    for f in (1.0, 0.5, 1.0 / 7):
        al = f * amax
        lam = opt.lambda_plus(al, E0, E0d, C0)
        un = (1 + lam * al) * u0 - al * ud
        assert abs(P.energy(un) - E0) < 1e-12 * E0      # before the rescale
        # lambda solves E0 x^2 - al C0 x + al^2 E0d - E0 = 0 with x = 1 + lam al
        x = 1 + lam * al
        assert abs(E0 * x * x - al * C0 * x + al * al * E0d - E0) < 1e-12 * E0


def test_gradient_matches_central_differences():
    P = Pipe(12, 6, 12, 2 * np.pi, 1500, 8, 1.0, 0.02, 0.3)
    E0 = 1e-3
    u0 = opt.normalise(P, opt.project(P, synth.solenoidal_modes(P.r, P.M, P.K, P.lz, 1)), E0)
    J, _, lam = P.gradient(u0, 6)
    g = opt.project(P, lam)
    for s in (100, 101, 102):
        d = opt.project(P, synth.random_field(P.shape, s))
        d = d * math.sqrt(P.wdot(u0, u0) / P.wdot(d, d))
        eps = 1e-4
        fd = (P.energy(P.forward(u0 + eps * d, 6)) - P.energy(P.forward(u0 - eps * d, 6))) / (2 * eps)
        an = P.wdot(g, d)
        assert abs(fd - an) / math.sqrt(P.wdot(g, g) * P.wdot(d, d)) < 1e-8


def test_linear_regime_loop_converges_to_top_singular_value():
    # E0 -> 0 and a steady base flow: the step is linear and mode-diagonal, so
    # the optimum over one (k, m) mode is the top singular value of the
    # discrete propagator restricted to admissible fields (W norm).
    P = Pipe(12, 6, 6, 2 * np.pi, 1000, 8, 0.0, 0.05, 0.0)
    m, kk, nsteps = 1, 1, 20
    n3 = 3 * P.nr
    G = opt.constraint_rows(P, m, P.alpha[kk])
    wv = np.tile(P.w, 3)
    sw = np.sqrt(wv)
    # W-orthonormal basis of the admissible subspace
    B = G / sw[None, :]
    _, s, Vh = np.linalg.svd(B)
    Q = Vh[np.sum(s > 1e-12 * s[0]):].conj().T                 # null space of G W^{-1/2}
    basis = Q / sw[:, None]
    A = np.zeros((n3, basis.shape[1]), dtype=complex)
    for i in range(basis.shape[1]):
        v = P.zeros()
        v[:, :, m, kk] = basis[:, i].reshape(3, P.nr)
        for n in range(nsteps):
            v = P.step_tan(P.zeros(), n, v)
        A[:, i] = v[:, :, m, kk].reshape(-1)
    smax2 = np.linalg.svd(sw[:, None] * A, compute_uv=False)[0] ** 2
    E0 = 1e-20
    u = P.zeros()
    rng = np.random.default_rng(3)
    u[:, :, m, kk] = (basis @ (rng.standard_normal(basis.shape[1]) + 1j * rng.standard_normal(basis.shape[1]))).reshape(3, P.nr)
    u = opt.normalise(P, u, E0)
    Gs = []
    for it in range(40):
        u, Gn, info = opt.iterate(P, u, E0, nsteps)
        Gs.append(Gn)
        if info['status'] == 'converged':
            break
    assert Gs[-1] <= smax2 * (1 + 1e-9)
    assert abs(Gs[-1] / smax2 - 1) < 1e-7


def test_checkpoint_closed_form_equals_brute_force():
    for l in range(1, 40):
        for s in range(1, 8):
            assert ck.dp_advances(l, s) == ck.closed_form(l, s)[0]


def test_checkpoint_worked_cases():
    g = json.load(open(os.path.join(GOLD, "checkpoint_counts.json")))
    for c in g["cases"]:
        assert ck.closed_form(c["nsteps"], c["ng"]) == (c["nrec"], c["S"])
