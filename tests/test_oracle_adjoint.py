"""Pins of the oracle's discrete adjoint: dot-product and Taylor tests."""
import numpy as np
import pytest

from oracle.pipe import Pipe
from oracle import optimize as opt
from paper_2509_10103_amd import synth


@pytest.fixture(scope="module")
def prob():
    P = Pipe(16, 12, 12, 2 * np.pi, 1500, 8, 1.0, 0.02, 0.3)
    u = opt.normalise(P, opt.project(P, synth.solenoidal_modes(P.r, P.M, P.K, P.lz, 1)), 1e-2)
    v = synth.random_field(P.shape, 2)
    y = synth.random_field(P.shape, 3)
    return P, u, v, y


def rel(a, b):
    return abs(a - b) / max(abs(a), abs(b))


@pytest.mark.parametrize("kind", ["S", "E", "C"])
def test_linear_pieces_dot_product(prob, kind):
    P, u, v, y = prob
    a = P.wdot(y, P.apply_modes(v, kind))
    b = P.wdot(P.apply_modes(y, kind, adjoint=True), v)
    assert rel(a, b) < 1e-13


def test_materialised_solve_matches_literal_solve(prob):
    P, u, v, y = prob
    a, b = P.S(v), P.S_direct(v)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_direct_adjoints_match_materialised_definition(prob):
    P, u, v, y = prob
    a = P.S_adj_direct(y)
    b = P.apply_modes(y, 'S', adjoint=True)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))
    a = P.E_adj_direct(y)
    b = P.apply_modes(y, 'E', adjoint=True)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


def test_nonlinear_term_dot_product(prob):
    P, u, v, y = prob
    a = P.wdot(y, P.N_tan(u, 0.7, v))
    b = P.wdot(P.N_adj(u, 0.7, y), v)
    assert abs(a) > 1e-3
    assert rel(a, b) < 1e-12


def test_step_dot_product(prob):
    P, u, v, y = prob
    a = P.wdot(y, P.step_tan(u, 3, v))
    b = P.wdot(P.step_adj(u, 3, y), v)
    assert rel(a, b) < 1e-11


@pytest.mark.parametrize("ncorr", [1, 3])
def test_step_dot_product_other_corrector_counts(prob, ncorr):
    P0, u, v, y = prob
    P = Pipe(16, 12, 12, 2 * np.pi, 1500, 8, 1.0, 0.02, 0.3, ncorr=ncorr)
    a = P.wdot(y, P.step_tan(u, 3, v))
    b = P.wdot(P.step_adj(u, 3, y), v)
    assert rel(a, b) < 1e-11


def test_two_corrector_passes_damp_fast_axial_advection():
    # one fast axial mode: with a single pass (Heun) the explicit advection
    # grows by ~(a U dt)^4/8 per step, more than the viscous decay; two passes damp it
    def radius(ncorr):
        P = Pipe(24, 6, 6, 2 * np.pi / 40.0, 2000, 8, 0.0, 0.03, 0.0, ncorr=ncorr)
        n3 = 3 * P.nr
        A = np.zeros((n3, n3), dtype=complex)
        for i in range(n3):
            v = P.zeros()
            v[:, :, 0, 1] = np.eye(n3)[i].reshape(3, P.nr)
            A[:, i] = P.step_tan(P.zeros(), 0, v)[:, :, 0, 1].reshape(-1)
        return np.max(np.abs(np.linalg.eigvals(A)))
    assert radius(1) > 1.0 > radius(2)


def test_tangent_matches_finite_differences(prob):
    P, u, v, y = prob
    tl = P.step_tan(u, 3, v)
    errs = []
    for eps in (1e-3, 1e-4):
        fd = (P.step(u + eps * v, 3) - P.step(u - eps * v, 3)) / (2 * eps)
        errs.append(np.sqrt(P.wdot(fd - tl, fd - tl) / P.wdot(tl, tl)))
    assert errs[1] < 1e-4
    assert 80 < errs[0] / errs[1] < 120          # second-order central difference


def test_nonlinear_tangent_matches_finite_differences(prob):
    P, u, v, y = prob
    eps = 1e-5
    fd = (P.N(u + eps * v, 0.7) - P.N(u - eps * v, 0.7)) / (2 * eps)
    tl = P.N_tan(u, 0.7, v)
    # N is quadratic in u, so the central difference is exact up to rounding
    assert np.max(np.abs(fd - tl)) < 1e-8 * np.max(np.abs(tl))
