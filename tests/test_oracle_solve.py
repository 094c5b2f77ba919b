"""Pins of the oracle's implicit solve and time stepper."""
import numpy as np
import pytest
from scipy.special import jv, jn_zeros

from oracle.pipe import Pipe
from paper_2509_10103_amd import synth


def small():
    return Pipe(24, 12, 12, 2 * np.pi, 1500, 8, 1.0, 0.02, 0.5)


@pytest.mark.parametrize("m,kk", [(0, 1), (1, 0), (1, 2), (3, 5), (2, 0)])
def test_solve_satisfies_momentum_continuity_and_wall(m, kk):
    P = small()
    a = P.alpha[kk]
    rng = np.random.default_rng(m * 10 + kk)
    R = rng.standard_normal((3, P.nr, 2)) + 1j * rng.standard_normal((3, P.nr, 2))
    u, p = P.S_mode(m, a, R, return_p=True)
    r = P.r[:, None]
    assert np.max(np.abs(u[:, -1])) == 0.0
    # wall divergence (one-sided d/dr of u_r) is zero
    D1o = P.rad.D1[P.rad.parity(m + 1)]
    D1e = P.rad.D1[P.rad.parity(m)]
    div = (D1o @ u[0] + u[0] / r + 1j * m / r * u[1] + 1j * a * u[2])
    scale = np.max(np.abs(R))
    assert np.max(np.abs(div[-1])) < 1e-9 * scale * P.nr ** 2
    # H u + grad p = R at interior nodes, in the (+, -, z) basis
    c = 1.0 / (2 * P.re)
    up, um = u[0] + 1j * u[1], u[0] - 1j * u[1]
    Hp = up / P.dt - c * P.lap(m + 1, a) @ up
    Hm = um / P.dt - c * P.lap(m - 1, a) @ um
    Hz = u[2] / P.dt - c * P.lap(m, a) @ u[2]
    gp = D1e @ p - m / r * p
    gm = D1e @ p + m / r * p
    gz = 1j * a * p
    Rp, Rm = R[0] + 1j * R[1], R[0] - 1j * R[1]
    for lhs, rhs in ((Hp + gp, Rp), (Hm + gm, Rm), (Hz + gz, R[2])):
        assert np.max(np.abs((lhs - rhs)[:-1])) < 1e-9 * scale


def test_mean_mode_zero_flux_no_radial_velocity():
    P = small()
    rng = np.random.default_rng(0)
    R = rng.standard_normal((3, P.nr, 1)) + 0j
    u = P.S_mode(0, 0.0, R)
    assert np.all(u[0] == 0)
    assert abs(P.w @ u[2, :, 0]) < 1e-15 * np.max(np.abs(u[2]))


def test_interior_divergence_converges_with_radial_resolution():
    errs = []
    for nr in (24, 48):
        P = Pipe(nr, 12, 12, 2 * np.pi, 1500, 8, 1.0, 0.02)
        r = P.r
        m, kk = 2, 1
        a = P.alpha[kk]
        R = np.zeros((3, nr, 1), dtype=complex)
        R[0, :, 0] = r * (1 - r ** 2) * np.cos(2 * r)
        R[1, :, 0] = 1j * r * np.cos(3 * r)          # parities of m = 2: u_r, u_t odd, u_z even
        R[2, :, 0] = r ** 2 * np.exp(-r * r)
        u = P.S_mode(m, a, R)
        D1o = P.rad.D1[-1]
        div = D1o @ u[0, :, 0] + u[0, :, 0] / r + 1j * m / r * u[1, :, 0] + 1j * a * u[2, :, 0]
        errs.append(np.max(np.abs(div)) / np.max(np.abs(u)))
    assert errs[1] < errs[0] / 8


def decay_rate(P, u, comp, m, kk, nsteps):
    es = []
    for n in range(nsteps):
        u = P.step(u, n)
        es.append(np.sum(P.w * np.abs(u[comp, :, m, kk]) ** 2))
    g = np.sqrt(es[-1] / es[-2])
    return (2.0 / P.dt) * (1 - g) / (1 + g)


@pytest.mark.parametrize("case", ["swirl", "axial_mean", "axial_m2"])
def test_stokes_mode_decay_matches_bessel_roots(case):
    # Steady base flow, tiny amplitude, k = 0: decay per step (1-s dt/2)/(1+s dt/2),
    # s = lambda^2/Re with lambda a Bessel root.
    # The k = 0 base-flow terms are a gradient only up to the O(h^6) error of
    # the discrete product rule, so the m = 2 axial case needs 48 nodes.
    re = 100.0
    P = Pipe(48 if case == "axial_m2" else 32, 12, 12, 2 * np.pi, re, 8, 0.0, 0.05)
    r = P.r
    u = P.zeros()
    if case == "swirl":
        lam = jn_zeros(1, 1)[0]
        u[1, :, 0, 0] = jv(1, lam * r)
        comp, m = 1, 0
    elif case == "axial_mean":
        lam = jn_zeros(2, 1)[0]                 # J2(lam) = 0 <=> zero-flux J0 mode
        u[2, :, 0, 0] = jv(0, lam * r) - jv(0, lam)
        comp, m = 2, 0
    else:
        lam = jn_zeros(2, 1)[0]
        u[2, :, 2, 0] = jv(2, lam * r)
        comp, m = 2, 2
    u *= 1e-8
    s = decay_rate(P, u, comp, m, 0, 400)
    assert abs(s * re / lam ** 2 - 1) < (3e-6 if case == "axial_m2" else 1e-6)


def test_time_stepper_second_order():
    from oracle import optimize as opt

    def run(dt, T=0.4):
        P = Pipe(32, 12, 12, 2 * np.pi, 1500, 8, 1.0, dt, 0.3)
        u = opt.normalise(P, opt.project(P, synth.solenoidal_modes(P.r, P.M, P.K, P.lz, 4)), 1e-3)
        for n in range(int(round(T / dt))):
            u = P.step(u, n)
        return u
    a, b, c = run(0.04), run(0.02), run(0.01)
    ratio = np.max(np.abs(a - b)) / np.max(np.abs(b - c))
    assert 3.6 < ratio < 4.4
