"""Pins of the oracle's Sexl-Womersley base flow."""
import json
import os

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

from oracle import womersley as wm

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def bulk(re, wo, amp, t):
    x, g = leggauss(80)
    r = 0.5 * (x + 1.0)
    U, _ = wm.base_flow(r, t, re, wo, amp)
    return 2.0 * np.sum(0.5 * g * U * r)


@pytest.mark.parametrize("re,wo,amp", [(2000, 8, 1.0), (1500, 10, 1.0), (1000, 18, 1.5), (3000, 4, 0.25)])
def test_bulk_velocity_and_wall(re, wo, amp):
    T = wm.period(re, wo)
    for t in np.linspace(0, T, 7):
        ub = 0.5 * (1 + amp * np.sin(2 * np.pi * t / T))
        assert abs(bulk(re, wo, amp, t) - ub) < 1e-13
        U, _ = wm.base_flow(np.array([1.0]), t, re, wo, amp)
        assert abs(U[0]) < 1e-13


def test_momentum_residual_is_uniform_pressure_gradient():
    # dU/dt - (1/Re)(U'' + U'/r) must not depend on r (it is -dP/dz(t))
    re, wo, amp = 2000.0, 8.0, 1.0
    r = np.linspace(0.05, 0.95, 7)
    t, h = 37.0, 1e-3
    dUdt = (wm.base_flow(r, t + h, re, wo, amp)[0] - wm.base_flow(r, t - h, re, wo, amp)[0]) / (2 * h)
    hr = 1e-4
    Up = wm.base_flow(r + hr, t, re, wo, amp)[0]
    Um = wm.base_flow(r - hr, t, re, wo, amp)[0]
    U0 = wm.base_flow(r, t, re, wo, amp)[0]
    lap = (Up - 2 * U0 + Um) / hr ** 2 + (Up - Um) / (2 * hr) / r
    res = dUdt - lap / re
    assert np.ptp(res) < 1e-6 * np.max(np.abs(dUdt)) + 1e-7


def test_derivative_matches_finite_difference():
    r = np.linspace(0.1, 0.9, 5)
    h = 1e-6
    _, Om = wm.base_flow(r, 11.0, 2000, 8, 1.0)
    dU = (wm.base_flow(r + h, 11.0, 2000, 8, 1.0)[0] - wm.base_flow(r - h, 11.0, 2000, 8, 1.0)[0]) / (2 * h)
    assert np.max(np.abs(-Om - dU)) < 1e-8


def test_quasi_steady_limit_is_poiseuille_shaped():
    r = np.linspace(0, 1, 11)
    ut, _ = wm.profile(r, 1e-3, 1.0)
    assert np.max(np.abs(ut - (-0.5j) * 2 * (1 - r ** 2))) < 1e-6


def test_period_in_paper_units_matches_printed_consistency_point():
    g = json.load(open(os.path.join(GOLD, "period_pin.json")))
    T = wm.period(g["re"], g["wo"])
    assert abs(g["fraction_of_period"] * T - g["t_peak"]) / g["t_peak"] < g["rel_tol"]
    # the printed formula pi Re / (2 Wo^2) is the same period in diameter/bulk units
    assert abs(T - 4 * np.pi * g["re"] / (2 * g["wo"] ** 2)) < 1e-12 * T
