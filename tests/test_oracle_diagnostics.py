"""Pins of the oracle's energy diagnostics (growth decompositions of Sec. 3-4,
resolution measures of Sec. 2.3): the parts add up to E(u), and single-mode
fields have closed-form energies."""
import math

import numpy as np

from oracle.pipe import Pipe
from paper_2509_10103_amd import synth


def test_components_and_modes_add_up_to_the_energy():
    P = Pipe(16, 12, 24, 9.0, 2000.0, 8.0, 1.0, 0.02)
    u = synth.random_field(P.shape, 4)
    E = P.energy(u)
    assert abs(P.component_energies(u).sum() / E - 1.0) < 1e-14
    assert abs(P.mode_energies(u).sum() / E - 1.0) < 1e-14


def test_single_mode_energies_closed_form():
    """u_z = r^m (1 - r^2) cos(m theta + alpha z): E = pi L_z m! / (2 (m+3)!),
    all of it axial, all in stored mode (m, k) (for m = 0 half at +k, half at -k)."""
    lz = 7.0
    P = Pipe(32, 12, 24, lz, 2000.0, 8.0, 1.0, 0.02)
    for m, kk in ((3, 2), (0, 5), (P.M, 1), (1, P.K)):
        f = P.r ** m * (1.0 - P.r ** 2)
        u = P.zeros()
        u[2, :, m, kk % P.nk] += 0.5 * f
        if m == 0:
            u[2, :, 0, (-kk) % P.nk] += 0.5 * f
        exact = math.pi * lz * math.factorial(m) / (2 * math.factorial(m + 3))
        ce = P.component_energies(u)
        assert abs(ce[2] / exact - 1) < 1e-13 and ce[0] == 0.0 and ce[1] == 0.0
        me = P.mode_energies(u)
        if m == 0:
            assert abs(me[0, kk] / exact - 0.5) < 1e-13 and abs(me[0, P.nk - kk] / exact - 0.5) < 1e-13
        else:
            assert abs(me[m, kk % P.nk] / exact - 1) < 1e-13
        eM, eK = P.band_energies(u)
        assert abs(eM - (exact if m == P.M else 0.0)) < 1e-13 * exact
        assert abs(eK - (exact if kk == P.K else 0.0)) < 1e-13 * exact
