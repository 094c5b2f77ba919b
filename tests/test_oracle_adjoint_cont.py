"""Pins of the oracle's continuous adjoint (paper Sec. 2, adjoint Navier-Stokes
equations integrated backwards with the direct stepper of Sec. 2.3).

The continuous adjoint is not the transpose of the discrete step, so there is
no exact dot-product identity to test.  What the mathematics fixes instead:
in the continuum, Omega x y + curl(y x V) is the L2 adjoint of the linearised
convective term v x Omega + V x curl v for fields that vanish at the wall, so
the mismatch <N'(u) v, y>_W - <v, Nc(u; y)>_W is a pure discretisation error
and must fall at the order of the radial differences (sixth) as N_r grows; the
same holds for one backward step against the tangent of the forward step,
provided the backward step takes the direct field at the right time levels
(the predictor at t_{n+1}, the correctors at t_n).  A sign error or a dropped
term leaves an O(1) mismatch, and wrong time levels leave a floor that does
not fall with N_r.  Over a short sweep the projected continuous-adjoint
gradient must approach the exact discrete gradient as N_r grows."""
import numpy as np
import pytest

from oracle.pipe import Pipe
from oracle import optimize as opt
from paper_2509_10103_amd import synth


def _case(nr, dt=0.01):
    P = Pipe(nr, 12, 12, 2 * np.pi, 1500.0, 8.0, 1.0, dt, 0.3)
    u = opt.normalise(P, opt.project(P, synth.solenoidal_modes(P.r, P.M, P.K, P.lz, 5)), 1e-2)
    v = opt.project(P, synth.solenoidal_modes(P.r, P.M, P.K, P.lz, 7))
    y = opt.project(P, synth.solenoidal_modes(P.r, P.M, P.K, P.lz, 8))
    return P, u, v, y


def _term_mismatch(nr):
    P, u, v, y = _case(nr)
    Nv = P.N_tan(u, 0.7, v)
    a, b = P.wdot(Nv, y), P.wdot(v, P.N_adj_cont(u, 0.7, y))
    return abs(a - b) / np.sqrt(P.wdot(Nv, Nv) * P.wdot(y, y))


def _step_mismatch(nr):
    P, u, v, y = _case(nr)
    sv = P.step_tan(u, 0, v)
    a, b = P.wdot(sv, y), P.wdot(v, P.step_adj_cont(u, P.step(u, 0), 0, y))
    return abs(a - b) / np.sqrt(P.wdot(sv, sv) * P.wdot(y, y))


def test_convective_term_is_the_adjoint_up_to_sixth_order_radial_error():
    e24, e48 = _term_mismatch(24), _term_mismatch(48)
    assert e24 < 1e-4 and e48 < 1e-6
    assert e24 / e48 > 30, (e24, e48)          # sixth order: 2^6 = 64 for twice the nodes


def test_backward_step_is_the_adjoint_of_the_step_tangent_up_to_discretisation():
    e24, e48 = _step_mismatch(24), _step_mismatch(48)
    assert e48 < 1e-8, e48
    assert e24 / e48 > 30, (e24, e48)


def test_discrete_term_is_exact():
    """The same mismatch for the exact discrete adjoint is rounding only, so
    the continuous mismatch above is the discretisation of the curl."""
    P, u, v, y = _case(16)
    Nv = P.N_tan(u, 0.7, v)
    a, b = P.wdot(Nv, y), P.wdot(v, P.N_adj(u, 0.7, y))
    assert abs(a - b) / np.sqrt(P.wdot(Nv, Nv) * P.wdot(y, y)) < 1e-13


@pytest.mark.parametrize("nsteps", [4])
def test_continuous_gradient_approaches_the_discrete_one(nsteps):
    def gap(nr):
        P, u, _, _ = _case(nr, dt=0.02)
        _, uN_c, gc = P.gradient_cont(u, nsteps)
        _, uN_d, gd = P.gradient(u, nsteps)
        assert np.array_equal(uN_c, uN_d)               # the same forward sweep
        pc, pd = opt.project(P, gc), opt.project(P, gd)
        d = pc - pd
        return np.sqrt(P.wdot(d, d) / P.wdot(pd, pd))
    g16, g32 = gap(16), gap(32)
    assert g16 < 0.03 and g32 < 0.01, (g16, g32)
    assert g16 / g32 > 2, (g16, g32)
