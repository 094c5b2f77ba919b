"""Pins of the oracle's radial discretisation (nodes, quadrature, FD)."""
import numpy as np
import pytest

from oracle.radial import Radial, nodes, quad_weights


@pytest.mark.parametrize("nr", [16, 32, 48, 64])
def test_quadrature_exact_on_even_polynomials(nr):
    # int_0^1 r^{2p} r dr = 1/(2p+2), exact for the interpolatory rule in s=r^2
    r, w = nodes(nr), quad_weights(nr)
    assert np.all(w > 0)
    for p in range(nr):
        assert abs(np.sum(w * r ** (2 * p)) - 1.0 / (2 * p + 2)) < 2e-15


def test_nodes_layout():
    r = nodes(32)
    assert r[-1] == 1.0 and r[0] > 0 and np.all(np.diff(r) > 0)
    # positive half of the 64-point Chebyshev-Gauss-Lobatto grid
    full = np.cos(np.pi * np.arange(64) / 63)
    assert np.allclose(np.sort(full[full > 0]), r, atol=0, rtol=1e-15)


@pytest.mark.parametrize("nr", [16, 33, 64])
def test_fd_exact_on_parity_polynomials(nr):
    R = Radial(nr)
    r = R.r
    for q in range(0, 7):
        p = 1 if q % 2 == 0 else -1
        f = r ** q
        d1 = q * r ** (q - 1) if q >= 1 else 0 * r
        d2 = q * (q - 1) * r ** (q - 2) if q >= 2 else 0 * r
        assert np.max(np.abs(R.D1[p] @ f - d1)) < 1e-9 * max(1, np.max(np.abs(d1)))
        assert np.max(np.abs(R.D2[p] @ f - d2)) < 1e-7 * max(1, np.max(np.abs(d2)))


def test_fd_sixth_order_convergence():
    errs = []
    for nr in (24, 48):
        R = Radial(nr)
        r = R.r
        f = np.cos(3 * r)                       # even
        errs.append(np.max(np.abs(R.D1[1] @ f + 3 * np.sin(3 * r))[:-3]))
    order = np.log2(errs[0] / errs[1])
    assert order > 5.0


def test_wall_rows_one_sided_any_parity():
    R = Radial(20)
    r = R.r
    for q in range(7):
        f = (r - 0.3) ** q
        d1 = q * (r - 0.3) ** (q - 1) if q else 0 * r
        for p in (1, -1):
            assert np.max(np.abs((R.D1[p] @ f - d1)[-3:])) < 1e-8


def test_poisson_conditioning_at_64_nodes_bounds_the_solve_tolerance():
    """The kernel-level parity bound at 64 radial nodes (1e-10 for the solves,
    ten times the others) rests on the conditioning of the interior Poisson
    operator: kappa_2 ~ 2e6 for m = 0, alpha = 0 on the clustered nodes, so two
    backward-stable double-precision solves (the oracle's pivoted LAPACK one,
    the library's unpivoted banded one with long-double factors) may differ by
    up to ~2 kappa eps ~ 5e-10 relative; the Helmholtz operators are benign."""
    import numpy as np
    R = Radial(64)
    L = R.lap(0, 0.0)[:-1, :-1]
    k = np.linalg.cond(L)
    assert 1e6 < k < 1e7
    assert 2 * k * np.finfo(float).eps > 1e-10
    H = np.eye(63) / 0.02 - L / (2 * 2000.0)
    assert np.linalg.cond(H) < 1e2
