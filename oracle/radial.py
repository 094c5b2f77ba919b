"""Radial discretisation of the oracle: nodes, quadrature and sixth-order FD.

Sec. 2.3 of the paper: the radial direction uses high-order (sixth-order)
finite differences on points placed at Chebyshev collocation points.  The
paper leaves the stencil, the axis treatment, the relaxation of the points and
the radial quadrature unstated; the readings taken here are

* nodes: the positive half of a 2N-point Chebyshev-Gauss-Lobatto grid,
  r_j = cos(pi (N-1-j) / (2N-1)), j = 0..N-1, so r_{N-1} = 1 is the wall and
  the axis is not a node (no relaxation);
* sixth-order derivatives from 7-point stencils centred on the node index in
  the grid mirrored through the axis; a mirrored node -r_i carries the field
  value p * f(r_i), where p = +-1 is the field's parity in r; the last three
  rows use the last seven nodes (one-sided);
* quadrature: interpolatory weights in s = r^2 on the nodes s_j = r_j^2, so
  that sum_j w_j g(r_j) approximates int_0^1 g r dr.

Everything is built from first principles: FD weights from the Taylor
(moment) conditions solved exactly in rationals, quadrature weights from
exact Chebyshev moments.
"""
import math

import numpy as np


def nodes(nr):
    """Radial nodes r_j, j = 0..nr-1, ascending, r_{nr-1} = 1."""
    j = np.arange(nr)
    return np.cos(np.pi * (nr - 1 - j) / (2 * nr - 1))


def quad_weights(nr):
    """Weights w_j with sum_j w_j g(r_j) ~ int_0^1 g(r) r dr.

    With s = r^2, int_0^1 g r dr = 1/2 int_0^1 g(sqrt s) ds.  The weights are
    the interpolatory rule on the nodes s_j, found by matching the exact
    moments of the shifted Chebyshev polynomials T_n(2s-1), n < nr.
    """
    s = nodes(nr) ** 2
    x = 2.0 * s - 1.0
    n = np.arange(nr)
    V = np.cos(np.outer(n, np.arccos(np.clip(x, -1.0, 1.0))))   # V[n, j] = T_n(x_j)
    mom = np.zeros(nr)
    even = n % 2 == 0
    mom[even] = 1.0 / (1.0 - n[even].astype(float) ** 2)         # int_0^1 T_n(2s-1) ds
    W = np.linalg.solve(V, mom)
    return 0.5 * W


def fd_weights(x0, xs, order):
    """Weights c with sum_i c_i f(xs_i) = f^(order)(x0), exact for deg <= len(xs)-1.

    The Taylor (moment) conditions sum_i c_i (xs_i - x0)^q / q! = delta_{q, order}
    are solved exactly in rational arithmetic on the (exactly representable)
    double values of the nodes; only the final weights are rounded.
    """
    from fractions import Fraction
    d = [Fraction(float(x)) - Fraction(float(x0)) for x in xs]
    npt = len(d)
    A = [[d[i] ** q / math.factorial(q) for i in range(npt)] + [Fraction(int(q == order))] for q in range(npt)]
    for k in range(npt):
        piv = next(i for i in range(k, npt) if A[i][k] != 0)
        A[k], A[piv] = A[piv], A[k]
        for i in range(npt):
            if i != k and A[i][k] != 0:
                f = A[i][k] / A[k][k]
                A[i] = [a - f * b for a, b in zip(A[i], A[k])]
    return np.array([float(A[i][npt] / A[i][i]) for i in range(npt)])


def stencil(nr, j):
    """Column indices (in the mirrored numbering) of the 7-point stencil of row j.

    A negative index c stands for the mirror image -r_{-c-1} of node -c-1.
    """
    if j >= nr - 3:
        return list(range(nr - 7, nr))
    return list(range(j - 3, j + 4))


def fd_matrix(nr, order, parity):
    """Dense nr x nr matrix of the order-th derivative for a field of given parity."""
    r = nodes(nr)
    D = np.zeros((nr, nr))
    for j in range(nr):
        cols = stencil(nr, j)
        xs = [r[c] if c >= 0 else -r[-c - 1] for c in cols]
        c = fd_weights(r[j], xs, order)
        for cc, wgt in zip(cols, c):
            if cc >= 0:
                D[j, cc] += wgt
            else:
                D[j, -cc - 1] += parity * wgt
    return D


class Radial:
    """Radial grid, weights and FD matrices for both parities."""

    def __init__(self, nr):
        if nr < 8:
            raise ValueError("need at least 8 radial nodes for 7-point stencils")
        self.nr = nr
        self.r = nodes(nr)
        self.w = quad_weights(nr)
        self.D1 = {p: fd_matrix(nr, 1, p) for p in (1, -1)}
        self.D2 = {p: fd_matrix(nr, 2, p) for p in (1, -1)}

    @staticmethod
    def parity(n):
        """Parity in r of a scalar carrying azimuthal index n: (-1)^n."""
        return 1 if n % 2 == 0 else -1

    def lap(self, n, alpha):
        """Scalar Laplacian D2 + D1/r - n^2/r^2 - alpha^2 for azimuthal index n."""
        p = self.parity(n)
        r = self.r
        return (self.D2[p] + self.D1[p] / r[:, None]
                - np.diag(n * n / r ** 2) - alpha * alpha * np.eye(self.nr))
