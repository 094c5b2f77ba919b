"""Oracle: admissible-set projection, energy-preserving update and one
adjoint-looping iteration (paper Sec. 2.1 and 2.2).

* ``project``: the W-orthogonal projector P_h onto admissible perturbations:
  zero wall velocity, discrete divergence zero at every radial node, and for
  the mean mode u_r = 0 and zero flux (Sec. 2, continuity and zero bulk
  velocity).  Formed per mode from a QR factorisation of W^{-1/2} G^H, with G
  the constraint rows, so that P_h = W^{-1/2} (I - Q Q^H) W^{1/2}.
* ``update``: the gradient step of Sec. 2.2, u' = (1 + lambda alpha) u0 -
  alpha u0_dag with lambda the '+' root of the energy constraint (Sec. 2.2,
  quadratic for lambda) and alpha_max from the reality condition; the result
  is rescaled to E0 to remove rounding drift.
* ``iterate``: forward sweep, compatibility condition u_dag(T) = -u(T),
  backward adjoint sweep, projection, and the backtracking line search of
  Sec. 2.2 (start at alpha_max, halve while G does not increase, stop when
  |dG/G| < tol).
"""
import math

import numpy as np


def constraint_rows(P, m, alpha):
    """Rows G of the admissible-set constraints of one mode (on 3nr unknowns)."""
    nr = P.nr
    r = P.r
    rows = []
    eye = np.eye(nr)
    for c in range(3):                                  # wall velocity
        g = np.zeros(3 * nr, dtype=complex)
        g[c * nr + nr - 1] = 1.0
        rows.append(g)
    if m == 0 and alpha == 0.0:
        for j in range(nr - 1):                         # u_r = 0 (wall row above)
            g = np.zeros(3 * nr, dtype=complex)
            g[j] = 1.0
            rows.append(g)
        g = np.zeros(3 * nr, dtype=complex)             # zero flux
        g[2 * nr:] = P.w
        rows.append(g)
        return np.array(rows)
    D1o = P.rad.D1[P.rad.parity(m + 1)]
    div = np.hstack([D1o + np.diag(1.0 / r), 1j * m * np.diag(1.0 / r), 1j * alpha * eye])
    return np.vstack([np.array(rows), div])


def project(P, u):
    """P_h u: W-orthogonal projection onto the admissible subspace."""
    out = np.empty_like(u)
    wv = np.tile(P.w, 3)
    sw = np.sqrt(wv)
    for m, kk, a in P.modes():
        G = constraint_rows(P, m, a)
        B = (G / sw[None, :]).conj().T                  # W^{-1/2} G^H
        Q, _ = np.linalg.qr(B)
        y = sw * u[:, :, m, kk].reshape(-1)
        v = (y - Q @ (Q.conj().T @ y)) / sw
        out[:, :, m, kk] = v.reshape(3, P.nr)
    return out


def lambda_plus(alpha, E0, E0d, C0):
    """'+' root of the energy constraint for the multiplier (Sec. 2.2)."""
    a = (alpha * C0 - 2.0 * E0) / (2.0 * alpha * E0)
    disc = ((-alpha * C0 + 2.0 * E0) / (2.0 * alpha * E0)) ** 2 - (alpha * E0d - C0) / (alpha * E0)
    return a + math.sqrt(max(disc, 0.0))


def alpha_max(E0, E0d, C0):
    q = E0d / E0 - C0 * C0 / (4.0 * E0 * E0)
    return math.inf if q <= 0.0 else q ** -0.5


def update(P, u0, udag, E0, alpha):
    """u' = (1 + lambda+ alpha) u0 - alpha udag, rescaled to energy E0."""
    E0d = 0.5 * P.wdot(udag, udag)
    C0 = P.wdot(u0, udag)
    lam = lambda_plus(alpha, E0, E0d, C0)
    un = (1.0 + lam * alpha) * u0 - alpha * udag
    return un * math.sqrt(E0 / P.energy(un)), dict(E0dag=E0d, C0=C0, lam=lam)


def normalise(P, u, E0):
    return u * math.sqrt(E0 / P.energy(u))


def iterate(P, u0, E0, nsteps, G=None, tol=1e-8, max_halvings=30):
    """One adjoint-looping iteration from u0 (energy E0).

    Returns (u0_next, G_next, info).  If G is None the forward gain at u0 is
    computed first.  info['status'] is 'accepted' or 'converged'.
    """
    J, uN, lam0 = P.gradient(u0, nsteps)
    G0 = J / E0
    g = project(P, lam0)
    udag = -g                                            # u_dag = -lambda (compatibility)
    E0d = 0.5 * P.wdot(udag, udag)
    C0 = P.wdot(u0, udag)
    amax = alpha_max(E0, E0d, C0)
    info = dict(G=G0, E0dag=E0d, C0=C0, alpha_max=amax, trials=[])
    if not math.isfinite(amax):
        info['status'] = 'converged'
        return u0, G0, info
    alpha = amax
    for _ in range(max_halvings + 1):
        un, _ = update(P, u0, udag, E0, alpha)
        Gn = P.energy(P.forward(un, nsteps)) / E0
        info['trials'].append((alpha, Gn))
        if Gn > G0:
            info['status'] = 'accepted'
            info['alpha'] = alpha
            return un, Gn, info
        if abs((Gn - G0) / Gn) < tol:
            break
        alpha *= 0.5
    info['status'] = 'converged'
    return u0, G0, info
