"""Pins of the oracle's dealiased nonlinear term."""
import numpy as np
import pytest

from oracle.pipe import Pipe
from paper_2509_10103_amd import synth


def full_hermitian(F, M, K):
    """dict (k, m) -> coefficient over |m| <= M, |k| <= K from the m >= 0 storage."""
    nk = 2 * K + 1
    d = {}
    for m in range(M + 1):
        for kk in range(nk):
            k = kk if kk <= K else kk - nk
            d[(k, m)] = F[..., m, kk]
            if m > 0:
                d[(-k, -m)] = np.conj(F[..., m, kk])
    return d


def brute_product(A, B, M, K):
    a, b = full_hermitian(A, M, K), full_hermitian(B, M, K)
    nk = 2 * K + 1
    out = np.zeros(A.shape, dtype=complex)
    for m in range(M + 1):
        for kk in range(nk):
            k = kk if kk <= K else kk - nk
            s = 0
            for (k1, m1), x in a.items():
                y = b.get((k - k1, m - m1))
                if y is not None:
                    s = s + x * y
            out[..., m, kk] = s
    return out


@pytest.mark.parametrize("nt,nz", [(6, 6), (9, 12), (12, 8), (8, 16)])
def test_padded_product_equals_brute_force_convolution(nt, nz):
    P = Pipe(8, nt, nz, 3.0, 1000, 5, 0.5, 0.01)
    A = synth.random_field(P.shape, 11)[0]
    B = synth.random_field(P.shape, 12)[0]
    A[:, 0, 0] = A[:, 0, 0].real
    B[:, 0, 0] = B[:, 0, 0].real
    fast = P.to_spec(P.to_phys(A) * P.to_phys(B))
    slow = brute_product(A, B, P.M, P.K)
    assert np.max(np.abs(fast - slow)) < 1e-13 * np.max(np.abs(slow))


def test_transform_round_trip():
    P = Pipe(8, 24, 48, 4 * np.pi, 2000, 8, 0.5, 0.04)
    F = synth.random_field(P.shape, 5)
    assert np.max(np.abs(P.to_spec(P.to_phys(F)) - F)) < 1e-14 * np.max(np.abs(F))


def test_convective_term_does_no_work():
    # u . (u x w) = 0 pointwise, and <y, P_K F f>_W = <Y, f>_phys for band-limited y
    P = Pipe(16, 12, 18, 2 * np.pi, 2000, 8, 1.0, 0.02)
    u = synth.smooth_modes(P.r, P.M, P.K, 3)
    w = P.curl(u)
    nl = P.to_spec(P.cross(P.to_phys(u), P.to_phys(w)))
    scale = np.sqrt(P.wdot(u, u) * P.wdot(nl, nl))
    assert abs(P.wdot(u, nl)) < 1e-14 * scale


def test_curl_of_gradient_vanishes():
    # curl grad phi = 0 for phi = f(r) e^{i(m theta + alpha z)}, exact when f is a low polynomial
    P = Pipe(24, 12, 12, 2 * np.pi, 2000, 8, 1.0, 0.02)
    r = P.r
    u = P.zeros()
    m, kk = 2, 1
    a = P.alpha[kk]
    f = r ** 2 * (1 - r ** 2)           # parity of m = 2 scalar
    fp = 2 * r - 4 * r ** 3
    u[0, :, m, kk] = fp
    u[1, :, m, kk] = 1j * m / r * f
    u[2, :, m, kk] = 1j * a * f
    w = P.curl(u)
    assert np.max(np.abs(w)) < 1e-10
