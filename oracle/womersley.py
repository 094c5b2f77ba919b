"""Sexl-Womersley laminar base flow of the oracle (Sec. 2, base flow).

Lengths are scaled by the radius and velocities by twice the mean bulk
velocity, so the steady part is 1 - r^2 and the enforced bulk velocity is
u_b(t) = 1/2 [1 + A sin(2 pi t / T)] (Sec. 2).  In these units the angular
frequency is Wo^2 / Re and the period T = 2 pi Re / Wo^2; the paper prints the
period in diameter/mean-velocity units (Appendix A, pulsatile validation).

The oscillating part is the classical Womersley solution driven so that its
flux is the prescribed oscillation:
    U(r, t) = 1 - r^2 + Re[ Ut(r) exp(i w t) ],
    Ut(r)   = b [1 - J0(k r)/J0(k)] / [1 - 2 J1(k)/(k J0(k))],
    k = Wo exp(3 i pi / 4),  b = -i A / 2,  w = Wo^2 / Re,
with J0, J1 taken from scipy on complex arguments.
"""
import numpy as np
from scipy.special import jv


def omega(re, wo):
    return wo * wo / re


def period(re, wo):
    return 2.0 * np.pi * re / (wo * wo)


def profile(r, wo, amp):
    """Complex amplitude Ut(r) and its radial derivative Ut'(r)."""
    r = np.asarray(r, dtype=float)
    if amp == 0.0:
        z = np.zeros_like(r, dtype=complex)
        return z, z.copy()
    kap = wo * np.exp(0.75j * np.pi)
    b = -0.5j * amp
    j0k = jv(0, kap)
    den = 1.0 - 2.0 * jv(1, kap) / (kap * j0k)
    ut = b * (1.0 - jv(0, kap * r) / j0k) / den
    dut = b * kap * jv(1, kap * r) / j0k / den
    return ut, dut


def base_flow(r, t, re, wo, amp):
    """U(r,t) and Omega_theta(r,t) = -dU/dr at the nodes r."""
    ut, dut = profile(r, wo, amp)
    ph = np.exp(1j * omega(re, wo) * t) if amp != 0.0 else 0.0
    U = 1.0 - r * r + np.real(ut * ph)
    dU = -2.0 * r + np.real(dut * ph)
    return U, -dU
