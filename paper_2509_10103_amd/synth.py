"""Seeded synthetic perturbations (raw random coefficients).

This module only draws random numbers and shapes them with smooth radial and
axial envelopes; it holds none of the method's arithmetic (no projection, no
normalisation, no solver).  Both the HIP path and the CPU oracle take its
arrays as input and project/normalise them with their own code.

Layout: complex128 [3][nr][M+1][2K+1], components (u_r, u_theta, u_z), axial
index in FFT order (k = 0..K, -K..-1); the m = 0 column is Hermitian in k.
"""
import numpy as np


def kvalues(K):
    kk = np.arange(2 * K + 1)
    return np.where(kk <= K, kk, kk - (2 * K + 1))


def _hermitian_m0(a, K):
    """Make the m = 0 column Hermitian: a(-k) = conj(a(k)), a(0) real."""
    nk = 2 * K + 1
    for k in range(1, K + 1):
        a[:, :, 0, nk - k] = np.conj(a[:, :, 0, k])
    a[:, :, 0, 0] = a[:, :, 0, 0].real
    return a


def smooth_modes(r, M, K, seed, decay=4.0, mset=None, kmask=None):
    """Random smooth coefficients, one polynomial profile per mode/component.

    u_c(r) = r^{s_c} (1 - r^2) (a0 + a1 r^2 + a2 r^4 + a3 r^6) * amp(k, m)
    with complex Gaussian a_i, s_r = s_theta = |m-1|, s_z = |m| (regular at
    the axis with the parity of each component) and amp = exp(-(|k|+m)/decay).
    ``mset`` restricts the azimuthal indices, ``kmask`` (bool per kk) the
    axial ones.
    """
    r = np.asarray(r, dtype=float)
    nr = len(r)
    nk = 2 * K + 1
    kv = kvalues(K)
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal((3, 4, M + 1, nk)) + 1j * rng.standard_normal((3, 4, M + 1, nk))
    out = np.zeros((3, nr, M + 1, nk), dtype=complex)
    r2 = r * r
    poly = np.stack([r2 ** i for i in range(4)])          # (4, nr)
    for m in range(M + 1):
        if mset is not None and m not in mset:
            continue
        s = [abs(m - 1), abs(m - 1), m]
        for c in range(3):
            prof = np.einsum('in,ik->nk', poly, coef[c, :, m, :])   # (nr, nk)
            prof *= (r ** s[c] * (1.0 - r2))[:, None]
            amp = np.exp(-(np.abs(kv) + m) / decay)
            if kmask is not None:
                amp = amp * kmask
            out[c, :, m, :] = prof * amp[None, :]
    return _hermitian_m0(out, K)


def z_envelope(a, lz, nz_phys, sigma, centre):
    """Multiply each (c, j, m) axial series by a periodic Gaussian in z.

    Done on an nz_phys-point grid in z and truncated back to |k| <= K.
    """
    K = (a.shape[-1] - 1) // 2
    kv = kvalues(K)
    z = np.arange(nz_phys) * lz / nz_phys
    d = (z - centre + 0.5 * lz) % lz - 0.5 * lz
    g = np.exp(-0.5 * (d / sigma) ** 2)
    pos = np.where(kv >= 0, kv, nz_phys + kv)
    Z = np.zeros(a.shape[:-1] + (nz_phys,), dtype=complex)
    Z[..., pos] = a
    f = np.fft.ifft(Z, axis=-1) * nz_phys
    b = np.fft.fft(f * g, axis=-1) / nz_phys
    return np.ascontiguousarray(_hermitian_m0(b[..., pos], K))   # C order: device copies keep the layout


def localized_oblique(r, M, K, lz, nz_phys, seed, amin=3.5, amax=6.5, sigma=6.0):
    """|m| = 1 oblique pair with |alpha_k| in [amin, amax], Gaussian in z."""
    kv = kvalues(K)
    al = np.abs(kv) * 2.0 * np.pi / lz
    kmask = ((al >= amin) & (al <= amax)).astype(float)
    a = smooth_modes(r, M, K, seed, decay=1e9, mset={1}, kmask=kmask)
    # equal weight of +m and -m: |a(k, 1)| = |a(-k, 1)|
    nk = 2 * K + 1
    for k in range(1, K + 1):
        mag = 0.5 * (np.abs(a[:, :, 1, k]) + np.abs(a[:, :, 1, nk - k]))
        a[:, :, 1, k] = mag * np.exp(1j * np.angle(a[:, :, 1, k]))
        a[:, :, 1, nk - k] = mag * np.exp(1j * np.angle(a[:, :, 1, nk - k]))
    return z_envelope(a, lz, nz_phys, sigma, 0.5 * lz)


def random_field(shape, seed):
    """Plain complex Gaussian field (for dot-product and direction tests)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    K = (shape[-1] - 1) // 2
    return _hermitian_m0(a, K)


def _poly_eval(c, r):
    """sum_i c[i] r^i for coefficient arrays c of shape (deg+1, ...)."""
    out = np.zeros(np.broadcast(r[:, None], c[0][None, ...]).shape if c.ndim > 1 else r.shape, dtype=complex)
    for i in range(len(c) - 1, -1, -1):
        out = out * (r[:, None] if c.ndim > 1 else r) + (c[i][None, ...] if c.ndim > 1 else c[i])
    return out


def solenoidal_modes(r, M, K, lz, seed, decay=4.0, mset=None, kmask=None):
    """Smooth, divergence-free, wall-compatible random coefficients.

    Per mode (k, m) the field is u = curl(psi e_z) + curl curl(phi e_z) with
        psi = r^m (1 - r^2)^2 p(r^2),  phi = r^m (1 - r^2)^3 q(r^2),
    p, q cubic with complex Gaussian coefficients, so that
        u_r = (i m / r) psi + i a phi',  u_theta = -psi' - (m a / r) phi,
        u_z = -(phi'' + phi'/r - m^2 phi / r^2)
    vanishes at r = 1, is regular at the axis and has zero divergence (and,
    for the mean mode, zero flux) in the continuum.  Amplitude
    exp(-(|k|+m)/decay); ``mset``/``kmask`` restrict the modes.
    """
    from numpy.polynomial import polynomial as Pl
    r = np.asarray(r, dtype=float)
    nr = len(r)
    nk = 2 * K + 1
    kv = kvalues(K)
    al = kv * 2.0 * np.pi / lz
    rng = np.random.default_rng(seed)
    cp = rng.standard_normal((4, M + 1, nk)) + 1j * rng.standard_normal((4, M + 1, nk))
    cq = rng.standard_normal((4, M + 1, nk)) + 1j * rng.standard_normal((4, M + 1, nk))
    out = np.zeros((3, nr, M + 1, nk), dtype=complex)
    w2 = Pl.polypow([1.0, 0.0, -1.0], 2)          # (1 - r^2)^2
    w3 = Pl.polypow([1.0, 0.0, -1.0], 3)          # (1 - r^2)^3
    for m in range(M + 1):
        if mset is not None and m not in mset:
            continue
        for kk in range(nk):
            amp = np.exp(-(abs(kv[kk]) + m) / decay)
            if kmask is not None:
                amp *= kmask[kk]
            if amp == 0.0:
                continue
            a = al[kk]
            pe = np.zeros(7, dtype=complex)
            qe = np.zeros(7, dtype=complex)
            pe[0:7:2] = cp[:, m, kk]
            qe[0:7:2] = cq[:, m, kk]
            mono = np.zeros(m + 1)
            mono[m] = 1.0
            psi = Pl.polymul(Pl.polymul(mono, w2), pe)
            phi = Pl.polymul(Pl.polymul(mono, w3), qe)
            dpsi, dphi = Pl.polyder(psi), Pl.polyder(phi)
            d2phi = Pl.polyder(phi, 2)
            # the 1/r terms are exact polynomial divisions (psi, phi ~ r^m)
            if m > 0:
                psi_r = psi[1:]
                phi_r = phi[1:]
                phi_r2 = phi[2:]
            else:
                psi_r = phi_r = phi_r2 = np.zeros(1)
            dphi_r = dphi[1:] if len(dphi) > 1 else np.zeros(1)
            ur = 1j * m * Pl.polyval(r, psi_r) + 1j * a * Pl.polyval(r, dphi)
            ut = -Pl.polyval(r, dpsi) - m * a * Pl.polyval(r, phi_r)
            uz = -(Pl.polyval(r, d2phi) + Pl.polyval(r, dphi_r) - m * m * Pl.polyval(r, phi_r2))
            out[0, :, m, kk] = amp * ur
            out[1, :, m, kk] = amp * ut
            out[2, :, m, kk] = amp * uz
    return _hermitian_m0(out, K)
