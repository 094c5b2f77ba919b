"""Oracle: discrete perturbation Navier-Stokes step for pulsatile pipe flow,
its tangent and its exact discrete adjoint (all FP64, NumPy/SciPy).

What is computed (paper Sec. 2 and 2.3; readings listed in the design notes):

Fields are Fourier-Galerkin series in theta and z (Sec. 2.3, Fourier
expansion), stored as complex coefficients F[c, j, m, kk] with component c in
(r, theta, z), radial node j, azimuthal index m = 0..M and axial index kk in
FFT order (k = 0..K, -K..-1); the m = 0 column is Hermitian in k.  The
retained band |m| <= M = (N_theta-1)//3, |k| <= K = (N_z-1)//3 makes the
N_theta x N_z physical grid a 3/2-rule dealiasing grid.

The perturbation equation (Sec. 2, direct Navier-Stokes equations) is taken
in rotational form,
    du/dt = u x w + U x w + u x Om - grad p' - f_z e_z + (1/Re) lap u,
with w = curl u, U = U(r,t) e_z the Womersley flow and Om = curl U; the
gradient of (|u|^2/2 + U.u) is absorbed in the pressure.  Time stepping is the
second-order predictor-corrector of Sec. 2.3: Crank-Nicolson on the viscous
term, explicit Euler predictor and trapezoidal corrector for the convective
terms, the pressure and the flux-holding gradient f_z implicit in every stage,
the corrector iterated ncorr times (default 2):
    w_0     = S(E u^n + N(u^n, t_n))
    w_c     = S(E u^n + (N(u^n, t_n) + N(w_{c-1}, t_{n+1})) / 2),  c = 1..ncorr
    u^{n+1} = w_ncorr.
A single corrector pass is Heun's method on the convective terms, whose
amplification on the imaginary axis exceeds one (by (a U dt)^4 / 8 per step);
two passes are dissipative there for |a U dt| < 2.
S is the per-mode solve of H u + grad p = R, div u = 0, u(1) = 0 with the
influence-matrix correction for the wall (Sec. 2.3, wall boundary conditions)
and, for the mean mode, the zero-flux constraint (Sec. 2, zero bulk velocity).

The adjoint is the exact transpose of this discrete step in the W inner
product <a,b>_W = 2 pi L_z sum_{k,m} c_m sum_j w_j Re(conj a . b), c_0 = 1,
c_{m>0} = 2 (Sec. 2, definition of <...>).  Linear per-mode maps (E, curl,
S) are materialised as dense matrices A, and their adjoints are formed as
W^{-1} A^H W.  The convective adjoint uses the identity
    <y, P_K F[a x b]>_W = <Y, a x b>_phys
for band-limited y, which gives
    N'(u)^dag y = P_K F[(Om + w_u) x Y] + curl^dag P_K F[Y x (U + u)].

Beside it, the continuous adjoint of the paper (Sec. 2, adjoint Navier-Stokes
equations, integrated backwards from the compatibility condition): with
V = U + u the total velocity and Omega = curl V, the adjoint convective term
-(V . grad) y + (grad V)^T y equals, up to a gradient that the adjoint
pressure absorbs, -(Omega x y + curl(y x V)), since curl(y x V) =
(V . grad) y - (y . grad) V and Omega x y = (y . grad) V - (grad V)^T y for
solenoidal V and y.  Integrated backwards in s = t_N - t, the adjoint field
obeys dy/ds = Omega x y + curl(y x V) - grad p' + f'_z e_z + (1/Re) lap y with
y = 0 at the wall and zero flux, the same form as the direct equation, so it
is discretised with the same stepper (Sec. 2.3) and the same S and E: the
pseudo-spectral term Nc(u; y) = P_K F[Omega x Y] + curl P_K F[Y x V] is the
discrete adjoint term with curl in place of curl^dag, the predictor taking the
direct field at t_{n+1} and the correctors the one at t_n.  Its gradient
differs from the exact discrete one by the discretisation error.
"""
import numpy as np
import scipy.linalg as sl

from .radial import Radial
from . import womersley


def sizes(ntheta, nz):
    """Retained band (M, K) of a N_theta x N_z 3/2-rule physical grid."""
    return (ntheta - 1) // 3, (nz - 1) // 3


class Pipe:
    """One discretised problem: grid, flow parameters, time step."""

    def __init__(self, nr, ntheta, nz, lz, re, wo, amp, dt, tau0=0.0, ncorr=2):
        if ncorr < 1:
            raise ValueError("at least one corrector pass")
        self.ncorr = int(ncorr)
        self.nr, self.ntheta, self.nz = nr, ntheta, nz
        self.lz, self.re, self.wo, self.amp = float(lz), float(re), float(wo), float(amp)
        self.dt, self.tau0 = float(dt), float(tau0)
        self.M, self.K = sizes(ntheta, nz)
        self.nk = 2 * self.K + 1
        kk = np.arange(self.nk)
        self.kint = np.where(kk <= self.K, kk, kk - self.nk)
        self.k0 = 2.0 * np.pi / self.lz
        self.alpha = self.kint * self.k0
        self.rad = Radial(nr)
        self.r, self.w = self.rad.r, self.rad.w
        self.cm = np.array([1.0] + [2.0] * self.M)
        self.shape = (3, nr, self.M + 1, self.nk)
        self._lu = {}
        self._mats = {}
        self.cache_bytes = 0
        self.cache_limit = 4 << 30

    # ------------------------------------------------------------------ basics
    def zeros(self):
        return np.zeros(self.shape, dtype=complex)

    def wdot(self, a, b):
        """<a, b>_W, the discrete form of the paper's volume integral."""
        s = np.einsum('j,m,cjmk->', self.w, self.cm, (np.conj(a) * b).real)
        return 2.0 * np.pi * self.lz * s

    def energy(self, u):
        return 0.5 * self.wdot(u, u)

    def component_energies(self, u):
        """E_r, E_theta, E_z: half the W inner product of each component with
        itself (their sum is E(u)); the decomposition of the growth into its
        axial and cross-sectional parts (Sec. 3-4)."""
        return np.array([0.5 * 2.0 * np.pi * self.lz *
                         np.einsum('j,m,jmk->', self.w, self.cm, np.abs(u[c]) ** 2) for c in range(3)])

    def mode_energies(self, u):
        """Energy of every stored mode (m, kk): 1/2 2 pi L_z c_m sum_j w_j |u|^2."""
        return np.pi * self.lz * self.cm[:, None] * np.einsum('j,cjmk->mk', self.w, np.abs(u) ** 2)

    def band_energies(self, u):
        """Energy in the highest azimuthal modes m = M and in the highest axial
        modes |k| = K (the quantities of the resolution criterion, Sec. 2.3)."""
        e = self.mode_energies(u)
        return e[self.M, :].sum(), e[:, self.K].sum() + e[:, self.nk - self.K].sum()

    def time(self, n):
        return self.tau0 + n * self.dt

    def base(self, t):
        return womersley.base_flow(self.r, t, self.re, self.wo, self.amp)

    def modes(self):
        """Iterate (m, kk, alpha) over all stored modes."""
        for m in range(self.M + 1):
            for kk in range(self.nk):
                yield m, kk, self.alpha[kk]

    # ------------------------------------------------------- radial operators
    def lap(self, n, alpha):
        return self.rad.lap(n, alpha)

    def _factor(self, kind, n, alpha):
        key = (kind, abs(n), round(abs(alpha), 14))
        f = self._lu.get(key)
        if f is None:
            L = self.lap(n, alpha)
            if kind == 'H':
                A = np.eye(self.nr) / self.dt - L / (2.0 * self.re)
            else:
                A = L
            f = sl.lu_factor(A[:-1, :-1])
            self._lu[key] = f
        return f

    def _inv(self, kind, n, alpha, b):
        """Interior solve with wall column removed; b complex (nr-1, ...)."""
        f = self._factor(kind, n, alpha)
        return sl.lu_solve(f, b.real) + 1j * sl.lu_solve(f, b.imag)

    def _inv_T(self, kind, n, alpha, b):
        """Transposed interior solve A^T x = b (A real), b complex."""
        f = self._factor(kind, n, alpha)
        return sl.lu_solve(f, b.real, trans=1) + 1j * sl.lu_solve(f, b.imag, trans=1)

    def _par(self, n):
        return self.rad.parity(n)

    # ----------------------------------------------------- per-mode linear maps
    def curl_mode(self, m, alpha, u):
        """Spectral curl of one mode; u has shape (3, nr, ...)."""
        r = self.r.reshape((-1,) + (1,) * (u.ndim - 2))
        D1z = self.rad.D1[self._par(m)]
        D1t = self.rad.D1[self._par(m + 1)]
        ur, ut, uz = u[0], u[1], u[2]
        wr = 1j * m / r * uz - 1j * alpha * ut
        wt = 1j * alpha * ur - np.tensordot(D1z, uz, axes=(1, 0))
        wz = np.tensordot(D1t, ut, axes=(1, 0)) + ut / r - 1j * m / r * ur
        return np.stack([wr, wt, wz])

    def E_mode(self, m, alpha, u):
        """E u = u/dt + lap(u)/(2 Re), vector Laplacian in the (u+, u-) basis."""
        up = u[0] + 1j * u[1]
        um = u[0] - 1j * u[1]
        c = 1.0 / (2.0 * self.re)
        Ep = up / self.dt + c * np.tensordot(self.lap(m + 1, alpha), up, axes=(1, 0))
        Em = um / self.dt + c * np.tensordot(self.lap(m - 1, alpha), um, axes=(1, 0))
        Ez = u[2] / self.dt + c * np.tensordot(self.lap(m, alpha), u[2], axes=(1, 0))
        return np.stack([0.5 * (Ep + Em), (Ep - Em) / 2j, Ez])

    def S_mode(self, m, alpha, R, return_p=False):
        """Solve H u + grad p = R, div u = 0, u(1) = 0 for one mode.

        R has shape (3, nr, ncol).  Steps (Sec. 2.3 influence-matrix method):
        particular pressure from lap p = div R with p(1) = 0, particular
        velocities from H u = R - grad p with u(1) = 0; homogeneous pressure
        lap p_h = 0, p_h(1) = 1, and H u_h = -grad p_h; the multiple of the
        homogeneous pair that zeroes d(u_r)/dr at the wall (the discrete wall
        divergence) is added.  The mean mode (0, 0) has u_r = 0 and its axial
        part carries the flux-holding gradient f_z (Sec. 2, pressure split).
        """
        nr = self.nr
        r = self.r[:, None]
        ncol = R.shape[2]
        u = np.zeros((3, nr, ncol), dtype=complex)
        if m == 0 and alpha == 0.0:
            u[1, :-1] = self._inv('H', 1, 0.0, R[1, :-1])
            uz = self._inv('H', 0, 0.0, R[2, :-1])
            g = self._inv('H', 0, 0.0, np.ones((nr - 1, 1), dtype=complex))
            wi = self.w[:-1]
            c = -(wi @ uz) / (wi @ g)
            u[2, :-1] = uz + g * c[None, :]
            return u
        D1o = self.rad.D1[self._par(m + 1)]      # parity of u_r, u_theta, u+-
        D1e = self.rad.D1[self._par(m)]          # parity of u_z and p
        Rp = R[0] + 1j * R[1]
        Rm = R[0] - 1j * R[1]
        div = 0.5 * (D1o @ Rp + (1 + m) / r * Rp + D1o @ Rm + (1 - m) / r * Rm) + 1j * alpha * R[2]
        p = np.zeros((nr, ncol), dtype=complex)
        p[:-1] = self._inv('P', m, alpha, div[:-1])
        gp = (D1e @ p - m / r * p)[:-1]
        gm = (D1e @ p + m / r * p)[:-1]
        gz = 1j * alpha * p[:-1]
        up = np.zeros((nr, ncol), dtype=complex)
        um = np.zeros((nr, ncol), dtype=complex)
        uz = np.zeros((nr, ncol), dtype=complex)
        up[:-1] = self._inv('H', m + 1, alpha, Rp[:-1] - gp)
        um[:-1] = self._inv('H', m - 1, alpha, Rm[:-1] - gm)
        uz[:-1] = self._inv('H', m, alpha, R[2, :-1] - gz)
        # homogeneous pair
        L = self.lap(m, alpha)
        ph = np.zeros((nr, 1), dtype=complex)
        ph[-1] = 1.0
        ph[:-1] = -self._inv('P', m, alpha, L[:-1, -1:].astype(complex))
        hp = np.zeros((nr, 1), dtype=complex)
        hm = np.zeros((nr, 1), dtype=complex)
        hz = np.zeros((nr, 1), dtype=complex)
        hp[:-1] = self._inv('H', m + 1, alpha, -(D1e @ ph - m / r * ph)[:-1])
        hm[:-1] = self._inv('H', m - 1, alpha, -(D1e @ ph + m / r * ph)[:-1])
        hz[:-1] = self._inv('H', m, alpha, -(1j * alpha * ph)[:-1])
        s = D1o[-1] @ (up + um)
        sh = (D1o[-1] @ (hp + hm))[0]
        a = -s / sh
        up = up + hp * a[None, :]
        um = um + hm * a[None, :]
        uz = uz + hz * a[None, :]
        u[0] = 0.5 * (up + um)
        u[1] = (up - um) / 2j
        u[2] = uz
        if return_p:
            return u, p + ph * a[None, :]
        return u

    def mode_matrix(self, kind, m, alpha):
        """Dense 3nr x 3nr matrix of a per-mode linear map."""
        n3 = 3 * self.nr
        eye = np.eye(n3, dtype=complex).reshape(3, self.nr, n3)
        if kind == 'S':
            A = self.S_mode(m, alpha, eye)
        elif kind == 'E':
            A = self.E_mode(m, alpha, eye)
        elif kind == 'C':
            A = self.curl_mode(m, alpha, eye)
        else:
            raise ValueError(kind)
        return A.reshape(n3, n3)

    def adjoint_matrix(self, kind, m, alpha):
        """W^{-1} A^H W for the per-mode map A (the W-adjoint)."""
        A = self.mode_matrix(kind, m, alpha)
        wv = np.tile(self.w, 3)
        return (A.conj().T * wv[None, :]) / wv[:, None]

    def _stack_m(self, kind, adjoint, m):
        """Matrices of all axial modes at azimuthal index m, (nk, 3nr, 3nr)."""
        key = (kind, adjoint, m)
        A = self._mats.get(key)
        if A is None:
            f = self.adjoint_matrix if adjoint else self.mode_matrix
            A = np.stack([f(kind, m, a) for a in self.alpha])
            if self.cache_bytes + A.nbytes <= self.cache_limit:
                self._mats[key] = A
                self.cache_bytes += A.nbytes
        return A

    def apply_modes(self, F, kind, adjoint=False):
        """Apply a per-mode map (kind in 'S', 'E', 'C') to a whole field."""
        n3 = 3 * self.nr
        out = np.empty_like(F)
        for m in range(self.M + 1):
            A = self._stack_m(kind, adjoint, m)
            x = F[:, :, m, :].reshape(n3, self.nk)
            out[:, :, m, :] = np.einsum('kab,bk->ak', A, x).reshape(3, self.nr, self.nk)
        return out

    def _fits(self):
        """Whether one kind of per-mode matrix for all modes fits the cache."""
        n3 = 3 * self.nr
        return (self.M + 1) * self.nk * n3 * n3 * 16 <= self.cache_limit // 4

    def S(self, R):
        # the same linear map either way: materialised when it fits in memory
        return self.apply_modes(R, 'S') if self._fits() else self.S_direct(R)

    def S_direct(self, R):
        """S applied mode by mode through the literal solve (no matrices)."""
        out = np.empty_like(R)
        for m in range(self.M + 1):
            for kk in range(self.nk):
                out[:, :, m, kk:kk + 1] = self.S_mode(m, self.alpha[kk], R[:, :, m, kk:kk + 1])
        return out

    def S_adj_mode(self, m, alpha, Y):
        """W^{-1} S^H W Y for one mode, applied as the reversed chain of
        conjugate-transposed steps of S_mode (pinned against the materialised
        W^{-1} S^H W in the tests).  Y has shape (3, nr, ncol)."""
        nr = self.nr
        r = self.r[:-1, None]
        wi = self.w[:-1]
        y = Y * self.w[None, :, None]
        y[:, -1] = 0.0                                   # the solve's wall output is identically zero
        out = np.zeros_like(Y)
        if m == 0 and alpha == 0.0:
            out[1, :-1] = self._inv_T('H', 1, 0.0, y[1, :-1])
            g = self._inv('H', 0, 0.0, np.ones((nr - 1, 1), dtype=complex))[:, 0].real
            yz = y[2, :-1] - wi[:, None] * (g @ y[2, :-1])[None, :] / (wi @ g)
            out[2, :-1] = self._inv_T('H', 0, 0.0, yz)
            return out / self.w[None, :, None]
        D1o = self.rad.D1[self._par(m + 1)]
        D1e = self.rad.D1[self._par(m)]
        yp = 0.5 * (y[0, :-1] + 1j * y[1, :-1])
        ym = 0.5 * (y[0, :-1] - 1j * y[1, :-1])
        yz = y[2, :-1]
        # homogeneous pair (forward operators)
        L = self.lap(m, alpha)
        ph = np.zeros(nr, dtype=complex)
        ph[-1] = 1.0
        ph[:-1] = -self._inv('P', m, alpha, L[:-1, -1:].astype(complex))[:, 0]
        rr = self.r
        hp = self._inv('H', m + 1, alpha, (-(D1e @ ph - m / rr * ph)[:-1])[:, None])[:, 0]
        hm = self._inv('H', m - 1, alpha, (-(D1e @ ph + m / rr * ph)[:-1])[:, None])[:, 0]
        hz = self._inv('H', m, alpha, (-(1j * alpha * ph)[:-1])[:, None])[:, 0]
        s = D1o[-1, :-1]
        sh = s @ (hp + hm)
        c = (np.conj(hp) @ yp + np.conj(hm) @ ym + np.conj(hz) @ yz) / sh
        yp = yp - s[:, None] * c[None, :]
        ym = ym - s[:, None] * c[None, :]
        wp = self._inv_T('H', m + 1, alpha, yp)
        wm = self._inv_T('H', m - 1, alpha, ym)
        wz = self._inv_T('H', m, alpha, yz)
        q = D1e[:-1, :-1].T @ (wp + wm) - m / r * (wp - wm) - 1j * alpha * wz
        phi = self._inv_T('P', m, alpha, q)
        DT = D1o[:-1, :].T @ phi
        Rp = -0.5 * DT
        Rm = -0.5 * DT
        Rp[:-1] += wp - 0.5 * (1 + m) / r * phi
        Rm[:-1] += wm - 0.5 * (1 - m) / r * phi
        out[0] = Rp + Rm
        out[1] = -1j * (Rp - Rm)
        out[2, :-1] = wz + 1j * alpha * phi
        return out / self.w[None, :, None]

    def S_adj_direct(self, Y):
        out = np.empty_like(Y)
        for m in range(self.M + 1):
            for kk in range(self.nk):
                out[:, :, m, kk:kk + 1] = self.S_adj_mode(m, self.alpha[kk], Y[:, :, m, kk:kk + 1])
        return out

    def E_adj_direct(self, Z):
        """W^{-1} E^H W Z with E^H = C^H diag(E_{m+1}^T, E_{m-1}^T) (C/2) and E_m^T."""
        out = np.empty_like(Z)
        c = 1.0 / (2.0 * self.re)
        for m in range(self.M + 1):
            for kk in range(self.nk):
                a = self.alpha[kk]
                z = Z[:, :, m, kk] * self.w[None, :]
                zp = 0.5 * (z[0] + 1j * z[1])
                zm = 0.5 * (z[0] - 1j * z[1])
                ep = zp / self.dt + c * self.lap(m + 1, a).T @ zp
                em = zm / self.dt + c * self.lap(m - 1, a).T @ zm
                ez = z[2] / self.dt + c * self.lap(m, a).T @ z[2]
                out[:, :, m, kk] = np.stack([ep + em, -1j * (ep - em), ez]) / self.w[None, :]
        return out

    def S_adj(self, Y):
        return self.apply_modes(Y, 'S', adjoint=True) if self._fits() else self.S_adj_direct(Y)

    def E_adj(self, Z):
        return self.apply_modes(Z, 'E', adjoint=True) if self._fits() else self.E_adj_direct(Z)

    def curl(self, u):
        out = np.empty_like(u)
        for m in range(self.M + 1):
            out[:, :, m, :] = self.curl_mode(m, self.alpha[None, :], u[:, :, m, :])
        return out

    def E(self, u):
        if self._fits():
            return self.apply_modes(u, 'E')
        out = np.empty_like(u)
        for m in range(self.M + 1):
            for kk in range(self.nk):
                out[:, :, m, kk] = self.E_mode(m, self.alpha[kk], u[:, :, m, kk])
        return out

    # ---------------------------------------------------------- transforms
    def to_phys(self, F):
        """f(theta_a, z_b) = sum_{m,k} F e^{i(m theta_a + alpha_k z_b)}, real.

        F has shape (..., M+1, nk); the m = 0 column enters through its real
        part after the z transform (Hermitian series in theta)."""
        lead = F.shape[:-2]
        Z = np.zeros(lead + (self.nz, self.ntheta // 2 + 1), dtype=complex)
        kpos = np.where(self.kint >= 0, self.kint, self.nz + self.kint)
        Z[..., kpos, :self.M + 1] = np.swapaxes(F, -1, -2)
        Z = np.fft.ifft(Z, axis=-2) * self.nz
        Z[..., 0] = Z[..., 0].real
        return np.fft.irfft(Z, n=self.ntheta, axis=-1) * self.ntheta   # (..., nz, ntheta)

    def to_spec(self, f):
        """P_K F f: coefficients (1/(Nt Nz)) sum f e^{-i(...)} on the retained band."""
        X = np.fft.fft(np.fft.rfft(f, axis=-1), axis=-2) / (self.ntheta * self.nz)
        kpos = np.where(self.kint >= 0, self.kint, self.nz + self.kint)
        return np.swapaxes(X[..., kpos, :self.M + 1], -1, -2)

    @staticmethod
    def cross(a, b):
        return np.stack([a[1] * b[2] - a[2] * b[1],
                         a[2] * b[0] - a[0] * b[2],
                         a[0] * b[1] - a[1] * b[0]])

    # ------------------------------------------------------ nonlinear terms
    def base_terms(self, v, wv, t):
        """U x curl(v) + v x Om, mode-diagonal (U and Om depend on r only)."""
        U, Om = self.base(t)
        U = U[:, None, None]
        Om = Om[:, None, None]
        return np.stack([-U * wv[1] - Om * v[2], U * wv[0], Om * v[0]])

    def N(self, u, t):
        """N(u, t) = P_K F[u x w] + U x w + u x Om."""
        w = self.curl(u)
        nl = self.to_spec(self.cross(self.to_phys(u), self.to_phys(w)))
        return nl + self.base_terms(u, w, t)

    def N_tan(self, u, t, v):
        """Tangent of N at u in direction v."""
        wu, wv = self.curl(u), self.curl(v)
        pu, pv = self.to_phys(u), self.to_phys(v)
        nl = self.to_spec(self.cross(pv, self.to_phys(wu)) + self.cross(pu, self.to_phys(wv)))
        return nl + self.base_terms(v, wv, t)

    def N_adj(self, u, t, y):
        """W-adjoint of the tangent of N at u, applied to y."""
        U, Om = self.base(t)
        wu = self.curl(u)
        Y = self.to_phys(y)
        a = self.to_spec(self.cross(self.to_phys(wu), Y))
        b = self.to_spec(self.cross(Y, self.to_phys(u)))
        Uc = U[:, None, None]
        Oc = Om[:, None, None]
        a = a + np.stack([Oc * y[2], np.zeros_like(y[1]), -Oc * y[0]])       # Om x y
        b = b + np.stack([Uc * y[1], -Uc * y[0], np.zeros_like(y[2])])       # y x U
        return a + self.apply_modes(b, 'C', adjoint=True)

    def N_adj_cont(self, u, t, y):
        """Continuous-adjoint convective term Omega x y + curl(y x V), V = U + u
        (Sec. 2, adjoint momentum equation, in rotational form): the products
        of N_adj with the discrete curl applied to the second one."""
        U, Om = self.base(t)
        wu = self.curl(u)
        Y = self.to_phys(y)
        a = self.to_spec(self.cross(self.to_phys(wu), Y))
        b = self.to_spec(self.cross(Y, self.to_phys(u)))
        Uc = U[:, None, None]
        Oc = Om[:, None, None]
        a = a + np.stack([Oc * y[2], np.zeros_like(y[1]), -Oc * y[0]])       # Om x y
        b = b + np.stack([Uc * y[1], -Uc * y[0], np.zeros_like(y[2])])       # y x U
        return a + self.curl(b)

    # ------------------------------------------------------------ stepping
    def stages(self, u, n):
        """Predictor and corrector iterates w_0..w_C of the step from u^n.

        w_0 = S(E u + N(u, t_n)); w_c = S(E u + (N(u, t_n) + N(w_{c-1}, t_{n+1}))/2),
        c = 1..C (C = ncorr corrector passes); w_C = u^{n+1}."""
        t0, t1 = self.time(n), self.time(n + 1)
        Nn = self.N(u, t0)
        Eu = self.E(u)
        ws = [self.S(Eu + Nn)]
        for _ in range(self.ncorr):
            ws.append(self.S(Eu + 0.5 * (Nn + self.N(ws[-1], t1))))
        return ws

    def step(self, u, n):
        """u^n -> u^{n+1} (predictor and ncorr corrector passes)."""
        return self.stages(u, n)[-1]

    def predictor(self, u, n):
        return self.stages(u, n)[0]

    def step_tan(self, u, n, v):
        """Tangent of the step at u^n in direction v."""
        t0, t1 = self.time(n), self.time(n + 1)
        ws = self.stages(u, n)
        Ev = self.E(v)
        Nv = self.N_tan(u, t0, v)
        vs = self.S(Ev + Nv)
        for c in range(self.ncorr):
            vs = self.S(Ev + 0.5 * (Nv + self.N_tan(ws[c], t1, vs)))
        return vs

    def step_adj(self, u, n, lam):
        """W-adjoint of the step tangent at u^n applied to lam^{n+1}:
        mu_C = S^+ lam, mu_{c-1} = S^+ (N'(w_{c-1})^+ mu_c / 2),
        lam^n = E^+ (sum_c mu_c) + N'(u^n)^+ (mu_0 + sum_{c>=1} mu_c / 2)."""
        t0, t1 = self.time(n), self.time(n + 1)
        ws = self.stages(u, n)
        mu = self.S_adj(lam)
        Z = mu.copy()
        Y = 0.5 * mu
        for c in range(self.ncorr, 0, -1):
            mu = self.S_adj(0.5 * self.N_adj(ws[c - 1], t1, mu))
            Z = Z + mu
            Y = Y + (mu if c == 1 else 0.5 * mu)
        return self.E_adj(Z) + self.N_adj(u, t0, Y)

    def step_adj_cont(self, u, u_next, n, y):
        """One backward step of the continuous adjoint (Sec. 2 adjoint equations
        with the Sec. 2.3 stepper): y^{n+1} at t_{n+1} -> y^n at t_n, with the
        direct fields u^n and u^{n+1}:
            v_0 = S(E y + Nc(u^{n+1}, t_{n+1}; y)),
            v_c = S(E y + (Nc(u^{n+1}, t_{n+1}; y) + Nc(u^n, t_n; v_{c-1})) / 2),
            y^n = v_ncorr."""
        t0, t1 = self.time(n), self.time(n + 1)
        Nn = self.N_adj_cont(u_next, t1, y)
        Ey = self.E(y)
        v = self.S(Ey + Nn)
        for _ in range(self.ncorr):
            v = self.S(Ey + 0.5 * (Nn + self.N_adj_cont(u, t0, v)))
        return v

    def gradient_cont(self, u0, nsteps):
        """J = E(u^N) and the continuous-adjoint gradient y^0 (unprojected),
        from y^N = u^N (the compatibility condition with the sign that makes
        y the ascent direction)."""
        uN, hist = self.forward(u0, nsteps, keep=True)
        states = hist + [uN]
        y = uN.copy()
        for n in range(nsteps - 1, -1, -1):
            y = self.step_adj_cont(states[n], states[n + 1], n, y)
        return self.energy(uN), uN, y

    def forward(self, u0, nsteps, keep=False):
        """Integrate nsteps; returns u^N (and all u^n, n < N, if keep)."""
        u = u0
        hist = []
        for n in range(nsteps):
            if keep:
                hist.append(u)
            u = self.step(u, n)
        return (u, hist) if keep else u

    def gradient(self, u0, nsteps):
        """J = E(u^N) and its W-gradient lam^0 (unprojected)."""
        uN, hist = self.forward(u0, nsteps, keep=True)
        lam = uN.copy()
        for n in range(nsteps - 1, -1, -1):
            lam = self.step_adj(hist[n], n, lam)
        return self.energy(uN), uN, lam
