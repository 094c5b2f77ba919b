"""The HIP optimisation loop in the linear regime (paper App. A validation
idea, taken to an exact pin): with E0 = 1e-20 and a steady base flow the step
is linear and mode-diagonal, so over one (k, m) mode the adjoint-looping
iteration (Sec. 2.1-2.2) converges to the square of the top singular value of
the discrete propagator restricted to admissible fields, in the W norm.  The
singular value comes from a dense SVD of the oracle's tangent propagator."""
import numpy as np
import pytest

from tests.gpu_common import to_dev
from oracle.pipe import Pipe
from oracle import optimize as opt

pytestmark = pytest.mark.gpu


def test_hip_loop_converges_to_top_singular_value():
    from paper_2509_10103_amd import npo
    cfg = dict(nr=12, nt=6, nz=6, lz=2 * np.pi, re=1000.0, wo=8.0, amp=0.0, dt=0.05, t0=0.0)
    m, kk, nsteps, E0 = 1, 1, 20, 1e-20
    P = Pipe(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"], cfg["dt"], cfg["t0"])
    n3 = 3 * P.nr
    G = opt.constraint_rows(P, m, P.alpha[kk])
    sw = np.sqrt(np.tile(P.w, 3))
    _, s, Vh = np.linalg.svd(G / sw[None, :])
    basis = Vh[np.sum(s > 1e-12 * s[0]):].conj().T / sw[:, None]     # W-orthonormal admissible basis
    A = np.zeros((n3, basis.shape[1]), dtype=complex)
    for i in range(basis.shape[1]):
        v = P.zeros()
        v[:, :, m, kk] = basis[:, i].reshape(3, P.nr)
        for n in range(nsteps):
            v = P.step_tan(P.zeros(), n, v)
        A[:, i] = v[:, :, m, kk].reshape(-1)
    smax2 = np.linalg.svd(sw[:, None] * A, compute_uv=False)[0] ** 2
    rng = np.random.default_rng(3)
    u = P.zeros()
    u[:, :, m, kk] = (basis @ (rng.standard_normal(basis.shape[1]) +
                               1j * rng.standard_normal(basis.shape[1]))).reshape(3, P.nr)
    u = opt.normalise(P, u, E0)

    Gp = npo.Plan(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"], cfg["dt"],
                  cfg["t0"], nsteps)
    u0 = to_dev(u)
    uN = Gp.field()
    ck = Gp.arena(nsteps)
    npo.npo_forward_run(Gp.handle, Gp.ws, ck, nsteps, u0, uN)
    gains = []
    for it in range(40):
        st = npo.npo_iterate(Gp.handle, Gp.ws, ck, nsteps, u0, uN, E0)
        gains.append(st["G_new"])
        if not st["accepted"]:
            break
    print(f"[linear] G history {gains[:3]} ... {gains[-1]:.12g}, sigma_max^2 {smax2:.12g}", flush=True)
    assert not st["accepted"]                        # the loop stopped (|dG/G| below its tolerance)
    assert gains[-1] <= smax2 * (1 + 1e-9)
    assert abs(gains[-1] / smax2 - 1) < 1e-8
    Gp.close()
