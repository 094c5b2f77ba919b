"""Write the oracle's expected values for the full-size prefix parity tests.

Calls only the CPU oracle (and the seeded input generator).  Two workloads, in
the paper's units, each over a short prefix of its horizon:

* paper-like: L_z = 50 radii, 64 x 96 x 768, Re = 2000, Wo = 8, A = 1,
  tau0 = T/2, dt = 0.02, localised oblique seed 2, E0 = 1e-5; 8 forward steps
  and the adjoint sweep back over them from lambda^N = u^N;
* differentiation: L_z = 24 radii, 48 x 64 x 384, Re = 1500, Wo = 10, A = 1,
  tau0 = T/2, dt = 0.02, smooth seed 3, E0 = 1e-5; 6 steps and the gradient.

The fields are too large to store whole, so the fixture keeps every radial
node and component of a fixed set of (m, kk) modes (u^0, u^N and lambda^0 on
those modes) plus whole-field scalars (energies and inner products), and the
scale that normalises the raw seed after the oracle's projection.

Usage: python tests/golden/make_fullsize_fixtures.py [c2|c3]  (about 20 and 5
minutes on one CPU core)
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.pipe import Pipe                      # noqa: E402
from oracle import optimize as opt                # noqa: E402
from oracle.radial import nodes                   # noqa: E402
from paper_2509_10103_amd import synth            # noqa: E402

T2 = 2.0 * math.pi * 2000.0 / 64.0
T3 = 2.0 * math.pi * 1500.0 / 100.0
CASES = {
    "c2": dict(nr=64, nt=96, nz=768, lz=50.0, re=2000.0, wo=8.0, amp=1.0, dt=0.02, t0=0.5 * T2, nsteps=8,
               e0=1e-5, seed=2, gen="oblique"),
    "c3": dict(nr=48, nt=64, nz=384, lz=24.0, re=1500.0, wo=10.0, amp=1.0, dt=0.02, t0=0.5 * T3, nsteps=6,
               e0=1e-5, seed=3, gen="smooth"),
}


def raw_seed(c):
    r = nodes(c["nr"])
    M, K = (c["nt"] - 1) // 3, (c["nz"] - 1) // 3
    if c["gen"] == "oblique":
        return synth.localized_oblique(r, M, K, c["lz"], c["nz"], c["seed"])
    return synth.solenoidal_modes(r, M, K, c["lz"], c["seed"])


def sample_modes(M, K):
    """(m, kk) pairs kept in the fixture: the axis and wall of the band, the
    oblique seed's band |k| ~ 28..52 at L_z = 50, and 24 seeded random pairs."""
    nk = 2 * K + 1
    ms = sorted({0, 1, 2, 3, M // 2, M})
    ks = sorted({0, 1, 2, min(30, K), min(40, K), K // 2, K, nk - 1, nk - min(40, K), nk - K})
    pairs = {(m, k) for m in ms for k in ks}
    rng = np.random.default_rng(12345)
    while len(pairs) < len(ms) * len(ks) + 24:
        pairs.add((int(rng.integers(0, M + 1)), int(rng.integers(0, nk))))
    return np.array(sorted(pairs), dtype=np.int64)


def main(which):
    c = CASES[which]
    P = Pipe(c["nr"], c["nt"], c["nz"], c["lz"], c["re"], c["wo"], c["amp"], c["dt"], c["t0"])
    P.cache_limit = 0
    t = time.time()
    raw = raw_seed(c)
    pr = opt.project(P, raw)
    scale = math.sqrt(c["e0"] / P.energy(pr))
    u0 = pr * scale
    print(f"{which}: seed projected ({time.time() - t:.0f} s)", flush=True)
    J, uN, lam0 = P.gradient(u0, c["nsteps"])
    print(f"{which}: forward + adjoint over {c['nsteps']} steps ({time.time() - t:.0f} s)", flush=True)
    sm = sample_modes(P.M, P.K)
    pick = lambda f: np.stack([f[:, :, m, k] for m, k in sm], axis=-1)    # (3, nr, nsamples)
    np.savez_compressed(os.path.join(HERE, f"{which}_prefix_oracle.npz"), config=np.array(repr(c)), modes=sm,
                        u0=pick(u0), uN=pick(uN), lam0=pick(lam0), J=J, E0=P.energy(u0),
                        lam_norm2=P.wdot(lam0, lam0), lam_u0=P.wdot(lam0, u0), uN_u0=P.wdot(uN, u0))


if __name__ == "__main__":
    for w in (sys.argv[1:] or ["c3", "c2"]):
        main(w)
