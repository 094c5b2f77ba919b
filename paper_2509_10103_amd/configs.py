"""Workloads of the benchmark and the tests, in the solver's units.

The solver uses the paper's scaling (Sec. 2): lengths in radii R = D/2,
velocities in 2 U_bar, time in R/(2 U_bar).  Workloads quoted in diameter /
bulk-velocity units convert as L_R = 2 L_D, t_R = 4 t_D, dt_R = 4 dt_D; the
pulsation period is T = 2 pi Re / Wo^2 (the printed pi Re / (2 Wo^2) is the
same period in D/U_bar units).
"""
import math


def period(re, wo):
    return 2.0 * math.pi * re / (wo * wo)


def _mk(name, nr, nt, nz, lz, re, wo, amp, dt, t0, nsteps, e0, seed, n_ckpt, iters, gen):
    return dict(name=name, nr=nr, nt=nt, nz=nz, lz=lz, re=re, wo=wo, amp=amp, dt=dt, t0=t0, nsteps=nsteps,
                e0=e0, seed=seed, n_ckpt=n_ckpt, iters=iters, gen=gen)


# Plain method, one instance, one iteration: L = 2 pi D, 32 x 24 x 48,
# Re 2000, Wo 8, A 0.5, 5 D/U time units at dt_D = 0.01, E0 = 1e-4, seed 1.
C1 = _mk("plain-32x24x48", 32, 24, 48, 4 * math.pi, 2000.0, 8.0, 0.5, 0.04, 0.0, 500, 1e-4, 1, 500, 1, "smooth")

# Plain method at paper-like scale: L = 25 D, 64 x 96 x 768, Re 2000, Wo 8,
# A 1, one pulsation period at dt_D = 0.005 from tau0 = T/2 (deceleration),
# localised oblique seed with E0 = 1e-5, seed 2.  Checkpoints: as many as the
# HBM holds (n_ckpt None; about 5300 slots of 50 MB on a 288 GB device).
_T2 = period(2000.0, 8.0)
C2 = _mk("paper-64x96x768", 64, 96, 768, 50.0, 2000.0, 8.0, 1.0, 0.02, 0.5 * _T2, int(round(_T2 / 0.02)),
         1e-5, 2, None, 10, "oblique")

# Differentiation workload: L = 12 D, 48 x 64 x 384, Re 1500, Wo 10, A 1,
# 20 D/U units at dt_D = 0.005 from tau0 = T/2, E0 = 1e-5, seed 3.
_T3 = period(1500.0, 10.0)
C3 = _mk("autograd-48x64x384", 48, 64, 384, 24.0, 1500.0, 10.0, 1.0, 0.02, 0.5 * _T3, 4000, 1e-5, 3, 128, 1,
         "smooth")

WORKLOADS = {"c1": C1, "c2": C2, "c3": C3}


def batch_instances(n=64, seed0=1000, hbm_budget=200e9, nsteps=2000, dt=0.02):
    """The batched workload: n instances of uneven size, seed seed0 + i.

    Per instance: N_r in {32, 48, 64}, N_theta in {24, 48, 96}, N_z in
    {96, ..., 768} with L_D = 25 N_z / 768 (the paper-like axial spacing),
    Re ~ U[1000, 3000], Wo ~ U[4, 18], A ~ U[0.25, 1.5], log10 E0 ~ U[-7, -3],
    tau0 in {0, T/4, T/2, 3T/4}; horizon 10 D/U (nsteps at dt); checkpoint
    slots so that all arenas together fit the HBM budget."""
    import numpy as np
    out = []
    sizes = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        nr = int(rng.choice([32, 48, 64]))
        nt = int(rng.choice([24, 48, 96]))
        nz = int(rng.choice([96, 144, 192, 288, 384, 576, 768]))
        re = float(rng.uniform(1000, 3000))
        wo = float(rng.uniform(4, 18))
        amp = float(rng.uniform(0.25, 1.5))
        e0 = float(10 ** rng.uniform(-7, -3))
        T = period(re, wo)
        t0 = float(rng.choice([0.0, 0.25, 0.5, 0.75])) * T
        M, K = (nt - 1) // 3, (nz - 1) // 3
        fbytes = 3 * nr * (M + 1) * (2 * K + 1) * 16
        sizes.append(fbytes)
        out.append(_mk(f"batch-{i}-{nr}x{nt}x{nz}", nr, nt, nz, 50.0 * nz / 768.0, re, wo, amp, dt, t0, nsteps,
                       e0, seed0 + i, 0, 1, "smooth"))
    per = hbm_budget / n
    for c, fb in zip(out, sizes):
        c["n_ckpt"] = int(max(2, min(c["nsteps"], per // fb)))
    return out


def field_bytes(c):
    M, K = (c["nt"] - 1) // 3, (c["nz"] - 1) // 3
    return 3 * c["nr"] * (M + 1) * (2 * K + 1) * 16
