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
# localised oblique seed with E0 = 1e-5, 4000 checkpoints, seed 2.
_T2 = period(2000.0, 8.0)
C2 = _mk("paper-64x96x768", 64, 96, 768, 50.0, 2000.0, 8.0, 1.0, 0.02, 0.5 * _T2, int(round(_T2 / 0.02)),
         1e-5, 2, 4000, 10, "oblique")

# Differentiation workload: L = 12 D, 48 x 64 x 384, Re 1500, Wo 10, A 1,
# 20 D/U units at dt_D = 0.005 from tau0 = T/2, E0 = 1e-5, seed 3.
_T3 = period(1500.0, 10.0)
C3 = _mk("autograd-48x64x384", 48, 64, 384, 24.0, 1500.0, 10.0, 1.0, 0.02, 0.5 * _T3, 4000, 1e-5, 3, 128, 1,
         "smooth")

WORKLOADS = {"c1": C1, "c2": C2, "c3": C3}
