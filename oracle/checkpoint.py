"""Oracle: binomial checkpointing counts (paper Sec. 2.4).

With N_G memory checkpoints (the stored initial state included) and
N_steps forward steps, the minimal number of forward advances needed to
recover every direct field during the backward sweep is
    N_rec = S N_steps - beta(N_G + 1, S - 1),
    beta(N_G, S - 1) < N_steps <= beta(N_G, S),
    beta(n, s) = C(n + s, n).
Advances are forward steps taken from a stored state; the step being
reversed is not counted.  ``dp_advances`` is the brute-force minimum over all
checkpoint placements, used to pin the closed form.
"""
from functools import lru_cache
from math import comb


def beta(n, s):
    return comb(n + s, n)


def closed_form(nsteps, ng):
    """N_rec of Sec. 2.4 and the repetition number S."""
    if nsteps <= 1:
        return 0, 0
    s = 0
    while beta(ng, s) < nsteps:
        s += 1
    return s * nsteps - beta(ng + 1, s - 1), s


@lru_cache(maxsize=None)
def dp_advances(l, s):
    """Minimal advances to reverse l steps from a stored state with s slots.

    Reversing one step costs nothing extra.  With a single slot (the start)
    every step i must be re-reached from the start: sum_{i<l} i.  Otherwise
    advance m steps, store, reverse the last l - m steps with one slot less,
    then the first m steps with all slots.
    """
    if l <= 1:
        return 0
    if s <= 1:
        return l * (l - 1) // 2
    return min(m + dp_advances(l - m, s - 1) + dp_advances(m, s) for m in range(1, l))
