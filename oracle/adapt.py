"""Adaptive penalties and step for Algorithm 6 (test infrastructure: FP64 reference only).

Section 4 runs every problem at mu = nu = 10, eps = 2 and remarks that tuning mu, nu, eps to a problem
could smooth the convergence profiles.  This mode tunes them during the run.  The three are scaled
together, (mu, nu, eps) = c (mu_0, nu_0, eps_0), so the ratio of the X step to the penalties stays the
starting one (the iteration turns unstable once eps exceeds about 0.4 mu), and c follows a step-size rule
on the two quantities whose vanishing certifies the optimum: the equality residual feasErr (eq. feasErr)
and the relative primal-dual gap |E_p - LB| / |LB| (E_p the energy of the marginals, LB the Lagrangian
bound).  Every `every` iterations, after iteration t, each is compared with its value at the previous
check: it "fell" if it dropped by more than the relative dead band DEAD, "rose" if it grew by more, and is
neutral in between or when both values lie below FLOOR (rounding level).  c is multiplied by GROW when
both fell, by SHRINK when either rose, kept otherwise, and held within [1, CMAX].
The first check only records the two values.

The multipliers Lambda, Lambda^(1), Lambda^(2) of Algorithm 6 are unscaled and the X step is a projected
gradient step, so a change of c needs no rescaling of the state and leaves every fixed point of the
iteration fixed; the limit is the same SDP optimum.
"""
from __future__ import annotations

import copy

from . import alg6

GROW = 1.25
SHRINK = 0.5
CMAX = 8.0
DEAD = 1e-6
FLOOR = 1e-12


def _trend(x: float, x_prev: float) -> int:
    """-1 fell, +1 rose, 0 neutral (within the dead band, or both at the rounding floor)."""
    if x <= FLOOR and x_prev <= FLOOR:
        return 0
    if x < x_prev * (1.0 - DEAD):
        return -1
    if x > x_prev * (1.0 + DEAD):
        return 1
    return 0


def next_scale(c: float, f: float, g: float, f_prev: float, g_prev: float) -> float:
    """One decision of the rule from feasErr and the gap now (f, g) and at the last check."""
    tf, tg = _trend(f, f_prev), _trend(g, g_prev)
    if tf > 0 or tg > 0:
        c *= SHRINK
    elif tf < 0 and tg < 0:
        c *= GROW
    return min(max(c, 1.0), CMAX)


def gap(p: alg6.Problem, s: alg6.State) -> float:
    lb = alg6.lower_bound(p, s)
    return abs(alg6.energy_per_site(p, s) - lb) / abs(lb)


def solve(p: alg6.Problem, iters: int, every: int, state: alg6.State | None = None, scale: float = 1.0,
          last: tuple | None = None):
    """Algorithm 6 with the joint scale adapted every `every` iterations (every <= 0: fixed, as alg6.solve).

    `scale` and `last` (feasErr, gap at the last check) resume a run.  Returns (final state, history,
    problem): history holds (t, feasErr, gap, scale after the decision) of each check; the returned
    problem is a copy carrying the final parameters (the argument is not changed)."""
    mu0, nu0, eps0 = p.mu, p.nu, p.eps
    q = copy.copy(p)
    c = float(scale)
    q.mu, q.nu, q.eps = c * mu0, c * nu0, c * eps0
    s = state.copy() if state is not None else alg6.initial_state(q)
    history = []
    for _ in range(iters):
        s = alg6.step(q, s)
        if every > 0 and s.t % every == 0:
            f, g = alg6.feasibility_error(q, s), gap(q, s)
            if last is not None:
                c = next_scale(c, f, g, *last)
                q.mu, q.nu, q.eps = c * mu0, c * nu0, c * eps0
            last = (f, g)
            history.append((s.t, f, g, c))
    return s, history, q
