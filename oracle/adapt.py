"""Adaptive penalties and step for Algorithm 6 (test infrastructure: FP64 reference only).

Section 4 runs every problem at mu = nu = 10, eps = 2 and remarks that tuning mu, nu, eps to a problem
could smooth the convergence profiles.  This mode tunes them during the run.  The three are scaled
together, (mu, nu, eps) = c (mu_0, nu_0, eps_0), so the ratio of the X step to the penalties stays the
starting one (the iteration turns unstable once eps exceeds about 0.4 mu), and c follows a
step-size rule on the equality residual of eq. feasErr: every `every` iterations, after iteration t,
feasErr(t) is compared with its value at the previous check; c is multiplied by GROW when it fell by
more than the relative dead band DEAD, by SHRINK when it rose by more than DEAD, and kept otherwise
(also when both values lie below FLOOR, at the rounding level), and held within [1, CMAX].  The first
check only records feasErr.

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


def next_scale(c: float, f: float, f_prev: float) -> float:
    """One decision of the rule: the new scale from the current one and feasErr now / at the last check."""
    if f <= FLOOR and f_prev <= FLOOR:
        return c
    if f < f_prev * (1.0 - DEAD):
        c *= GROW
    elif f > f_prev * (1.0 + DEAD):
        c *= SHRINK
    return min(max(c, 1.0), CMAX)


def solve(p: alg6.Problem, iters: int, every: int, state: alg6.State | None = None, scale: float = 1.0,
          f_prev: float | None = None):
    """Algorithm 6 with the joint scale adapted every `every` iterations (every <= 0: fixed, as alg6.solve).

    `scale` and `f_prev` resume a run (the scale in force and feasErr at its last check).  Returns
    (final state, history, problem): history holds (t, feasErr, scale after the decision) of each check;
    the returned problem is a copy carrying the final parameters (the argument is not changed)."""
    mu0, nu0, eps0 = p.mu, p.nu, p.eps
    q = copy.copy(p)
    c = float(scale)
    q.mu, q.nu, q.eps = c * mu0, c * nu0, c * eps0
    s = state.copy() if state is not None else alg6.initial_state(q)
    history = []
    for _ in range(iters):
        s = alg6.step(q, s)
        if every > 0 and s.t % every == 0:
            f = alg6.feasibility_error(q, s)
            if f_prev is not None:
                c = next_scale(c, f, f_prev)
                q.mu, q.nu, q.eps = c * mu0, c * nu0, c * eps0
            f_prev = f
            history.append((s.t, f, c))
    return s, history, q
