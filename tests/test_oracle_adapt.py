"""Pins of the oracle's adaptive mode (oracle/adapt.py): the joint scale of (mu, nu, eps) tuned during
the run (Section 4's remark that tuning the three to a problem could smooth convergence)."""
import numpy as np
import pytest

import synth
from oracle import adapt, alg6, exact

KEYS = ("X", "rho0", "rho", "rho_t", "Lam", "Lam1", "Lam2")


def _same(a, b, tol):
    for k in KEYS:
        x, y = getattr(a, k), getattr(b, k)
        assert np.abs(x - y).max() <= tol * max(1.0, np.abs(y).max()), k


def test_without_adaptation_it_is_algorithm6():
    p = alg6.Problem.from_workload(synth.tfi_ring(8, 2, 1.0))
    s1, hist, q = adapt.solve(p, 25, 0)
    s2, _ = alg6.solve(p, 25)
    _same(s1, s2, 0.0)
    assert hist == [] and (q.mu, q.nu, q.eps) == (p.mu, p.nu, p.eps)


def test_a_fixed_point_stays_fixed_when_the_scale_changes():
    """The multipliers are unscaled and the X step is a projected gradient step: a converged iterate
    of the fixed-parameter run does not move when (mu, nu, eps) are scaled (a scaled-multiplier form
    would have to rescale Lambda, and an un-rescaled one would leave the fixed point)."""
    p = alg6.Problem.from_workload(synth.tfi_ring(6, 1, 1.0))
    s, _ = alg6.solve(p, 3000)
    assert alg6.feasibility_error(p, s) < 1e-13
    for c in (4.0, 0.5):
        q = alg6.Problem.from_workload(synth.tfi_ring(6, 1, 1.0))
        q.mu, q.nu, q.eps = c * p.mu, c * p.nu, c * p.eps
        t, _ = alg6.solve(q, 20, state=s)
        _same(t, s, 1e-10)


def test_adaptive_run_reaches_the_certified_optimum():
    """XXZ ring N = 8, 2-site clusters: the adaptive run closes the duality gap (E_p = LB, feasErr at
    rounding: a certified optimum of the relaxation) at the value a fixed-parameter run converges to,
    below the exact ground-state energy, and gets there well before the paper's fixed parameters do."""
    w = synth.xxz_ring(8, 2, 0.5)
    p = alg6.Problem.from_workload(w)
    s, hist, q = adapt.solve(p, 3000, 50)
    lb, e, f = alg6.lower_bound(q, s), alg6.energy_per_site(q, s), alg6.feasibility_error(q, s)
    assert f < 1e-12 and abs(e - lb) < 1e-10
    # the same optimum from a fixed scale (8 x the paper's parameters, which converges on this instance)
    r = alg6.Problem.from_workload(w)
    r.mu, r.nu, r.eps = 8 * r.mu, 8 * r.nu, 8 * r.eps
    t, _ = alg6.solve(r, 3000)
    assert alg6.feasibility_error(r, t) < 1e-12
    assert abs(alg6.lower_bound(r, t) - lb) < 1e-10
    E0, _ = exact.ground_state(w.terms, w.extent)
    assert lb <= E0 / 8 + 1e-12
    # the paper's fixed parameters are still far from it at 3000 iterations
    u, _ = alg6.solve(p, 3000)
    assert alg6.feasibility_error(p, u) > 1e3 * f
    assert all(1.0 <= c <= adapt.CMAX for _, _, c in hist)


def test_scale_history_follows_the_residual():
    """Each recorded feasErr (eq. feasErr) and decision agrees with a plain Algorithm 6 run that applies
    the recorded scales window by window, and that run ends in the same state."""
    w = synth.tfi_ring(12, 2, 0.5)
    p = alg6.Problem.from_workload(w)
    s, hist, q = adapt.solve(p, 600, 50)
    # replay: plain Algorithm 6 steps with the parameters each window used
    r = alg6.Problem.from_workload(w)
    st = alg6.initial_state(r)
    c = 1.0
    prev = None
    for t, f, c_after in hist:
        r.mu, r.nu, r.eps = c * p.mu, c * p.nu, c * p.eps
        st, _ = alg6.solve(r, t - st.t, state=st)
        f_replay = alg6.feasibility_error(r, st)
        assert abs(f_replay - f) <= 1e-12 * f
        if prev is not None:
            if f < prev * (1 - adapt.DEAD):
                assert c_after == min(c * adapt.GROW, adapt.CMAX)
            elif f > prev * (1 + adapt.DEAD):
                assert c_after == max(c * adapt.SHRINK, 1.0)
        prev, c = f, c_after
    _same(st, s, 1e-12)


@pytest.mark.parametrize("f,f_prev,c,want", [(1.0, 2.0, 1.0, 1.25), (2.0, 1.0, 4.0, 2.0), (2.0, 1.0, 1.0, 1.0),
                                              (1.0, 2.0, 8.0, 8.0), (1.0, 1.0 + 1e-9, 2.0, 2.0),
                                              (1e-13, 2e-13, 2.0, 2.0), (1e-13, 5e-12, 2.0, 2.5)])
def test_rule_cases(f, f_prev, c, want):
    assert adapt.next_scale(c, f, f_prev) == pytest.approx(want, rel=0, abs=0)
