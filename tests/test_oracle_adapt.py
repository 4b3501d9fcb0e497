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


def test_adaptive_run_approaches_the_certified_optimum_sooner():
    """XXZ ring N = 8, 2-site clusters: after 6000 iterations the adaptive run has closed feasErr and the
    primal-dual gap to 1e-9 at the value a converged fixed-scale run certifies (8 x the paper's
    parameters, which converges on this instance: gap and feasErr at rounding), below the exact
    ground-state energy, and its feasErr is an order of magnitude below the paper's fixed parameters'."""
    w = synth.xxz_ring(8, 2, 0.5)
    p = alg6.Problem.from_workload(w)
    s, hist, q = adapt.solve(p, 6000, 50)
    lb, e, f = alg6.lower_bound(q, s), alg6.energy_per_site(q, s), alg6.feasibility_error(q, s)
    assert f < 1e-9 and abs(e - lb) < 1e-9 * abs(lb)
    r = alg6.Problem.from_workload(w)
    r.mu, r.nu, r.eps = 8 * r.mu, 8 * r.nu, 8 * r.eps
    t, _ = alg6.solve(r, 3000)
    lb8 = alg6.lower_bound(r, t)
    assert alg6.feasibility_error(r, t) < 1e-12 and abs(alg6.energy_per_site(r, t) - lb8) < 1e-12
    assert abs(lb - lb8) < 1e-8 * abs(lb8)
    E0, _ = exact.ground_state(w.terms, w.extent)
    assert lb8 <= E0 / 8 + 1e-12
    u, _ = alg6.solve(p, 6000)
    assert alg6.feasibility_error(p, u) > 10 * f
    assert all(1.0 <= c <= adapt.CMAX for *_, c in hist)


def test_scale_history_follows_the_residuals():
    """Each recorded feasErr (eq. feasErr) and gap agrees with a plain Algorithm 6 run that applies the
    recorded scales window by window, each decision with the rule's trends of the replayed values, and
    the replay ends in the same state."""
    w = synth.tfi_ring(12, 2, 0.5)
    p = alg6.Problem.from_workload(w)
    s, hist, q = adapt.solve(p, 600, 50)
    r = alg6.Problem.from_workload(w)
    st = alg6.initial_state(r)
    c = 1.0
    prev = None
    for t, f, g, c_after in hist:
        r.mu, r.nu, r.eps = c * p.mu, c * p.nu, c * p.eps
        st, _ = alg6.solve(r, t - st.t, state=st)
        f_r = alg6.feasibility_error(r, st)
        lb = alg6.lower_bound(r, st)
        g_r = abs(alg6.energy_per_site(r, st) - lb) / abs(lb)
        assert abs(f_r - f) <= 1e-12 * f and abs(g_r - g) <= 1e-12 * g
        if prev is not None:
            fp, gp = prev
            rose = f > fp * (1 + adapt.DEAD) or g > gp * (1 + adapt.DEAD)
            fell = f < fp * (1 - adapt.DEAD) and g < gp * (1 - adapt.DEAD)
            want = max(c * adapt.SHRINK, 1.0) if rose else (min(c * adapt.GROW, adapt.CMAX) if fell else c)
            assert c_after == want, (t, c, c_after)
        prev, c = (f, g), c_after
    _same(st, s, 1e-12)
    assert len({c for *_, c in hist}) > 2  # the scale moved


@pytest.mark.parametrize("f,g,fp,gp,c,want", [
    (1.0, 1.0, 2.0, 2.0, 1.0, 1.25),  # both fell
    (1.0, 2.0, 2.0, 2.0, 2.0, 2.0),  # one fell, one flat
    (1.0, 3.0, 2.0, 2.0, 4.0, 2.0),  # one rose
    (3.0, 1.0, 2.0, 2.0, 1.0, 1.0),  # one rose, held at 1
    (1.0, 1.0, 2.0, 2.0, 8.0, 8.0),  # held at 8
    (1.0, 1.0, 1.0 + 1e-9, 1.0 - 1e-9, 2.0, 2.0),  # within the dead band
    (1e-13, 1e-13, 2e-13, 5e-14, 2.0, 2.0),  # both at the rounding floor
    (1e-13, 0.5, 5e-12, 1.0, 2.0, 2.5),  # feasErr fell to the floor, the gap fell
])
def test_rule_cases(f, g, fp, gp, c, want):
    assert adapt.next_scale(c, f, g, fp, gp) == want
