"""Pins of the dense Algorithm 5 oracle with one-site fields (no translation invariance):
exact marginals reproduce the exact energy, the bound lies below the exact energy at every
iterate, a single pair spanning the system is tight, and uniform fields reproduce the
translation-invariant iteration with the shifted field."""
import numpy as np
import pytest

import synth
from oracle import alg5, alg6, exact


def _fields(N, seed, scale=0.8):
    rng = np.random.default_rng([synth.BASE_SEED, 17, seed])
    return [("X", (x, 0), float(scale * rng.uniform(-1, 1))) for x in range(N)]


def _problem(N, L, h, fields):
    w = synth.tfi_ring(N, L, h)
    p = alg6.Problem.from_workload(w)
    return w, p, alg5.DenseProblem(p, fields)


@pytest.mark.parametrize("N,L", [(6, 2), (8, 2), (6, 3)])
def test_exact_marginals_give_exact_energy(N, L):
    f = _fields(N, N + L)
    w, p, dp = _problem(N, L, 1.0, f)
    e0, psi = exact.ground_state(w.terms, w.extent, f)
    rho, pairs = exact.all_marginals(psi, w.extent, w.cluster)
    st = {"rho": rho, "rho_p": pairs}
    assert abs(alg5.energy_dense(dp, st) - e0 / N) < 1e-12


def test_bound_below_exact_energy_at_every_iterate():
    N, L = 8, 2
    f = _fields(N, 3)
    w, p, dp = _problem(N, L, 0.9, f)
    e0 = exact.ground_state(w.terms, w.extent, f)[0] / N
    st = alg5.initial_dense(dp)
    for it in range(120):
        if it % 20 == 0:
            assert alg5.lower_bound_dense(dp, st) <= e0 + 1e-12
        st = alg5.dense_step(dp, st)
    lb = alg5.lower_bound_dense(dp, st)
    assert lb <= e0 + 1e-12 and lb > e0 - 0.2


def test_single_pair_spanning_the_system_is_tight():
    N, L = 4, 2  # M = 2: one pair holds the whole ring
    f = _fields(N, 5)
    w, p, dp = _problem(N, L, 1.2, f)
    e0 = exact.ground_state(w.terms, w.extent, f)[0] / N
    st = alg5.initial_dense(dp)
    for _ in range(3000):
        st = alg5.dense_step(dp, st)
    lb = alg5.lower_bound_dense(dp, st)
    assert lb <= e0 + 1e-12
    assert abs(lb - e0) < 1e-6
    assert abs(alg5.energy_dense(dp, st) - e0) < 1e-5


def test_uniform_fields_match_the_invariant_iteration():
    """delta X on every site shifts h by -delta (TFI is -h sum X - sum ZZ): the dense iterates
    from the invariant start equal Algorithm 6 with h - delta."""
    N, L, h, delta = 8, 2, 1.0, 0.3
    f = [("X", (x, 0), delta) for x in range(N)]
    w, p, dp = _problem(N, L, h, f)
    p2 = alg6.Problem.from_workload(synth.tfi_ring(N, L, h - delta))
    st = alg5.initial_dense(dp)
    s = alg6.initial_state(p2)
    for _ in range(30):
        st = alg5.dense_step(dp, st)
        s = alg6.step(p2, s)
    assert abs(alg5.lower_bound_dense(dp, st) - alg6.lower_bound(p2, s)) < 1e-10
    assert abs(alg5.energy_dense(dp, st) - alg6.energy_per_site(p2, s)) < 1e-10
    # and the first block row of X agrees
    k = p.n_op
    for d in range(p.M):
        assert np.abs(st["X"][0:k, d * k:(d + 1) * k] - s.X[d]).max() < 1e-10
