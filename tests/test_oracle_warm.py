"""Pins of the warm-start encoding oracle (oracle/warm.py): exact round trip on a solver state
whose offsets are all represented, validity invariants of decoded random vectors, and the
Lagrangian bound at a decoded random point below the exact ground-state energy."""
import numpy as np
import pytest

import synth
from oracle import alg6, warm
from oracle.exact import tfi_ring_energy_jw


@pytest.fixture(scope="module")
def ring8():
    w = synth.tfi_ring(16, 2, 0.8)  # M = 8 clusters of 2 sites
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, 150)
    return p, s


def test_round_trip_on_solver_state(ring8):
    p, s = ring8
    vec = warm.encode(p, s)
    assert vec.size == warm.sizes(p)[0]
    s2 = warm.decode(p, vec)
    for k in ("X", "rho0", "rho_t", "Lam", "Lam1", "Lam2"):
        a, b = getattr(s, k), getattr(s2, k)
        assert np.abs(a - b).max() <= 1e-11 * max(1.0, np.abs(a).max()), k
    assert alg6.lower_bound(p, s2) == pytest.approx(alg6.lower_bound(p, s), abs=1e-11)


def test_slot_assignment():
    assert [warm.slot_of(d, 8) for d in range(1, 8)] == [(0, 0), (0, 1), (0, 2), (0, 3), (1, 2), (1, 1), (1, 0)]
    assert [warm.slot_of(d, 11) for d in (1, 4, 5, 6, 7, 10)] == [(0, 0), (0, 3), (0, 3), (1, 3), (1, 3), (1, 0)]
    assert [warm.slot_of(d, 11, 5) for d in (4, 5, 6, 7)] == [(0, 3), (0, 4), (1, 4), (1, 3)]


def test_encoding_needs_more_clusters_than_near_distances():
    p = alg6.Problem.from_workload(synth.tfi_ring(6, 2, 1.0))  # M = 3
    with pytest.raises(ValueError):
        warm.encode(p, alg6.initial_state(p), near=3)
    warm.encode(p, alg6.initial_state(p), near=1)


@pytest.mark.parametrize("N", [22, 32])
def test_exact_round_trip_with_all_distances(N):
    w = synth.tfi_ring(N, 2, 1.3)  # M = 11 (odd) and 16 (even)
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, 60)
    near = p.M // 2
    s2 = warm.decode(p, warm.encode(p, s, near), near)
    for k in ("X", "rho0", "rho_t", "Lam", "Lam1", "Lam2"):
        a, b = getattr(s, k), getattr(s2, k)
        assert np.abs(a - b).max() <= 1e-11 * max(1.0, np.abs(a).max()), k


def _random_vec(p, seed):
    return np.random.default_rng(seed).standard_normal(warm.sizes(p)[0]) * 0.3


@pytest.mark.parametrize("M", [8, 11, 16])
def test_decoded_random_vectors_are_valid(M):
    p = alg6.Problem.from_workload(synth.tfi_ring(2 * M, 2, 1.0))
    s = warm.decode(p, _random_vec(p, M))
    # X symmetric block-circulant and PSD: the dense matrix built from the block row
    n = p.n_op
    big = np.zeros((M * n, M * n))
    for i in range(M):
        for j in range(M):
            big[i * n:(i + 1) * n, j * n:(j + 1) * n] = s.X[(j - i) % M]
    assert np.abs(big - big.T).max() < 1e-12
    assert np.linalg.eigvalsh(big).min() > -1e-10
    assert abs(np.trace(s.rho0) - 1.0) < 1e-14
    for a in (s.rho_t, s.Lam, s.Lam1, s.Lam2):
        assert np.abs(a - a.transpose(0, 2, 1)).max() == 0.0


def test_bound_at_decoded_random_point_is_below_ground_energy():
    N, h = 16, 1.0
    p = alg6.Problem.from_workload(synth.tfi_ring(N, 2, h))
    e0 = tfi_ring_energy_jw(N, h)
    for seed in range(3):
        s = warm.decode(p, _random_vec(p, 100 + seed))
        assert alg6.lower_bound(p, s) <= e0 + 1e-12


def test_far_offsets_start_cold():
    """decode(far_cold=True): offsets at distances up to `near` keep their slots exactly as the plain decode
    gives them, every farther offset is Section 4's cold start (multipliers 0, rho~ = I/n, X' block 0 before
    the projection), the projected X is PSD, and with no far offsets (near >= M/2) nothing changes."""
    w = synth.tfi_ring(32, 2, 1.1)  # M = 16 clusters
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, 40)
    near = 3
    vec = warm.encode(p, s, near)
    plain = warm.decode(p, vec, near)
    cold = warm.decode(p, vec, near, far_cold=True)
    cold0 = alg6.initial_state(p)
    M = p.M
    for d in range(1, M):
        r = min(d, M - d)
        if r <= near:
            for k in ("Lam", "Lam1", "Lam2", "rho_t"):
                assert np.array_equal(getattr(cold, k)[d - 1], getattr(plain, k)[d - 1]), (d, k)
        else:
            for k in ("Lam", "Lam1", "Lam2", "rho_t", "rho"):
                assert np.array_equal(getattr(cold, k)[d - 1], getattr(cold0, k)[d - 1]), (d, k)
    assert alg6.min_momentum_eig(p, cold) >= -1e-12
    full = M // 2
    vec_full = warm.encode(p, s, full)
    a, b = warm.decode(p, vec_full, full), warm.decode(p, vec_full, full, far_cold=True)
    for k in ("X", "rho0", "rho_t", "Lam", "Lam1", "Lam2"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
