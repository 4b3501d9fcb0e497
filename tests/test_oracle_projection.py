"""Pins of the PSD projection Pi (Section 3, definition of Pi as the Frobenius-nearest PSD matrix).

The oracle's Pi clips eigenvalues; these tests check it against what the
definition fixes independently of that route: Moreau's decomposition
(C = Pi(C) - Pi(-C) with Pi(C) ⟂ Pi(-C)), idempotence, special cases, and a
brute-force search over PSD matrices for 2x2 and 4x4 inputs.
"""
import numpy as np
import pytest

from oracle.maps import psd_project


def _sym(rng, n):
    A = rng.standard_normal((n, n))
    return 0.5 * (A + A.T)


def _min_eig(A):
    return np.linalg.eigvalsh(0.5 * (A + A.conj().T))[0]


@pytest.mark.parametrize("n", [2, 3, 4, 16, 64])
def test_moreau_and_idempotence(n):
    rng = np.random.default_rng([1, n])
    for _ in range(5):
        C = _sym(rng, n)
        P = psd_project(C)
        N = P - C
        scale = np.linalg.norm(C)
        assert _min_eig(P) >= -1e-12 * scale
        assert _min_eig(N) >= -1e-12 * scale
        assert abs(np.sum(P * N)) <= 1e-12 * scale ** 2
        assert np.abs(psd_project(P) - P).max() <= 1e-12 * scale
        # Moreau: Pi(C) - Pi(-C) = C
        assert np.abs(P - psd_project(-C) - C).max() <= 1e-12 * scale


def test_complex_hermitian_moreau():
    rng = np.random.default_rng(5)
    n = 8
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    C = 0.5 * (A + A.conj().T)
    P = psd_project(C)
    N = P - C
    assert _min_eig(P) >= -1e-12 and _min_eig(N) >= -1e-12
    assert abs(np.vdot(P, N)) <= 1e-12
    assert np.abs(P - P.conj().T).max() == 0.0


def test_special_cases():
    rng = np.random.default_rng(7)
    B = rng.standard_normal((6, 6))
    S = B @ B.T
    assert np.allclose(psd_project(S), S, atol=1e-12)
    assert np.abs(psd_project(-S)).max() < 1e-12
    D = np.diag([3.0, -1.0, 0.5, -2.0])
    assert np.allclose(psd_project(D), np.diag([3.0, 0.0, 0.5, 0.0]), atol=1e-15)
    assert np.abs(psd_project(np.zeros((5, 5)))).max() == 0.0


def test_bruteforce_2x2_grid():
    """Exhaustive grid over PSD [[a, b], [b, c]] (a, c >= 0, b^2 <= ac): nothing beats Pi."""
    rng = np.random.default_rng(11)
    a = np.linspace(0.0, 3.0, 121)
    A, Cc, Bb = np.meshgrid(a, a, np.linspace(-3.0, 3.0, 241), indexing="ij")
    ok = Bb ** 2 <= A * Cc
    for _ in range(4):
        C = _sym(rng, 2) * 1.5
        P = psd_project(C)
        best_proj = np.linalg.norm(P - C)
        dist = np.sqrt((A - C[0, 0]) ** 2 + (Cc - C[1, 1]) ** 2 + 2 * (Bb - C[0, 1]) ** 2)
        grid_best = dist[ok].min()
        assert best_proj <= grid_best + 1e-12
        assert grid_best - best_proj < 0.05  # the grid comes close to the optimum


@pytest.mark.parametrize("n", [2, 4])
def test_bruteforce_random_search(n):
    """Random PSD matrices of every rank plus rank-1 local moves never get closer than Pi(C)."""
    rng = np.random.default_rng([13, n])
    for _ in range(3):
        C = _sym(rng, n)
        P = psd_project(C)
        d0 = np.linalg.norm(P - C)
        for r in range(1, n + 1):
            B = rng.standard_normal((2000, n, r))
            S = B @ np.swapaxes(B, 1, 2)
            d = np.linalg.norm(S - C, axis=(1, 2))
            assert d.min() >= d0 - 1e-12
        # local search around the projection: P + t v v^T and PSD-preserving shrink moves
        for _ in range(2000):
            v = rng.standard_normal(n)
            t = rng.uniform(-0.3, 0.3)
            S = P + t * np.outer(v, v)
            if _min_eig(S) < 0:
                continue
            assert np.linalg.norm(S - C) >= d0 - 1e-12
