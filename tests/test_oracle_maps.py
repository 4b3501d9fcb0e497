"""Pins of the operator maps (Sections 2.2, 3.1 and 3.3).

* partial traces against their defining property Tr[A rho_S] = Tr[(A (x) I) rho];
* adjoint identities of A_1, A_2;
* the closed-form inverse of eq. rhoijUpdate against a dense superoperator solve;
* the matrix-unit realignments against the generic trace definitions of G and
  of the effective-Hamiltonian corrections (eq. effHam), and their duality;
* G of true marginals is PSD (it is a Gram matrix of operator expectations);
* the FFT route of Section 3.3 against a dense projection of the
  block-circulant X'.
"""
import numpy as np
import pytest

import synth
from oracle import exact
from oracle.alg6 import Problem, inverse_blocks, momentum_blocks
from oracle.maps import (
    C0_complete, C0_generic, G0_complete, G0_generic, Gd_complete, Gd_generic, OperatorMaps, Rd_complete,
    Rd_generic, adj1, adj2, operator_collection, pair_solve, pair_superoperator, psd_project, ptrace1, ptrace2,
)


def _sym(rng, n):
    A = rng.standard_normal((n, n))
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("m", [2, 3, 4])
def test_partial_trace_definition(m):
    rng = np.random.default_rng([20, m])
    rho = _sym(rng, m * m)
    A = rng.standard_normal((m, m))
    # Tr[A rho_1] = Tr[(A (x) I) rho]  and  Tr[A rho_2] = Tr[(I (x) A) rho]
    assert np.isclose(np.trace(A @ ptrace2(rho, m)), np.trace(np.kron(A, np.eye(m)) @ rho), atol=1e-13)
    assert np.isclose(np.trace(A @ ptrace1(rho, m)), np.trace(np.kron(np.eye(m), A) @ rho), atol=1e-13)
    # product states: Tr_2 (a (x) b) = a Tr b
    a, b = _sym(rng, m), _sym(rng, m)
    assert np.allclose(ptrace2(np.kron(a, b), m), a * np.trace(b), atol=1e-13)
    assert np.allclose(ptrace1(np.kron(a, b), m), b * np.trace(a), atol=1e-13)


@pytest.mark.parametrize("m", [2, 3])
def test_adjoints(m):
    rng = np.random.default_rng([21, m])
    rho = rng.standard_normal((m * m, m * m))
    tau = rng.standard_normal((m, m))
    assert np.isclose(np.sum(ptrace2(rho, m) * tau), np.sum(rho * adj1(tau, m)), atol=1e-13)
    assert np.isclose(np.sum(ptrace1(rho, m) * tau), np.sum(rho * adj2(tau, m)), atol=1e-13)


@pytest.mark.parametrize("m,mu,nu", [(2, 10.0, 10.0), (3, 10.0, 10.0), (2, 1.7, 0.3), (3, 0.5, 4.0)])
def test_closed_form_inverse_vs_dense(m, mu, nu):
    rng = np.random.default_rng([22, m])
    n = m * m
    S = pair_superoperator(m, mu, nu)
    for _ in range(3):
        R = rng.standard_normal((n, n))
        want = np.linalg.solve(S, R.ravel()).reshape(n, n)
        got = pair_solve(R, m, mu, nu)
        assert np.abs(got - want).max() < 1e-12 * max(1.0, np.abs(want).max())
    # the operator itself: mu rho + nu (Tr_2 rho (x) I) + nu (I (x) Tr_1 rho) reproduces R
    rho = pair_solve(R, m, mu, nu)
    back = mu * rho + nu * adj1(ptrace2(rho, m), m) + nu * adj2(ptrace1(rho, m), m)
    assert np.abs(back - R).max() < 1e-12


@pytest.mark.parametrize("L", [1, 2])
def test_complete_maps_match_trace_definitions(L):
    m = 2 ** L
    n = m * m
    ops = operator_collection("complete", L)
    # orthonormality in the Hilbert-Schmidt inner product
    gram = np.einsum("aij,bij->ab", ops, ops)
    assert np.allclose(gram, np.eye(n))
    rng = np.random.default_rng([23, L])
    rho0 = _sym(rng, m)
    rho = _sym(rng, n)
    X0 = _sym(rng, n)
    Xd = rng.standard_normal((n, n))
    assert np.allclose(G0_complete(rho0, m), G0_generic(rho0, ops), atol=1e-13)
    assert np.allclose(Gd_complete(rho, m), Gd_generic(rho, ops), atol=1e-13)
    assert np.allclose(C0_complete(X0, m), C0_generic(X0, ops), atol=1e-13)
    assert np.allclose(Rd_complete(Xd, m), Rd_generic(Xd, ops), atol=1e-13)


@pytest.mark.parametrize("opset,L", [("complete", 1), ("complete", 2), ("pauli1", 1), ("pauli1", 2)])
def test_effective_hamiltonian_duality(opset, L):
    """<R(X_d) + R(X_d)^T, rho> = 2 <X_d, G_d(rho)> and <C_0(X_0), rho_0> = <X_0, G_0(rho_0)>.

    This is the blockwise split of the Lagrangian term -Tr[X G] (Section 2.4).
    """
    maps = OperatorMaps(opset, L)
    m, k = maps.m, maps.n_op
    rng = np.random.default_rng([24, L, len(opset)])
    rho = _sym(rng, m * m)
    rho0 = _sym(rng, m)
    Xd = rng.standard_normal((k, k))
    X0 = _sym(rng, k)
    R = maps.Rd(Xd)
    assert np.isclose(np.sum((R + R.T) * rho), 2 * np.sum(Xd * maps.Gd(rho)), atol=1e-12)
    assert np.isclose(np.sum(maps.C0(X0) * rho0), np.sum(X0 * maps.G0(rho0)), atol=1e-12)


def test_pauli1_collection():
    ops = operator_collection("pauli1", 2)
    assert ops.shape == (6, 4, 4)
    assert np.allclose(np.einsum("aij,bij->ab", ops, ops), np.eye(6))
    assert np.isrealobj(ops)


@pytest.mark.parametrize("model,opset,L,N", [
    ("tfi", "complete", 1, 6), ("tfi", "complete", 2, 8), ("tfi", "pauli1", 1, 6),
    ("xxz", "complete", 1, 6), ("xxz", "complete", 2, 8), ("xxz", "pauli1", 1, 6),
    ("afh", "complete", 1, 6), ("afh", "complete", 1, 8), ("afh", "complete", 2, 6), ("afh", "complete", 2, 8),
])
def test_global_matrix_of_true_marginals_is_psd(model, opset, L, N):
    """For marginals of a real state, G is the Gram matrix of the O_{i,a} expectations: PSD.

    The XXZ (J_z = 0.5) and AFH (eq. AFH) ground states have off-diagonal XX + YY bonds, so their
    marginals exercise the realignment G_0d on entries that the diagonal TFI bonds leave at zero."""
    w = {"tfi": lambda: synth.tfi_ring(N, L, 0.8, opset), "xxz": lambda: synth.xxz_ring(N, L, 0.5, opset),
         "afh": lambda: synth.xxz_ring(N, L, 1.0, opset)}[model]()
    p = Problem.from_workload(w)
    _, psi = exact.ground_state(w.terms, w.extent)
    rho0, rhos = exact.cluster_marginals(psi, w.extent, w.cluster)
    M, k = p.M, p.n_op
    G = np.zeros((M * k, M * k))

    def off(i, j):
        return (j - i) % M

    for i in range(M):
        G[i * k:(i + 1) * k, i * k:(i + 1) * k] = p.maps.G0(rho0)
        for j in range(i + 1, M):
            g = p.maps.Gd(rhos[off(i, j) - 1])
            G[i * k:(i + 1) * k, j * k:(j + 1) * k] = g
            G[j * k:(j + 1) * k, i * k:(i + 1) * k] = g.T
    assert np.linalg.eigvalsh(G)[0] > -1e-10
    # and the block-circulant first row is consistent with the X-step layout: G_{0,-d} = G_{0,d}^T
    for d in range(1, M):
        assert np.allclose(p.maps.Gd(rhos[(M - d) % M - 1]), p.maps.Gd(rhos[d - 1]).T, atol=1e-12)


@pytest.mark.parametrize("Mx,My,k", [(5, 1, 3), (8, 1, 4), (3, 2, 3), (2, 2, 4)])
def test_fft_projection_equals_dense_block_circulant(Mx, My, k):
    """Section 3.3: projecting the momentum blocks equals projecting the dense block-circulant X'."""
    rng = np.random.default_rng([25, Mx, My, k])
    M = Mx * My

    class _P:
        pass

    p = _P()
    p.Mx, p.My, p.M, p.n_op = Mx, My, M, k
    B = rng.standard_normal((M, k, k))
    # enforce X'_{0,-d} = X'_{0,d}^T so the dense matrix is symmetric
    Xp = np.zeros_like(B)
    for d in range(M):
        dx, dy = divmod(d, My)
        nd = ((-dx) % Mx) * My + ((-dy) % My)
        Xp[d] = 0.5 * (B[d] + B[nd].T)
    dense = np.zeros((M * k, M * k))
    for i in range(M):
        ix, iy = divmod(i, My)
        for j in range(M):
            jx, jy = divmod(j, My)
            d = ((jx - ix) % Mx) * My + ((jy - iy) % My)
            dense[i * k:(i + 1) * k, j * k:(j + 1) * k] = Xp[d]
    want = psd_project(dense)[:k, :]
    Y = psd_project(momentum_blocks(p, Xp))
    got = inverse_blocks(p, Y)
    assert np.abs(got.imag).max() < 1e-13
    got = np.concatenate(list(got.real), axis=1)
    assert np.abs(got - want).max() < 1e-12
