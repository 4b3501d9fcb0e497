"""Physics pins of the oracle's Algorithm 6 (Sections 2-4 of the paper).

* the local Hamiltonians and the per-cluster energy formula reproduce the
  exact ground-state energy from exact marginals;
* the Jordan-Wigner closed form agrees with exact diagonalisation;
* the Lagrangian lower bound stays at or below E_0 at every iterate;
* one cluster pair spanning the ring (M = 2) makes the relaxation tight;
* h = 0 is exact (Section 4, caption of the TFI figure);
* larger clusters tighten the bound (Section 4);
* the paper's printed energies (Tables tfi_size_energies, tfi_100x1_energies,
  and the AFH tables) are reproduced;
* invariants of the iteration (unit trace, swap symmetry, PSD momentum blocks);
* the translation-invariant iteration equals the dense non-invariant
  Algorithm 5 from the same start;
* Algorithm 4 with X frozen converges to its own Lagrangian bound;
* the printed "+ eps G" sign diverges (why the oracle reads it as - eps G).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import alg5, alg6, exact
from oracle.maps import ptrace1, ptrace2

GOLD = os.path.join(os.path.dirname(__file__), "golden")
with open(os.path.join(GOLD, "exact_energies.json")) as f:
    EXACT = json.load(f)
with open(os.path.join(GOLD, "paper_tables.json")) as f:
    TABLES = json.load(f)


def _run(w, iters, every=0):
    p = alg6.Problem.from_workload(w)
    s, tr = alg6.solve(p, iters, every=every)
    return p, s, tr


# ---------------------------------------------------------------------------
# Hamiltonian assembly and exact references
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("w", [
    synth.tfi_ring(8, 1, 1.0), synth.tfi_ring(8, 2, 0.7), synth.tfi_ring(8, 4, 1.3), synth.xxz_ring(8, 2, 0.5),
    synth.tfi_ring(6, 3, 1.0), synth.tfi_ring(2, 1, 1.0), synth.tfi_torus(4, 2, 2, 1, 1.0), synth.afh_torus(2, 4, 1, 2),
], ids=lambda w: w.name)
def test_energy_formula_on_exact_marginals(w):
    """Per-cluster energy Tr H_0 rho_0 + 1/2 sum_d Tr H_0d rho_0d of exact marginals equals E_0/N."""
    E0, psi = exact.ground_state(w.terms, w.extent)
    p = alg6.Problem.from_workload(w)
    rho0, rhos = exact.cluster_marginals(psi, w.extent, w.cluster)
    st = alg6.initial_state(p)
    st.rho0, st.rho = rho0, rhos
    N = w.extent[0] * w.extent[1]
    assert abs(alg6.energy_per_site(p, st) - E0 / N) < 1e-12
    # the exact marginals are feasible: consistent partial traces
    assert np.abs(ptrace2(rhos, p.m) - rho0).max() < 1e-12
    assert np.abs(ptrace1(rhos, p.m) - rho0).max() < 1e-12


@pytest.mark.parametrize("N", [4, 6, 8, 10, 12])
@pytest.mark.parametrize("h", [0.5, 1.0, 1.5, 3.0])
def test_jordan_wigner_matches_ed(N, h):
    E0, _ = exact.ground_state(synth.tfi_terms(h, 1.0, 1), (N, 1))
    assert abs(exact.tfi_ring_energy_jw(N, h) - E0 / N) < 1e-12


def test_golden_exact_values_reproduce():
    E0, _ = exact.ground_state(synth.afh_terms(1), (8, 1))
    assert abs(E0 / 8 - EXACT["afh_ring_N8"]["E0_per_site"]) < 1e-12
    assert abs(exact.tfi_ring_energy_jw(8, 1.0) - EXACT["tfi_ring_N8_h1"]["E0_per_site"]) < 1e-12


def test_invalid_instances_rejected():
    with pytest.raises(ValueError):
        alg6.Problem(synth.tfi_terms(1.0), (8, 1), (3, 1))  # does not tile
    with pytest.raises(ValueError):
        alg6.Problem(synth.tfi_terms(1.0), (4, 1), (4, 1))  # one cluster: M = 1
    with pytest.raises(ValueError):
        alg6.Problem([(1.0, (("Y", (0, 0)),))], (4, 1), (1, 1))  # complex term


# ---------------------------------------------------------------------------
# Lower bound
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("w,key", [
    (synth.tfi_ring(8, 1, 1.0), "tfi_ring_N8_h1"),
    (synth.tfi_ring(8, 2, 1.0), "tfi_ring_N8_h1"),
    (synth.tfi_ring(8, 1, 1.0, "pauli1"), "tfi_ring_N8_h1"),
    (synth.xxz_ring(8, 1, 1.0), "afh_ring_N8"),
    (synth.xxz_ring(8, 2, 1.0), "afh_ring_N8"),
    (synth.xxz_ring(8, 2, 0.5), "xxz_ring_N8_Jz0.5"),
    (synth.tfi_torus(4, 4, 2, 1, 1.0, 300), "tfi_torus_4x4_h1"),
], ids=lambda x: getattr(x, "name", x))
def test_bound_below_exact_energy_every_iterate(w, key):
    E0 = EXACT[key]["E0_per_site"]
    p = alg6.Problem.from_workload(w)
    s = alg6.initial_state(p)
    for _ in range(300):
        s = alg6.step(p, s)
        assert alg6.lower_bound(p, s) <= E0 + 1e-12


def test_bound_below_jordan_wigner():
    for N, L in [(10, 1), (12, 2), (10, 2)]:
        p, s, _ = _run(synth.tfi_ring(N, L, 1.0), 1500)
        assert alg6.lower_bound(p, s) <= exact.tfi_ring_energy_jw(N, 1.0)


@pytest.mark.parametrize("N,L", [(2, 1), (4, 2)])
def test_tight_when_one_pair_spans_the_ring(N, L):
    """M = 2: the single pair marginal is the whole state, so the bound reaches E_0."""
    w = synth.tfi_ring(N, L, 1.0)
    E0, _ = exact.ground_state(w.terms, w.extent)
    p, s, _ = _run(w, 4000)
    assert abs(alg6.lower_bound(p, s) - E0 / N) < 1e-8
    assert abs(alg6.energy_per_site(p, s) - E0 / N) < 1e-8


@pytest.mark.slow
@pytest.mark.parametrize("N,L,eps,tol", [(6, 3, 2.0, 1e-5), (8, 4, 0.5, 2e-5)])
def test_tight_m2_large_clusters(N, L, eps, tol):
    """M = 2 with 3- and 4-site clusters: the bound approaches E_0 / N sublinearly (10,000 iterations).
    The 4-site case does not converge at the paper's eps = 2 (the bound stays ~9 per site below E_0),
    so it runs at eps = 0.5; the relaxation's value does not depend on the step."""
    w = synth.tfi_ring(N, L, 1.0)
    E0, _ = exact.ground_state(w.terms, w.extent)
    p = alg6.Problem(w.terms, w.extent, w.cluster, "complete", 10.0, 10.0, eps)
    s, _ = alg6.solve(p, 10000)
    lb = alg6.lower_bound(p, s)
    assert lb <= E0 / N + 1e-12 and abs(lb - E0 / N) < tol


@pytest.mark.parametrize("w,target", [
    (synth.tfi_ring(8, 1, 0.0), -1.0), (synth.tfi_ring(8, 2, 0.0), -1.0),
    (synth.tfi_torus(4, 4, 1, 1, 0.0), -2.0),
], ids=lambda x: getattr(x, "name", str(x)))
def test_exact_at_zero_field(w, target):
    p, s, _ = _run(w, 1500)
    assert abs(alg6.lower_bound(p, s) - target) < 1e-8
    assert abs(alg6.energy_per_site(p, s) - target) < 1e-8


def test_larger_clusters_tighten_the_bound():
    """Converged relaxation values increase with cluster size; the complete collection beats single-site Paulis."""
    E0 = EXACT["tfi_ring_N8_h1"]["E0_per_site"]
    p1, s1, _ = _run(synth.tfi_ring(8, 1, 1.0), 3000)
    pp, sp, _ = _run(synth.tfi_ring(8, 1, 1.0, "pauli1"), 3000)
    p2, s2, _ = _run(synth.tfi_ring(8, 2, 1.0), 2000)
    lb1, lbp, lb2 = (alg6.lower_bound(p1, s1), alg6.lower_bound(pp, sp), alg6.lower_bound(p2, s2))
    e1 = alg6.energy_per_site(p1, s1)
    ep = alg6.energy_per_site(pp, sp)
    assert abs(e1 - lb1) < 1e-7 and abs(ep - lbp) < 1e-6  # converged L = 1 values
    assert lbp <= lb1 + 1e-7  # complete >= single-site Pauli collection
    assert e1 < lb2 <= E0  # L = 1 optimum below a valid L = 2 bound, itself below E_0


# ---------------------------------------------------------------------------
# Paper tables
# ---------------------------------------------------------------------------

def test_table_size_energies_N20_h1():
    """Table tfi_size_energies, 20x1 lattice, h = 1, 2x1 clusters, 10000 iterations: -1.283534."""
    want = TABLES["tfi_size_energies"]["N"]["20"][1]
    p, s, _ = _run(synth.tfi_ring(20, 2, 1.0), 10000)
    assert abs(alg6.energy_per_site(p, s) - want) < 2e-6
    assert abs(alg6.lower_bound(p, s) - want) < 2e-6


@pytest.mark.slow
@pytest.mark.parametrize("N", ["20", "40", "60", "80", "100"])
@pytest.mark.parametrize("hi", [0, 1, 2])
def test_table_size_energies(N, hi):
    want = TABLES["tfi_size_energies"]["N"][N][hi]
    h = TABLES["tfi_size_energies"]["h"][hi]
    p, s, _ = _run(synth.tfi_ring(int(N), 2, h), 40000)
    assert abs(alg6.energy_per_site(p, s) - want) < 2e-6


@pytest.mark.slow
@pytest.mark.parametrize("L", ["1", "2"])
@pytest.mark.parametrize("hi", [0, 1, 2])
def test_table_100x1_energies(L, hi):
    want = TABLES["tfi_100x1_energies"]["L"][L][hi]
    h = TABLES["tfi_100x1_energies"]["h"][hi]
    p, s, _ = _run(synth.tfi_ring(100, int(L), h), 10000)
    assert abs(alg6.energy_per_site(p, s) - want) < 1e-4


def test_table_100x1_one_site_clusters_h1_and_energy_change():
    """Table tfi_100x1_energies, 1x1 clusters, h = 1: -1.3084 (4 printed decimals, so 1e-4), reached
    by 6000 iterations; and Section 4's convergence claim for this run: the per-site energy change of
    one iteration is below 1e-6 well within 10^4 iterations."""
    want = TABLES["tfi_100x1_energies"]["L"]["1"][1]
    p, s, _ = _run(synth.tfi_ring(100, 1, 1.0), 6000)
    e = alg6.energy_per_site(p, s)
    assert abs(e - want) < 1e-4
    s2 = alg6.step(p, s)
    assert abs(alg6.energy_per_site(p, s2) - e) < 1e-6


@pytest.mark.slow
@pytest.mark.parametrize("hi", [0, 1, 2])
def test_table_100x1_energies_four_site_clusters(hi):
    """Table tfi_100x1_energies, 4x1 clusters (pair marginals 256 x 256): -1.0636 / -1.2761 / -1.6720."""
    want = TABLES["tfi_100x1_energies"]["L"]["4"][hi]
    h = TABLES["tfi_100x1_energies"]["h"][hi]
    p, s, _ = _run(synth.tfi_ring(100, 4, h), 10000)
    assert abs(alg6.energy_per_site(p, s) - want) < 1e-4


@pytest.mark.slow
@pytest.mark.parametrize("L", [1, 2, 4])
def test_energy_change_below_1e6_within_1e4_iterations(L):
    """Section 4 (convergence on the 100x1 TFI lattice, h = 1): the per-site energy change between
    consecutive iterations falls below 1e-6 within 10^4 iterations for every cluster size."""
    p = alg6.Problem.from_workload(synth.tfi_ring(100, L, 1.0))
    s = alg6.initial_state(p)
    e_prev = None
    reached = None
    for t in range(1, 10001):
        s = alg6.step(p, s)
        e = alg6.energy_per_site(p, s)
        if e_prev is not None and abs(e - e_prev) < 1e-6 and t > 100:
            reached = t
            break
        e_prev = e
    assert reached is not None


def test_certified_interval_afh_ring():
    """At convergence the relaxation value is bracketed: LB <= E0^(2) <= energy of a feasible point.

    Feasibility = small eq. feasErr, PSD pair marginals (rho~) and G >= 0 (eq. sdpC4).
    """
    p, s, _ = _run(synth.xxz_ring(8, 2, 1.0), 5000)
    lb, e = alg6.lower_bound(p, s), alg6.energy_per_site(p, s)
    assert alg6.feasibility_error(p, s) < 1e-10
    assert alg6.primal_G_min_eig(p, s) > -1e-9
    assert lb <= e + 1e-9 and e - lb < 1e-8  # e is feasible only up to feasErr
    assert e <= EXACT["afh_ring_N8"]["E0_per_site"]


# ---------------------------------------------------------------------------
# Invariants and structure
# ---------------------------------------------------------------------------

def test_invariants_along_iteration():
    w = synth.tfi_ring(10, 2, 1.2)
    p = alg6.Problem.from_workload(w)
    s = alg6.initial_state(p)
    m, M = p.m, p.M
    swap = np.zeros((p.n, p.n))
    for a in range(m):
        for b in range(m):
            swap[b * m + a, a * m + b] = 1.0
    for _ in range(60):
        s = alg6.step(p, s)
        assert abs(np.trace(s.rho0) - 1.0) < 1e-13
        for d in range(1, M):
            nd = M - d
            assert np.abs(s.rho[nd - 1] - swap @ s.rho[d - 1] @ swap).max() < 1e-12
            assert np.abs(s.X[nd] - s.X[d].T).max() < 1e-12
        Y = alg6.momentum_blocks(p, s.X)
        ev = np.linalg.eigvalsh(Y)
        assert ev.min() >= -1e-13 * max(1.0, np.abs(ev).max())


def test_min_momentum_eig_is_the_dense_minimum():
    """min_momentum_eig = the smallest eigenvalue of the dense block-circulant X built from the first
    block row (its plain definition) divided by sqrt(M): the momentum blocks of step 7 carry the
    M^{-1/2} normalisation, the block-diagonalisation of the dense matrix has none.  Checked on a
    perturbed iterate of a 2-D lattice (not PSD, so the minimum is a genuine negative eigenvalue)."""
    w = synth.tfi_torus(4, 2, 2, 1, 1.3)
    p = alg6.Problem.from_workload(w)
    s = alg6.initial_state(p)
    for _ in range(5):
        s = alg6.step(p, s)
    X = s.X + 1e-3 * np.random.default_rng([210602682, 61]).standard_normal(s.X.shape)
    for d in range(p.M):  # keep X_{0,-d} = X_{0,d}^T so the dense matrix is symmetric
        dx, dy = divmod(d, p.My)
        nd = ((-dx) % p.Mx) * p.My + ((-dy) % p.My)
        if nd < d:
            X[d] = X[nd].T
        elif nd == d:
            X[d] = 0.5 * (X[d] + X[d].T)
    k, M = p.n_op, p.M
    dense = np.zeros((M * k, M * k))
    for i in range(M):
        ix, iy = divmod(i, p.My)
        for j in range(M):
            jx, jy = divmod(j, p.My)
            d = ((jx - ix) % p.Mx) * p.My + ((jy - iy) % p.My)
            dense[i * k:(i + 1) * k, j * k:(j + 1) * k] = X[d]
    s.X = X
    lam = np.linalg.eigvalsh(dense)[0]
    assert lam < -1e-4
    assert abs(alg6.min_momentum_eig(p, s) * np.sqrt(M) - lam) < 1e-12


@pytest.mark.parametrize("model,N,L,opset", [("tfi", 8, 1, "complete"), ("tfi", 8, 2, "complete"),
                                             ("tfi", 6, 1, "pauli1"), ("tfi", 4, 1, "complete"),
                                             ("xxz", 8, 1, "complete"), ("xxz", 8, 2, "complete"),
                                             ("xxz", 6, 1, "pauli1"), ("afh", 8, 2, "complete")])
def test_translation_invariant_equals_dense_algorithm5(model, N, L, opset):
    """Algorithm 6 iterates equal those of the dense Algorithm 5 from the same start; the XXZ
    (J_z = 0.7) and AFH instances carry off-diagonal XX + YY bonds through every map."""
    w = {"tfi": lambda: synth.tfi_ring(N, L, 1.1, opset), "xxz": lambda: synth.xxz_ring(N, L, 0.7, opset),
         "afh": lambda: synth.xxz_ring(N, L, 1.0, opset)}[model]()
    p = alg6.Problem.from_workload(w)
    dp = alg5.DenseProblem(p)
    s = alg6.initial_state(p)
    ds = alg5.initial_dense(dp)
    k = p.n_op
    for _ in range(50):
        s = alg6.step(p, s)
        ds = alg5.dense_step(dp, ds)
    for d in range(1, p.M):
        assert np.abs(ds["rho_t"][(0, d)] - s.rho_t[d - 1]).max() < 1e-12
        assert np.abs(ds["Lam"][(0, d)] - s.Lam[d - 1]).max() < 1e-11
        assert np.abs(ds["Lam2"][(0, d)] - s.Lam2[d - 1]).max() < 1e-11
        assert np.abs(ds["X"][:k, d * k:(d + 1) * k] - s.X[d]).max() < 1e-12
    for i in range(p.M):
        assert np.abs(ds["rho"][i] - s.rho0).max() < 1e-12


def test_algorithm4_with_fixed_X_closes_its_gap():
    """Algorithm 4 (X frozen at the start value I): residuals vanish and the bound meets the inner objective."""
    w = synth.tfi_ring(8, 1, 1.0)
    p = alg6.Problem.from_workload(w)
    s = alg6.initial_state(p)
    for _ in range(3000):
        s = alg6.step(p, s, x_step=False)
    H0p, Hdp = alg6.effective_hamiltonians(p, s.X)
    inner = (np.trace(H0p @ s.rho0) + 0.5 * np.einsum("dij,dji->", Hdp, s.rho)) / p.L
    assert alg6.feasibility_error(p, s) < 1e-9
    assert abs(inner - alg6.lower_bound(p, s)) < 1e-9


def test_printed_plus_sign_diverges():
    w = synth.tfi_ring(8, 1, 1.0)
    p = alg6.Problem.from_workload(w)
    with np.errstate(all="ignore"):
        s, _ = alg6.solve(p, 200, sign=+1)
        assert not np.isfinite(alg6.lower_bound(p, s)) or alg6.feasibility_error(p, s) > 1e6
    s, _ = alg6.solve(p, 200, sign=-1)
    assert alg6.feasibility_error(p, s) < 1e-3
