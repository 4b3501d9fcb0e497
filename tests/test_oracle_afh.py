"""The antiferromagnetic Heisenberg model (eq. AFH) in the oracle, and why its printed tables are not
this relaxation's optimum.

Two independent facts pin the oracle's off-diagonal (XX + YY) bond path:

* 1x1 clusters.  The two-marginal SDP (eqs. sdpObj-sdpC4, complete operator collection) and the AFH
  Hamiltonian are invariant under a global SU(2) rotation of every site, and under lattice
  translations; averaging a feasible point over both keeps it feasible (G transforms by a unitary
  congruence) with the same energy.  So some optimum has rho_i = I/2 and isotropic pair marginals:
  Werner states with <sigma^a_i sigma^b_j> = c_d delta_ab, where PSD two-site marginals allow exactly
  c_d in [-1, 1/3].  Then G is the all-ones block of the identity operators plus C (x) I_3 with C the
  circulant of (1, c_1, c_2, ...), so G >= 0 is C >= 0, i.e. nonnegative lattice Fourier sums of c.
  The SDP optimum per site is min sum_bonds 3 c_bond over that polytope: a small linear program,
  solved here with scipy, independent of the oracle.  The oracle's Lagrangian bound must never exceed
  it (the bound is below the SDP optimum at every iterate).
* 2x1 clusters on the 20x1 ring.  The iteration converges; the point it reaches is certified: the
  bound equals the primal energy to 1e-10, the equality residual (eq. feasErr) is at rounding level
  and the global matrix G of the marginals is PSD, so that value is the SDP optimum as the oracle
  builds it.

Tables afh_benchmark_20x1 / afh_benchmark_4x4 print errors below these optima (0.5383 and 0.0521 on
the ring, 0.6634 on the torus), i.e. bounds above the relaxation's own optimum, which a converged lower
bound of this SDP cannot reach; the TFI tables, which share every map but the XX + YY terms, do
reproduce.  The AFH rows stay an expected failure (see the reading in the design notes).
"""
import json
import os

import numpy as np
import pytest
from scipy.optimize import linprog

import synth
from oracle import alg6

GOLD = os.path.join(os.path.dirname(__file__), "golden")
with open(os.path.join(GOLD, "exact_energies.json")) as f:
    EXACT = json.load(f)
with open(os.path.join(GOLD, "paper_tables.json")) as f:
    TABLES = json.load(f)


def su2_lp_optimum(extent):
    """Per-site optimum of the AFH two-marginal SDP with 1x1 clusters on a periodic lattice, by the
    SU(2)- and translation-reduced linear program described in the module docstring."""
    Nx, Ny = extent
    offs = [(dx, dy) for dx in range(Nx) for dy in range(Ny) if (dx, dy) != (0, 0)]
    cls = {}
    for d in offs:
        key = min(d, ((-d[0]) % Nx, (-d[1]) % Ny))  # c_d = c_{-d}
        cls.setdefault(key, len(cls))
    A = np.zeros((Nx * Ny, len(cls)))
    for kx in range(Nx):
        for ky in range(Ny):
            for (dx, dy) in offs:
                key = min((dx, dy), ((-dx) % Nx, (-dy) % Ny))
                A[kx * Ny + ky, cls[key]] -= np.cos(2 * np.pi * (dx * kx / Nx + dy * ky / Ny))
    cost = np.zeros(len(cls))
    cost[cls[(1, 0) if Nx > 1 else (0, 1)]] += 3.0  # bond along x: 3 c per site
    if Ny > 1 and Nx > 1:
        cost[cls[(0, 1)]] += 3.0  # bond along y on a torus
    r = linprog(cost, A_ub=A, b_ub=np.ones(Nx * Ny), bounds=[(-1.0, 1.0 / 3.0)] * len(cls), method="highs")
    assert r.status == 0
    return float(r.fun)


def test_lp_reduction_reproduces_known_limits():
    """Sanity of the reduction against exact diagonalisation: on the rings of 2 and 4 sites the LP
    optimum equals exact E_0/N (there the relaxation is tight); for 6 and 8 sites it lies below E_0/N;
    N = 8 gives -(1 + sqrt 2) and the 4x4 torus -4 (isotropic c = -2/3 on both bonds)."""
    from oracle import exact

    for N in (2, 4, 6, 8):
        E0, _ = exact.ground_state(synth.afh_terms(1), (N, 1))
        lp = su2_lp_optimum((N, 1))
        if N <= 4:
            assert abs(lp - E0 / N) < 1e-9
        else:
            assert lp < E0 / N - 0.1
    assert abs(su2_lp_optimum((8, 1)) - (-(1.0 + np.sqrt(2.0)))) < 1e-9
    assert abs(su2_lp_optimum((4, 4)) - (-4.0)) < 1e-9


@pytest.mark.parametrize("extent,mu,eps,iters", [((8, 1), 10.0, 2.0, 600), ((8, 1), 1.0, 0.2, 600),
                                                 ((20, 1), 10.0, 2.0, 300)])
def test_bound_never_exceeds_the_su2_optimum(extent, mu, eps, iters):
    """1x1 clusters: the Lagrangian bound of every iterate stays at or below the LP optimum (the SDP
    optimum); the iteration itself oscillates for this model at these step sizes (it does not converge)."""
    lp = su2_lp_optimum(extent)
    w = synth.xxz_ring(extent[0], 1, 1.0)
    p = alg6.Problem(w.terms, w.extent, w.cluster, "complete", mu, mu, eps)
    s = alg6.initial_state(p)
    best = -np.inf
    for _ in range(iters):
        s = alg6.step(p, s)
        lb = alg6.lower_bound(p, s)
        assert lb <= lp + 1e-10
        best = max(best, lb)
    assert best > lp - 0.5  # the bound does approach the optimum


def test_printed_one_site_errors_lie_above_the_relaxation_optimum():
    """Table afh_benchmark_20x1 (1x1: 0.5383) and Table afh_benchmark_4x4 (1x1: 0.6634) would put the
    bound above the SDP optimum: E_0/N - printed error > LP optimum, by 0.094 and 0.529 per site."""
    ring = EXACT["afh_ring_N20"]["E0_per_site"] - TABLES["afh_20x1_errors"]["L"]["1"]
    torus = EXACT["afh_torus_4x4"]["E0_per_site"] - TABLES["afh_4x4_errors"]["cluster"]["1x1"]
    assert ring > su2_lp_optimum((20, 1)) + 0.09
    assert torus > su2_lp_optimum((4, 4)) + 0.5


def test_afh_20x1_two_site_clusters_certified_optimum():
    """2x1 clusters, 5000 iterations at the paper's parameters: bound = energy, residuals at rounding
    level, G(marginals) PSD.  The certified optimum -1.853374 per site is 0.0725 below exact E_0,
    against the printed 0.0521."""
    w = synth.xxz_ring(20, 2, 1.0)
    p = alg6.Problem.from_workload(w)
    s, _ = alg6.solve(p, 5000)
    lb, e = alg6.lower_bound(p, s), alg6.energy_per_site(p, s)
    assert abs(lb - e) < 1e-10
    assert alg6.feasibility_error(p, s) < 1e-12
    assert alg6.primal_G_min_eig(p, s) > -1e-12
    assert alg6.min_momentum_eig(p, s) > -1e-12
    err = EXACT["afh_ring_N20"]["E0_per_site"] - lb
    assert abs(err - 0.0725) < 5e-4
    assert err > TABLES["afh_20x1_errors"]["L"]["2"] + 0.02


@pytest.mark.xfail(reason="Table afh_benchmark_20x1 is not this SDP's optimum: with 2x1 clusters the oracle's "
                          "certified optimum (bound = energy, feasErr ~1e-14, G >= 0) has error 0.0725, not "
                          "0.0521, and the 1x1 entry lies above the SU(2)-reduced LP optimum",
                   strict=True)
def test_table_afh_20x1_two_site_clusters():
    E0 = EXACT["afh_ring_N20"]["E0_per_site"]
    err = TABLES["afh_20x1_errors"]["L"]["2"]
    p = alg6.Problem.from_workload(synth.xxz_ring(20, 2, 1.0))
    s, _ = alg6.solve(p, 5000)
    assert abs(alg6.energy_per_site(p, s) - (E0 - err)) < 1e-4
