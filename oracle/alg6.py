"""Algorithm 6 (translation-invariant ADMM / projected dual gradient ascent), FP64.

Oracle; test infrastructure only.  One call of :func:`step` performs one pass
of the while-loop of Algorithm 6 (Section 3.3) in the paper's order:

1. effective Hamiltonians H'_0 = H_0[X_00], H'_0d = H_0d[X_0d]        (eq. effHam)
2. pair update rho_0d by the closed-form inverse                       (eq. rhoijUpdate)
3. rho~_0d = Pi(rho_0d - Lambda_0d / mu)                               (eq. rhoijTildeUpdate)
4. rho'_0 = [sum_d (nu A_1 rho_0d + Lambda1_0d) - H'_0] / (nu (M-1)),
   rho_0 = rho'_0 + (1 - Tr rho'_0)/m I                                (eq. rhoiUpdate)
5. multiplier updates Lambda, Lambda1, Lambda2 with the new rho_0
6. X'_00 = X_00 - eps G_00(rho_0), X'_0d = X_0d - eps G_0d(rho_0d)
7. momentum blocks Xhat_k = M^{-1/2} sum_d exp(-2 pi i d.k/M) X'_0d
8. Y_k = Pi(Hermitian part of Xhat_k)
9. X_0d = Re M^{-1/2} sum_k exp(+2 pi i d.k/M) Y_k

Readings where the text is silent, garbled or at odds with itself:
* X step sign: the paper's gradient of F is -G (eq. gradX) and the effective
  Hamiltonian subtracts the X terms, so ascent on F is X <- Pi(X - eps G);
  the printed "+ eps G" is read as a sign slip.  ``sign=+1`` keeps the
  printed form for the divergence test.
* eq. effHam prints "H_ij[X_ij] := H_i - ... O_{i,a}^dag (x) O_{i,b}"; read
  H_ij and O_{j,b}.  Real case: conj(X) = X.
* M in the rho_0 update and in the FFT normalisation is the total number of
  clusters; the FFT runs per lattice axis.
* The inverse transform of the last step sums over k (the printed sum runs
  over j).
* All M-1 directed offsets d carry variables; H_0d is the full interaction
  between clusters 0 and d; energy per cluster is Tr H_0 rho_0 +
  1/2 sum_d Tr H_0d rho_0d.
* Initialisation (Section 4): rho_0 = I/m, rho~ = I/n, all multipliers 0,
  X_00 = I, X_0d = 0 for d != 0.  mu = nu = 10, eps = 2.
* Symmetric inputs to Pi are symmetrised first.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from .maps import OperatorMaps, lambda_min, pair_solve, psd_project, ptrace1, ptrace2
from .model import Geometry, local_hamiltonians


class Problem:
    """Fixed data of one instance: geometry, local Hamiltonians, operator maps, parameters."""

    def __init__(self, terms, extent, cluster, opset="complete", mu=10.0, nu=10.0, eps=2.0, fermionic=False):
        self.geom = Geometry(tuple(extent), tuple(cluster))
        g = self.geom
        self.M, self.L, self.m, self.n = g.M, g.L, g.m, g.n
        self.Mx, self.My = g.Mx, g.My
        self.P = self.M - 1
        self.fermionic = bool(fermionic)
        if self.fermionic:
            from .fermion import local_hamiltonians as fermion_hamiltonians

            self.H0, self.Hd = fermion_hamiltonians(terms, g)
        else:
            self.H0, self.Hd = local_hamiltonians(terms, g)
        self.maps = OperatorMaps(opset, g.L, self.fermionic)
        self.n_op = self.maps.n_op
        self.mu, self.nu, self.eps = float(mu), float(nu), float(eps)

    @classmethod
    def from_workload(cls, w):
        return cls(w.terms, w.extent, w.cluster, w.opset, w.mu, w.nu, w.eps, getattr(w, "fermionic", False))


@dataclass
class State:
    t: int
    X: np.ndarray  # (M, n_op, n_op): first block row X_0d, d = 0..M-1 (flat cluster index)
    rho0: np.ndarray  # (m, m)
    rho: np.ndarray  # (P, n, n): rho_0d from the latest pair update
    rho_t: np.ndarray  # (P, n, n): rho~_0d
    Lam: np.ndarray  # (P, n, n)
    Lam1: np.ndarray  # (P, m, m)
    Lam2: np.ndarray  # (P, m, m)

    def copy(self):
        return replace(self, **{k: np.array(v, copy=True) for k, v in self.__dict__.items() if isinstance(v, np.ndarray)})


def initial_state(p: Problem) -> State:
    """Section 4: multipliers zero, marginals identity with unit trace, X identity."""
    X = np.zeros((p.M, p.n_op, p.n_op))
    X[0] = np.eye(p.n_op)
    rho_t = np.broadcast_to(np.eye(p.n) / p.n, (p.P, p.n, p.n)).copy()
    return State(
        t=0,
        X=X,
        rho0=np.eye(p.m) / p.m,
        rho=rho_t.copy(),
        rho_t=rho_t,
        Lam=np.zeros((p.P, p.n, p.n)),
        Lam1=np.zeros((p.P, p.m, p.m)),
        Lam2=np.zeros((p.P, p.m, p.m)),
    )


def effective_hamiltonians(p: Problem, X):
    """eq. effHam with the readings above: H'_0 = H_0 - C0(X_00); H'_0d = H_0d - (R + R^T)(X_0d)."""
    H0p = p.H0 - p.maps.C0(X[0])
    R = p.maps.Rd(X[1:])
    Hdp = p.Hd - R - np.swapaxes(R, -1, -2)
    return H0p, Hdp


def momentum_blocks(p: Problem, Xp):
    """Xhat_k = M^{-1/2} sum_d exp(-2 pi i d.k/M) X'_0d over the Mx x My cluster lattice (Section 3.3)."""
    Xg = Xp.reshape(p.Mx, p.My, p.n_op, p.n_op)
    return np.fft.fftn(Xg, axes=(0, 1), norm="ortho").reshape(p.M, p.n_op, p.n_op)


def inverse_blocks(p: Problem, Y):
    """X_0d = M^{-1/2} sum_k exp(+2 pi i d.k/M) Y_k; returns the complex result."""
    Yg = Y.reshape(p.Mx, p.My, p.n_op, p.n_op)
    return np.fft.ifftn(Yg, axes=(0, 1), norm="ortho").reshape(p.M, p.n_op, p.n_op)


def project_X(p: Problem, Xp):
    """Steps 7-9: Pi over the block-circulant X' through its momentum blocks."""
    Xh = momentum_blocks(p, Xp)
    Y = psd_project(Xh)
    Xc = inverse_blocks(p, Y)
    scale = max(1.0, np.abs(Xc).max())
    if np.abs(Xc.imag).max() > 1e-9 * scale:
        raise FloatingPointError("inverse transform left an imaginary part above rounding")
    return Xc.real.copy(), Y


def step(p: Problem, s: State, sign: int = -1, x_step: bool = True) -> State:
    """One iteration of Algorithm 6.  ``x_step=False`` freezes X (Algorithm 4 with X fixed)."""
    m, mu, nu, eps = p.m, p.mu, p.nu, p.eps
    X = s.X
    # 1. effective Hamiltonians from the current X
    H0p, Hdp = effective_hamiltonians(p, X)
    # 2. pair update (eq. rhoijUpdate); uses the previous rho_0
    A1s = nu * s.rho0[None] - s.Lam1
    A2s = nu * s.rho0[None] - s.Lam2
    Im = np.eye(m)
    R = mu * s.rho_t + np.stack([np.kron(a, Im) + np.kron(Im, b) for a, b in zip(A1s, A2s)]) + s.Lam - Hdp
    rho = pair_solve(R, m, mu, nu)
    # 3. PSD projection (eq. rhoijTildeUpdate)
    rho_t = psd_project(rho - s.Lam / mu)
    # 4. cluster marginal (eq. rhoiUpdate)
    tr2 = ptrace2(rho, m)
    tr1 = ptrace1(rho, m)
    rho0p = (np.sum(nu * tr2 + s.Lam1, axis=0) - H0p) / (nu * (p.M - 1))
    z = (1.0 - np.trace(rho0p)) / m
    rho0 = rho0p + z * Im
    # 5. multipliers
    Lam = s.Lam + mu * (rho_t - rho)
    Lam1 = s.Lam1 + nu * (tr2 - rho0[None])
    Lam2 = s.Lam2 + nu * (tr1 - rho0[None])
    # 6-9. X step and projection
    if x_step:
        Xp = np.empty_like(X)
        Xp[0] = X[0] + sign * eps * p.maps.G0(rho0)
        Xp[1:] = X[1:] + sign * eps * p.maps.Gd(rho)
        Xn, _ = project_X(p, Xp)
    else:
        Xn = X.copy()
    return State(s.t + 1, Xn, rho0, rho, rho_t, Lam, Lam1, Lam2)


# ---------------------------------------------------------------------------
# Diagnostics
# ---------------------------------------------------------------------------

def energy_per_site(p: Problem, s: State) -> float:
    """[Tr(H_0 rho_0) + 1/2 sum_d Tr(H_0d rho_0d)] / L (primal objective of eq. sdpObj per site)."""
    e = np.trace(p.H0 @ s.rho0) + 0.5 * np.einsum("dij,dji->", p.Hd, s.rho)
    return float(e) / p.L


def feasibility_error(p: Problem, s: State) -> float:
    """eq. feasErr: per-cluster equality-constraint residual."""
    m = p.m
    r1 = ptrace2(s.rho, m) - s.rho0[None]
    r2 = ptrace1(s.rho, m) - s.rho0[None]
    r3 = s.rho - s.rho_t
    tot = np.sum(r1 ** 2) + np.sum(r2 ** 2) + np.sum(r3 ** 2)
    return float(np.sqrt(tot / (p.M - 1)))


def lower_bound(p: Problem, s: State) -> float:
    """Lagrangian lower bound per site, valid for any PSD X and any symmetric Lambda1, Lambda2.

    For feasible translation-invariant marginals, energy >= energy - <X, G>/M
    (X, G both PSD) = Tr H'_0 rho_0 + 1/2 sum_d Tr H'_0d rho_0d (Section 2.4,
    the Lagrangian term -Tr[X G]); adding the vanishing consistency terms
    1/2 sum_d <Lambda1_d, A_1 rho_0d - rho_0> + <Lambda2_d, A_2 rho_0d - rho_0>
    and bounding each trace by the smallest eigenvalue gives
    (1/L)[lmin(H'_0 - 1/2 sum_d (Lambda1_d + Lambda2_d))
          + 1/2 sum_d lmin(H'_0d + Lambda1_d (x) I + I (x) Lambda2_d)].
    """
    m = p.m
    H0p, Hdp = effective_hamiltonians(p, s.X)
    L1 = 0.5 * (s.Lam1 + np.swapaxes(s.Lam1, -1, -2))
    L2 = 0.5 * (s.Lam2 + np.swapaxes(s.Lam2, -1, -2))
    K0 = H0p - 0.5 * np.sum(L1 + L2, axis=0)
    Im = np.eye(m)
    Kd = Hdp + np.stack([np.kron(a, Im) + np.kron(Im, b) for a, b in zip(L1, L2)])
    val = lambda_min(K0) + 0.5 * np.sum(lambda_min(Kd))
    return float(val) / p.L


def min_momentum_eig(p: Problem, s: State) -> float:
    """Smallest eigenvalue over the momentum blocks of the current X (>= -rounding)."""
    return float(np.min(lambda_min(momentum_blocks(p, s.X))))


def primal_G_min_eig(p: Problem, s: State) -> float:
    """Smallest eigenvalue of the global matrix G of the current marginals (eq. sdpC4).

    G is block-circulant with first block row (G_00(rho_0), G_0d(rho_0d)); its
    momentum blocks come from the same transform as X.  Together with a small
    feasibility error, G >= 0 makes the energy an upper bound on the relaxation.
    """
    Gp = np.empty((p.M, p.n_op, p.n_op))
    Gp[0] = p.maps.G0(s.rho0)
    Gp[1:] = p.maps.Gd(s.rho)
    return float(np.min(lambda_min(momentum_blocks(p, Gp))))


def diagnostics(p: Problem, s: State) -> dict:
    e = energy_per_site(p, s)
    lb = lower_bound(p, s)
    return {
        "t": s.t,
        "energy": e,
        "lb": lb,
        "gap": (e - lb) / abs(lb) if lb != 0 else np.inf,
        "feas": feasibility_error(p, s),
        "min_eig_X": min_momentum_eig(p, s),
    }


def solve(p: Problem, iters: int, every: int = 0, state: State | None = None, sign: int = -1):
    """Run ``iters`` iterations; returns (final state, list of diagnostics every ``every`` iterations)."""
    s = state.copy() if state is not None else initial_state(p)
    trace = []
    for _ in range(iters):
        s = step(p, s, sign=sign)
        if every and s.t % every == 0:
            trace.append(diagnostics(p, s))
    return s, trace
