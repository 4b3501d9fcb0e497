"""Dense Algorithm 5 (no translation invariance), FP64.

Oracle; test infrastructure only.  It pins the translation-invariant reduction
of Algorithm 6 (started from the same translation-invariant point, both produce
the same iterates) and is the reference of the library's dense variant, which
also takes one-site fields that break translation invariance (disorder).  Every unordered cluster pair i < j has
its own rho_ij, rho~_ij, Lambda_ij, Lambda1_ij, Lambda2_ij (Section 3.2), the
rho_i update collects A_1 terms of pairs (i, j > i) and A_2 terms of pairs
(j < i, i) (eq. rhoiUpdate), and X is one dense (M n_op) x (M n_op) matrix
projected by a full eigendecomposition (last step of Algorithm 5, with the
X - eps G reading of the sign).
"""
from __future__ import annotations

import numpy as np

from .maps import pair_solve, psd_project, ptrace1, ptrace2


class DenseProblem:
    """Non-translation-invariant view of an Algorithm 6 problem (same H_0, H_0d, maps), with
    optional one-site fields (letter, (x, y), coeff) added to the cluster Hamiltonians."""

    def __init__(self, p, fields=()):
        self.p = p
        M = p.M
        self.pairs = [(i, j) for i in range(M) for j in range(i + 1, M)]
        g = p.geom
        from .model import site_operator

        self.Hc = {i: np.array(p.H0, dtype=float) for i in range(M)}
        for letter, (x, y), coeff in fields:
            c, loc = g.locate(x, y)
            self.Hc[c] = self.Hc[c] + coeff * site_operator({loc: letter}, g.L).real

        def offset(i, j):
            ix, iy = divmod(i, g.My)
            jx, jy = divmod(j, g.My)
            return ((jx - ix) % g.Mx) * g.My + ((jy - iy) % g.My)

        self.offset = offset
        # H_ij = H_{0, j-i} by translation invariance
        self.H = {(i, j): p.Hd[offset(i, j) - 1] for (i, j) in self.pairs}


def initial_dense(dp):
    p = dp.p
    M, m, n, k = p.M, p.m, p.n, p.n_op
    st = {
        "rho": {i: np.eye(m) / m for i in range(M)},
        "rho_t": {e: np.eye(n) / n for e in dp.pairs},
        "rho_p": {e: np.eye(n) / n for e in dp.pairs},
        "Lam": {e: np.zeros((n, n)) for e in dp.pairs},
        "Lam1": {e: np.zeros((m, m)) for e in dp.pairs},
        "Lam2": {e: np.zeros((m, m)) for e in dp.pairs},
        "X": np.eye(M * k),
    }
    return st


def dense_step(dp, st):
    """One iteration of Algorithm 5 in the paper's order."""
    p = dp.p
    M, m, k = p.M, p.m, p.n_op
    mu, nu, eps = p.mu, p.nu, p.eps
    X = st["X"]

    def blk(i, j):
        return X[i * k:(i + 1) * k, j * k:(j + 1) * k]

    Hp_i = {i: dp.Hc[i] - p.maps.C0(blk(i, i)) for i in range(M)}
    Hp_ij = {}
    for (i, j) in dp.pairs:
        R = p.maps.Rd(blk(i, j))
        Hp_ij[(i, j)] = dp.H[(i, j)] - R - R.T
    Im = np.eye(m)
    rho_p = {}
    for e in dp.pairs:
        i, j = e
        R = (mu * st["rho_t"][e] + np.kron(nu * st["rho"][i] - st["Lam1"][e], Im)
             + np.kron(Im, nu * st["rho"][j] - st["Lam2"][e]) + st["Lam"][e] - Hp_ij[e])
        rho_p[e] = pair_solve(R, m, mu, nu)
    rho_t = {e: psd_project(rho_p[e] - st["Lam"][e] / mu) for e in dp.pairs}
    rho = {}
    for i in range(M):
        acc = np.zeros((m, m))
        for (a, b) in dp.pairs:
            if a == i:
                acc += nu * ptrace2(rho_p[(a, b)], m) + st["Lam1"][(a, b)]
            elif b == i:
                acc += nu * ptrace1(rho_p[(a, b)], m) + st["Lam2"][(a, b)]
        r = (acc - Hp_i[i]) / (nu * (M - 1))
        rho[i] = r + (1.0 - np.trace(r)) / m * Im
    Lam = {e: st["Lam"][e] + mu * (rho_t[e] - rho_p[e]) for e in dp.pairs}
    Lam1 = {e: st["Lam1"][e] + nu * (ptrace2(rho_p[e], m) - rho[e[0]]) for e in dp.pairs}
    Lam2 = {e: st["Lam2"][e] + nu * (ptrace1(rho_p[e], m) - rho[e[1]]) for e in dp.pairs}
    G = np.zeros_like(X)
    for i in range(M):
        G[i * k:(i + 1) * k, i * k:(i + 1) * k] = p.maps.G0(rho[i])
    for (i, j) in dp.pairs:
        g = p.maps.Gd(rho_p[(i, j)])
        G[i * k:(i + 1) * k, j * k:(j + 1) * k] = g
        G[j * k:(j + 1) * k, i * k:(i + 1) * k] = g.T
    Xn = psd_project(X - eps * G)
    return {"rho": rho, "rho_t": rho_t, "rho_p": rho_p, "Lam": Lam, "Lam1": Lam1, "Lam2": Lam2, "X": Xn}


def energy_dense(dp, st):
    """Energy per site of the latest pair update: [sum_i Tr H_i rho_i + sum_{i<j} Tr H_ij rho_ij] / N."""
    p = dp.p
    e = sum(np.trace(dp.Hc[i] @ st["rho"][i]) for i in range(p.M))
    e += sum(np.trace(dp.H[pair] @ st["rho_p"][pair]) for pair in dp.pairs)
    return float(e) / (p.M * p.L)


def feasibility_dense(dp, st):
    """eq. feasErr summed over all pairs: consistency and rho = rho~ residuals, per cluster."""
    m = dp.p.m
    tot = 0.0
    for (i, j) in dp.pairs:
        r = st["rho_p"][(i, j)]
        tot += np.sum((ptrace2(r, m) - st["rho"][i]) ** 2) + np.sum((ptrace1(r, m) - st["rho"][j]) ** 2)
        tot += np.sum((r - st["rho_t"][(i, j)]) ** 2)
    return float(np.sqrt(tot / dp.p.M))


def lower_bound_dense(dp, st):
    """Lagrangian lower bound per site for the dense problem, valid for any PSD X and any
    symmetric Lambda1, Lambda2 (Section 2.4 applied pair by pair):

      E >= sum_i lmin(H'_i - sum_{(i,b)} L1_(i,b) - sum_{(a,i)} L2_(a,i))
           + sum_{i<j} lmin(H'_ij + L1_ij x I + I x L2_ij),

    with H'_i = H_i - C_0(X_ii), H'_ij = H_ij - R(X_ij) - R(X_ij)^T; divided by N.
    Minimising the Lagrangian over trace-one PSD marginals gives the smallest eigenvalues."""
    p = dp.p
    M, m, k = p.M, p.m, p.n_op
    X = st["X"]
    Im = np.eye(m)

    def sym(a):
        return 0.5 * (a + a.T)

    tot = 0.0
    for i in range(M):
        A = dp.Hc[i] - p.maps.C0(X[i * k:(i + 1) * k, i * k:(i + 1) * k])
        for (a, b) in dp.pairs:
            if a == i:
                A = A - sym(st["Lam1"][(a, b)])
            elif b == i:
                A = A - sym(st["Lam2"][(a, b)])
        tot += np.linalg.eigvalsh(sym(A))[0]
    for (i, j) in dp.pairs:
        R = p.maps.Rd(X[i * k:(i + 1) * k, j * k:(j + 1) * k])
        K = dp.H[(i, j)] - R - R.T + np.kron(sym(st["Lam1"][(i, j)]), Im) + np.kron(Im, sym(st["Lam2"][(i, j)]))
        tot += np.linalg.eigvalsh(sym(K))[0]
    return float(tot) / (M * p.L)
