"""Spinless fermions (appendix on fermions), FP64.

Oracle; test infrastructure only.  The two-marginal relaxation of a fermionic
pairwise Hamiltonian fixes a Jordan-Wigner transformation (JWT) per cluster
(sites in local order) and per cluster pair (the first cluster's sites, then
the second's); no global JWT enters the relaxation.  After the JWT the SDP has
the form of the spin case, with two changes:

* the local Hamiltonians are the JW images of the fermionic terms: hopping
  a_i^dag a_j + h.c. inside a cluster in the cluster's JWT, and between two
  clusters in the pair's JWT (strings over the sites in between);
* an operator of the second cluster of a pair, taken to the pair's JWT,
  carries the parity string of the first cluster when it is odd, so the
  off-diagonal blocks of G (and the matching corrections of eq. effHam) change
  by signs.

Conventions: a site is empty (|0>) or occupied (|1>); a = |0><1| on its site
(sigma^-), n = a^dag a = (1 - Z)/2.  The JW image of a_k in an ordered set of
sites is Z x ... x Z (the sites before k) x sigma^- x I x ... .

The library's fast forms (sign masks on the realignment) are pinned against
the definitions here, which build every operator from the JWT itself.
"""
from __future__ import annotations

import numpy as np

from .model import Geometry, site_operator

SIGMA_MINUS = np.array([[0.0, 1.0], [0.0, 0.0]])
PAULI_Z = np.diag([1.0, -1.0])


def annihilators(nsites: int) -> list:
    """JW images of a_0 .. a_{nsites-1} on 2^nsites states (site 0 the most significant factor)."""
    out = []
    for k in range(nsites):
        op = np.ones((1, 1))
        for s in range(nsites):
            op = np.kron(op, PAULI_Z if s < k else (SIGMA_MINUS if s == k else np.eye(2)))
        out.append(op)
    return out


def hopping(nsites: int, p: int, q: int) -> np.ndarray:
    """a_p^dag a_q + a_q^dag a_p in the JWT of `nsites` ordered sites."""
    a = annihilators(nsites)
    return a[p].T @ a[q] + a[q].T @ a[p]


def unit_image(c: int, e: int, ops) -> np.ndarray:
    """Image of the fermionic operator whose JW image on len(ops) sites is the matrix unit
    E_ce, under the map sending the k-th annihilator to ops[k] (any operators obeying the
    anticommutation relations; with the sites' own JW annihilators this returns E_ce).

    Per site k, with row bit c_k and column bit e_k, E_ce is the tensor product of
    |c_k><e_k|: 1 - n_k, n_k, sigma^+_k or sigma^-_k, and the bare sigma^-_k equals
    (prod_{j<k} (1 - 2 n_j)) a_k in terms of the annihilators."""
    L = len(ops)
    dim = ops[0].shape[0]
    eye = np.eye(dim)
    num = [a.T @ a for a in ops]
    out = eye
    for k in range(L):
        ck = (c >> (L - 1 - k)) & 1
        ek = (e >> (L - 1 - k)) & 1
        if ck == ek:
            f = num[k] if ck else eye - num[k]
        else:
            string = eye
            for j in range(k):
                string = string @ (eye - 2.0 * num[j])
            f = string @ (ops[k].T if ck else ops[k])
        out = out @ f
    return out


def pair_images(L: int):
    """JW images in the pair's JWT of the matrix units of the first cluster (A, offset 0) and of
    the second cluster (B, offset L): lists indexed by a*m + b."""
    m = 2 ** L
    b = annihilators(2 * L)
    first, second = b[:L], b[L:]
    A = [unit_image(a_, b_, first) for a_ in range(m) for b_ in range(m)]
    B = [unit_image(c_, e_, second) for c_ in range(m) for e_ in range(m)]
    return A, B


def Gd_generic(rho: np.ndarray, L: int) -> np.ndarray:
    """(G_0d)_{alpha beta} = Tr[J(A_0,alpha)^T J(A_d,beta) rho] with both operators in the pair's JWT
    (appendix on fermions, definition of G; real operators: dagger = transpose)."""
    A, B = pair_images(L)
    return np.array([[np.trace(Aa.T @ Bb @ rho) for Bb in B] for Aa in A])


def Rd_generic(X: np.ndarray, L: int) -> np.ndarray:
    """sum_{alpha beta} X_{alpha beta} J(A_0,alpha)^T J(A_d,beta): the pair correction of eq. effHam
    (before adding its transpose), adjoint of Gd_generic."""
    A, B = pair_images(L)
    n = (2 ** L) ** 2
    R = np.zeros((n, n))
    for i, Aa in enumerate(A):
        for j, Bb in enumerate(B):
            if X[i, j] != 0.0:
                R += X[i, j] * (Aa.T @ Bb)
    return R


def _parity(x: np.ndarray) -> np.ndarray:
    return np.array([bin(int(v)).count("1") & 1 for v in np.ravel(x)]).reshape(np.shape(x))


def sign_mask(m: int) -> np.ndarray:
    """s(a)^(p(c) + p(e)) over the matrix-unit indices ((a, b), (c, e)), s(a) = (-1)^popcount(a),
    p = popcount mod 2: the parity string of the first cluster met by odd units of the second."""
    idx = np.arange(m)
    s = 1 - 2 * _parity(idx)
    p = _parity(idx)
    mask = np.ones((m, m, m, m))
    for a in range(m):
        for c in range(m):
            for e in range(m):
                if (p[c] + p[e]) & 1:
                    mask[a, :, c, e] = s[a]
    return mask.reshape(m * m, m * m)


def Gd_complete(rho: np.ndarray, m: int) -> np.ndarray:
    """Fast form: (G_0d)_(a,b),(c,e) = s(a)^(p(c)+p(e)) rho_(a,e),(b,c); works on stacks."""
    from .maps import Gd_complete as spin_gd

    return spin_gd(rho, m) * sign_mask(m)


def Rd_complete(X: np.ndarray, m: int) -> np.ndarray:
    """Fast form: R_(x,y),(x',y') = s(x')^(p(y)+p(y')) X_(x',x),(y,y'); works on stacks."""
    from .maps import Rd_complete as spin_rd

    # R_(x,y),(x',y') = X_(a,b),(c,e) with a = x', b = x, c = y, e = y': the mask of (a, c, e)
    n = m * m
    mk = sign_mask(m).reshape(m, m, m, m)  # [a, b, c, e]
    rmask = np.einsum("abce->bcae", mk).reshape(n, n)  # [(x=b, y=c), (x'=a, y'=e)]
    return spin_rd(X, m) * rmask


def local_hamiltonians(terms, geom: Geometry):
    """H_0 (cluster JWT) and H_0d, d = 1..M-1 (pair JWT, cluster 0 first), of a fermionic term list:
    ("F", "F") two-site terms are hoppings t (a_i^dag a_j + h.c.); "Z" letters are 1 - 2n (even,
    no strings).  Term instances are collected as in the spin case (every translate touching
    cluster 0)."""
    L, m, n, M = geom.L, geom.m, geom.n, geom.M
    H0 = np.zeros((m, m))
    Hd = np.zeros((M, n, n))
    for coeff, factors in terms:
        letters = [p for p, _ in factors]
        hop = letters == ["F", "F"]
        if not hop and any(p not in ("Z",) for p in letters):
            raise ValueError("fermionic models take hoppings ('F', 'F') and density letters 'Z' only")
        for x in range(geom.Nx):
            for y in range(geom.Ny):
                placed = [(p, geom.locate(x + o[0], y + o[1])) for p, o in factors]
                clusters = [c for _, (c, _) in placed]
                if len(placed) == 2 and placed[0][1] == placed[1][1]:
                    raise ValueError("a two-site term folds onto one site on this lattice")
                if 0 not in clusters:
                    continue
                if all(c == 0 for c in clusters):
                    if hop:
                        H0 += coeff * hopping(L, placed[0][1][1], placed[1][1][1])
                    else:
                        op = np.eye(m)
                        for p, (_, loc) in placed:
                            op = op @ site_operator({loc: p}, L).real
                        H0 += coeff * op
                else:
                    (p0, (c0, l0)), (p1, (c1, l1)) = placed
                    if c0 != 0:
                        (p0, (c0, l0)), (p1, (c1, l1)) = (p1, (c1, l1)), (p0, (c0, l0))
                    if hop:
                        Hd[c1] += coeff * hopping(2 * L, l0, L + l1)
                    else:
                        Hd[c1] += coeff * np.kron(site_operator({l0: p0}, L).real, site_operator({l1: p1}, L).real)
    return H0, Hd[1:].copy()


# ---------------------------------------------------------------------------
# Exact references
# ---------------------------------------------------------------------------

def full_hamiltonian_sparse(terms, extent, fields=()):
    """Fock-space Hamiltonian of the whole lattice (sites in flat order x * Ny + y, site 0 the most
    significant bit).  A hopping a_s^dag a_t moves a particle from t to s with the sign
    (-1)^(number of occupied sites strictly between s and t), the anticommutation sign of the
    global ordering; "Z" is 1 - 2n.  fields: one-site (letter "Z", (x, y), coeff)."""
    import scipy.sparse as sp

    Nx, Ny = extent
    N = Nx * Ny
    dim = 2 ** N
    idx = np.arange(dim, dtype=np.int64)

    def mask(s):
        return np.int64(1) << (N - 1 - s)

    def occ(s):
        return (idx >> (N - 1 - s)) & 1

    rows, cols, vals = [], [], []

    def hop(s, t, coeff):
        # a_s^dag a_t on every basis state with t occupied and s empty
        sel = (occ(t) == 1) & (occ(s) == 0)
        src = idx[sel]
        lo, hi = min(s, t), max(s, t)
        between = np.zeros(src.shape, dtype=np.int64)
        for k in range(lo + 1, hi):
            between += (src >> (N - 1 - k)) & 1
        sign = 1.0 - 2.0 * (between & 1)
        rows.append(src ^ mask(s) ^ mask(t))
        cols.append(src)
        vals.append(coeff * sign)

    def diag(sites, coeff):
        v = np.full(dim, coeff, dtype=float)
        for s in sites:
            v *= 1.0 - 2.0 * occ(s)
        rows.append(idx)
        cols.append(idx)
        vals.append(v)

    for coeff, factors in terms:
        letters = [p for p, _ in factors]
        for x in range(Nx):
            for y in range(Ny):
                sites = [((x + o[0]) % Nx) * Ny + ((y + o[1]) % Ny) for _, o in factors]
                if letters == ["F", "F"]:
                    hop(sites[0], sites[1], coeff)
                    hop(sites[1], sites[0], coeff)
                elif all(p == "Z" for p in letters):
                    diag(sites, coeff)
                else:
                    raise ValueError("fermionic models take hoppings ('F', 'F') and density letters 'Z' only")
    for p, (x, y), coeff in fields:
        if p != "Z":
            raise ValueError("fermionic one-site fields are 'Z' (a potential on 1 - 2n)")
        diag([(x % Nx) * Ny + (y % Ny)], coeff)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(dim, dim))
    return H


def ground_state(terms, extent, fields=()):
    """(E_0, psi) over the whole Fock space (all particle numbers)."""
    H = full_hamiltonian_sparse(terms, extent, fields)
    if H.shape[0] <= 1024:
        w, V = np.linalg.eigh(H.toarray())
        return float(w[0]), V[:, 0]
    from scipy.sparse.linalg import eigsh

    w, V = eigsh(H, k=1, which="SA", tol=1e-13)
    return float(w[0]), V[:, 0]


def free_fermion_energy(terms, extent) -> float:
    """Ground-state energy of a hopping-only Hamiltonian: the sum of the negative eigenvalues of the
    one-particle hopping matrix (every mode below zero filled; no particle-number constraint)."""
    Nx, Ny = extent
    N = Nx * Ny
    h = np.zeros((N, N))
    for coeff, factors in terms:
        if [p for p, _ in factors] != ["F", "F"]:
            if coeff != 0.0:
                raise ValueError("free fermions: hopping terms only")
            continue
        for x in range(Nx):
            for y in range(Ny):
                s, t = [((x + o[0]) % Nx) * Ny + ((y + o[1]) % Ny) for _, o in factors]
                h[s, t] += coeff
                h[t, s] += coeff
    w = np.linalg.eigvalsh(h)
    return float(np.sum(w[w < 0]))


def global_annihilators(N: int):
    """Sparse JW images of a_0 .. a_{N-1} in the global site order."""
    import scipy.sparse as sp

    Zs = sp.diags([1.0, -1.0])
    Sm = sp.csr_matrix(SIGMA_MINUS)
    I2 = sp.identity(2, format="csr")
    out = []
    for k in range(N):
        op = sp.identity(1, format="csr")
        for s in range(N):
            op = sp.kron(op, Zs if s < k else (Sm if s == k else I2), format="csr")
        out.append(op)
    return out


def _sparse_unit_image(c, e, ops):
    import scipy.sparse as sp

    L = len(ops)
    dim = ops[0].shape[0]
    eye = sp.identity(dim, format="csr")
    num = [(a.T @ a).tocsr() for a in ops]
    out = eye
    for k in range(L):
        ck = (c >> (L - 1 - k)) & 1
        ek = (e >> (L - 1 - k)) & 1
        if ck == ek:
            f = num[k] if ck else eye - num[k]
        else:
            string = eye
            for j in range(k):
                string = string @ (eye - 2.0 * num[j])
            f = string @ (ops[k].T if ck else ops[k])
        out = out @ f
    return out


def marginal(psi, site_list, gops):
    """rho_S of |psi><psi| in the JWT of the ordered site list S: rho_uv = <psi| J(E_vu) |psi>,
    with E_vu mapped to the global JWT through the annihilators of the listed sites."""
    ops = [gops[s] for s in site_list]
    d = 2 ** len(site_list)
    rho = np.zeros((d, d))
    for u in range(d):
        for v in range(d):
            rho[u, v] = float(psi @ (_sparse_unit_image(v, u, ops) @ psi))
    return rho


def cluster_marginals(psi, extent, cluster):
    """rho_0 (cluster JWT) and rho_0d, d = 1..M-1 (pair JWT, cluster 0 first) of |psi><psi|."""
    g = Geometry(extent, cluster)
    gops = global_annihilators(extent[0] * extent[1])

    def sites_of(c):
        cx, cy = divmod(c, g.My)
        return [(cx * g.Lx + lx) * extent[1] + (cy * g.Ly + ly) for lx in range(g.Lx) for ly in range(g.Ly)]

    rho0 = marginal(psi, sites_of(0), gops)
    rhos = np.stack([marginal(psi, sites_of(0) + sites_of(d), gops) for d in range(1, g.M)])
    return rho0, rhos
