"""Lattice, clusters and local Hamiltonians (oracle; test infrastructure only).

Conventions
-----------
* Periodic lattice ``Nx x Ny`` (``Ny = 1`` for a ring), tiled exactly by
  rectangular clusters ``Lx x Ly`` (Section 2.3: clusters used as supersites).
  Cluster grid ``Mx x My``, ``M = Mx*My``, ``L = Lx*Ly`` sites per cluster,
  ``m = 2**L`` states per cluster, pair dimension ``n = m*m``.
* Site ``(x, y)`` lies in cluster ``(x // Lx, y // Ly)``; its local index is
  ``(x % Lx) * Ly + (y % Ly)``; flat cluster index ``cx * My + cy``.
* Kronecker order: local site 0 is the most significant tensor factor; in a
  pair (0, d) cluster 0 is the first factor.
* H_0 holds every term instance whose sites all lie in cluster 0.  H_{0,d}
  holds every term instance with one site in cluster 0 and the other in
  cluster d, written on (cluster 0) x (cluster d).  With translation
  invariance (Section 3.3) the energy per cluster is
  ``Tr(H_0 rho_0) + 1/2 sum_{d != 0} Tr(H_{0,d} rho_{0,d})``.
"""
from __future__ import annotations

import numpy as np

PAULI = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


class Geometry:
    """Cluster tiling of a periodic lattice (Section 2.3, Section 3.3)."""

    def __init__(self, extent, cluster):
        Nx, Ny = extent
        Lx, Ly = cluster
        if Nx % Lx or Ny % Ly:
            raise ValueError("clusters must tile the lattice exactly")
        self.Nx, self.Ny, self.Lx, self.Ly = Nx, Ny, Lx, Ly
        self.Mx, self.My = Nx // Lx, Ny // Ly
        self.M = self.Mx * self.My
        self.L = Lx * Ly
        self.m = 2 ** self.L
        self.n = self.m * self.m
        if self.M < 2:
            raise ValueError("at least two clusters are required")

    def locate(self, x, y):
        x %= self.Nx
        y %= self.Ny
        c = (x // self.Lx) * self.My + (y // self.Ly)
        loc = (x % self.Lx) * self.Ly + (y % self.Ly)
        return c, loc

    def cluster_coords(self, c):
        return divmod(c, self.My)


def site_operator(letters_at: dict, L: int) -> np.ndarray:
    """Kronecker product over L sites with the given Pauli letters (identity elsewhere)."""
    out = np.ones((1, 1), dtype=complex)
    for s in range(L):
        out = np.kron(out, PAULI[letters_at.get(s, "I")])
    return out


def local_hamiltonians(terms, geom: Geometry):
    """H_0 (m x m) and H_{0,d} for d = 1..M-1 ((M-1) x n x n), real float64.

    Each term is translated to every lattice site; term instances touching
    cluster 0 are kept, as described in the module header.
    """
    L, m, n, M = geom.L, geom.m, geom.n, geom.M
    H0 = np.zeros((m, m), dtype=complex)
    Hd = np.zeros((M, n, n), dtype=complex)  # index 0 unused
    for coeff, factors in terms:
        if len(factors) > 2:
            raise ValueError("only one- and two-site terms are pairwise")
        for x in range(geom.Nx):
            for y in range(geom.Ny):
                placed = [(p, geom.locate(x + o[0], y + o[1])) for p, o in factors]
                clusters = [c for _, (c, _) in placed]
                if len(placed) == 2 and placed[0][1] == placed[1][1]:
                    raise ValueError("a two-site term folds onto one site on this lattice")
                if 0 not in clusters:
                    continue
                if all(c == 0 for c in clusters):
                    op = np.eye(m, dtype=complex)
                    for p, (_, loc) in placed:
                        op = op @ site_operator({loc: p}, L)
                    H0 += coeff * op
                else:
                    # one factor in cluster 0, the other in cluster d != 0
                    (p0, (c0, l0)), (p1, (c1, l1)) = placed
                    if c0 != 0:
                        (p0, (c0, l0)), (p1, (c1, l1)) = (p1, (c1, l1)), (p0, (c0, l0))
                    d = c1
                    Hd[d] += coeff * np.kron(site_operator({l0: p0}, L), site_operator({l1: p1}, L))
    if np.abs(H0.imag).max() > 1e-14 or np.abs(Hd.imag).max() > 1e-14:
        raise ValueError("complex Hamiltonian terms are not supported (real case of Section 3)")
    return H0.real.copy(), Hd[1:].real.copy()


def full_hamiltonian_sparse(terms, extent, fields=()):
    """Sparse 2^N x 2^N Hamiltonian on the whole lattice (for exact diagonalisation pins).

    Site ordering: flat site index ``x * Ny + y``, site 0 the most significant bit.
    ``fields``: extra one-site terms (letter, (x, y), coeff) at single sites (not
    translated), for Hamiltonians without translation invariance.
    """
    import scipy.sparse as sp

    Nx, Ny = extent
    N = Nx * Ny
    dim = 2 ** N
    idx = np.arange(dim, dtype=np.int64)

    def bit(s):
        return (idx >> (N - 1 - s)) & 1

    H = sp.csr_matrix((dim, dim), dtype=complex)
    for coeff, factors in terms:
        for x in range(Nx):
            for y in range(Ny):
                flip = np.zeros(dim, dtype=np.int64)
                phase = np.ones(dim, dtype=complex)
                for p, o in factors:
                    s = ((x + o[0]) % Nx) * Ny + ((y + o[1]) % Ny)
                    b = bit(s)
                    if p == "X":
                        flip ^= 1 << (N - 1 - s)
                    elif p == "Z":
                        phase *= 1 - 2 * b
                    elif p == "Y":
                        # Y|0> = i|1>, Y|1> = -i|0>: column index j, entry at row j^mask
                        flip ^= 1 << (N - 1 - s)
                        phase *= 1j * (1 - 2 * b)
                rows = idx ^ flip
                H = H + sp.csr_matrix((coeff * phase, (rows, idx)), shape=(dim, dim))
    for p, (x, y), coeff in fields:
        s = (x % Nx) * Ny + (y % Ny)
        b = bit(s)
        flip = np.zeros(dim, dtype=np.int64)
        phase = np.ones(dim, dtype=complex)
        if p == "X":
            flip ^= 1 << (N - 1 - s)
        elif p == "Z":
            phase = phase * (1 - 2 * b)
        else:
            raise ValueError("one-site fields are X or Z (real)")
        H = H + sp.csr_matrix((coeff * phase, (idx ^ flip, idx)), shape=(dim, dim))
    if abs(H.imag).max() > 1e-12:
        raise ValueError("complex Hamiltonian")
    return H.real.tocsr()
