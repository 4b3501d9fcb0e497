"""Exact references for the pins (oracle; test infrastructure only).

* Exact diagonalisation of the full lattice Hamiltonian (eq. groundstate).
* The Jordan-Wigner free-fermion ground-state energy of the periodic
  transverse-field Ising ring (eq. TFI with J = 1).
* Cluster marginals of a state vector by partial trace (Section 2.2), used to
  check that the local Hamiltonians and the energy formula reproduce E_0.
"""
from __future__ import annotations

import numpy as np

from .model import full_hamiltonian_sparse


def ground_state(terms, extent, fields=()):
    """(E_0, psi) of the full Hamiltonian by sparse Lanczos (dense eigh for tiny sizes)."""
    H = full_hamiltonian_sparse(terms, extent, fields)
    dim = H.shape[0]
    if dim <= 256:
        w, V = np.linalg.eigh(H.toarray())
        return float(w[0]), V[:, 0]
    from scipy.sparse.linalg import eigsh

    w, V = eigsh(H, k=1, which="SA", tol=1e-13)
    return float(w[0]), V[:, 0]


def tfi_ring_energy_jw(N: int, h: float) -> float:
    """E_0/N of -h sum X - sum Z Z on a periodic ring of N sites (J = 1).

    The ground state lies in the even-parity sector, whose fermion modes obey
    antiperiodic boundary conditions: k = pi (2j+1)/N, with single-mode energy
    2 sqrt(1 + h^2 - 2 h cos k); E_0 = -1/2 sum_k of it.
    """
    k = np.pi * (2 * np.arange(N) + 1) / N
    return float(-np.sum(np.sqrt(1.0 + h * h - 2.0 * h * np.cos(k))) / N)


def cluster_marginals(psi, extent, cluster):
    """rho_0 and rho_{0,d} (d = 1..M-1) of |psi><psi| in the oracle's basis conventions."""
    Nx, Ny = extent
    Lx, Ly = cluster
    N = Nx * Ny
    My = Ny // Ly
    M = (Nx // Lx) * My

    def sites_of(c):
        cx, cy = divmod(c, My)
        out = []
        for lx in range(Lx):
            for ly in range(Ly):
                x, y = cx * Lx + lx, cy * Ly + ly
                out.append(x * Ny + y)  # flat site index used by full_hamiltonian_sparse
        return out  # local index order lx*Ly + ly

    T = psi.reshape((2,) * N)

    def reduced(site_list):
        rest = [s for s in range(N) if s not in site_list]
        A = np.transpose(T, site_list + rest).reshape(2 ** len(site_list), -1)
        return A @ A.conj().T

    rho0 = reduced(sites_of(0)).real
    rhos = np.stack([reduced(sites_of(0) + sites_of(d)).real for d in range(1, M)])
    return rho0, rhos


def all_marginals(psi, extent, cluster):
    """rho_i for every cluster and rho_ij for every pair i < j of |psi><psi| (dense Algorithm 5 layout)."""
    Nx, Ny = extent
    Lx, Ly = cluster
    N = Nx * Ny
    My = Ny // Ly
    M = (Nx // Lx) * My

    def sites_of(c):
        cx, cy = divmod(c, My)
        return [(cx * Lx + lx) * Ny + (cy * Ly + ly) for lx in range(Lx) for ly in range(Ly)]

    T = psi.reshape((2,) * N)

    def reduced(site_list):
        rest = [s for s in range(N) if s not in site_list]
        A = np.transpose(T, site_list + rest).reshape(2 ** len(site_list), -1)
        return (A @ A.conj().T).real

    rho = {i: reduced(sites_of(i)) for i in range(M)}
    pairs = {(i, j): reduced(sites_of(i) + sites_of(j)) for i in range(M) for j in range(i + 1, M)}
    return rho, pairs
