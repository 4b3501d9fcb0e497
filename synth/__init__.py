"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module holds no arithmetic of the solver.  It only fixes *what* is solved:
model Hamiltonians as lists of real Pauli-string terms on a periodic lattice,
the workload configurations, the seeded parameter draws of the batched sweep
and the warm-start sets, and seeded random symmetric matrices that imitate
ADMM iterates for the isolated projection benchmark.  Random numbers that the
method itself would draw do not exist (the iteration is deterministic).

Term format (used by both sides)
--------------------------------
A term is ``(coeff, ((pauli, (ox, oy)), ...))``: a real coefficient times a
product of Pauli letters ``"X" | "Y" | "Z"`` placed at site offsets ``(ox, oy)``
relative to a lattice origin.  The Hamiltonian is the sum of every term
translated to every lattice site (periodic boundary conditions).

Fermionic models (spinless fermions, appendix on fermions) use the letter
``"F"``: a two-site term ``(t, (("F", o1), ("F", o2)))`` is the hopping
``t (a_i^dag a_j + a_j^dag a_i)`` between the sites at o1 and o2, and
``"Z"`` stands for 1 - 2 n (so (n_i - 1/2)(n_j - 1/2) = Z_i Z_j / 4).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

BASE_SEED = 210602682

Term = Tuple[float, Tuple[Tuple[str, Tuple[int, int]], ...]]


def tfi_terms(h: float, J: float = 1.0, ndim: int = 1) -> list:
    """Transverse-field Ising model: -h sum X_i - J sum_<ij> Z_i Z_j (Section 2.1, eq. TFI)."""
    terms = [(-float(h), (("X", (0, 0)),))]
    terms.append((-float(J), (("Z", (0, 0)), ("Z", (1, 0)))))
    if ndim == 2:
        terms.append((-float(J), (("Z", (0, 0)), ("Z", (0, 1)))))
    return terms


def xxz_terms(Jz: float, ndim: int = 1) -> list:
    """XXZ chain sum_<ij> (X_i X_j + Y_i Y_j + Jz Z_i Z_j); Jz = 1 is the AFH model (eq. AFH)."""
    bonds = [(1, 0)] + ([(0, 1)] if ndim == 2 else [])
    terms = []
    for b in bonds:
        terms.append((1.0, (("X", (0, 0)), ("X", b))))
        terms.append((1.0, (("Y", (0, 0)), ("Y", b))))
        terms.append((float(Jz), (("Z", (0, 0)), ("Z", b))))
    return terms


def afh_terms(ndim: int = 1) -> list:
    return xxz_terms(1.0, ndim)


def sf_terms(U: float, ndim: int = 1) -> list:
    """Spinless fermions (eq. spinlessFerm): sum over nearest-neighbour bonds of
    -(a_i^dag a_j + a_j^dag a_i) + U (n_i - 1/2)(n_j - 1/2)."""
    bonds = [(1, 0)] + ([(0, 1)] if ndim == 2 else [])
    terms = []
    for b in bonds:
        terms.append((-1.0, (("F", (0, 0)), ("F", b))))
        terms.append((0.25 * float(U), (("Z", (0, 0)), ("Z", b))))
    return terms


def lrsf_terms(U: float, N: int) -> list:
    """Long-range spinless fermions on a ring of N sites (eq. spinlessFermLR): nearest-neighbour
    hopping plus U sum over ordered pairs i != j of (n_i - 1/2)(n_j - 1/2) / d(i, j), d the
    periodic (minimum-image) distance.  Each unordered pair at distance r carries 2U/r; the term
    at offset r translated to every site meets each such pair once (twice for r = N/2, whose
    coefficient is halved)."""
    terms = [(-1.0, (("F", (0, 0)), ("F", (1, 0))))]
    for r in range(1, N // 2 + 1):
        c = 2.0 * float(U) / r * 0.25
        if 2 * r == N:
            c *= 0.5
        terms.append((c, (("Z", (0, 0)), ("Z", (r, 0)))))
    return terms


@dataclass(frozen=True)
class Workload:
    """One solver instance: model terms on an Nx x Ny torus tiled by Lx x Ly clusters."""

    name: str
    terms: tuple
    extent: Tuple[int, int]
    cluster: Tuple[int, int]
    opset: str = "complete"  # "complete" | "pauli1"
    iters: int = 2000
    mu: float = 10.0
    nu: float = 10.0
    eps: float = 2.0
    meta: dict = field(default_factory=dict, compare=False, hash=False)
    fermionic: bool = False  # "F" hopping terms; pair operators Jordan-Wigner ordered per cluster pair

    @property
    def ndim(self) -> int:
        return 1 if self.extent[1] == 1 else 2

    @property
    def L(self) -> int:
        return self.cluster[0] * self.cluster[1]

    @property
    def M(self) -> int:
        return (self.extent[0] // self.cluster[0]) * (self.extent[1] // self.cluster[1])

    @property
    def m(self) -> int:
        return 2 ** self.L

    @property
    def n(self) -> int:
        return self.m * self.m

    @property
    def n_op(self) -> int:
        return self.m * self.m if self.opset == "complete" else 3 * self.L


def tfi_ring(N: int, L: int, h: float, opset: str = "complete", iters: int = 2000, name=None) -> Workload:
    return Workload(name or f"tfi_ring_N{N}_L{L}_h{h}_{opset}", tuple(tfi_terms(h, 1.0, 1)),
                    (N, 1), (L, 1), opset, iters, meta={"model": "tfi", "h": h, "Jz": 0.0})


def xxz_ring(N: int, L: int, Jz: float, opset: str = "complete", iters: int = 2000, name=None) -> Workload:
    return Workload(name or f"xxz_ring_N{N}_L{L}_Jz{Jz}_{opset}", tuple(xxz_terms(Jz, 1)),
                    (N, 1), (L, 1), opset, iters, meta={"model": "xxz", "h": 0.0, "Jz": Jz})


def tfi_torus(Nx: int, Ny: int, Lx: int, Ly: int, h: float, iters: int = 2000, name=None) -> Workload:
    return Workload(name or f"tfi_torus_{Nx}x{Ny}_{Lx}x{Ly}_h{h}", tuple(tfi_terms(h, 1.0, 2)),
                    (Nx, Ny), (Lx, Ly), "complete", iters, meta={"model": "tfi", "h": h, "Jz": 0.0})


def sf_ring(N: int, L: int, U: float, iters: int = 2000, name=None, long_range: bool = False) -> Workload:
    """Spinless fermions (short- or long-range density interaction) on a ring of N sites."""
    terms = lrsf_terms(U, N) if long_range else sf_terms(U, 1)
    tag = "lrsf" if long_range else "sf"
    return Workload(name or f"{tag}_ring_N{N}_L{L}_U{U}", tuple(terms), (N, 1), (L, 1), "complete", iters,
                    meta={"model": tag, "U": U}, fermionic=True)


def sf_torus(Nx: int, Ny: int, Lx: int, Ly: int, U: float, iters: int = 2000, name=None) -> Workload:
    return Workload(name or f"sf_torus_{Nx}x{Ny}_{Lx}x{Ly}_U{U}", tuple(sf_terms(U, 2)), (Nx, Ny), (Lx, Ly),
                    "complete", iters, meta={"model": "sf", "U": U}, fermionic=True)


def afh_torus(Nx: int, Ny: int, Lx: int, Ly: int, iters: int = 2000, name=None) -> Workload:
    return Workload(name or f"afh_torus_{Nx}x{Ny}_{Lx}x{Ly}", tuple(afh_terms(2)),
                    (Nx, Ny), (Lx, Ly), "complete", iters, meta={"model": "xxz", "h": 0.0, "Jz": 1.0})


# ---------------------------------------------------------------------------
# Workload configurations (the paper's method at the shapes of the five configs)
# ---------------------------------------------------------------------------

def config_c1() -> list:
    """Ring N=8, J=1, h=1, 2000 iterations; four cluster choices (L=1 Pauli, L=1, 2, 4 complete)."""
    return [tfi_ring(8, 1, 1.0, "pauli1", 2000, "C1a"), tfi_ring(8, 1, 1.0, "complete", 2000, "C1b"),
            tfi_ring(8, 2, 1.0, "complete", 2000, "C1c"), tfi_ring(8, 4, 1.0, "complete", 2000, "C1d")]


def config_c2(h: float = 1.0) -> list:
    """Ring, J=1, h in {0.5, 1, 1.5}, 5000 iterations: N=128 with L=1 Pauli; N=384 with L=3."""
    return [tfi_ring(128, 1, h, "pauli1", 5000, f"C2a_h{h}"), tfi_ring(384, 3, h, "complete", 5000, f"C2b_h{h}")]


def config_c3() -> list:
    """16x16 torus, J=1, h=3: 2x1 clusters and 2x2 plaquettes."""
    return [tfi_torus(16, 16, 2, 1, 3.0, 2000, "C3a"), tfi_torus(16, 16, 2, 2, 3.0, 2000, "C3b")]


def draw_instance(rng: np.random.Generator) -> dict:
    """One batched-sweep draw; all five numbers are always drawn so streams stay aligned."""
    model = int(rng.integers(2))
    N = int(rng.integers(32, 513))
    L = int(rng.integers(2, 5))
    h = float(rng.uniform(0.2, 2.0))
    Jz = float(rng.uniform(0.0, 2.0))
    return {"model": "tfi" if model == 0 else "xxz", "N": N, "L": L, "h": h, "Jz": Jz}


def instance_workload(d: dict, iters: int = 5000, name: str = "") -> Workload:
    M = d["N"] // d["L"]
    N_eff = M * d["L"]
    if d["model"] == "tfi":
        terms = tfi_terms(d["h"], 1.0, 1)
    else:
        terms = xxz_terms(d["Jz"], 1)
    return Workload(name or f"{d['model']}_N{N_eff}_L{d['L']}", tuple(terms), (N_eff, 1), (d["L"], 1),
                    "complete", iters, meta=dict(d, N_eff=N_eff))


def c4_instances(count: int = 64) -> list:
    return [draw_instance(np.random.default_rng([BASE_SEED, 4, i])) for i in range(count)]


def c5_train_instances(count: int = 4096) -> list:
    return [draw_instance(np.random.default_rng([BASE_SEED, 5, 0, i])) for i in range(count)]


def c5_heldout_instances(count: int = 512) -> list:
    return [draw_instance(np.random.default_rng([BASE_SEED, 5, 1, j])) for j in range(count)]


# ---------------------------------------------------------------------------
# Random symmetric inputs shaped like ADMM iterates (isolated projection benchmark)
# ---------------------------------------------------------------------------

def admm_like_batch(n: int, batch: int, mu: float = 10.0, tag: int = 0) -> np.ndarray:
    """(batch, n, n) float64: W/Tr W - S/mu with W = G G^T, S = (Z + Z^T)/(2 sqrt n).

    Roughly half of the eigenvalues come out negative, like rho - Lambda/mu.
    """
    rng = np.random.default_rng([BASE_SEED, tag, n, batch])
    G = rng.standard_normal((batch, n, n))
    W = G @ np.swapaxes(G, 1, 2)
    tr = np.trace(W, axis1=1, axis2=2)[:, None, None]
    Z = rng.standard_normal((batch, n, n))
    S = (Z + np.swapaxes(Z, 1, 2)) / (2.0 * np.sqrt(n))
    return W / tr - S / mu


def hermitian_batch(n: int, batch: int, tag: int = 1) -> np.ndarray:
    """(batch, n, n) complex128 Hermitian matrices with a spread of signed eigenvalues."""
    rng = np.random.default_rng([BASE_SEED, tag, n, batch, 7])
    A = rng.standard_normal((batch, n, n)) + 1j * rng.standard_normal((batch, n, n))
    return (A + np.conj(np.swapaxes(A, 1, 2))) / (2.0 * np.sqrt(n))


# ---------------------------------------------------------------------------
# Learned warm start: seeded initial network parameters and input features
# ---------------------------------------------------------------------------

def family_draws(count: int, N: int, L: int, split: int = 0) -> list:
    """Draws of the learned-start recipe (model, h, J_z from the same streams as the
    training / held-out draws) on one ring: N sites in clusters of L (a parameter sweep)."""
    out = []
    for i in range(count):
        d = draw_instance(np.random.default_rng([BASE_SEED, 5, split, i]))
        d["N"], d["L"] = N, L
        out.append(d)
    return out


def cross_draws(count: int, split: int = 0, Ls=(2, 3)) -> list:
    """Draws of the learned start's cross-size family: model, N ~ U{32..512}, h, J_z from the training
    (split 0) / held-out (split 1) streams as in the batched sweep, clusters of L sites alternating over
    Ls (one network for every ring size and cluster size, k = 2L an input)."""
    out = []
    for i in range(count):
        d = draw_instance(np.random.default_rng([BASE_SEED, 5, split, i]))
        d["L"] = Ls[i % len(Ls)]
        out.append(d)
    return out


def mlp_init(dims, tag: int = 0) -> np.ndarray:
    """Initial parameters, flat FP32 in the layout W_0 (out x in, row-major), b_0, W_1, b_1, ...
    drawn uniform in +-1/sqrt(fan_in) from a seeded stream."""
    rng = np.random.default_rng([BASE_SEED, 13, tag])
    parts = []
    for l in range(len(dims) - 1):
        k = 1.0 / np.sqrt(dims[l])
        parts.append(rng.uniform(-k, k, size=dims[l + 1] * dims[l]))
        parts.append(rng.uniform(-k, k, size=dims[l + 1]))
    return np.concatenate(parts).astype(np.float32)


def mlp_features(d: dict) -> np.ndarray:
    """Network input of one instance draw, a fixed featurisation of (model, h, J_z, k = 2L):
    one-hot model, the model's parameter p (h for TFI, J_z for XXZ), p^2, |p - 1|,
    tanh(4 (p - 1)) (both models change phase at p = 1) and k / 8."""
    tfi = d["model"] == "tfi"
    p = d["h"] if tfi else d["Jz"]
    return np.array([1.0 if tfi else 0.0, 0.0 if tfi else 1.0, p, p * p, abs(p - 1.0), np.tanh(4.0 * (p - 1.0)),
                     2 * d["L"] / 8.0], dtype=np.float32)


N_FEATURES = 7


def mlp_batch(n_in: int, batch: int, tag: int = 0) -> np.ndarray:
    """Seeded FP32 inputs for network parity tests."""
    return np.random.default_rng([BASE_SEED, 14, tag]).standard_normal((batch, n_in)).astype(np.float32)


def disorder_fields(w: Workload, scale: float, letters=("X",), tag: int = 0) -> list:
    """Random one-site fields (letter, (x, y), coeff) with coeff ~ U[-scale, scale] on every site
    of the workload's lattice, one per letter: the disordered instances of the dense solver."""
    rng = np.random.default_rng([BASE_SEED, 29, tag])
    return [(letter, (x, y), float(scale * rng.uniform(-1.0, 1.0)))
            for x in range(w.extent[0]) for y in range(w.extent[1]) for letter in letters]


def dense_bench() -> tuple:
    """Dense (non-invariant) benchmark instance: TFI ring N = 32, J = 1, h = 1, 2-site clusters
    (M = 16, 120 pair marginals 16 x 16, dense X 256 x 256), random transverse fields
    U[-0.5, 0.5] added site by site."""
    w = tfi_ring(32, 2, 1.0, "complete", 2000, "dense_ring32_L2")
    return w, disorder_fields(w, 0.5, ("X",), tag=1)
