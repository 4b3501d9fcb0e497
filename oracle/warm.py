"""FP64 reference of the learned warm start's state encoding (test infrastructure).

A converged state of Algorithm 6 on a ring of M clusters is summarised by a
fixed-size vector that does not depend on M, and any such vector is turned back
into a valid starting state for a ring of any M.

Offsets d = 1..M-1 are read as a direction and a distance: d <= M/2 is direction
'+' at distance r = d, otherwise direction '-' at distance r = M - d.  Distances
1..near have blocks of their own; every distance > near shares one 'far' block.
Per (direction, slot):
    X_0d (n_op x n_op), Lambda_d (n x n), Lambda1_d (m x m), Lambda2_d (m x m), rho~_d (n x n).
The vector is [X_00, rho_0, then for direction '+', '-': slots r = 1..near, far],
each matrix row-major.  With near >= M/2 the encoding is exact (no far offsets);
a smaller `near` gives a vector independent of M at the price of averaging.

Encoding (M >= near + 1) takes the blocks at d = r (direction '+') and d = M - r
(direction '-') and, for the far slot, the mean over the distances near+1..M/2
(zeros when there are none).

Decoding assigns each offset its slot's blocks and makes the state valid:
  * X_00 symmetrised; X_0d and X_0,M-d made transposes of each other (X symmetric),
    then X is projected onto the PSD cone through its momentum blocks (Section 3.3),
    so the Lagrangian bound of the decoded point is a valid lower bound;
  * rho_0 symmetrised and shifted along the identity to unit trace;
  * rho~_d, Lambda_d, Lambda1_d, Lambda2_d symmetrised;  rho_d = rho~_d;  t = 0.

Pins (tests/test_oracle_warm.py): decode(encode(s)) = s for a solver state, both with
near = M/2 and with near = 3 on a ring whose only far offset is d = M/2 (M = 8); invariants of decoded random vectors (X PSD,
unit trace of rho_0, symmetry); the bound at a decoded random point lies below the
Jordan-Wigner ground-state energy.
"""
from __future__ import annotations

import numpy as np

from .alg6 import Problem, State, project_X

NEAR = 3  # default number of distances with blocks of their own


def sizes(p: Problem, near: int = NEAR):
    n_op, n, m = p.n_op, p.n, p.m
    block = n_op * n_op + 2 * n * n + 2 * m * m
    return n_op * n_op + m * m + 2 * (near + 1) * block, block


def slot_of(d: int, M: int, near: int = NEAR):
    """(direction 0 for '+' / 1 for '-', slot 0..near) of offset d; slot `near` is 'far'."""
    if 2 * d <= M:
        direction, r = 0, d
    else:
        direction, r = 1, M - d
    return direction, min(r, near + 1) - 1


def _block_views(p: Problem, vec, near):
    n_op, n, m = p.n_op, p.n, p.m
    X00 = vec[:n_op * n_op].reshape(n_op, n_op)
    o = n_op * n_op
    rho0 = vec[o:o + m * m].reshape(m, m)
    o += m * m
    blocks = []
    for _ in range(2 * (near + 1)):
        parts = []
        for shape in ((n_op, n_op), (n, n), (m, m), (m, m), (n, n)):
            k = shape[0] * shape[1]
            parts.append(vec[o:o + k].reshape(shape))
            o += k
        blocks.append(parts)
    return X00, rho0, blocks


def encode(p: Problem, s: State, near: int = NEAR) -> np.ndarray:
    if p.My != 1:
        raise ValueError("the warm-start encoding covers rings (one-dimensional cluster lattices)")
    if near < 1 or p.M < near + 1:
        raise ValueError(f"encoding with {near} near distances needs M >= {near + 1} clusters")
    total, _ = sizes(p, near)
    vec = np.zeros(total)
    X00, rho0, blocks = _block_views(p, vec, near)
    S = near + 1
    X00[...] = s.X[0]
    rho0[...] = s.rho0
    M = p.M

    def grab(d):
        return (s.X[d], s.Lam[d - 1], s.Lam1[d - 1], s.Lam2[d - 1], s.rho_t[d - 1])

    for direction in (0, 1):
        for r in range(1, near + 1):
            d = r if direction == 0 else M - r
            for dst, src in zip(blocks[direction * S + r - 1], grab(d)):
                dst[...] = src
        far = range(near + 1, M // 2 + 1)
        if len(far):
            for k, dst in enumerate(blocks[direction * S + near]):
                dst[...] = np.mean([grab(r if direction == 0 else M - r)[k] for r in far], axis=0)
    return vec


def _sym(a):
    return 0.5 * (a + a.T)


def _unit_trace(a):
    k = a.shape[0]
    return a + (1.0 - np.trace(a)) / k * np.eye(k)


def decode(p: Problem, vec, near: int = NEAR, far_cold: bool = False) -> State:
    """State from a vector (the inverse of encode for near >= M/2).  far_cold: the offsets at distances
    above `near` take the cold start of Section 4 (X_0d = 0, multipliers 0, rho~_d = I/n) instead of
    the far slot."""
    if p.My != 1:
        raise ValueError("the warm-start encoding covers rings (one-dimensional cluster lattices)")
    if near < 1:
        raise ValueError("near must be >= 1")
    vec = np.asarray(vec, np.float64)
    X00, rho0, blocks = _block_views(p, vec, near)
    M, P = p.M, p.P
    raw = {}
    cold = (np.zeros((p.n_op, p.n_op)), np.zeros((p.n, p.n)), np.zeros((p.m, p.m)), np.zeros((p.m, p.m)),
            np.eye(p.n) / p.n)
    for d in range(1, M):
        direction, slot = slot_of(d, M, near)
        raw[d] = cold if (far_cold and slot == near) else blocks[direction * (near + 1) + slot]
    Xp = np.zeros((M, p.n_op, p.n_op))
    Xp[0] = _sym(X00)
    for d in range(1, M):
        Xp[d] = 0.5 * (raw[d][0] + raw[M - d][0].T)
    X, _ = project_X(p, Xp)
    Lam = np.stack([_sym(raw[d][1]) for d in range(1, M)]) if P else np.zeros((0, p.n, p.n))
    Lam1 = np.stack([_sym(raw[d][2]) for d in range(1, M)]) if P else np.zeros((0, p.m, p.m))
    Lam2 = np.stack([_sym(raw[d][3]) for d in range(1, M)]) if P else np.zeros((0, p.m, p.m))
    rho_t = np.stack([_sym(raw[d][4]) for d in range(1, M)]) if P else np.zeros((0, p.n, p.n))
    return State(0, X, _unit_trace(_sym(rho0)), rho_t.copy(), rho_t, Lam, Lam1, Lam2)
