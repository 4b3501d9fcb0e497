"""Linear maps of the two-marginal SDP (oracle; test infrastructure only).

All arrays are float64 (or complex128 for momentum blocks).  Pair operators
act on (cluster 0) x (cluster d) with cluster 0 the first Kronecker factor, so
a pair index is ``(x, y) -> x * m + y``.

Operator collections (Section 2.2, definition of G):
* ``complete``: the m*m matrix units ``O_(a,b) = E_ab`` (index ``a*m + b``),
  orthonormal in the Hilbert-Schmidt inner product; they span all operators on
  a cluster, the choice used in the paper's experiments.
* ``pauli1``: ``sigma^alpha_s / sqrt(m)`` for every site s of the cluster and
  alpha in {x, z, xz} with ``sigma^xz = sigma^x sigma^z`` (a real multiple of
  sigma^y); real and Hilbert-Schmidt orthonormal, spanning single-site X, Y, Z.

Generic maps use the definitions directly; the ``complete`` fast forms are
index permutations pinned against the generic ones in the tests.
"""
from __future__ import annotations

import numpy as np

from .model import PAULI, site_operator


# ---------------------------------------------------------------------------
# Operator collections
# ---------------------------------------------------------------------------

def operator_collection(opset: str, L: int) -> np.ndarray:
    """(n_op, m, m) real array of the cluster operators O_alpha."""
    m = 2 ** L
    if opset == "complete":
        ops = np.zeros((m * m, m, m))
        for a in range(m):
            for b in range(m):
                ops[a * m + b, a, b] = 1.0
        return ops
    if opset == "pauli1":
        xz = (PAULI["X"] @ PAULI["Z"]).real
        singles = {"x": PAULI["X"].real, "z": PAULI["Z"].real, "xz": xz}
        ops = []
        for s in range(L):
            for key in ("x", "z", "xz"):
                out = np.ones((1, 1))
                for t in range(L):
                    out = np.kron(out, singles[key] if t == s else np.eye(2))
                ops.append(out / np.sqrt(m))
        return np.array(ops)
    raise ValueError(f"unknown operator collection {opset!r}")


# ---------------------------------------------------------------------------
# Partial traces (Section 3.1: A_1 = Tr_2, A_2 = Tr_1) and adjoints
# ---------------------------------------------------------------------------

def ptrace2(rho: np.ndarray, m: int) -> np.ndarray:
    """A_1[rho] = Tr_2 rho: (A_1 rho)_ab = sum_c rho_(a,c),(b,c).  Works on stacks."""
    r = rho.reshape(rho.shape[:-2] + (m, m, m, m))
    return np.einsum("...acbc->...ab", r)


def ptrace1(rho: np.ndarray, m: int) -> np.ndarray:
    """A_2[rho] = Tr_1 rho: (A_2 rho)_ab = sum_c rho_(c,a),(c,b).  Works on stacks."""
    r = rho.reshape(rho.shape[:-2] + (m, m, m, m))
    return np.einsum("...cacb->...ab", r)


def adj1(tau: np.ndarray, m: int) -> np.ndarray:
    """A_1^* tau = tau (x) I_m."""
    return np.kron(tau, np.eye(m)) if tau.ndim == 2 else np.stack([np.kron(t, np.eye(m)) for t in tau])


def adj2(tau: np.ndarray, m: int) -> np.ndarray:
    """A_2^* tau = I_m (x) tau."""
    return np.kron(np.eye(m), tau) if tau.ndim == 2 else np.stack([np.kron(np.eye(m), t) for t in tau])


# ---------------------------------------------------------------------------
# Global-matrix blocks G (Section 2.2) and effective Hamiltonians (eq. effHam)
# ---------------------------------------------------------------------------

def G0_generic(rho0, ops):
    """(G_00)_ab = Tr[O_a^T O_b rho_0] (real operators: dagger = transpose)."""
    return np.einsum("aij,bjk,ki->ab", ops.transpose(0, 2, 1), ops, rho0)


def Gd_generic(rho, ops):
    """(G_0d)_ab = Tr[(O_a^T (x) O_b) rho_0d]."""
    n_op, m, _ = ops.shape
    r = rho.reshape(m, m, m, m)  # rho_(x,y),(x',y') -> r[x, y, x', y']
    # Tr[(A (x) B) rho] = sum A_{x x'} B_{y y'} rho_(x',y'),(x,y)
    return np.einsum("aij,bkl,jlik->ab", ops.transpose(0, 2, 1), ops, r)


def C0_generic(X0, ops):
    """sum_ab X0_ab O_a^T O_b, the correction in H_i[X_ii] (eq. effHam)."""
    return np.einsum("ab,aij,bjk->ik", X0, ops.transpose(0, 2, 1), ops)


def Rd_generic(Xd, ops):
    """sum_ab Xd_ab (O_a^T (x) O_b), the correction in H_ij[X_ij] before adding h.c. (eq. effHam)."""
    n_op, m, _ = ops.shape
    R = np.einsum("ab,aij,bkl->ikjl", Xd, ops.transpose(0, 2, 1), ops)
    return R.reshape(m * m, m * m)


def G0_complete(rho0, m):
    """Matrix units: (G_00)_(a,b),(c,e) = Tr[E_ba E_ce rho_0] = delta_ac rho0_eb."""
    return np.einsum("ac,eb->abce", np.eye(m), rho0).reshape(m * m, m * m)


def Gd_complete(rho, m):
    """Matrix units: (G_0d)_(a,b),(c,e) = Tr[(E_ba (x) E_ce) rho] = rho_(a,e),(b,c) (a realignment)."""
    r = rho.reshape(rho.shape[:-2] + (m, m, m, m))  # axes [a, e, b, c]
    nd = r.ndim
    perm = tuple(range(nd - 4)) + (nd - 4, nd - 2, nd - 1, nd - 3)
    return r.transpose(perm).reshape(rho.shape[:-2] + (m * m, m * m))


def C0_complete(X0, m):
    """Matrix units: sum X0_(a,b),(c,e) E_ba E_ce = sum_a X0_(a,b),(a,e) E_be."""
    return np.einsum("abae->be", X0.reshape(m, m, m, m))


def Rd_complete(Xd, m):
    """Matrix units: R_(x,y),(x',y') = Xd_(x',x),(y,y')."""
    X = Xd.reshape(Xd.shape[:-2] + (m, m, m, m))  # axes [x', x, y, y']
    nd = X.ndim
    perm = tuple(range(nd - 4)) + (nd - 3, nd - 2, nd - 4, nd - 1)
    return X.transpose(perm).reshape(Xd.shape[:-2] + (m * m, m * m))


class OperatorMaps:
    """G blocks and effective-Hamiltonian corrections for one operator collection.  fermionic:
    the off-diagonal blocks carry the Jordan-Wigner parity signs of the appendix on fermions
    (complete collection only; see ``oracle.fermion``)."""

    def __init__(self, opset: str, L: int, fermionic: bool = False):
        self.opset = opset
        self.L = L
        self.m = 2 ** L
        self.ops = operator_collection(opset, L)
        self.n_op = self.ops.shape[0]
        self.fermionic = bool(fermionic)
        if self.fermionic and opset != "complete":
            raise ValueError("fermionic problems use the complete operator collection")

    def G0(self, rho0):
        return G0_complete(rho0, self.m) if self.opset == "complete" else G0_generic(rho0, self.ops)

    def Gd(self, rho):
        if self.fermionic:
            from .fermion import Gd_complete as fermion_gd

            return fermion_gd(rho, self.m)
        if self.opset == "complete":
            return Gd_complete(rho, self.m)
        if rho.ndim == 2:
            return Gd_generic(rho, self.ops)
        return np.stack([Gd_generic(r, self.ops) for r in rho])

    def C0(self, X0):
        return C0_complete(X0, self.m) if self.opset == "complete" else C0_generic(X0, self.ops)

    def Rd(self, Xd):
        if self.fermionic:
            from .fermion import Rd_complete as fermion_rd

            return fermion_rd(Xd, self.m)
        if self.opset == "complete":
            return Rd_complete(Xd, self.m)
        if Xd.ndim == 2:
            return Rd_generic(Xd, self.ops)
        return np.stack([Rd_generic(x, self.ops) for x in Xd])


# ---------------------------------------------------------------------------
# Closed-form solution of the pair system (eq. rhoijUpdate)
# ---------------------------------------------------------------------------

def pair_solve(R, m, mu, nu):
    """(mu + nu A_1^*A_1 + nu A_2^*A_2)^{-1} R in closed form.

    T_1 = A_1^*A_1/m and T_2 = A_2^*A_2/m are commuting orthogonal projectors
    with T_1 T_2 R = Tr(R) I/m^2, so the inverse is a Id + b (T_1+T_2) + c T_1T_2
    with a = 1/mu, b = 1/(mu+nu m) - 1/mu, c = 1/(mu+2 nu m) - 2/(mu+nu m) + 1/mu.
    Pinned against the dense superoperator inverse in the tests.
    """
    a = 1.0 / mu
    b = 1.0 / (mu + nu * m) - 1.0 / mu
    c = 1.0 / (mu + 2 * nu * m) - 2.0 / (mu + nu * m) + 1.0 / mu
    n = m * m
    t2 = ptrace2(R, m)  # Tr_2 R
    t1 = ptrace1(R, m)  # Tr_1 R
    tr = np.trace(R, axis1=-2, axis2=-1)
    out = a * R + (b / m) * (adj1(t2, m) + adj2(t1, m))
    out = out + (c / (m * m)) * tr[..., None, None] * np.eye(n)
    return out


def pair_superoperator(m, mu, nu):
    """Dense (n*n x n*n) matrix of mu + nu A_1^*A_1 + nu A_2^*A_2 acting on vec(rho) (row-major)."""
    n = m * m
    S = np.zeros((n * n, n * n))
    for k in range(n * n):
        E = np.zeros((n, n))
        E.flat[k] = 1.0
        img = mu * E + nu * adj1(ptrace2(E, m), m) + nu * adj2(ptrace1(E, m), m)
        S[:, k] = img.ravel()
    return S


# ---------------------------------------------------------------------------
# Projection onto the PSD cone (Section 3, definition of Pi)
# ---------------------------------------------------------------------------

def _eigh(A, vectors=True):
    """Eigendecomposition of stacked symmetric / Hermitian matrices by LAPACK.  numpy's driver
    (divide and conquer) can stop with "did not converge" on rare finite matrices; those matrices are
    then decomposed one by one by the implicit QL/QR driver of the same library (same definition)."""
    try:
        return np.linalg.eigh(A) if vectors else (np.linalg.eigvalsh(A), None)
    except np.linalg.LinAlgError:
        import scipy.linalg

        flat = A.reshape((-1,) + A.shape[-2:])
        ws, Vs = [], []
        for M in flat:
            if vectors:
                w, V = scipy.linalg.eigh(M, driver="ev")
                Vs.append(V)
            else:
                w = scipy.linalg.eigh(M, driver="ev", eigvals_only=True)
            ws.append(w)
        w = np.stack(ws).reshape(A.shape[:-1])
        return (w, np.stack(Vs).reshape(A.shape)) if vectors else (w, None)


def psd_project(C):
    """argmin_{S >= 0} ||S - C||_F for symmetric / Hermitian C (stacked): clip negative eigenvalues."""
    Ch = 0.5 * (C + np.conj(np.swapaxes(C, -1, -2)))
    w, V = _eigh(Ch)
    wp = np.maximum(w, 0.0)
    P = (V * wp[..., None, :]) @ np.conj(np.swapaxes(V, -1, -2))
    return 0.5 * (P + np.conj(np.swapaxes(P, -1, -2)))


def lambda_min(A):
    """Smallest eigenvalue of a symmetric / Hermitian matrix (stacked)."""
    Ah = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    return _eigh(Ah, vectors=False)[0][..., 0]
