"""Smallest strictly positive eigenvalues of the compensated operator.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The kernel-compensation formulation asks for the first m smallest POSITIVE eigenvalues of
A M A^H + gamma B^H B (eq (2.13)).  For k != 0 the operator is HPD (Prop 2.5 (1)); for k = 0
it has exactly the three constant fields as null space, which are removed here.  Dense LAPACK
(eigvalsh) serves small n; larger n use shift-invert Lanczos (ARPACK via scipy eigsh) about
sigma = -1, so that the factored matrix Op + I is HPD even at k = 0.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import kspace, yee


def op_norm_bound(Op) -> float:
    """Max absolute row sum: an upper bound of the 2-norm of a Hermitian matrix."""
    return float(np.abs(Op).sum(axis=1).max())


def smallest_positive(Op, m: int, method: str = "auto", return_vectors: bool = False,
                      zero_rel: float = 1e-10):
    """m smallest eigenvalues of Op that are larger than zero_rel*||Op|| (ascending)."""
    n = Op.shape[0]
    extra = 3  # at most three zero modes (Prop 2.5 (1))
    want = min(m + extra, n)
    if method == "auto":
        method = "dense" if n <= 3 * 12 ** 3 else "shift_invert"
    if method == "dense":
        Ad = Op.toarray()
        if return_vectors:
            w, V = sla.eigh(Ad, subset_by_index=[0, want - 1])
        else:
            w = sla.eigh(Ad, subset_by_index=[0, want - 1], eigvals_only=True)
            V = None
    elif method == "shift_invert":
        w, V = spla.eigsh(Op.tocsc(), k=want, sigma=-1.0, which="LM", tol=1e-14,
                          return_eigenvectors=True)
        order = np.argsort(w)
        w, V = w[order], V[:, order]
    else:
        raise ValueError(method)
    thr = zero_rel * op_norm_bound(Op)
    keep = w > thr
    w = w[keep][:m]
    if return_vectors:
        return w, V[:, keep][:, :m]
    return w


def all_eigenvalues(Op) -> np.ndarray:
    """Whole spectrum by dense LAPACK (brute force for tiny grids)."""
    return np.linalg.eigvalsh(Op.toarray())


def smallest_positive_matfree(N: int, k, ids: np.ndarray, table: np.ndarray, scheme: str, m: int,
                              gamma: float | None = None, stencil_m: int = 1, sigma: float = -1.0,
                              cg_rtol: float = 1e-12, arpack_tol: float = 1e-10,
                              return_vectors: bool = False, lattice=None):
    """m smallest strictly positive eigenvalues of Op = A M A^H + gamma B^H B (eq (2.13)) for
    grids too large to factor: shift-invert Lanczos (ARPACK) about sigma = -1, the inner solves
    of (Op - sigma I) y = b by conjugate gradients on the product of the sparse factors A, M, B
    (eqs (2.7), (3.3)-(3.8)); a Rayleigh-Ritz step with Op on the returned vectors gives the
    final values.  CG is preconditioned per frequency by the inverse of
    c K_A K_A^H + gamma K_B + |sigma| I (eq (2.31) with the curl part scaled by the mean diagonal
    inverse permittivity c), which changes the speed of the inner solves, not their solution."""
    if gamma is None:
        gamma = yee.gamma_rule(k)
    A = yee.curl_matrix(N, k, stencil_m, lattice)
    AH = A.conj().T.tocsr()
    B = yee.div_matrix(N, k, stencil_m, lattice)
    BH = B.conj().T.tocsr()
    Mx = yee.eps_matrix(N, ids, table, scheme)
    n = 3 * N ** 3

    def op(x):
        return A @ (Mx @ (AH @ x)) + gamma * (BH @ (B @ x))

    # curl part scaled by the mean diagonal inverse permittivity over the edge points
    P = yee.point_tensors(ids, table)
    c = float(np.mean([P[a][:, a, a].real.mean() for a in range(3)]))
    K = kspace.symbols_3d(N, k, stencil_m, lattice)
    KA = kspace.curl_symbol(K)
    KP = c * (KA @ KA.conj().transpose(0, 2, 1)) + gamma * kspace.div_symbol_gram(K) - sigma * np.eye(3)[None]
    KPinv = np.linalg.inv(KP)                                  # (N^3, 3, 3)

    def prec(v):
        xk = kspace.F3H(np.asarray(v, dtype=np.complex128).reshape(1, 3, N ** 3), N)[0]
        zk = np.einsum("pab,bp->ap", KPinv, xk)
        return kspace.F3(zk[None], N)[0].reshape(n)

    Lop = spla.LinearOperator((n, n), matvec=lambda v: op(v) - sigma * v, dtype=np.complex128)
    Pop = spla.LinearOperator((n, n), matvec=prec, dtype=np.complex128)

    def solve(b):
        y, info = spla.cg(Lop, b, rtol=cg_rtol, atol=0.0, M=Pop, maxiter=5000)
        if info != 0:
            raise RuntimeError("inner CG did not converge (info=%d)" % info)
        return y

    want = m + 3 + 2
    OPinv = spla.LinearOperator((n, n), matvec=solve, dtype=np.complex128)
    Aop = spla.LinearOperator((n, n), matvec=op, dtype=np.complex128)
    _, V = spla.eigsh(Aop, k=want, sigma=sigma, which="LM", OPinv=OPinv, tol=arpack_tol,
                      ncv=min(n, max(4 * want, 24)))
    # Rayleigh-Ritz with Op on the Lanczos vectors (orthonormalised)
    Q, _ = np.linalg.qr(V)
    OQ = np.stack([op(Q[:, j]) for j in range(Q.shape[1])], axis=1)
    G = Q.conj().T @ OQ
    w, C = np.linalg.eigh(0.5 * (G + G.conj().T))
    thr = 1e-10 * max(1.0, float(np.abs(w).max()))
    keep = np.nonzero(w > thr)[0][:m]
    if return_vectors:
        X = Q @ C[:, keep]
        R = np.stack([op(X[:, j]) - w[j_] * X[:, j] for j, j_ in enumerate(keep)], axis=1)
        return w[keep], X, np.linalg.norm(R, axis=0)
    return w[keep]
