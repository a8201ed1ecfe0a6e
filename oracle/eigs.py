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
