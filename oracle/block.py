"""Dense block steps of the LOBPCG iteration (Section 4, the block eigensolver, and the
convergence test of eq (4.3)) written out from their definitions, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A block is a complex128 array of shape (nb, nc, n): k-point b, column j, entry r.
"""
from __future__ import annotations

import numpy as np


def gram(S: np.ndarray, AS: np.ndarray):
    """Gram matrices of the search space: GA_b = S_b^H AS_b, GB_b = S_b^H S_b, entry (i, j) the
    inner product of column i of S_b with column j of AS_b (resp. S_b)."""
    Sc = np.conj(S)
    GA = np.matmul(Sc, np.transpose(AS, (0, 2, 1)))
    GB = np.matmul(Sc, np.transpose(S, (0, 2, 1)))
    return GA, GB


def update(S: np.ndarray, AS: np.ndarray, C: np.ndarray, theta: np.ndarray):
    """One Rayleigh-Ritz update: with S_b = [X W P], AS_b = [AX AW AP] (3mb columns each) and
    C_b = [C1 | Cp] (3mb x 2mb), the new X = S_b C1, P = S_b Cp and their images AX = AS_b C1,
    AP = AS_b Cp take the places of X and P (W, AW unchanged); then the residuals
    R_j = AX_j - theta_j X_j, Res_j = |R_j| / |X_j| (eq (4.3); 0 for a zero column) and |X_j|^2.
    Returns (S_new, AS_new, R, res, xnorm2)."""
    nb, nc, n = S.shape
    mb = nc // 3
    # Y_b = (S_b^T C_b)^T: output column q is sum_c C_b[c, q] S_b[c, :]
    Y = np.matmul(np.transpose(C, (0, 2, 1)), S)
    AY = np.matmul(np.transpose(C, (0, 2, 1)), AS)
    S_new, AS_new = S.copy(), AS.copy()
    S_new[:, :mb], S_new[:, 2 * mb:] = Y[:, :mb], Y[:, mb:]
    AS_new[:, :mb], AS_new[:, 2 * mb:] = AY[:, :mb], AY[:, mb:]
    X, AX = Y[:, :mb], AY[:, :mb]
    R = AX - theta[:, :, None] * X
    xnorm2 = np.sum(np.abs(X) ** 2, axis=2)
    rn2 = np.sum(np.abs(R) ** 2, axis=2)
    res = np.sqrt(np.divide(rn2, xnorm2, out=np.zeros_like(rn2), where=xnorm2 > 0))
    return S_new, AS_new, R, res, xnorm2
