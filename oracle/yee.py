"""Explicit sparse FP64 matrices of the Yee discretisation and kernel compensation.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every matrix here is built
from its definition in the paper, entry by entry, with scipy.sparse; there is no
FFT anywhere in this module.

Index order: a scalar grid function is a vector of length N^3 with index
i + N j + N^2 k (x fastest), as in the Kronecker embeddings of Section 2.1,
eq (2.6): D_{s,1} = I_{N^2} (x) D_s acts on x, D_{s,2} = I_N (x) D_s (x) I_N on y and
D_{s,3} = D_s (x) I_{N^2} on z.  A vector field is the concatenation of its three
components (eq (2.1)).
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np
import scipy.sparse as sp

SCHEMES = ("diagonal", "trivial", "crossdof")


def shift_matrix(N: int) -> sp.csr_matrix:
    """(S u)_i = u_{i-1} (periodic)."""
    rows = np.arange(N)
    cols = (rows - 1) % N
    return sp.csr_matrix((np.ones(N), (rows, cols)), shape=(N, N))


def circulant_d1(N: int) -> sp.csr_matrix:
    """D1 of eq (2.5): first row (1, 0, ..., 0, -1)/h, i.e. (D1 u)_i = (u_i - u_{i-1})/h."""
    h = 1.0 / N
    return ((sp.identity(N, format="csr") - shift_matrix(N)) / h).tocsr()


def circulant_d0(N: int) -> sp.csr_matrix:
    """D0 of eq (2.5): first row (1, 0, ..., 0, 1)/2, i.e. (D0 u)_i = (u_i + u_{i-1})/2."""
    return ((sp.identity(N, format="csr") + shift_matrix(N)) * 0.5).tocsr()


def embed(M1: sp.spmatrix, axis: int, N: int) -> sp.csr_matrix:
    """Kronecker embedding of a 1D N x N matrix acting along `axis` (0=x, 1=y, 2=z), eq (2.6)."""
    I = sp.identity(N, format="csr")
    if axis == 0:
        return sp.kron(sp.identity(N * N, format="csr"), M1, format="csr")
    if axis == 1:
        return sp.kron(I, sp.kron(M1, I, format="csr"), format="csr")
    return sp.kron(M1, sp.identity(N * N, format="csr"), format="csr")


def deriv_blocks(N: int, k: Sequence[float]):
    """D_i = D_{1,i} + i k_i D_{0,i}, i = 1, 2, 3 (eq (2.6)), complex sparse N^3 x N^3."""
    D1, D0 = circulant_d1(N), circulant_d0(N)
    return [(embed(D1, a, N) + 1j * k[a] * embed(D0, a, N)).tocsr() for a in range(3)]


def curl_matrix(N: int, k: Sequence[float]) -> sp.csr_matrix:
    """Outer curl A (edge -> face), eq (2.7): [[0, -D3, D2], [D3, 0, -D1], [-D2, D1, 0]]."""
    D1, D2, D3 = deriv_blocks(N, k)
    return sp.bmat([[None, -D3, D2], [D3, None, -D1], [-D2, D1, None]], format="csr")


def div_matrix(N: int, k: Sequence[float]) -> sp.csr_matrix:
    """Divergence B (face -> volume), eq (2.7): [D1, D2, D3]."""
    D1, D2, D3 = deriv_blocks(N, k)
    return sp.hstack([D1, D2, D3], format="csr")


def transfer_matrices(N: int):
    """Cross-DoF transfer matrices of eqs (3.5)-(3.7), read geometrically: T12 averages the four
    y-edges around an x-edge (x in {i-1, i}, y-edge rows j, j+1), T13 the four z-edges around an
    x-edge, T23 the four z-edges around a y-edge.  D0 acts on the axis of the row component,
    D0^T on the axis of the column component, the identity on the third axis."""
    D0 = circulant_d0(N)
    D0T = D0.T.tocsr()
    T12 = (embed(D0, 0, N) @ embed(D0T, 1, N)).tocsr()
    T13 = (embed(D0, 0, N) @ embed(D0T, 2, N)).tocsr()
    T23 = (embed(D0, 1, N) @ embed(D0T, 2, N)).tocsr()
    return {(0, 1): T12, (0, 2): T13, (1, 2): T23}


def point_tensors(ids: np.ndarray, table: np.ndarray) -> np.ndarray:
    """Inverse permittivity at the four point sets: complex (4, N^3, 3, 3) (input lookup)."""
    return np.asarray(table, dtype=np.complex128)[np.asarray(ids, dtype=np.int64)]


def eps_matrix(N: int, ids: np.ndarray, table: np.ndarray, scheme: str) -> sp.csr_matrix:
    """Discrete inverse-permittivity matrix M, 3N^3 x 3N^3.

    diagonal block c: diag of (eps^-1)_cc sampled at the c-edge points (eq (3.3));
    'diagonal' : off-diagonal blocks zero (eq (3.3));
    'trivial'  : block (c,d) = diag of (eps^-1)_cd at the volume points (eq (3.4));
    'crossdof' : block (c,d), c<d, = 1/2 (Q_c T_cd + T_cd Q_d), Q_e = diag of (eps^-1)_cd at the
                 e-edge points (eq (3.8); with one material Q_e = eps_cd I_e, which is eq (3.8)
                 verbatim).  Lower blocks are the conjugate transposes.
    """
    if scheme not in SCHEMES:
        raise ValueError(scheme)
    P = point_tensors(ids, table)  # (4, n3, 3, 3): ex, ey, ez, vol
    n3 = N ** 3
    blocks = [[None] * 3 for _ in range(3)]
    for c in range(3):
        blocks[c][c] = sp.diags(P[c][:, c, c].real.astype(np.complex128), format="csr")
    T = transfer_matrices(N) if scheme == "crossdof" else None
    for c in range(3):
        for d in range(c + 1, 3):
            if scheme == "diagonal":
                U = sp.csr_matrix((n3, n3), dtype=np.complex128)
            elif scheme == "trivial":
                U = sp.diags(P[3][:, c, d], format="csr")
            else:
                Qc = sp.diags(P[c][:, c, d], format="csr")
                Qd = sp.diags(P[d][:, c, d], format="csr")
                U = (0.5 * (Qc @ T[(c, d)] + T[(c, d)] @ Qd)).tocsr()
            blocks[c][d] = U
            blocks[d][c] = U.conj().T.tocsr()
    return sp.bmat(blocks, format="csr")


def gamma_rule(k: Sequence[float]) -> float:
    """Practical penalty coefficient of Remark 2.6, eq (2.26): 4 pi^2 if k = 0 or |k| >= 1,
    else 4 pi^2 / |k|^2 (both branches agree at |k| = 1)."""
    kn2 = float(np.dot(k, k))
    if kn2 == 0.0 or kn2 >= 1.0:
        return 4.0 * math.pi ** 2
    return 4.0 * math.pi ** 2 / kn2


def compensated_operator(N: int, k: Sequence[float], ids: np.ndarray, table: np.ndarray,
                         scheme: str, gamma: float | None = None) -> sp.csr_matrix:
    """Op = A M A^H + gamma B^H B, eq (2.13); gamma defaults to eq (2.26)."""
    if gamma is None:
        gamma = gamma_rule(k)
    A = curl_matrix(N, k)
    B = div_matrix(N, k)
    M = eps_matrix(N, ids, table, scheme)
    Op = (A @ M @ A.conj().T + gamma * (B.conj().T @ B)).tocsr()
    return Op
