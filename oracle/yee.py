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


def stencil_coefficients(m: int):
    """Coefficients c_s^(1), c_s^(0), s = 1..m, of the order-2m stencils of eq (2.34), as exact
    rationals: the solution of the m x m system of eq (2.35),
        sum_t ((2t - 1)/2)^(2s + kind - 2) c_t^(kind) = 1/2 if s = 1 else 0,
    by Gaussian elimination over the rationals.  Returns (c1, c0), lists of Fraction."""
    from fractions import Fraction

    if m < 1:
        raise ValueError("stencil order 2m needs m >= 1")
    out = []
    for kind in (1, 0):
        A = [[Fraction(2 * t - 1, 2) ** (2 * s + kind - 2) for t in range(1, m + 1)] + [Fraction(1, 2) if s == 1 else Fraction(0)]
             for s in range(1, m + 1)]
        for col in range(m):
            piv = next(r for r in range(col, m) if A[r][col] != 0)
            A[col], A[piv] = A[piv], A[col]
            for r in range(m):
                if r != col and A[r][col] != 0:
                    f = A[r][col] / A[col][col]
                    A[r] = [a - f * b for a, b in zip(A[r], A[col])]
        out.append([A[r][m] / A[r][r] for r in range(m)])
    return out[0], out[1]


def circulant_from_taps(N: int, taps) -> sp.csr_matrix:
    """Periodic N x N matrix with (C u)_j = sum over (offset, weight) of weight * u_{j + offset}
    (repeated columns add up)."""
    rows, cols, vals = [], [], []
    for off, w in taps:
        rows.append(np.arange(N))
        cols.append((np.arange(N) + off) % N)
        vals.append(np.full(N, float(w)))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def circulant_d1(N: int, m: int = 1) -> sp.csr_matrix:
    """D1 of eq (2.5) (m = 1: first row (1, 0, ..., 0, -1)/h, (D1 u)_j = (u_j - u_{j-1})/h), and
    its order-2m form of eq (2.34): (D1 u)_j = (1/h) sum_s c_s^(1) (u_{j+s-1} - u_{j-s})."""
    h = 1.0 / N
    c1, _ = stencil_coefficients(m)
    taps = []
    for s, c in enumerate(c1, start=1):
        taps += [(s - 1, float(c) / h), (-s, -float(c) / h)]
    return circulant_from_taps(N, taps)


def circulant_d0(N: int, m: int = 1) -> sp.csr_matrix:
    """D0 of eq (2.5) (m = 1: first row (1, 0, ..., 0, 1)/2, (D0 u)_j = (u_j + u_{j-1})/2), and
    its order-2m form of eq (2.34): (D0 u)_j = sum_s c_s^(0) (u_{j+s-1} + u_{j-s})."""
    _, c0 = stencil_coefficients(m)
    taps = []
    for s, c in enumerate(c0, start=1):
        taps += [(s - 1, float(c)), (-s, float(c))]
    return circulant_from_taps(N, taps)


def embed(M1: sp.spmatrix, axis: int, N: int) -> sp.csr_matrix:
    """Kronecker embedding of a 1D N x N matrix acting along `axis` (0=x, 1=y, 2=z), eq (2.6)."""
    I = sp.identity(N, format="csr")
    if axis == 0:
        return sp.kron(sp.identity(N * N, format="csr"), M1, format="csr")
    if axis == 1:
        return sp.kron(I, sp.kron(M1, I, format="csr"), format="csr")
    return sp.kron(M1, sp.identity(N * N, format="csr"), format="csr")


def lattice_inverse(lattice) -> np.ndarray:
    """b = A^{-1} for the lattice matrix A = (a_1, a_2, a_3) whose COLUMNS are the primitive
    vectors (Section 2.2, eq (2.8)); `lattice` lists the vectors as rows (None: simple cubic)."""
    if lattice is None:
        return np.eye(3)
    A = np.asarray(lattice, dtype=np.float64).reshape(3, 3).T
    return np.linalg.inv(A)


def deriv_blocks(N: int, k: Sequence[float], m: int = 1, lattice=None):
    """D_i = D_{1,i} + i k_i D_{0,i}, i = 1, 2, 3 (eq (2.6)), complex sparse N^3 x N^3, with the
    order-2m first rows of eq (2.34) (m = 1 is eq (2.5)).  For a general lattice (Section 2.2,
    eq (2.12)) the difference part follows the transformed gradient of eq (2.11):
    D_i = sum_j b_ji D_{1,j} + i k_i D_{0,i}, b = A^{-1} (the printed eq (2.12) has D_{1,i} under
    the sum over j; the derivative along lattice axis j is D_{1,j})."""
    D1, D0 = circulant_d1(N, m), circulant_d0(N, m)
    b = lattice_inverse(lattice)
    E1 = [embed(D1, j, N) for j in range(3)]
    out = []
    for i in range(3):
        Di = 1j * k[i] * embed(D0, i, N)
        for j in range(3):
            if b[j, i] != 0.0:
                Di = Di + b[j, i] * E1[j]
        out.append(Di.tocsr())
    return out


def curl_matrix(N: int, k: Sequence[float], m: int = 1, lattice=None) -> sp.csr_matrix:
    """Outer curl A (edge -> face), eq (2.7): [[0, -D3, D2], [D3, 0, -D1], [-D2, D1, 0]]."""
    D1, D2, D3 = deriv_blocks(N, k, m, lattice)
    return sp.bmat([[None, -D3, D2], [D3, None, -D1], [-D2, D1, None]], format="csr")


def div_matrix(N: int, k: Sequence[float], m: int = 1, lattice=None) -> sp.csr_matrix:
    """Divergence B (face -> volume), eq (2.7): [D1, D2, D3]."""
    D1, D2, D3 = deriv_blocks(N, k, m, lattice)
    return sp.hstack([D1, D2, D3], format="csr")


def transfer_matrices(N: int):
    """Cross-DoF transfer matrices of eqs (3.5)-(3.7), read geometrically: T12 averages the four
    y-edges around an x-edge (x in {i-1, i}, y-edge rows j, j+1), T13 the four z-edges around an
    x-edge, T23 the four z-edges around a y-edge.  D0 acts on the axis of the row component,
    D0^T on the axis of the column component, the identity on the third axis.  The transfer
    keeps the two-point average of eq (2.5) whatever the order of the curl stencils: eq (3.5)
    defines it on the four nearest edges, and the bounds of Props 3.7-3.10 rest on its
    non-negative weights."""
    D0 = circulant_d0(N, 1)
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
                         scheme: str, gamma: float | None = None, m: int = 1, lattice=None) -> sp.csr_matrix:
    """Op = A M A^H + gamma B^H B, eq (2.13); gamma defaults to eq (2.26); curl and divergence
    with the order-2m stencils of eq (2.34) (Remark 2.10: the penalty rule is unchanged) and the
    lattice's transformed blocks of eq (2.12) (lattice vectors as rows, None: simple cubic)."""
    if gamma is None:
        gamma = gamma_rule(k)
    A = curl_matrix(N, k, m, lattice)
    B = div_matrix(N, k, m, lattice)
    M = eps_matrix(N, ids, table, scheme)
    Op = (A @ M @ A.conj().T + gamma * (B.conj().T @ B)).tocsr()
    return Op
