"""The compensated operator on k-space coefficients, the diagonal-block preconditioner and a
direct DFT.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The eigenproblem is solved for x = F3^H H (Section 2.4, eq (2.30)), where F3 = diag(F, F, F),
F = F (x) F (x) F and F is the unitary DFT of Lemma 2.1, F_ab = omega^(a b)/sqrt(N),
omega = exp(+2 pi i/N).  The oracle's k-space operator is the plain conjugation
F3^H Op F3 of the explicit sparse operator; the DFT is a library step (numpy.fft), with
F u = sqrt(N) * ifft(u) per axis, so F applied along all three axes is N^(3/2) ifftn.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from . import yee


def F3(v: np.ndarray, N: int) -> np.ndarray:
    """Unitary 3D DFT F (x) F (x) F of Lemma 2.1 applied to the trailing N^3 axis (x fastest)."""
    shp = v.shape[:-1]
    a = v.reshape(shp + (N, N, N))
    return (np.fft.ifftn(a, axes=(-3, -2, -1)) * N ** 1.5).reshape(shp + (N ** 3,))


def F3H(v: np.ndarray, N: int) -> np.ndarray:
    """Inverse of F3: F^H (x) F^H (x) F^H = fftn / N^(3/2)."""
    shp = v.shape[:-1]
    a = v.reshape(shp + (N, N, N))
    return (np.fft.fftn(a, axes=(-3, -2, -1)) / N ** 1.5).reshape(shp + (N ** 3,))


def kspace_apply(Op, x: np.ndarray, N: int) -> np.ndarray:
    """y = F3^H Op F3 x for a block x of shape (nvec, 3, N^3) (Prop 2.8, eq (2.30))."""
    x = np.asarray(x, dtype=np.complex128)
    H = F3(x, N).reshape(x.shape[0], 3 * N ** 3)
    Y = (Op @ H.T).T.reshape(x.shape)
    return F3H(Y, N)


def circulant_eigenvalues(first_row: np.ndarray) -> np.ndarray:
    """Eigenvalues lambda_q = sum_j c_j omega^(q j), omega = exp(2 pi i/N), of the circulant
    matrix with first row c, by the definition in Lemma 2.1 (direct sum)."""
    c = np.asarray(first_row, dtype=np.complex128)
    N = c.shape[0]
    q = np.arange(N)
    W = np.exp(2j * math.pi * np.outer(q, q) / N)
    return W @ c


def symbols_1d(N: int, k: Sequence[float], m: int = 1):
    """Diagonal of Lambda_1 + i k_a Lambda_0 for each axis a (Prop 2.8, eq (2.28)), from the
    first rows of D1 and D0 (eq (2.5), or their order-2m forms of eq (2.34)) through Lemma 2.1.
    Returns three complex arrays (N,)."""
    D1 = yee.circulant_d1(N, m).toarray()
    D0 = yee.circulant_d0(N, m).toarray()
    l1 = circulant_eigenvalues(D1[0])
    l0 = circulant_eigenvalues(D0[0])
    return [l1 + 1j * k[a] * l0 for a in range(3)]


def symbols_3d(N: int, k: Sequence[float], m: int = 1, lattice=None) -> np.ndarray:
    """K_1, K_2, K_3 as full diagonals over the k-space index p = qx + N qy + N^2 qz (eq (2.28)),
    complex (3, N^3).  For a general lattice, the eigenvalues of the blocks of eq (2.12):
    K_i(p) = sum_j b_ji Lambda_1(q_j) + i k_i Lambda_0(q_i), b = A^{-1} (Lemma 2.1 per axis)."""
    qz, qy, qx = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    q = [qx.ravel(), qy.ravel(), qz.ravel()]
    if lattice is None:
        s = symbols_1d(N, k, m)
        return np.stack([s[0][q[0]], s[1][q[1]], s[2][q[2]]])
    D1 = yee.circulant_d1(N, m).toarray()
    D0 = yee.circulant_d0(N, m).toarray()
    l1 = circulant_eigenvalues(D1[0])
    l0 = circulant_eigenvalues(D0[0])
    b = yee.lattice_inverse(lattice)
    K = np.zeros((3, N ** 3), dtype=np.complex128)
    for i in range(3):
        K[i] = 1j * k[i] * l0[q[i]] + sum(b[j, i] * l1[q[j]] for j in range(3))
    return K


def curl_symbol(K: np.ndarray) -> np.ndarray:
    """K_A per frequency, (N^3, 3, 3): [[0, -K3, K2], [K3, 0, -K1], [-K2, K1, 0]] (eq (2.29))."""
    n3 = K.shape[1]
    A = np.zeros((n3, 3, 3), dtype=np.complex128)
    A[:, 0, 1], A[:, 0, 2] = -K[2], K[1]
    A[:, 1, 0], A[:, 1, 2] = K[2], -K[0]
    A[:, 2, 0], A[:, 2, 1] = -K[1], K[0]
    return A


def div_symbol_gram(K: np.ndarray) -> np.ndarray:
    """K_B = [K1^H; K2^H; K3^H][K1 K2 K3] per frequency, (N^3, 3, 3) (eq (2.29))."""
    return np.einsum("ap,bp->pab", K.conj(), K)


def precond_matrices(N: int, k: Sequence[float], gamma: float, m: int = 1, lattice=None) -> np.ndarray:
    """K_P = K_A K_A^H + gamma K_B per frequency, (N^3, 3, 3) (eq (2.31))."""
    K = symbols_3d(N, k, m, lattice)
    A = curl_symbol(K)
    return A @ A.conj().transpose(0, 2, 1) + gamma * div_symbol_gram(K)


def precond_apply(N: int, k: Sequence[float], gamma: float, r: np.ndarray, m: int = 1,
                  lattice=None) -> np.ndarray:
    """z = K_P^{-1} r per frequency (eq (2.32)), r of shape (nvec, 3, N^3).  Where K_P is
    singular (only the DC frequency at k = 0, whose modes are the constant fields of Prop 2.5)
    the output is zero."""
    KP = precond_matrices(N, k, gamma, m, lattice)
    r = np.asarray(r, dtype=np.complex128)
    z = np.zeros_like(r)
    scale = np.abs(KP).reshape(KP.shape[0], -1).max(axis=1)
    ok = scale > 0
    sing = np.zeros(KP.shape[0], dtype=bool)
    for p in np.nonzero(ok)[0]:
        if np.linalg.matrix_rank(KP[p]) < 3:
            sing[p] = True
    good = ok & ~sing
    rhs = r.transpose(2, 1, 0)[good]            # (np, 3, nvec)
    z_good = np.linalg.solve(KP[good], rhs)     # (np, 3, nvec)
    zt = z.transpose(2, 1, 0).copy()
    zt[good] = z_good
    return zt.transpose(2, 1, 0)


def direct_dft(u: np.ndarray, sign: int) -> np.ndarray:
    """Unnormalised DFT along the last axis by its definition: X_q = sum_j u_j exp(sign 2 pi i j q/N)."""
    u = np.asarray(u, dtype=np.complex128)
    N = u.shape[-1]
    j = np.arange(N)
    W = np.exp(sign * 2j * math.pi * np.outer(j, j) / N)
    return u @ W.T


def edge_permittivity(ids: np.ndarray, table: np.ndarray) -> np.ndarray:
    """E0_c = 1 / (eps^-1)_cc of the material at the c-edge points, (3, N^3): the field of the
    classical transverse-projection preconditioner (input lookup and a reciprocal)."""
    P = yee.point_tensors(ids, table)
    return np.stack([1.0 / P[c][:, c, c].real for c in range(3)])


def transverse_precond_apply(N: int, k: Sequence[float], gamma: float, E: np.ndarray,
                             r: np.ndarray, m: int = 1, lattice=None) -> np.ndarray:
    """z = T_E r with T_E = K_A^{+H} F3^H diag(E) F3 K_A^{+} + (gamma K_B)^{+}, the
    transverse-projection preconditioner (Johnson & Joannopoulos, Opt. Express 8 (2001) 173)
    written for the operator of eq (2.30): the curl part of Op with the inverse permittivity M
    replaced by the diagonal field E, each factor inverted by its Moore-Penrose pseudo-inverse
    per frequency (numpy.linalg.pinv), plus the pseudo-inverse of the penalty block.
    E: real (3, N^3) on the edge points (component c scales the c-edge values), one field for
    all vectors or (nvec, 3, N^3); r: (nvec, 3, N^3); m: stencil order 2m (eq (2.34))."""
    K = symbols_3d(N, k, m, lattice)
    A = curl_symbol(K)
    Ap = np.linalg.pinv(A, rcond=1e-12)                      # (N^3, 3, 3)
    Bp = np.linalg.pinv(gamma * div_symbol_gram(K), rcond=1e-12)
    r = np.asarray(r, dtype=np.complex128)
    E = np.asarray(E, dtype=np.float64)
    if E.ndim == 2:
        E = np.broadcast_to(E, r.shape)
    u = np.einsum("pab,vbp->vap", Ap, r)                     # K_A^+ r
    u = F3H(F3(u, N) * E, N)                                 # F3^H E F3
    z = np.einsum("pba,vbp->vap", Ap.conj(), u)              # K_A^{+H}
    return z + np.einsum("pab,vbp->vap", Bp, r)
