"""Pins of the oracle's block steps (oracle/block.py): brute-force sums on tiny inputs,
closed forms (orthonormal columns, exact eigenvectors) and selections that expose a transposed
or misplaced coefficient."""
import numpy as np

import workloads as W
from oracle import block


def test_gram_brute_force_tiny():
    S = W.random_complex(1, (2, 3, 5))
    AS = W.random_complex(2, (2, 3, 5))
    GA, GB = block.gram(S, AS)
    for b in range(2):
        for i in range(3):
            for j in range(3):
                a = sum(complex(S[b, i, r]).conjugate() * complex(AS[b, j, r]) for r in range(5))
                g = sum(complex(S[b, i, r]).conjugate() * complex(S[b, j, r]) for r in range(5))
                assert abs(GA[b, i, j] - a) < 1e-13 and abs(GB[b, i, j] - g) < 1e-13


def test_gram_orthonormal_columns_and_eigenvectors():
    """Columns from a QR factorisation give GB = I; eigenvectors of a Hermitian A with
    AS = A S give GA = diag(eigenvalues)."""
    n, nc = 40, 7
    M = W.random_complex(3, (n, n))
    A = M + M.conj().T
    lam, V = np.linalg.eigh(A)
    S = V[:, :nc].T[None]                 # columns = eigenvectors
    AS = (A @ V[:, :nc]).T[None]
    GA, GB = block.gram(S, AS)
    assert np.allclose(GB[0], np.eye(nc), atol=1e-13)
    assert np.allclose(GA[0], np.diag(lam[:nc]), atol=1e-12)
    Q, _ = np.linalg.qr(W.random_complex(4, (n, nc)))
    _, GB = block.gram(Q.T[None], Q.T[None])
    assert np.allclose(GB[0], np.eye(nc), atol=1e-13)


def test_gram_hermitian():
    n, nc = 30, 6
    M = W.random_complex(5, (n, n))
    A = M + M.conj().T
    S = W.random_complex(6, (1, nc, n))
    GA, GB = block.gram(S, (A @ S[0].T).T[None])
    assert np.allclose(GA[0], GA[0].conj().T, atol=1e-12)
    assert np.allclose(GB[0], GB[0].conj().T, atol=1e-13)
    assert np.all(np.linalg.eigvalsh(GB[0]) > 0)


def test_update_single_coefficient():
    """C with one entry alpha at (c, q): output column q is alpha times input column c, in the
    X slots (q < mb) or the P slots (q >= mb -> column mb + q); W is untouched."""
    nb, mb, n = 2, 3, 8
    S = W.random_complex(7, (nb, 3 * mb, n))
    AS = W.random_complex(8, (nb, 3 * mb, n))
    for (c, q) in [(0, 0), (4, 1), (8, 2), (2, 3), (7, 5)]:
        C = np.zeros((nb, 3 * mb, 2 * mb), complex)
        C[:, c, q] = 0.5 - 2j
        S1, AS1, R, res, xn2 = block.update(S, AS, C, np.ones((nb, mb)))
        col = q if q < mb else mb + q
        assert np.allclose(S1[:, col], (0.5 - 2j) * S[:, c])
        assert np.allclose(AS1[:, col], (0.5 - 2j) * AS[:, c])
        assert np.array_equal(S1[:, mb:2 * mb], S[:, mb:2 * mb])
        others = [j for j in list(range(mb)) + list(range(2 * mb, 3 * mb)) if j != col]
        assert np.all(S1[:, others] == 0)


def test_update_exact_eigenvectors_zero_residual():
    """X from eigenvectors of a Hermitian A, AS = A S, C1 selecting X: R = 0, Res = 0, |x|^2 = 1;
    a wrong theta gives Res = |theta - lambda| exactly."""
    n, mb = 24, 4
    M = W.random_complex(9, (n, n))
    A = M + M.conj().T
    lam, V = np.linalg.eigh(A)
    S = W.random_complex(10, (1, 3 * mb, n))
    S[0, :mb] = V[:, :mb].T
    AS = (A @ S[0].T).T[None]
    C = np.zeros((1, 3 * mb, 2 * mb), complex)
    for j in range(mb):
        C[0, j, j] = 1.0
        C[0, 2 * mb + j, mb + j] = 1.0
    _, _, R, res, xn2 = block.update(S, AS, C, lam[None, :mb])
    assert np.max(np.abs(R)) < 1e-12 and np.max(res) < 1e-12
    assert np.allclose(xn2, 1.0)
    _, _, _, res2, _ = block.update(S, AS, C, lam[None, :mb] + 0.25)
    assert np.allclose(res2, 0.25, atol=1e-12)
