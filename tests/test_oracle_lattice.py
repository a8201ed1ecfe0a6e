"""Pins of the oracle's general-lattice operator (Section 2.2, eqs (2.8)-(2.12)) against facts the
mathematics fixes: the divergence of a curl vanishes (Prop 2.2) and A A^H + B^H B is block
diagonal (Lemma 2.4 (1)) for any lattice; a scaled cubic lattice is the unit one at a scaled wave
vector; and for a homogeneous medium the plane waves e^{i G.x} of the reciprocal lattice
(G = 2 pi A^{-T} n) span invariant 3-dimensional subspaces whose eigenvalues converge at second
order to the free-photon values c |k + G|^2 (twice) and gamma |k + G|^2 -- which fixes the lattice
matrix, its inverse and the orientation of b_ji in eq (2.12) (the triclinic cell is not
symmetric)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import kspace, yee

LATS = ["fcc", "bcc", "tric"]


@pytest.mark.parametrize("lat", LATS)
def test_divergence_of_curl_vanishes(lat):
    N = 5
    k = (0.4, -0.9, 1.3)
    A = yee.curl_matrix(N, k, 1, W.LATTICES[lat])
    B = yee.div_matrix(N, k, 1, W.LATTICES[lat])
    assert abs(B @ A).max() < 1e-9 * abs(A).max() ** 2


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("m", [1, 2])
def test_curl_curl_plus_grad_div_is_block_diagonal(lat, m):
    N = 5
    k = (0.7, 0.2, -0.5)
    A = yee.curl_matrix(N, k, m, W.LATTICES[lat])
    B = yee.div_matrix(N, k, m, W.LATTICES[lat])
    S = (A @ A.conj().T + B.conj().T @ B).toarray()
    n3 = N ** 3
    L = S[:n3, :n3]
    for c in range(3):
        for d in range(3):
            blk = S[c * n3:(c + 1) * n3, d * n3:(d + 1) * n3]
            assert np.abs(blk - (L if c == d else 0)).max() < 1e-9 * np.abs(L).max()


def test_scaled_cubic_lattice_is_the_unit_one_at_a_scaled_wave_vector():
    """A = a I: every difference picks up 1/a, so Op(aI, k) = Op(I, a k) / a^2 (same gamma and M)."""
    N, a = 6, 1.7
    wl = W.sphere_anisotropic(N=N, nk=3, m=4)
    k = np.array([0.3, -0.8, 1.1])
    g = 9.0
    Op_a = yee.compensated_operator(N, k, wl.ids, wl.table, "crossdof", gamma=g, lattice=a * np.eye(3))
    Op_1 = yee.compensated_operator(N, a * k, wl.ids, wl.table, "crossdof", gamma=g)
    assert abs(Op_a - Op_1 / a ** 2).max() < 1e-12 * abs(Op_1).max() / a ** 2


def _plane_wave_blocks(N, lat, k, c, g, ns):
    """3 x 3 blocks P^H Op P on the plane waves of integer vectors n (fractional-coordinate
    frequencies), from the oracle's sparse Op; also checks that span(P) is invariant."""
    ids = np.ones((4, N ** 3), dtype=np.uint8)
    tab = np.stack([np.eye(3, dtype=complex), c * np.eye(3, dtype=complex)])
    Op = yee.compensated_operator(N, k, ids, tab, "diagonal", gamma=g, lattice=W.LATTICES[lat])
    kk, jj, ii = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    idx = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    out = []
    for n in ns:
        ph = np.exp(2j * math.pi * (idx @ np.asarray(n)) / N) / N ** 1.5
        P = np.zeros((3 * N ** 3, 3), dtype=complex)
        for a in range(3):
            P[a * N ** 3:(a + 1) * N ** 3, a] = ph
        OP = Op @ P
        blk = P.conj().T @ OP
        assert np.abs(OP - P @ blk).max() < 1e-9 * np.abs(blk).max()
        out.append(np.sort(np.linalg.eigvalsh(0.5 * (blk + blk.conj().T))))
    return out


@pytest.mark.parametrize("lat", LATS)
def test_free_photon_limit(lat):
    c, g = 0.4, 3.0
    k = np.array([0.35, -0.6, 0.45])
    ns = [(0, 0, 0), (1, 0, 0), (0, -1, 0), (0, 0, 1), (1, -1, 0), (1, 1, -1)]
    b = np.linalg.inv(W.LATTICES[lat].T)       # A^{-1}, A = (a_1 a_2 a_3) as columns
    exact = [float(np.sum((k + 2 * math.pi * b.T @ np.asarray(n)) ** 2)) for n in ns]
    err = {}
    for N in (8, 16):
        ev = _plane_wave_blocks(N, lat, k, c, g, ns)
        err[N] = []
        for e, ex in zip(ev, exact):
            trans = np.sort(e)[:2] if c < g else np.sort(e)[1:]
            # the two transverse values and the longitudinal one
            assert abs(trans[0] - trans[1]) < 1e-9 * abs(trans[0]) + 1e-12
            lon = e[np.argmax(np.abs(e - trans[0]))]
            assert abs(lon / g - trans[0] / c) < 1e-9 * trans[0] / c
            err[N].append(abs(trans[0] / c - ex) / ex)
    err8, err16 = np.array(err[8]), np.array(err[16])
    assert err16.max() < 0.1
    # second order: halving h divides the error by about 4
    ratio = err8[1:] / err16[1:]
    assert np.all((ratio > 3.0) & (ratio < 5.5)), ratio


@pytest.mark.parametrize("lat", LATS)
def test_kspace_symbols_match_the_sparse_operator(lat):
    """The oracle's k-space symbols of eq (2.12) (Lemma 2.1 per axis) against its sparse operator
    conjugated by the unitary DFT, on a random field."""
    N = 6
    k = (0.2, 0.9, -0.4)
    L = W.LATTICES[lat]
    wl = W.sphere_anisotropic(N=N, nk=3, m=4)
    ids = np.ones((4, N ** 3), dtype=np.uint8)
    tab = np.stack([np.eye(3, dtype=complex), wl.table[1]])
    g = 5.0
    Op = yee.compensated_operator(N, k, ids, tab, "trivial", gamma=g, lattice=L)
    x = W.random_block(3, 1, N)
    y = kspace.kspace_apply(Op, x, N)[0]
    K = kspace.symbols_3d(N, k, 1, L)
    v = K.conj()
    e = -np.cross(v.T, x[0].T).T
    yy = np.cross(K.T, (tab[1] @ e).T).T + g * v * (K * x[0]).sum(axis=0)[None, :]
    assert np.abs(y - yy).max() < 1e-11 * np.abs(yy).max()
