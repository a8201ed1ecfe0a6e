"""Pins of the order-2m stencils of Section 2.5 in the oracle (eqs (2.34)-(2.35), Table 1,
Remark 2.10, Table 5).

The closed forms here are written from Lemma 2.1 and Taylor expansion, independently of the
oracle's circulant assembly: a wrong coefficient, a shifted tap or a dropped sign in the
high-order first rows fails at least one of them.
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import eigs, kspace, yee

# Table 1, with the m = 3 entry c_1^(1) read as 75/64 (the printed 25/64 does not satisfy
# eq (2.35): sum_s (2s - 1) c_s^(1) = 1 needs 75/64)
TABLE1 = {
    1: ([F(1)], [F(1, 2)]),
    2: ([F(9, 8), F(-1, 24)], [F(9, 16), F(-1, 16)]),
    3: ([F(75, 64), F(-25, 384), F(3, 640)], [F(75, 128), F(-25, 256), F(3, 256)]),
    4: ([F(1225, 1024), F(-245, 3072), F(49, 5120), F(-5, 7168)],
        [F(1225, 2048), F(-245, 2048), F(49, 2048), F(-5, 2048)]),
    5: ([F(19845, 16384), F(-735, 8192), F(567, 40960), F(-405, 229376), F(35, 294912)],
        [F(19845, 32768), F(-2205, 16384), F(567, 16384), F(-405, 65536), F(35, 65536)]),
}


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_table1_coefficients(m):
    """eq (2.35) solved exactly reproduces Table 1 (with the m = 3 reading above)."""
    c1, c0 = yee.stencil_coefficients(m)
    assert c1 == TABLE1[m][0]
    assert c0 == TABLE1[m][1]


def test_table1_printed_m3_entry_is_inconsistent():
    """The printed 25/64 breaks the first equation of eq (2.35) (consistency of the
    derivative); 75/64 satisfies it."""
    c1 = TABLE1[3][0]
    assert sum((2 * s - 1) * c for s, c in enumerate(c1, start=1)) == 1
    printed = [F(25, 64)] + c1[1:]
    assert sum((2 * s - 1) * c for s, c in enumerate(printed, start=1)) != 1


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_stencils_exact_on_polynomials(m):
    """Taylor expansion behind eq (2.34): the order-2m derivative stencil at the midpoint
    (j - 1/2) h is exact on polynomials of degree <= 2m, and the order-2m average on degree
    <= 2m - 1, but not one degree beyond; checked in grid units (h D1, D0 on phi_j = (j - c)^p)
    on interior points of a long grid, away from the periodic wrap."""
    N = 32
    D1h = yee.circulant_d1(N, m).toarray() / N
    D0 = yee.circulant_d0(N, m).toarray()
    j = np.arange(N, dtype=np.float64)
    inner = slice(2 * m, N - 2 * m)
    u = j - N / 2                     # |u| <= 16
    uc = u - 0.5                      # midpoints
    for p in range(0, 2 * m + 2):
        phi = u ** p
        scale = max(1.0, float(np.abs(phi).max()))
        d_exact = p * uc ** (p - 1) if p > 0 else np.zeros(N)
        err1 = np.abs((D1h @ phi)[inner] - d_exact[inner]).max() / scale
        err0 = np.abs((D0 @ phi)[inner] - (uc ** p)[inner]).max() / scale
        if p <= 2 * m:
            assert err1 < 1e-14, (p, err1)
        else:
            assert err1 > 1e-12, (p, err1)         # the order is exactly 2m
        if p <= 2 * m - 1:
            assert err0 < 1e-14, (p, err0)
        elif p == 2 * m:
            assert err0 > 1e-12, (p, err0)


def kappa_m(N, kk, m):
    """Real factor of the order-2m 1D symbol by Lemma 2.1 on the first rows of eq (2.34):
    K(q) = i e^{-i theta/2} kappa(q), kappa = (2/h) sum_s c1_s sin((s - 1/2) theta)
    + 2 k sum_s c0_s cos((s - 1/2) theta), theta = 2 pi q / N."""
    c1, c0 = TABLE1[m]
    th = 2 * math.pi * np.arange(N) / N
    s1 = sum(float(c) * np.sin((s - 0.5) * th) for s, c in enumerate(c1, start=1))
    s0 = sum(float(c) * np.cos((s - 0.5) * th) for s, c in enumerate(c0, start=1))
    return 2.0 * N * s1 + 2.0 * kk * s0


@pytest.mark.parametrize("m", [2, 3, 5])
@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (math.pi, math.pi, math.pi), (0.0, 0.0, 0.0)])
def test_highorder_symbols(m, k):
    """Lemma 2.1 on the order-2m circulants: their eigenvalues are i e^{-i theta/2} kappa."""
    N = 12
    th = 2 * math.pi * np.arange(N) / N
    syms = kspace.symbols_1d(N, k, m)
    for a in range(3):
        ref = 1j * np.exp(-0.5j * th) * kappa_m(N, k[a], m)
        assert np.allclose(syms[a], ref, rtol=0, atol=1e-10 * N)


@pytest.mark.parametrize("m", [2, 5])
@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (math.pi, 0.0, -2.0)])
def test_highorder_homogeneous_dispersion(m, k):
    """eps^-1 = c I everywhere: spec(Op) = {c s(p) (twice), gamma s(p)} with the order-2m
    s(p) = sum_i kappa_i(q_i)^2 (Prop 2.8 with the high-order symbols, Section 2.5)."""
    N = max(6, 2 * m)
    c = 1.0 / 13.0
    ids = np.ones((4, N ** 3), dtype=np.uint8)
    tab = W.eps_table([np.eye(3) / c])
    kx, ky, kz = (kappa_m(N, k[a], m) for a in range(3))
    s = (kx[None, None, :] ** 2 + ky[None, :, None] ** 2 + kz[:, None, None] ** 2).ravel()
    g = yee.gamma_rule(k)
    ref = np.sort(np.concatenate([c * s, c * s, g * s]))
    ev = np.sort(np.linalg.eigvalsh(yee.compensated_operator(N, k, ids, tab, "crossdof", m=m).toarray()))
    assert np.allclose(ev, ref, rtol=1e-10, atol=1e-10 * ref.max())


@pytest.mark.parametrize("m", [2, 5])
def test_remark_2_10_null_space_and_lambda_min(m):
    """Remark 2.10: the statements of Prop 2.5 hold for the order-2m stencils: at k = 0 the
    compensated operator's null space is the three constant fields, for k != 0 (|k_i| <= pi) it
    is trivial and lambda_min(L) = |k|^2, so eq (2.26) keeps its guarantee."""
    N = max(8, 2 * m)
    wl = W.sphere_anisotropic(N=N, nk=2, m=4)
    for k, dim in (((0.0, 0.0, 0.0), 3), ((0.3, -0.5, 0.7), 0)):
        Op = yee.compensated_operator(N, k, wl.ids, wl.table, "crossdof", m=m).toarray()
        ev = np.linalg.eigvalsh(Op)
        assert int((np.abs(ev) < 1e-10 * np.abs(ev).max()).sum()) == dim
    k = np.array([0.3, -0.5, 0.7])
    B = yee.div_matrix(N, k, m)
    L = (B @ B.conj().T).toarray()
    assert np.linalg.eigvalsh(L).min() == pytest.approx(float(k @ k), rel=1e-9)


def _sector_lowest(N, m, gamma=1.0):
    """Lowest eigenvalue of the smooth-permittivity operator of eq (4.7) at k = (pi, pi, pi) on
    the fields that depend on the grid index only through t = i + j + k (mod N).  The samples
    of eps depend on t alone and k is along (1, 1, 1), so the index translations that keep t
    commute with Op; the fields they leave invariant form an invariant subspace, reduced here
    to 3N unknowns.  gamma = 1 keeps the spurious spectrum (>= |k|^2 = 3 pi^2) far above."""
    wl = W.smooth_isotropic(N)
    k = wl.kpoints[0]
    A = yee.curl_matrix(N, k, m)
    B = yee.div_matrix(N, k, m)
    M = yee.eps_matrix(N, wl.ids, wl.table, "diagonal")
    n3 = N ** 3
    p = np.arange(n3)
    t = (p % N + (p // N) % N + p // (N * N)) % N
    rows = np.concatenate([c * n3 + p for c in range(3)])
    cols = np.concatenate([c * N + t for c in range(3)])
    P = sp.csr_matrix((np.full(rows.size, 1.0 / N), (rows, cols)), shape=(3 * n3, 3 * N))
    OP = A @ (M @ (A.conj().T @ P)) + gamma * (B.conj().T @ (B @ P))
    red = (P.T @ OP).toarray()
    assert np.abs((OP - P @ sp.csr_matrix(red)).toarray()).max() <= 1e-12 * np.abs(red).max()
    return np.linalg.eigvalsh(0.5 * (red + red.conj().T))[0]


def test_smooth_sector_holds_the_lowest_mode():
    """The invariant subspace above holds the lowest eigenvalue of the whole operator
    (checked against the dense spectrum at N = 8)."""
    N, m = 8, 5
    wl = W.smooth_isotropic(N)
    Op = yee.compensated_operator(N, wl.kpoints[0], wl.ids, wl.table, "diagonal", gamma=1.0, m=m)
    full = np.linalg.eigvalsh(Op.toarray())
    assert _sector_lowest(N, m) == pytest.approx(full[0], rel=1e-12)


def test_table5_smooth_permittivity_tenth_order():
    """Table 5: smooth eps of eq (4.7), k = (pi, pi, pi), order-10 stencils (m = 5); the first
    two eigenvalues change by 4.87e-09 between h = 1/16 and h = 1/32.  The printed differences
    are those of the normalised frequencies omega / (2 pi) = sqrt(lambda) / (2 pi) (the header
    says omega^2; the three eigenvalue groups of the h = 1/32 column all agree with the
    frequency reading).  The h = 1/64 and 1/128 columns sit at the accuracy floor of the
    eigensolves and are not used."""
    lam16 = _sector_lowest(16, 5)
    lam32 = _sector_lowest(32, 5)
    d = abs(math.sqrt(lam32) - math.sqrt(lam16)) / (2 * math.pi)
    assert d == pytest.approx(4.87e-9, rel=0.01)
    # the same eigenvalue with the second-order stencil moves by far more
    d2 = abs(math.sqrt(_sector_lowest(32, 1)) - math.sqrt(_sector_lowest(16, 1))) / (2 * math.pi)
    assert d2 > 1e-5


def test_matfree_oracle_matches_dense_highorder():
    """The shift-invert/CG eigen-solve on the sparse factors agrees with dense LAPACK on the
    assembled operator (order-4 stencils, anisotropic sphere, CrossDoF)."""
    N, m = 8, 2
    wl = W.sphere_anisotropic(N=N, nk=3, m=6)
    k = wl.kpoints[1]
    Op = yee.compensated_operator(N, k, wl.ids, wl.table, "crossdof", m=m)
    ref = eigs.smallest_positive(Op, 6, method="dense")
    got = eigs.smallest_positive_matfree(N, k, wl.ids, wl.table, "crossdof", 6, stencil_m=m)
    assert np.allclose(got, ref, rtol=1e-11, atol=0)
