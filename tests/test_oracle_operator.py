"""Pins of the oracle's operator against what the paper and the mathematics fix.

Each test names the statement it checks.  The closed forms used here are derived from
Lemma 2.1 (eigenvalues of circulant matrices) and are written independently of the oracle's
sparse assembly, so that a dropped term, a wrong sign or index or a transposed operand in
`oracle.yee` fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import eigs, kspace, yee

KS = [(0.3, 0.5, 0.7), (math.pi, math.pi, math.pi), (0.0, 0.0, 0.0), (-1.1, 0.2, 2.9)]


def kappa(N, kk):
    """kappa(q) = (2/h) sin(theta/2) + k cos(theta/2), theta = 2 pi q/N: the real part of the
    1D symbol (1 - e^{-i theta})/h + i k (1 + e^{-i theta})/2 = i e^{-i theta/2} kappa."""
    th = 2 * math.pi * np.arange(N) / N
    return 2.0 * N * np.sin(th / 2) + kk * np.cos(th / 2)


def s_of_p(N, k):
    kx, ky, kz = (kappa(N, k[a]) for a in range(3))
    return (kx[None, None, :] ** 2 + ky[None, :, None] ** 2 + kz[:, None, None] ** 2).ravel()


def homog(N, tensor):
    """Every point inside material 1 with permittivity `tensor` (the table stores its inverse)."""
    n3 = N ** 3
    ids = np.ones((4, n3), dtype=np.uint8)
    return ids, W.eps_table([tensor])


@pytest.mark.parametrize("N", [3, 4, 5])
@pytest.mark.parametrize("k", KS)
def test_BA_zero(N, k):
    """Prop 2.2: B A = 0 exactly."""
    A = yee.curl_matrix(N, k)
    B = yee.div_matrix(N, k)
    assert abs(B @ A).max() < 1e-9 * N * N


@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("k", KS)
def test_AAH_plus_BHB_block_diagonal(N, k):
    """Lemma 2.4 (1): A A^H + B^H B = diag(L, L, L), L = B B^H."""
    A = yee.curl_matrix(N, k)
    B = yee.div_matrix(N, k)
    L = B @ B.conj().T
    S = A @ A.conj().T + B.conj().T @ B
    assert abs(S - sp.block_diag([L, L, L])).max() < 1e-10 * N * N


@pytest.mark.parametrize("N", [4, 5, 6])
@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (math.pi, 0.0, -2.0), (0.0, 0.0, 0.01)])
def test_lambda_min_L_is_k_squared(N, k):
    """Lemma 2.4 (2): lambda_min(L) = |k|^2 for k != 0, max|k_i| <= pi, N > pi."""
    B = yee.div_matrix(N, k)
    L = (B @ B.conj().T).toarray()
    assert np.linalg.eigvalsh(L).min() == pytest.approx(float(np.dot(k, k)), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("N", [4, 6, 8])
def test_k0_second_eigenvalue_of_L(N):
    """Proof of Prop 2.5: at k = 0 the smallest nonzero eigenvalue of K^H K is (4/h^2) sin^2(pi h)."""
    B = yee.div_matrix(N, (0.0, 0.0, 0.0))
    ev = np.sort(np.linalg.eigvalsh((B @ B.conj().T).toarray()))
    assert abs(ev[0]) < 1e-9
    assert ev[1] == pytest.approx(4.0 * N * N * math.sin(math.pi / N) ** 2, rel=1e-12)


@pytest.mark.parametrize("k,dimAMA,dimOp", [((0.3, 0.5, 0.7), 64, 0), ((0.0, 0.0, 0.0), 66, 3)])
def test_null_space_dimensions(k, dimAMA, dimOp):
    """Prop 2.5 (1): without compensation ker(A M A^H) has dimension N^3 (k != 0) or N^3 + 2
    (k = 0); with compensation the null space is {0} or the three constant fields."""
    N = 4
    wl = W.sphere_anisotropic(N=N, nk=2, m=4)
    A = yee.curl_matrix(N, k)
    M = yee.eps_matrix(N, wl.ids, wl.table, "crossdof")
    AMA = (A @ M @ A.conj().T).toarray()
    ev = np.linalg.eigvalsh(AMA)
    tol = 1e-10 * abs(ev).max()
    assert int((abs(ev) < tol).sum()) == dimAMA
    Op = yee.compensated_operator(N, k, wl.ids, wl.table, "crossdof").toarray()
    ev2 = np.linalg.eigvalsh(Op)
    assert int((abs(ev2) < 1e-10 * abs(ev2).max()).sum()) == dimOp
    if dimOp == 3:
        # the null vectors are the constant fields o_1, o_2, o_3 (eq (2.24))
        n3 = N ** 3
        for c in range(3):
            o = np.zeros(3 * n3)
            o[c * n3:(c + 1) * n3] = 1.0
            assert np.abs(Op @ o).max() < 1e-9


@pytest.mark.parametrize("scheme", ["trivial", "crossdof"])
@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (0.0, 0.0, 0.0)])
def test_spectrum_union(scheme, k):
    """Prop 2.3: spec(Op) minus {0} = spec+(A M A^H) union gamma * spec+(B^H B)."""
    N = 4
    wl = W.sphere_anisotropic(N=N, nk=2, m=4)
    A = yee.curl_matrix(N, k)
    B = yee.div_matrix(N, k)
    M = yee.eps_matrix(N, wl.ids, wl.table, scheme)
    g = yee.gamma_rule(k)
    e1 = np.linalg.eigvalsh((A @ M @ A.conj().T).toarray())
    e2 = np.linalg.eigvalsh((B.conj().T @ B).toarray())
    e3 = np.linalg.eigvalsh(yee.compensated_operator(N, k, wl.ids, wl.table, scheme).toarray())
    t1, t2, t3 = 1e-9 * e1.max(), 1e-9 * e2.max(), 1e-9 * e3.max()
    union = np.sort(np.concatenate([e1[e1 > t1], g * e2[e2 > t2]]))
    pos = np.sort(e3[e3 > t3])
    assert union.shape == pos.shape
    assert np.allclose(union, pos, rtol=1e-9, atol=1e-9 * e3.max())


@pytest.mark.parametrize("N", [4, 5, 6])
@pytest.mark.parametrize("k", KS)
def test_homogeneous_isotropic_dispersion(N, k):
    """Closed form from Lemma 2.1 and Prop 2.8: for eps^-1 = c I everywhere,
    spec(Op) = {c s(p) (twice), gamma s(p) (once)}, s(p) = sum_i kappa_i(q_i)^2 (all schemes)."""
    c = 1.0 / 13.0
    ids, tab = homog(N, np.eye(3) / c)
    g = yee.gamma_rule(k)
    s = s_of_p(N, k)
    ref = np.sort(np.concatenate([c * s, c * s, g * s]))
    for scheme in yee.SCHEMES:
        Op = yee.compensated_operator(N, k, ids, tab, scheme)
        ev = np.sort(np.linalg.eigvalsh(Op.toarray()))
        assert np.allclose(ev, ref, rtol=1e-10, atol=1e-10 * ref.max())


def lam0(th):
    return 0.5 * (1.0 + np.exp(-1j * th))


@pytest.mark.parametrize("scheme", ["trivial", "crossdof"])
@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (-1.1, 0.2, 2.9)])
def test_homogeneous_anisotropic_per_frequency(scheme, k):
    """Homogeneous anisotropic medium: F^H M F is block diagonal per frequency p.  Trivial:
    M_p = eps1; CrossDoF: off-diagonal (c,d) entries eps_cd * t_cd(p) with
    t_cd = lambda0(theta_c) conj(lambda0(theta_d)), lambda0(theta) = (1 + e^{-i theta})/2 (the
    symbols of D0 and D0^T by Lemma 2.1, with D0 on the row component's axis).  Op_p =
    K_A M_p K_A^H + gamma conj(K) K^T, K = i e^{-i theta/2} kappa."""
    N = 4
    rng = np.random.default_rng(5)
    eps = W.rotated_eps(rng, 4.0, 14.0) + np.array([[0, 0.7j, 0], [-0.7j, 0, 0.3j], [0, -0.3j, 0]])
    eps1 = np.linalg.inv(eps)
    eps1 = 0.5 * (eps1 + eps1.conj().T)
    ids, tab = homog(N, eps)
    g = yee.gamma_rule(k)
    Op = yee.compensated_operator(N, k, ids, tab, scheme)
    ev = np.sort(np.linalg.eigvalsh(Op.toarray()))
    th = 2 * math.pi * np.arange(N) / N
    ref = []
    for qz in range(N):
        for qy in range(N):
            for qx in range(N):
                q = (qx, qy, qz)
                K = np.array([1j * np.exp(-1j * th[q[a]] / 2) * kappa(N, k[a])[q[a]] for a in range(3)])
                KA = np.array([[0, -K[2], K[1]], [K[2], 0, -K[0]], [-K[1], K[0], 0]])
                Mp = eps1.copy()
                if scheme == "crossdof":
                    for c in range(3):
                        for d in range(c + 1, 3):
                            t = lam0(th[q[c]]) * np.conj(lam0(th[q[d]]))
                            Mp[c, d] = eps1[c, d] * t
                            Mp[d, c] = np.conj(Mp[c, d])
                v = K.conj()
                Opp = KA @ Mp @ KA.conj().T + g * np.outer(v, v.conj())
                ref.extend(np.linalg.eigvalsh(Opp))
    ref = np.sort(np.array(ref))
    assert np.allclose(ev, ref, rtol=1e-10, atol=1e-10 * ref.max())


@pytest.mark.parametrize("N", [4, 7])
@pytest.mark.parametrize("k", KS)
def test_symbols_match_lemma_2_1(N, k):
    """Lemma 2.1 / Prop 2.8: D_i F_col(q) = K_i(q) F_col(q) with K_i(q) = i e^{-i theta/2} kappa."""
    K = kspace.symbols_1d(N, k)
    th = 2 * math.pi * np.arange(N) / N
    for a in range(3):
        closed = 1j * np.exp(-1j * th / 2) * kappa(N, k[a])
        assert np.allclose(K[a], closed, atol=1e-12 * N)
    # plane-wave check on the 3D blocks
    D = yee.deriv_blocks(N, k)
    rng = np.random.default_rng(0)
    q = rng.integers(0, N, size=3)
    i = np.arange(N)
    kk, jj, ii = np.meshgrid(i, i, i, indexing="ij")
    om = 2 * math.pi / N
    f = np.exp(1j * om * (q[0] * ii + q[1] * jj + q[2] * kk)).ravel()
    for a in range(3):
        closed = 1j * np.exp(-1j * th[q[a]] / 2) * kappa(N, k[a])[q[a]]
        assert np.allclose(D[a] @ f, closed * f, atol=1e-10 * N)


@pytest.mark.parametrize("k", KS)
def test_kspace_apply_matches_symbol_form(k):
    """Prop 2.8 / eq (2.30) for eps^-1 = c I: F3^H Op F3 x = K x (c(-conj K x x)) + gamma
    conj(K) (K . x) per frequency, with the DFT convention of Lemma 2.1 (omega = e^{+2 pi i/N})."""
    N = 4
    c = 1.0 / 13.0
    ids, tab = homog(N, np.eye(3) / c)
    g = yee.gamma_rule(k)
    Op = yee.compensated_operator(N, k, ids, tab, "crossdof")
    x = W.random_block(3, 2, N)
    y = kspace.kspace_apply(Op, x, N)
    th = 2 * math.pi * np.arange(N) / N
    qz, qy, qx = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    q = [qx.ravel(), qy.ravel(), qz.ravel()]
    K = np.stack([1j * np.exp(-1j * th[q[a]] / 2) * kappa(N, k[a])[q[a]] for a in range(3)])
    v = K.conj()
    for b in range(2):
        xb = x[b]
        e = -np.cross(v.T, xb.T).T
        yy = np.cross(K.T, (c * e).T).T + g * v * (K * xb).sum(axis=0)[None, :]
        assert np.allclose(y[b], yy, atol=1e-11 * abs(yy).max())


def test_unitary_dft_convention():
    """Lemma 2.1: F_ab = omega^{ab}/sqrt(N), omega = e^{2 pi i/N}; F3 is unitary and F3H is its
    inverse."""
    N = 5
    u = W.random_block(0, 1, N)[0, 0]
    Fd = np.exp(2j * math.pi * np.outer(np.arange(N), np.arange(N)) / N) / math.sqrt(N)
    ref = np.einsum("ai,bj,ck,kji->cba", Fd, Fd, Fd, u.reshape(N, N, N)).ravel()
    assert np.allclose(kspace.F3(u[None], N)[0], ref, atol=1e-12)
    assert np.allclose(kspace.F3H(kspace.F3(u[None], N), N)[0], u, atol=1e-12)
    assert np.linalg.norm(kspace.F3(u[None], N)) == pytest.approx(np.linalg.norm(u), rel=1e-13)


@pytest.mark.parametrize("sign", [-1, 1])
@pytest.mark.parametrize("N", [2, 3, 4, 6, 8, 12, 16])
def test_direct_dft_vs_library(sign, N):
    """The direct DFT definition against numpy.fft (a library routine)."""
    u = W.random_block(N, 1, N)[0, 0, : 4 * N].reshape(4, N)
    ref = np.fft.fft(u, axis=-1) if sign < 0 else np.fft.ifft(u, axis=-1) * N
    assert np.allclose(kspace.direct_dft(u, sign), ref, atol=1e-12 * N)


@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (0.0, 0.0, 0.0), (0.5, 0.0, 0.0)])
def test_gamma_separates_spurious_spectrum(k):
    """Remark 2.6 with Lemma 2.4: with gamma from eq (2.26) the smallest nonzero eigenvalue of
    gamma B^H B is at least 4 pi^2 (normalised frequency 1), for k = 0 and k != 0."""
    N = 6
    B = yee.div_matrix(N, k)
    ev = np.linalg.eigvalsh((B.conj().T @ B).toarray())
    g = yee.gamma_rule(k)
    lam1 = ev[ev > 1e-9 * ev.max()].min()
    assert g * lam1 >= 4 * math.pi ** 2 * (math.sin(1.0) ** 2) - 1e-9
    if np.dot(k, k) > 0:
        assert g * lam1 >= 4 * math.pi ** 2 * (1 - 1e-12)
