"""Pins of the oracle's inverse-permittivity matrices (Section 3) and of the preconditioner."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import kspace, yee


def _tensor_assump31(rng, sdd=False, one_zero=False):
    """Random Hermitian inverse permittivity with eigenvalues in (0, 1] (Assumption 3.1)."""
    for _ in range(1000):
        G = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        Q, _ = np.linalg.qr(G)
        e = rng.uniform(0.05, 1.0, size=3)
        T = (Q * e[None, :]) @ Q.conj().T
        T = 0.5 * (T + T.conj().T)
        if one_zero:
            # rotate in the xy-plane only -> eps13 = eps23 = 0 (Assumption 3.3)
            c, s = math.cos(rng.uniform(0, 6.3)), math.sin(rng.uniform(0, 6.3))
            R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
            T = R @ np.diag(e) @ R.T + 0j
            T[0, 1] += 0.3j * min(e[0], e[1]) * 0.5
            T[1, 0] = np.conj(T[0, 1])
            if np.linalg.eigvalsh(T).min() <= 0 or np.linalg.eigvalsh(T).max() > 1:
                continue
        if sdd:
            d = np.real(np.diag(T))
            off = np.abs(T).sum(axis=1) - np.abs(np.diag(T))
            if not np.all(d > off):
                continue
        return T
    raise RuntimeError("no sample")


def _geom(N, T, rng):
    ids = W.sample_ids(N, [W.Sphere(rng.uniform(0, 1, 3), 0.31, 1), W.Rod(1, rng.uniform(0, 1, 3), 0.17, 1)])
    tab = np.stack([np.eye(3, dtype=complex), T])
    return ids, tab


@pytest.mark.parametrize("seed", range(4))
def test_eps_matrices_hermitian(seed):
    """Eq (3.8): M_CrossDoF is Hermitian by construction; so are M_Trivial and the diagonal one."""
    rng = np.random.default_rng(seed)
    N = 4
    T = _tensor_assump31(rng)
    ids, tab = _geom(N, T, rng)
    for scheme in yee.SCHEMES:
        M = yee.eps_matrix(N, ids, tab, scheme)
        assert abs(M - M.conj().T).max() == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_trivial_lower_bound(seed):
    """Prop 3.6: lambda_min(M_Trivial) >= lambda_min(eps1_hat), eps1_hat_ii = min(eps_ii, 1)."""
    rng = np.random.default_rng(100 + seed)
    N = 4
    T = _tensor_assump31(rng)
    ids, tab = _geom(N, T, rng)
    M = yee.eps_matrix(N, ids, tab, "trivial").toarray()
    That = T.copy()
    for i in range(3):
        That[i, i] = min(T[i, i].real, 1.0)
    assert np.linalg.eigvalsh(M).min() >= np.linalg.eigvalsh(That).min() - 1e-13


@pytest.mark.parametrize("seed", range(4))
def test_crossdof_S_norms(seed):
    """Prop 3.7: ||S_ij||_1, ||S_ij||_2, ||S_ij||_inf <= 1, S_ij = (I_i T_ij + T_ij I_j)/2."""
    rng = np.random.default_rng(200 + seed)
    N = 5
    T = _tensor_assump31(rng)
    ids, _ = _geom(N, T, rng)
    Tm = yee.transfer_matrices(N)
    for (c, d), Tcd in Tm.items():
        Ic = sp.diags((ids[c] == 1).astype(float))
        Id = sp.diags((ids[d] == 1).astype(float))
        S = (0.5 * (Ic @ Tcd + Tcd @ Id)).toarray()
        assert np.abs(S).sum(axis=0).max() <= 1 + 1e-14
        assert np.abs(S).sum(axis=1).max() <= 1 + 1e-14
        assert np.linalg.norm(S, 2) <= 1 + 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_crossdof_sdd_under_assumption_32(seed):
    """Prop 3.8: under Assumptions 3.1 and 3.2 M_CrossDoF is strictly diagonally dominant."""
    rng = np.random.default_rng(300 + seed)
    N = 4
    T = _tensor_assump31(rng, sdd=True)
    ids, tab = _geom(N, T, rng)
    M = yee.eps_matrix(N, ids, tab, "crossdof").toarray()
    d = np.real(np.diag(M))
    off = np.abs(M).sum(axis=1) - np.abs(np.diag(M))
    assert np.all(d > off)
    assert np.linalg.eigvalsh(M).min() > 0


@pytest.mark.parametrize("seed", range(4))
def test_crossdof_hpd_under_assumption_33(seed):
    """Prop 3.10: under Assumptions 3.1 and 3.3 M_CrossDoF is HPD."""
    rng = np.random.default_rng(400 + seed)
    N = 4
    T = _tensor_assump31(rng, one_zero=True)
    assert abs(T[0, 2]) == 0 and abs(T[1, 2]) == 0
    ids, tab = _geom(N, T, rng)
    M = yee.eps_matrix(N, ids, tab, "crossdof").toarray()
    assert np.linalg.eigvalsh(M).min() > 0


def test_crossdof_transfer_template():
    """Eq (3.5) (with its duplicated term read as E2_{i-1,j+1/2,k}): (T12 E2) at the x-edge
    (i-1/2, j, k) averages the y-edges at x in {i-1, i}, y in {j-1/2, j+1/2}.  Checked on
    point-evaluated linear fields: the average of a linear field over the four neighbours is
    the value at the x-edge (exact), which fixes both the neighbours and the directions."""
    N = 6
    Tm = yee.transfer_matrices(N)
    pts = {w: W.point_coords(N, w) for w in W.POINT_SETS}
    rng = np.random.default_rng(0)
    a = rng.standard_normal(3)
    # a linear function evaluated away from the periodic seam: use small slopes and check
    # only target points whose stencil does not cross the seam.
    for (c, d), T in Tm.items():
        src = pts[("ex", "ey", "ez")[d]]
        dst = pts[("ex", "ey", "ez")[c]]
        f = src @ a
        g = T @ f
        ok = np.all((dst > 1.5 / N) & (dst < 1 - 1.5 / N), axis=1)
        assert np.allclose(g[ok], (dst @ a)[ok], atol=1e-12)
        gt = T.T @ (dst @ a)
        ok2 = np.all((src > 1.5 / N) & (src < 1 - 1.5 / N), axis=1)
        assert np.allclose(gt[ok2], (src @ a)[ok2], atol=1e-12)


@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (0.0, 0.0, 0.0), (math.pi, math.pi, math.pi)])
def test_preconditioner_closed_form(k):
    """Eq (2.31): K_P = K_A K_A^H + gamma K_B = s I + (gamma - 1) v v^H with v = conj(K),
    s = |K|^2 (Lemma 2.4 (1) per frequency); its inverse by Sherman-Morrison is
    (1/s)(I - v v^H/s) + 1/(gamma s) v v^H/s.  The oracle's solve must agree; at the k = 0 DC
    frequency the output is zero."""
    N = 4
    g = yee.gamma_rule(k)
    r = W.random_block(7, 2, N)
    z = kspace.precond_apply(N, k, g, r)
    K = kspace.symbols_3d(N, k)
    v = K.conj()
    s = (abs(K) ** 2).sum(axis=0)
    for b in range(2):
        rb = r[b]
        vh_r = (v.conj() * rb).sum(axis=0)
        with np.errstate(divide="ignore", invalid="ignore"):
            zz = (rb - v * vh_r / s) / s + v * vh_r / (g * s * s)
        zz[:, s == 0] = 0.0
        assert np.allclose(z[b], zz, atol=1e-12 * abs(zz).max())


@pytest.mark.parametrize("scheme", ["trivial", "crossdof"])
@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (-1.0, 2.0, 0.4)])
def test_preconditioned_rayleigh_bound(scheme, k):
    """Prop 2.9: the Rayleigh quotient of the preconditioned pencil (Op, F3 K_P F3^H) lies in the
    range of the spectrum of M (and of the identity, which the penalty term contributes)."""
    N = 4
    rng = np.random.default_rng(11)
    T = _tensor_assump31(rng, sdd=True)
    ids, tab = _geom(N, T, rng)
    g = yee.gamma_rule(k)
    Op = yee.compensated_operator(N, k, ids, tab, scheme).toarray()
    M = yee.eps_matrix(N, ids, tab, scheme).toarray()
    evM = np.linalg.eigvalsh(M)
    lo, hi = min(evM.min(), 1.0), max(evM.max(), 1.0)
    # P = F3 K_P F3^H assembled column by column through the oracle's preconditioner inverse
    n = 3 * N ** 3
    E = np.eye(n, dtype=complex).reshape(n, 3, N ** 3)
    Pinv_k = kspace.precond_apply(N, k, g, E).reshape(n, n).T  # columns = K_P^{-1} e_j
    Fm = kspace.F3(np.eye(n, dtype=complex).reshape(n, 3, N ** 3), N).reshape(n, n).T
    Pinv = Fm @ Pinv_k @ Fm.conj().T
    Pinv = 0.5 * (Pinv + Pinv.conj().T)
    # generalized eigenvalues of (Op, P) = eigenvalues of P^{-1/2} Op P^{-1/2}
    wP, VP = np.linalg.eigh(Pinv)
    Ph = (VP * np.sqrt(wP)[None, :]) @ VP.conj().T
    ev = np.linalg.eigvalsh(Ph @ Op @ Ph)
    assert ev.min() >= lo - 1e-10 and ev.max() <= hi + 1e-10


@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (0.0, 0.0, 0.0), (math.pi, math.pi, math.pi)])
def test_transverse_precond_unit_field_is_kp_inverse(k):
    """T_E with E = 1 is the pseudo-inverse of K_A K_A^H plus that of gamma K_B; the two ranges
    are orthogonal (K_B K_A = 0, Lemma 2.4), so the sum is K_P^{-1} of eq (2.32), zero at the
    k = 0 DC frequency."""
    N = 4
    g = yee.gamma_rule(k)
    r = W.random_block(8, 2, N)
    z = kspace.transverse_precond_apply(N, k, g, np.ones((3, N ** 3)), r)
    ref = kspace.precond_apply(N, k, g, r)
    assert np.allclose(z, ref, atol=1e-11 * abs(ref).max())


@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (-1.1, 0.2, 2.9)])
def test_transverse_precond_inverts_homogeneous_operator(k):
    """Homogeneous isotropic medium eps = e I: Op = (1/e) K_A K_A^H + gamma K_B in k-space, so
    T_E with E = e (the classical field 1/(eps^-1)_cc) is its exact inverse; checked as
    T_E Op x = x on random vectors, with Op the sparse operator conjugated by the DFT."""
    N = 4
    e = 9.0
    ids = np.ones((4, N ** 3), dtype=np.uint8)
    tab = W.eps_table([e * np.eye(3)])
    g = yee.gamma_rule(k)
    E0 = kspace.edge_permittivity(ids, tab)
    assert np.allclose(E0, e)
    Op = yee.compensated_operator(N, k, ids, tab, "crossdof")
    x = W.random_block(9, 2, N)
    y = kspace.kspace_apply(Op, x, N)
    z = kspace.transverse_precond_apply(N, k, g, E0, y)
    assert np.allclose(z, x, atol=1e-10 * abs(x).max())


@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (0.0, 0.0, 0.0)])
def test_transverse_precond_hermitian_psd(k):
    """For a positive field T_E is Hermitian positive semi-definite; its null space is the
    k = 0 DC frequency only (three vectors at k = 0, none otherwise)."""
    N = 3
    rng = np.random.default_rng(5)
    E = rng.uniform(1.0, 14.0, size=(3, N ** 3))
    g = yee.gamma_rule(k)
    n = 3 * N ** 3
    I = np.eye(n, dtype=complex).reshape(n, 3, N ** 3)
    T = kspace.transverse_precond_apply(N, k, g, E, I).reshape(n, n).T
    assert np.allclose(T, T.conj().T, atol=1e-12 * abs(T).max())
    ev = np.linalg.eigvalsh(0.5 * (T + T.conj().T))
    assert ev.min() > -1e-12 * ev.max()
    nz = int(np.sum(ev < 1e-10 * ev.max()))
    assert nz == (3 if np.allclose(k, 0) else 0)


def test_edge_permittivity_reads_edge_points():
    """E0_c comes from the material at the c-edge points, and is the reciprocal of the
    diagonal entry of the stored inverse tensor (not the diagonal of the tensor's inverse)."""
    N = 2
    T = np.array([[10.0, 2.0, 0.0], [2.0, 6.0, 0.0], [0.0, 0.0, 4.0]])
    tab = W.eps_table([T])
    ids = np.zeros((4, N ** 3), dtype=np.uint8)
    ids[1, 3] = 1  # one y-edge point inside material 1
    E0 = kspace.edge_permittivity(ids, tab)
    inv = np.linalg.inv(T)
    assert E0[1, 3] == pytest.approx(1.0 / inv[1, 1])
    assert np.allclose(np.delete(E0[1], 3), 1.0) and np.allclose(E0[0], 1.0) and np.allclose(E0[2], 1.0)
