"""Pins of WHERE the oracle samples the inverse permittivity, of the penalty rule and of the
domain in which the transverse preconditioner applies its field.

Every closed-form pin of the operator uses a homogeneous medium, where the sampling point of
a coefficient cannot matter.  The pins below use media that vary in space, so that a
coefficient read at the wrong Yee point (edge instead of volume, one edge set instead of
another) changes the result:

* a layered medium (the inverse permittivity depends on one coordinate only) reduces the 3D
  operator, on fields constant across the layers, to a 1D operator whose coefficients are read
  at the Yee positions of Section 2.1 (edges at integer, volume centres at half-integer
  coordinates along the layering axis);
* the CrossDoF entries near an interface (Section 3, eq (3.8)) are fixed by which of the two
  coupled edge points lies inside the inclusion;
* the Yee grid is mapped onto itself by a mirror plane, so the diagonal and CrossDoF operators
  of a mirrored structure have the same spectrum (Trivial, eq (3.4), pairs DoFs by index and
  is not mirror-covariant);
* eq (2.26) is eq (2.25) with the bound 4 pi^2 on the wanted eigenvalues (Remark 2.6);
* a real-space field commutes with a one-cell translation as the translation's phase
  (Lemma 2.1).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import kspace, yee


def _herm_tensor(rng):
    """Hermitian tensor with eigenvalues in (0, 1] and nonzero complex off-diagonals."""
    G = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    Q, _ = np.linalg.qr(G)
    e = rng.uniform(0.1, 1.0, size=3)
    T = (Q * e[None, :]) @ Q.conj().T
    return 0.5 * (T + T.conj().T)


# --- layered medium ------------------------------------------------------------------------

def _d1d(N, kk):
    """1D Bloch difference along the layering axis: (u_j - u_{j-1})/h + i kk (u_j + u_{j-1})/2."""
    h = 1.0 / N
    d = np.zeros((N, N), dtype=np.complex128)
    for j in range(N):
        d[j, j] += 1.0 / h + 0.5j * kk
        d[j, (j - 1) % N] += -1.0 / h + 0.5j * kk
    return d


def _layer_embedding(N, a):
    """3N^3 x 3N isometry: the 1D profile u (index j along axis a) of each component, spread
    uniformly over the two other axes (value u_j / N at every grid index whose a-th index is j)."""
    n3 = N ** 3
    p = np.arange(n3)
    idx = [p % N, (p // N) % N, p // (N * N)]   # x fastest
    rows, cols = [], []
    for c in range(3):
        rows.append(c * n3 + p)
        cols.append(c * N + idx[a])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    return sp.csr_matrix((np.full(rows.size, 1.0 / N), (rows, cols)), shape=(3 * n3, 3 * N))


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("scheme", ["diagonal", "trivial", "crossdof"])
def test_layered_medium_reduces_to_1d(axis, scheme):
    """Layer lo <= t < hi of a Hermitian inverse permittivity along axis a, air elsewhere, Bloch
    vector along a.  On fields constant in the two other directions, A, B and M (eqs (2.7),
    (3.3), (3.4), (3.8)) act through the 1D difference along a only, so P^H Op P must be
    A1 M1 A1^H + gamma B1^H B1 with A1, B1 built from that 1D difference alone and M1 holding,
    for the two components b, c != a:
      * (eps^-1)_bb, (eps^-1)_cc at the b- and c-edge points, which sit at the integer positions
        j h along a (the half-cell offset of an edge point is along its own axis);
      * the (b, c) coupling at the volume points (j - 1/2) h for Trivial (eq (3.4)), and for
        CrossDoF at j h: both coupled edge points lie at j h, and the transfer matrix averages
        only across the layers, where the field is constant (eq (3.8)).
    The layer edges 0.3 and 0.6 put some integer and half-integer positions on different sides,
    so a coefficient read at the wrong point set changes M1."""
    rng = np.random.default_rng(40 + axis)
    N = 8
    h = 1.0 / N
    lo, hi = 0.3, 0.6
    T = _herm_tensor(rng)
    ids = W.sample_ids(N, [W.Slab(axis, lo, hi, 1)])
    tab = np.stack([np.eye(3, dtype=np.complex128), T])
    kk = 0.7
    k = np.zeros(3)
    k[axis] = kk
    gamma = 5.0
    Op = yee.compensated_operator(N, k, ids, tab, scheme, gamma=gamma)

    def inside(t):
        t = t % 1.0
        return lo <= t < hi

    def coef(b, c, t):
        return T[b, c] if inside(t) else (1.0 if b == c else 0.0)

    edge_t = [j * h for j in range(N)]             # b-edge points, b != axis
    vol_t = [(j - 0.5) * h for j in range(N)]      # volume centres
    others = [b for b in range(3) if b != axis]
    M1 = np.zeros((3 * N, 3 * N), dtype=np.complex128)
    for b in others:
        M1[b * N:(b + 1) * N, b * N:(b + 1) * N] = np.diag([coef(b, b, t) for t in edge_t])
    b, c = others
    if scheme != "diagonal":
        pts = vol_t if scheme == "trivial" else edge_t
        U = np.diag([coef(b, c, t) for t in pts])
        M1[b * N:(b + 1) * N, c * N:(c + 1) * N] = U
        M1[c * N:(c + 1) * N, b * N:(b + 1) * N] = U.conj().T
    D = [np.zeros((N, N), dtype=np.complex128) for _ in range(3)]
    D[axis] = _d1d(N, kk)
    Z = np.zeros((N, N), dtype=np.complex128)
    A1 = np.block([[Z, -D[2], D[1]], [D[2], Z, -D[0]], [-D[1], D[0], Z]])
    B1 = np.hstack(D)
    ref = A1 @ M1 @ A1.conj().T + gamma * B1.conj().T @ B1

    P = _layer_embedding(N, axis)
    red = (P.T @ (Op @ P)).toarray()
    assert np.abs(red - ref).max() <= 1e-12 * np.abs(ref).max()
    # the subspace is invariant: Op P = P (P^H Op P)
    OpP = (Op @ P).toarray()
    assert np.abs(OpP - P @ ref).max() <= 1e-12 * np.abs(ref).max()


def test_layered_medium_schemes_differ():
    """The check above can tell the schemes apart: with the layer edges between integer and
    half-integer points the Trivial and CrossDoF couplings differ on the same layered medium."""
    rng = np.random.default_rng(41)
    N = 8
    T = _herm_tensor(rng)
    ids = W.sample_ids(N, [W.Slab(2, 0.3, 0.6, 1)])
    tab = np.stack([np.eye(3, dtype=np.complex128), T])
    k = np.array([0.0, 0.0, 0.7])
    a = yee.compensated_operator(N, k, ids, tab, "trivial", gamma=5.0)
    b = yee.compensated_operator(N, k, ids, tab, "crossdof", gamma=5.0)
    P = _layer_embedding(N, 2)
    assert np.abs((P.T @ (a - b) @ P).toarray()).max() > 1e-3


# --- CrossDoF entries at an interface ------------------------------------------------------

def _edge_position(N, c, p):
    """Yee position of the c-edge DoF with linear index p = i + N j + N^2 k (Section 2.1):
    the index coordinates times h, shifted by -h/2 along axis c."""
    i, j, k = p % N, (p // N) % N, p // (N * N)
    pos = np.array([i, j, k], dtype=np.float64) / N
    pos[c] -= 0.5 / N
    return pos % 1.0


def _min_image(d):
    return d - np.round(d)


@pytest.mark.parametrize("seed", range(3))
def test_crossdof_interface_entries(seed):
    """eq (3.8) with the indicator matrices of eq (3.2): block (c, d), c < d, is
    eps_cd (I_c T_cd + T_cd I_d) / 2 and T_cd averages the four d-edge points around a c-edge
    point.  Hence entry (P, S) is eps_cd / 8 * ([c-edge P inside] + [d-edge S inside]) when the
    d-edge point S is one of the four at distance h / sqrt(2) from the c-edge point P in the
    (c, d) plane, and zero otherwise.  Positions and membership are evaluated here from the
    geometry, independently of the material ids the oracle reads."""
    rng = np.random.default_rng(70 + seed)
    N = 5
    n3 = N ** 3
    T = _herm_tensor(rng)
    sph = W.Sphere(rng.uniform(0, 1, 3), 0.33, 1)
    ids = W.sample_ids(N, [sph])
    tab = np.stack([np.eye(3, dtype=np.complex128), T])
    M = yee.eps_matrix(N, ids, tab, "crossdof").toarray()
    h = 1.0 / N
    pos = [np.stack([_edge_position(N, c, p) for p in range(n3)]) for c in range(3)]
    ins = [sph.contains(pos[c]) for c in range(3)]
    n_mixed = 0
    for c in range(3):
        # diagonal blocks: (eps^-1)_cc at the c-edge point (eq (3.3))
        diag_ref = np.where(ins[c], T[c, c].real, 1.0)
        assert np.allclose(np.diag(M[c * n3:(c + 1) * n3, c * n3:(c + 1) * n3]), diag_ref,
                           rtol=0, atol=1e-15)
        for d in range(c + 1, 3):
            e = 3 - c - d
            blk = M[c * n3:(c + 1) * n3, d * n3:(d + 1) * n3]
            ref = np.zeros((n3, n3), dtype=np.complex128)
            for P in range(n3):
                dv = _min_image(pos[d] - pos[c][P])
                near = (np.abs(np.abs(dv[:, c]) - 0.5 * h) < 1e-12) & \
                       (np.abs(np.abs(dv[:, d]) - 0.5 * h) < 1e-12) & (np.abs(dv[:, e]) < 1e-12)
                assert near.sum() == 4
                ref[P, near] = T[c, d] / 8.0 * (float(ins[c][P]) + ins[d][near].astype(float))
                n_mixed += int(np.sum(ins[d][near] != ins[c][P]))
            assert np.abs(blk - ref).max() <= 1e-15
    assert n_mixed > 0  # the sphere cuts some stencils, so the interface rule is exercised


# --- mirror covariance ---------------------------------------------------------------------

@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("scheme", ["diagonal", "crossdof"])
def test_mirror_covariance(axis, scheme):
    """The mirror t -> -t along one axis maps the Yee grid onto itself (edge points to edge
    points of the same orientation, Section 2.1), the permittivity to R eps R and the Bloch
    vector to R k, R = diag(+-1).  The diagonal (eq (3.3)) and CrossDoF (eq (3.8)) matrices are
    built from positions only, so the mirrored structure has the same spectrum.  An asymmetric
    off-centre inclusion makes a coefficient read half a cell off the correct point break this."""
    rng = np.random.default_rng(90 + axis)
    N = 4
    T = _herm_tensor(rng)
    tab = np.stack([np.eye(3, dtype=np.complex128), T])
    ctr = np.array([0.31, 0.42, 0.23])
    r = 0.33
    k = np.array([0.4, -0.9, 0.6])
    R = np.eye(3)
    R[axis, axis] = -1.0
    cm = ctr.copy()
    cm[axis] = (1.0 - cm[axis]) % 1.0
    ids = W.sample_ids(N, [W.Sphere(ctr, r, 1)])
    idsm = W.sample_ids(N, [W.Sphere(cm, r, 1)])
    tabm = np.stack([R @ t @ R for t in tab])
    a = np.linalg.eigvalsh(yee.compensated_operator(N, k, ids, tab, scheme, gamma=7.0).toarray())
    b = np.linalg.eigvalsh(yee.compensated_operator(N, R @ k, idsm, tabm, scheme,
                                                    gamma=7.0).toarray())
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_trivial_is_not_mirror_covariant():
    """Trivial pairs the DoFs of equal index (eq (3.4)), which sit at different places, so the
    mirror test above has power: it fails for Trivial on the same structure."""
    rng = np.random.default_rng(90)
    N = 4
    T = _herm_tensor(rng)
    tab = np.stack([np.eye(3, dtype=np.complex128), T])
    ctr, r, k = np.array([0.31, 0.42, 0.23]), 0.33, np.array([0.4, -0.9, 0.6])
    R = np.diag([-1.0, 1.0, 1.0])
    cm = ctr.copy()
    cm[0] = 1.0 - cm[0]
    a = np.linalg.eigvalsh(yee.compensated_operator(
        N, k, W.sample_ids(N, [W.Sphere(ctr, r, 1)]), tab, "trivial", gamma=7.0).toarray())
    b = np.linalg.eigvalsh(yee.compensated_operator(
        N, R @ k, W.sample_ids(N, [W.Sphere(cm, r, 1)]), np.stack([R @ t @ R for t in tab]),
        "trivial", gamma=7.0).toarray())
    assert np.abs(a - b).max() > 1e-6 * np.abs(a).max()


# --- penalty rule --------------------------------------------------------------------------

def test_gamma_rule_is_the_sufficient_rule_at_its_bound():
    """Prop 2.5 (2), eq (2.25): gamma = max{1, lam_m} * max{1, |k|^-2} (k != 0) and
    max{1, lam_m} (k = 0) suffices; Remark 2.6 bounds lam_m by 4 pi^2, which gives eq (2.26).
    Checked on both sides of |k| = 1 and at k = 0."""
    lam_bound = 4.0 * math.pi ** 2
    rng = np.random.default_rng(5)
    ks = [np.zeros(3), np.array([1.0, 0.0, 0.0])]
    for scale in (0.05, 0.3, 0.8, 0.999, 1.001, 1.7, 3.0, 5.4):
        v = rng.standard_normal(3)
        ks.append(scale * v / np.linalg.norm(v))
    for k in ks:
        kn2 = float(k @ k)
        ref = max(1.0, lam_bound) * (1.0 if kn2 == 0.0 else max(1.0, 1.0 / kn2))
        assert abs(yee.gamma_rule(k) - ref) <= 1e-12 * ref, (k, yee.gamma_rule(k), ref)


def test_gamma_values():
    """eq (2.26) at two points: k = 2 pi (0.1, 0.2, 0.3) (|k| = 2.351 > 1) gives 4 pi^2 = 39.478;
    k = (0.5, 0, 0) gives 4 pi^2 / 0.25 = 16 pi^2 = 157.91."""
    k1 = 2.0 * math.pi * np.array([0.1, 0.2, 0.3])
    assert abs(yee.gamma_rule(k1) - 39.47841760435743) < 1e-12
    assert abs(yee.gamma_rule(np.array([0.5, 0.0, 0.0])) - 157.91367041742973) < 1e-10


# --- transverse preconditioner: the field acts in real space -------------------------------

@pytest.mark.parametrize("shift_axis", [0, 1, 2])
def test_transverse_precond_translation_covariance(shift_axis):
    """A one-cell translation S of real-space fields is, on k-space coefficients, the diagonal
    phase S_hat = F3^H S F3 (Lemma 2.1), which commutes with every per-frequency 3x3 block
    (K_A^+, K_B).  A field E applied in real space therefore satisfies
    T_{S E} = S_hat T_E S_hat^H; a field applied to k-space coefficients would not."""
    N = 6
    rng = np.random.default_rng(11 + shift_axis)
    k = np.array([0.3, -0.5, 0.8])
    gamma = yee.gamma_rule(k)
    E = rng.uniform(0.5, 3.0, size=(3, N ** 3))
    r = W.random_block(12 + shift_axis, 2, N)
    ax = 2 - shift_axis  # numpy axis of (z, y, x) arrays

    def roll(v):
        s = v.shape[:-1]
        return np.roll(v.reshape(s + (N, N, N)), 1, axis=len(s) + ax).reshape(v.shape)

    def S_hat(v):
        return kspace.F3H(roll(kspace.F3(v, N)), N)

    def S_hat_H(v):
        s = v.shape[:-1]
        back = np.roll(kspace.F3(v, N).reshape(s + (N, N, N)), -1, axis=len(s) + ax).reshape(v.shape)
        return kspace.F3H(back, N)

    z1 = kspace.transverse_precond_apply(N, k, gamma, roll(E), r)
    z2 = S_hat(kspace.transverse_precond_apply(N, k, gamma, E, S_hat_H(r)))
    assert np.abs(z1 - z2).max() <= 1e-12 * np.abs(z2).max()
    # and the field is not translation invariant, so the check has power
    z3 = kspace.transverse_precond_apply(N, k, gamma, E, r)
    assert np.abs(z1 - z3).max() > 1e-3 * np.abs(z3).max()
