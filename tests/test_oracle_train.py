"""Pins of the training quantities of the learned preconditioner (oracle.train), against facts
that do not use them: the closed-form inverse of the operator in a homogeneous isotropic medium,
the extremal property of the Rayleigh quotient, the orthogonality of the perturbation, and a
direct scan over the scale alpha."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import kspace, train, yee


def _homogeneous(N, eps):
    ids = np.zeros((4, N ** 3), dtype=np.uint8)
    tab = W.eps_table([np.eye(3) * eps])
    ids[:] = 1
    return ids, tab


def test_solve_is_the_transverse_inverse_in_a_homogeneous_medium():
    """With eps constant and isotropic, Op = (1/eps) K_A K_A^H + gamma K_B per frequency, whose
    inverse is eps K_A^{+H} K_A^{+} + (gamma K_B)^{+}: T_E with E = eps (Lemma 2.4: the two parts
    act on orthogonal subspaces).  The sparse direct solve must agree with that pseudo-inverse."""
    N, eps = 6, 4.0
    k = np.array([0.7, -0.4, 1.1])
    ids, tab = _homogeneous(N, eps)
    g = yee.gamma_rule(k)
    Op = yee.compensated_operator(N, k, ids, tab, "crossdof", gamma=g)
    r = W.random_block(3, 2, N)
    c = train.solve(Op, r, N)
    ref = kspace.transverse_precond_apply(N, k, g, np.full((3, N ** 3), eps), r)
    assert np.abs(c - ref).max() <= 1e-10 * np.abs(ref).max()


def test_perturbed_residuals_properties():
    """x - X is orthogonal to span(X) with length amp_j; r_j is orthogonal to x_j (theta_j is the
    Rayleigh quotient); amp = 0 on exact eigenvectors gives r = 0."""
    N = 4
    wl = W.sphere_anisotropic(N=N, nk=2, m=4)
    k = wl.kpoints[1]
    g = yee.gamma_rule(k)
    Op = yee.compensated_operator(N, k, wl.ids, wl.table, "crossdof", gamma=g)
    # exact eigenvectors of the k-space operator (dense)
    n = 3 * N ** 3
    I = np.eye(n, dtype=np.complex128).reshape(n, 3, N ** 3)
    Ok = kspace.kspace_apply(Op, I, N).reshape(n, n).T
    lam, V = np.linalg.eigh(0.5 * (Ok + Ok.conj().T))
    sel = np.nonzero(lam > 1e-8)[0][:3]
    X = V[:, sel].T.reshape(3, 3, N ** 3)
    noise = W.random_block(5, 3, N)
    amp = np.array([0.05, 0.2, 0.0])
    x, theta, r = train.perturbed_residuals(N, k, g, Op, X, noise, amp)
    d = (x - X).reshape(3, -1)
    Q = X.reshape(3, -1)
    assert np.abs(Q.conj() @ d.T).max() <= 1e-12
    assert np.allclose(np.linalg.norm(d, axis=1), amp, atol=1e-12)
    for j in range(3):
        assert abs(np.vdot(x[j], r[j])) <= 1e-10 * np.linalg.norm(r[j]) * np.linalg.norm(x[j]) + 1e-14 * lam.max()
    assert np.linalg.norm(r[2]) <= 1e-9 * lam[sel[2]]
    assert theta[2] == pytest.approx(lam[sel[2]], rel=1e-12)


@pytest.mark.parametrize("kind", ["energy", "euclidean"])
def test_misfit_is_the_minimum_over_alpha(kind):
    """The value at the closed-form alpha is the minimum of a direct scan over alpha, lies in
    [0, 1], and vanishes when z is a multiple of c."""
    N = 4
    wl = W.sphere_anisotropic(N=N, nk=2, m=4)
    k = wl.kpoints[1]
    Op = yee.compensated_operator(N, k, wl.ids, wl.table, "crossdof")
    r = W.random_block(7, 2, N)
    c = train.solve(Op, r, N)
    zn = W.random_block(8, 2, N)
    z = zn * (np.linalg.norm(c) / np.linalg.norm(zn)) + 0.5 * c  # the optimal alpha is O(1)
    val = train.misfit(Op, r, c, z, N, kind)
    assert np.all((val >= 0) & (val <= 1))
    for j in range(2):
        if kind == "energy":
            nrm = lambda v: np.vdot(v, kspace.kspace_apply(Op, v[None], N)[0]).real  # noqa: E731
        else:
            nrm = lambda v: np.vdot(v, v).real  # noqa: E731
        scan = min(nrm(a * z[j] - c[j]) / nrm(c[j]) for a in np.linspace(-3, 3, 6001))
        assert val[j] <= scan + 1e-12 and val[j] >= scan - 1e-5
    assert np.abs(train.misfit(Op, r, c, -2.5 * c, N, kind)).max() <= 1e-12


def test_field_loss_vanishes_for_the_exact_field_of_a_homogeneous_medium():
    """In a homogeneous isotropic medium T_E with E = eps is Op^{-1}, so z = c and both misfits
    are zero; another field gives a positive misfit."""
    N, eps = 4, 6.0
    k = np.array([0.9, 0.3, -0.5])
    ids, tab = _homogeneous(N, eps)
    g = yee.gamma_rule(k)
    Op = yee.compensated_operator(N, k, ids, tab, "crossdof", gamma=g)
    r = W.random_block(9, 2, N)
    c = train.solve(Op, r, N)
    E = np.full((3, N ** 3), eps)
    for kind in ("energy", "euclidean"):
        assert train.field_loss(N, k, g, E, Op, r, c, kind) <= 1e-12
        Eb = E * np.exp(0.3 * np.sin(np.arange(N ** 3) * 0.7))[None]
        assert train.field_loss(N, k, g, Eb, Op, r, c, kind) > 1e-4
