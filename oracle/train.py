"""Training quantities of the learned preconditioner, from their definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component.  These functions follow the design chosen for it: T_E is
the transverse-projection preconditioner with a per-cell field E (kspace.transverse_precond_apply)
and the network predicts E; its training inputs are residuals of perturbed eigenvector
iterates, its targets the exact corrections Op^{-1} r, and its loss the scale-free misfit of
T_E r against that target.  Everything is dense or explicit-sparse FP64 on small grids: the
operator is the explicit matrix of eq (2.13) (oracle.yee) conjugated by the unitary DFT
(Prop 2.8, eq (2.30)), the linear solve a sparse direct factorisation, the norms and inner
products plain numpy.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import scipy.sparse.linalg as spla

from . import kspace


def solve(Op, r: np.ndarray, N: int) -> np.ndarray:
    """c = F3^H Op^{-1} F3 r for a block r (nvec, 3, N^3): the exact correction of each residual
    (Op is Hermitian positive definite away from k = 0, Prop 2.3 with Remark 2.6)."""
    r = np.asarray(r, dtype=np.complex128)
    R = kspace.F3(r, N).reshape(r.shape[0], -1).T
    lu = spla.splu(Op.tocsc())
    Cm = lu.solve(R)
    return kspace.F3H(Cm.T.reshape(r.shape), N)


def perturbed_residuals(N: int, k: Sequence[float], gamma: float, Op, X: np.ndarray, noise: np.ndarray,
                        amp: np.ndarray, m: int = 1, lattice=None):
    """Training inputs of one k-point.  With X (nvec, 3, N^3) orthonormal k-space vectors:
    e = K_P^{-1} noise (eqs (2.31)-(2.32)), made orthogonal to span(X) by subtracting its
    orthogonal projection and scaled to unit length; x_j = X_j + amp_j e_j; theta_j the
    Rayleigh quotient <x_j, Op x_j> / <x_j, x_j>; r_j = Op x_j - theta_j x_j.
    Returns (x, theta, r)."""
    X = np.asarray(X, dtype=np.complex128)
    nv = X.shape[0]
    e = kspace.precond_apply(N, k, gamma, noise, m=m, lattice=lattice).reshape(nv, -1)
    Q = X.reshape(nv, -1)
    for j in range(nv):
        for i in range(nv):
            e[j] = e[j] - np.vdot(Q[i], e[j]) * Q[i]
        e[j] = e[j] / np.linalg.norm(e[j])
    x = (Q + np.asarray(amp, dtype=np.float64)[:, None] * e).reshape(X.shape)
    Ax = kspace.kspace_apply(Op, x, N)
    theta = np.array([np.vdot(x[j], Ax[j]).real / np.vdot(x[j], x[j]).real for j in range(nv)])
    r = Ax - theta[:, None, None] * x
    return x, theta, r


def misfit(Op, r: np.ndarray, c: np.ndarray, z: np.ndarray, N: int, kind: str = "energy") -> np.ndarray:
    """Scale-free misfit of each direction z_j against its target c_j, as the minimum over a
    real scale alpha:
        energy:    min_alpha |alpha z - c|_Op^2 / |c|_Op^2   (|v|_Op^2 = <v, Op v>)
        euclidean: min_alpha |alpha z - c|^2 / |c|^2
    The minimiser is alpha = Re<z, c>_W / <z, z>_W in the chosen inner product W; the value is
    evaluated at that alpha from the definition."""
    r = np.asarray(r, dtype=np.complex128)
    out = np.zeros(r.shape[0])
    for j in range(r.shape[0]):
        if kind == "energy":
            ip = lambda a, b: np.vdot(a, kspace.kspace_apply(Op, b[None], N)[0]).real  # noqa: E731
        else:
            ip = lambda a, b: np.vdot(a, b).real  # noqa: E731
        alpha = ip(z[j], c[j]) / ip(z[j], z[j])
        d = alpha * z[j] - c[j]
        out[j] = ip(d, d) / ip(c[j], c[j])
    return out


def field_loss(N: int, k: Sequence[float], gamma: float, E: np.ndarray, Op, r: np.ndarray, c: np.ndarray,
               kind: str = "energy") -> float:
    """Mean misfit of z = T_E r over the residuals of one k-point, as a function of the field E
    (3, N^3): the loss whose gradient trains the network."""
    z = kspace.transverse_precond_apply(N, k, gamma, E, r)
    return float(misfit(Op, r, c, z, N, kind).mean())
