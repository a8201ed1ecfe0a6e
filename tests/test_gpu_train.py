"""Training calls of the learned preconditioner (kc_pcg, kc_perturbed_residuals,
kc_net_loss_grad) through the C ABI against the oracle's definitions (oracle.train)."""
import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W
from oracle import train, yee

from gpu_util import note, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

N = 8
NNET = 16  # the network needs N % 16 == 0


def _setup(N=N):
    wl = W.sphere_anisotropic(N=N, nk=9, m=6)
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints[3:5])
    g = op.gamma()
    Op = [yee.compensated_operator(N, wl.kpoints[3 + i], wl.ids, wl.table, "crossdof", gamma=g[i]) for i in range(2)]
    return wl, op, g, Op


def _rand_net(seed, scale):
    net = kc.Net(seed=seed)
    rng = np.random.default_rng(seed)
    net.set_params((scale * rng.standard_normal(kc.Net.param_count())).astype(np.float32))
    return net


def test_pcg_matches_direct_solve():
    """c = Op^{-1} r for three vectors against a sparse direct factorisation of the explicit
    operator, at the second k-point of the handle."""
    wl, op, g, Op = _setup()
    r = W.random_block(11, 3, N)
    note("pcg")
    c, its, ok = op.pcg(to_dev(r), ik=1, tol=1e-12, maxit=3000)
    assert ok and 1 <= its < 3000
    ref = train.solve(Op[1], r, N)
    assert rel_err(to_host(c), ref) < 1e-9


def test_pcg_zero_right_hand_side():
    """A zero r_j gives c_j = 0 and does not hold back the others."""
    wl, op, g, Op = _setup()
    r = W.random_block(16, 3, N)
    r[1] = 0.0
    c, its, ok = op.pcg(to_dev(r), ik=0, tol=1e-11, maxit=3000)
    c = to_host(c)
    assert ok and np.all(c[1] == 0.0)
    ref = train.solve(Op[0], r, N)
    assert rel_err(c, ref) < 1e-8


def test_pcg_reports_no_convergence():
    wl, op, g, Op = _setup()
    r = W.random_block(12, 2, N)
    c, its, ok = op.pcg(to_dev(r), ik=0, tol=1e-14, maxit=3)
    assert not ok and its == 3


def test_perturbed_residuals_match_oracle():
    """x = X + amp e with e = K_P^{-1} noise projected off span(X) and normalised; r = Op x -
    theta x with the Rayleigh quotient theta; element by element against the oracle."""
    wl, op, g, Op = _setup()
    m = 4
    A = W.random_block(13, m, N).reshape(m, -1).T
    Q, _ = np.linalg.qr(A)
    X = Q.T.reshape(m, 3, N ** 3).copy()
    noise = W.random_block(14, m, N)
    amp = np.array([0.02, 0.1, 0.25, 0.3])
    note("perturbed residuals")
    x, r = op.perturbed_residuals(to_dev(X), to_dev(noise), amp, ik=0)
    xr, th, rr = train.perturbed_residuals(N, wl.kpoints[3], g[0], Op[0], X, noise, amp)
    assert rel_err(to_host(x), xr) < 1e-12
    assert rel_err(to_host(r), rr) < 1e-10


@pytest.mark.parametrize("kind", ["energy", "euclidean"])
def test_net_loss_and_gradient_match_oracle(kind):
    """The mean misfit of T_E r (E: the network's field) against the oracle's misfit with the same
    field; the gradient with respect to the network output against central differences of the
    oracle's loss along E -> E exp(t d) (every |y| < 3 here, so no clamp is active)."""
    import torch

    N = NNET
    wl, op, g, Op = _setup(N)
    net = _rand_net(23, 0.03)
    op.attach_net(net)
    m = 3
    r = W.random_block(15, m, N)
    c = train.solve(Op[1], r, N)
    note("net loss", kind)
    loss, gout = op.net_loss_grad(to_dev(r), to_dev(c), ik=1, kind=kind, grad=True, scale=2.0)
    E = to_host(op.net_efield(ik0=1, nk=1))[0].astype(np.float64)
    ref = train.field_loss(N, wl.kpoints[4], g[1], E, Op[1], r, c, kind)
    assert loss == pytest.approx(ref, rel=1e-9)
    y = to_host(net.forward(op.net_features(1, 1), N))[0]
    assert np.abs(y[:, :3]).max() < 3.0
    go = to_host(gout).astype(np.float64)
    assert np.all(go[:, 3:] == 0.0)
    rng = np.random.default_rng(4)
    for trial in range(2):
        d = rng.standard_normal((3, N ** 3))
        t = 1e-4
        lp = train.field_loss(N, wl.kpoints[4], g[1], E * np.exp(t * d), Op[1], r, c, kind)
        lm = train.field_loss(N, wl.kpoints[4], g[1], E * np.exp(-t * d), Op[1], r, c, kind)
        fd = (lp - lm) / (2 * t)
        lhs = float(np.sum(go[:, :3].T * d)) / 2.0
        assert lhs == pytest.approx(fd, rel=2e-3, abs=1e-7 * abs(ref)), (trial, lhs, fd)
    loss2, none = op.net_loss_grad(to_dev(r), to_dev(c), ik=1, kind=kind)
    assert none is None and loss2 == pytest.approx(loss, rel=1e-13)
    del torch
