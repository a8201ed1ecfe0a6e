"""The learned preconditioner's HIP kernels (through the C ABI) against the FP64 conv-net
reference in oracle/nn.py: forward, gradients, a short training run, the feature map and the
preconditioner application; and the eigen-solve with the learned preconditioner attached
against the oracle's eigenvalues."""
import json
import math
import os

import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W
from oracle import kspace, nn, yee

from gpu_util import note, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LAYERS = [(32, 18), (32, 32), (6, 32)]


def split(p):
    out, off = [], 0
    for co, ci in LAYERS:
        w = p[off:off + co * ci * 27].reshape(co, ci, 3, 3, 3).astype(np.float64)
        off += co * ci * 27
        b = p[off:off + co].astype(np.float64)
        off += co
        out.append((w, b))
    return out


def bf16(a):
    return nn.bf16_round(np.asarray(a, dtype=np.float32)).astype(np.float64)


def forward_bf16(params, x):
    """Reference forward with the kernels' rounding points: BF16 weights, inputs and hidden
    activations, FP64 sums."""
    ps = [(bf16(w), b) for w, b in params]
    h1 = bf16(nn.act(nn.conv3d(x, *ps[0])))
    h2 = bf16(nn.act(nn.conv3d(h1, *ps[1])))
    return nn.conv3d(h2, *ps[2])


def to_cl(a):
    """[C][N][N][N] -> channels-last [N^3][C]"""
    return a.reshape(a.shape[0], -1).T


def rand_net(seed, scale=0.08):
    net = kc.Net(seed=seed)
    rng = np.random.default_rng(seed)
    p = (scale * rng.standard_normal(kc.Net.param_count())).astype(np.float32)
    net.set_params(p)
    return net, p


def feats(rng, batch, N):
    x = rng.standard_normal((batch, N ** 3, 32)).astype(np.float32)
    x[:, :, 18:] = 0.0
    xb = bf16(x).astype(np.float32)
    return xb


def test_forward_matches_oracle():
    import torch

    N, batch = 16, 2
    net, p = rand_net(3)
    rng = np.random.default_rng(4)
    x = feats(rng, batch, N)
    note("nn forward")
    y = to_host(net.forward(to_dev(x).to(torch.bfloat16), N))
    params = split(p)
    for b in range(batch):
        xo = x[b, :, :18].T.reshape(18, N, N, N).astype(np.float64)
        ref = forward_bf16(params, xo)
        assert rel_err(y[b, :, :6], to_cl(ref)) < 5e-3
        assert np.all(y[b, :, 6:] == 0.0)


def test_gradients_match_oracle():
    import torch

    N, batch = 16, 2
    net, p = rand_net(5)
    rng = np.random.default_rng(6)
    x = feats(rng, batch, N)
    t = np.zeros((batch, N ** 3, 16), dtype=np.float32)
    t[:, :, :6] = rng.standard_normal((batch, N ** 3, 6))
    note("nn gradients")
    loss, g = net.gradients(to_dev(x).to(torch.bfloat16), to_dev(t), N)
    params = [(bf16(w), b) for w, b in split(p)]
    # reference: sum over the batch of per-sample gradients of the batch-mean MSE
    gsum = None
    L = 0.0
    for b in range(batch):
        xo = x[b, :, :18].T.reshape(18, N, N, N).astype(np.float64)
        to = t[b, :, :6].T.reshape(6, N, N, N).astype(np.float64)
        y, cache = nn.forward(params, xo)
        L += np.sum((y - to) ** 2)
        gy = 2.0 * (y - to) / (batch * N ** 3 * 6)
        gr, _ = nn.backward(params, xo, cache, gy)
        flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in gr])
        gsum = flat if gsum is None else gsum + flat
    L /= batch * N ** 3 * 6
    assert loss == pytest.approx(L, rel=2e-2)
    off = 0
    for co, ci in LAYERS:
        nw = co * ci * 27
        assert rel_err(g[off:off + nw], gsum[off:off + nw]) < 5e-2, (co, ci)
        assert rel_err(g[off + nw:off + nw + co], gsum[off + nw:off + nw + co]) < 5e-2
        off += nw + co


def test_training_reduces_loss():
    """Adam on the GPU fits a target produced by a fixed random network of the same shape."""
    import torch

    N, batch = 16, 2
    teacher, pt = rand_net(11, scale=0.05)
    rng = np.random.default_rng(12)
    x = to_dev(feats(rng, batch, N)).to(torch.bfloat16)
    t = teacher.forward(x, N).contiguous()
    net = kc.Net(seed=13)
    note("nn training")
    l0, _ = net.gradients(x, t, N, host_grads=False)
    for step in range(150):
        loss, _ = net.gradients(x, t, N, host_grads=False)
        net.adam_step(2e-3)
    assert loss < 0.2 * l0, (l0, loss)


def _op16():
    wl = W.sphere_anisotropic(N=16, nk=4, m=6)
    op = kc.Op(16, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints)
    return wl, op


def test_features_match_definition():
    import torch

    wl, op = _op16()
    net, p = rand_net(21)
    op.attach_net(net)
    N = 16
    r = W.random_block(22, 2, N)
    note("nn features")
    f = to_host(op.net_features(to_dev(r), ik0=1, vecs_per_k=1).to(torch.float32))
    P = yee.point_tensors(wl.ids, wl.table)
    for v in range(2):
        real = kspace.F3(r[v:v + 1], N)[0] * math.sqrt(3 * N ** 3) / np.linalg.norm(r[v])
        ref = np.zeros((N ** 3, 32))
        for c in range(3):
            ref[:, 2 * c] = real[c].real
            ref[:, 2 * c + 1] = real[c].imag
        ref[:, 6] = P[0][:, 0, 0].real
        ref[:, 7] = P[1][:, 1, 1].real
        ref[:, 8] = P[2][:, 2, 2].real
        for q, (a, b) in enumerate([(0, 1), (0, 2), (1, 2)]):
            ref[:, 9 + 2 * q] = P[3][:, a, b].real
            ref[:, 10 + 2 * q] = P[3][:, a, b].imag
        ref[:, 15:18] = wl.kpoints[1 + v] / math.pi
        assert np.max(np.abs(f[v] - ref)) <= 1e-2 * max(1.0, np.abs(ref).max())


def test_precond_learned_matches_definition():
    import torch

    wl, op = _op16()
    net, p = rand_net(31, scale=0.05)
    op.attach_net(net)
    N = 16
    r = W.random_block(32, 1, N)
    note("nn precond")
    z = to_host(op.precond_learned(to_dev(r), ik0=2))
    g = op.gamma()[2]
    base = kspace.precond_apply(N, wl.kpoints[2], g, r)
    # the network reads the diagonal-block preconditioned residual, in units of its RMS value
    real = kspace.F3(base, N)[0] * math.sqrt(3 * N ** 3) / np.linalg.norm(base[0])
    P = yee.point_tensors(wl.ids, wl.table)
    x = np.zeros((18, N ** 3))
    for c in range(3):
        x[2 * c], x[2 * c + 1] = real[c].real, real[c].imag
    x[6], x[7], x[8] = P[0][:, 0, 0].real, P[1][:, 1, 1].real, P[2][:, 2, 2].real
    for q, (a, b) in enumerate([(0, 1), (0, 2), (1, 2)]):
        x[9 + 2 * q], x[10 + 2 * q] = P[3][:, a, b].real, P[3][:, a, b].imag
    x[15:18] = (wl.kpoints[2] / math.pi)[:, None]
    y = forward_bf16(split(p), bf16(x).reshape(18, N, N, N)).reshape(6, -1)
    delta = np.stack([y[0] + 1j * y[1], y[2] + 1j * y[3], y[4] + 1j * y[5]])
    delta *= np.linalg.norm(base) / math.sqrt(3 * N ** 3)
    corr = kspace.F3H(delta[None], N)
    assert rel_err(z - base, corr) < 3e-2
    assert np.linalg.norm(corr) > 1e-3 * np.linalg.norm(base)


def test_solve_with_learned_preconditioner_matches_oracle():
    """Eigenvalues do not depend on the preconditioner: with a (random) network attached the
    solve still matches the oracle (and falls back to the diagonal one if it stalls)."""
    with open(os.path.join(GOLDEN, "sphere16_aniso.json")) as fh:
        g = json.load(fh)
    wl = W.sphere_anisotropic(N=16, nk=9, m=10)
    cases = [c for c in g["cases"] if c["scheme"] == "crossdof"][:3]
    op = kc.Op(16, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(np.array([c["k"] for c in cases]))
    net = kc.Net(seed=41)
    op.attach_net(net)
    note("solve learned")
    eig, res, its, st = op.solve(10, tol=1e-8, batch_k=3, guard=2, precond=kc.KC_PRECOND_LEARNED)
    assert st == 0 and res.max() <= 1e-8
    for i, c in enumerate(cases):
        ref = np.array(c["eigenvalues"])
        assert np.max(np.abs(eig[i] - ref) / ref) <= 1e-6
