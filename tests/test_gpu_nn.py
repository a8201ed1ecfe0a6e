"""The learned preconditioner's HIP kernels (through the C ABI) against the FP64 conv-net
reference in oracle/nn.py: forward, gradients (from a loss and from a given output gradient), a
short training run, the feature map, the learned field and the preconditioner application; and
the eigen-solve with the learned preconditioner attached against the oracle's eigenvalues."""
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
LAYERS = [(32, 15), (32, 32), (3, 32)]
NIN, NOUT = 15, 3


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
    x[:, :, NIN:] = 0.0
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
        xo = x[b, :, :NIN].T.reshape(NIN, N, N, N).astype(np.float64)
        ref = forward_bf16(params, xo)
        assert rel_err(y[b, :, :NOUT], to_cl(ref)) < 5e-3
        assert np.all(y[b, :, NOUT:] == 0.0)


def test_gradients_match_oracle():
    import torch

    N, batch = 16, 2
    net, p = rand_net(5)
    rng = np.random.default_rng(6)
    x = feats(rng, batch, N)
    t = np.zeros((batch, N ** 3, 16), dtype=np.float32)
    t[:, :, :NOUT] = rng.standard_normal((batch, N ** 3, NOUT))
    note("nn gradients")
    loss, g = net.gradients(to_dev(x).to(torch.bfloat16), to_dev(t), N)
    params = [(bf16(w), b) for w, b in split(p)]
    # reference: sum over the batch of per-sample gradients of the batch-mean MSE
    gsum = None
    L = 0.0
    for b in range(batch):
        xo = x[b, :, :NIN].T.reshape(NIN, N, N, N).astype(np.float64)
        to = t[b, :, :NOUT].T.reshape(NOUT, N, N, N).astype(np.float64)
        y, cache = nn.forward(params, xo)
        L += np.sum((y - to) ** 2)
        gy = 2.0 * (y - to) / (batch * N ** 3 * NOUT)
        gr, _ = nn.backward(params, xo, cache, gy)
        flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in gr])
        gsum = flat if gsum is None else gsum + flat
    L /= batch * N ** 3 * NOUT
    assert loss == pytest.approx(L, rel=2e-2)
    _compare_grads(g, gsum)


def _compare_grads(g, ref):
    """Weights within 5%; biases within 10% (a bias gradient sums BF16 back-propagated values
    over every cell of the batch, with heavy cancellation)."""
    off = 0
    for co, ci in LAYERS:
        nw = co * ci * 27
        assert rel_err(g[off:off + nw], ref[off:off + nw]) < 5e-2, (co, ci)
        assert rel_err(g[off + nw:off + nw + co], ref[off + nw:off + nw + co]) < 1e-1, (co, ci)
        off += nw + co


def test_backward_from_output_gradient_matches_oracle():
    import torch

    N, batch = 16, 2
    net, p = rand_net(7)
    rng = np.random.default_rng(8)
    x = feats(rng, batch, N)
    gout = np.zeros((batch, N ** 3, 16), dtype=np.float32)
    gout[:, :, :NOUT] = bf16(1e-3 * rng.standard_normal((batch, N ** 3, NOUT)))  # the kernel's rounding
    note("nn backward")
    g = net.backward(to_dev(x).to(torch.bfloat16), to_dev(gout), N)
    params = [(bf16(w), b) for w, b in split(p)]
    gsum = None
    for b in range(batch):
        xo = x[b, :, :NIN].T.reshape(NIN, N, N, N).astype(np.float64)
        y, cache = nn.forward(params, xo)
        gy = gout[b, :, :NOUT].T.reshape(NOUT, N, N, N).astype(np.float64)
        gr, _ = nn.backward(params, xo, cache, gy)
        flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in gr])
        gsum = flat if gsum is None else gsum + flat
    _compare_grads(g, gsum)


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
    for step in range(300):
        loss, _ = net.gradients(x, t, N, host_grads=False)
        net.adam_step(2e-3)
    assert loss < 0.2 * l0, (l0, loss)


def _op16():
    wl = W.sphere_anisotropic(N=16, nk=4, m=6)
    op = kc.Op(16, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints)
    return wl, op


def _ref_features(wl, ik):
    """Network input by its definition: inverse permittivity (9), log E0 (3), k/pi (3)."""
    N = wl.N
    P = yee.point_tensors(wl.ids, wl.table)
    ref = np.zeros((N ** 3, 32))
    ref[:, 0] = P[0][:, 0, 0].real
    ref[:, 1] = P[1][:, 1, 1].real
    ref[:, 2] = P[2][:, 2, 2].real
    for q, (a, b) in enumerate([(0, 1), (0, 2), (1, 2)]):
        ref[:, 3 + 2 * q] = P[3][:, a, b].real
        ref[:, 4 + 2 * q] = P[3][:, a, b].imag
    ref[:, 9:12] = np.log(kspace.edge_permittivity(wl.ids, wl.table)).T
    ref[:, 12:15] = wl.kpoints[ik] / math.pi
    return ref


def test_features_match_definition():
    import torch

    wl, op = _op16()
    note("nn features")
    f = to_host(op.net_features(ik0=1, nk=2).to(torch.float32))
    for b in range(2):
        ref = _ref_features(wl, 1 + b)
        assert np.max(np.abs(f[b] - ref)) <= 1e-2 * max(1.0, np.abs(ref).max())


def test_learned_field_and_precond_match_definition():
    """E = E0 exp(clamp(net, -3, 3)) against the oracle's conv net on the same features, and
    kc_precond_learned = T_E with that field against the oracle's pseudo-inverse definition."""
    wl, op = _op16()
    net, p = rand_net(31, scale=0.05)
    op.attach_net(net)
    N = 16
    note("nn efield")
    E = to_host(op.net_efield(ik0=2, nk=1))[0].astype(np.float64)
    x = bf16(_ref_features(wl, 2)[:, :NIN].T).reshape(NIN, N, N, N)
    y = forward_bf16(split(p), x).reshape(NOUT, -1)
    Eref = kspace.edge_permittivity(wl.ids, wl.table) * np.exp(np.clip(y, -3, 3))
    assert rel_err(E, Eref) < 5e-3
    assert np.abs(np.log(E / kspace.edge_permittivity(wl.ids, wl.table))).max() > 1e-2  # not trivial
    r = W.random_block(32, 2, N)
    note("nn precond")
    z = to_host(op.precond_learned(to_dev(r), ik0=2))
    ref = kspace.transverse_precond_apply(N, wl.kpoints[2], op.gamma()[2], E, r)
    assert rel_err(z, ref) < 1e-10


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("prec,tol", [(kc.KC_PREC_FP64, 1e-10), (kc.KC_PREC_FP32, 2e-6)])
def test_learned_precond_per_kpoint_fields(N, prec, tol):
    """kc_precond_learned over three k-points, two vectors each: every k-point's T_E takes its own
    learned field (FP32: through the yz-plane pass, which reads the x-major copy written beside
    the fields), against the oracle's pseudo-inverse definition of T_E with the field that
    kc_net_efield returns for that k-point."""
    wl = W.sphere_anisotropic(N=N, nk=9, m=6)
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints)
    net, _ = rand_net(37, scale=0.05)
    op.attach_net(net)
    note("nn precond per k N=%d prec=%d" % (N, prec))
    E = to_host(op.net_efield(ik0=1, nk=3)).astype(np.float64)
    assert np.abs(E[0] - E[2]).max() > 1e-3 * E.max()  # the fields differ between k-points
    r = W.random_block(90 + N, 6, N)
    z = to_host(op.precond_learned(to_dev(r), ik0=1, vecs_per_k=2, prec=prec))
    g = op.gamma()
    for b in range(3):
        ref = kspace.transverse_precond_apply(N, wl.kpoints[1 + b], g[1 + b], E[b], r[2 * b:2 * b + 2])
        assert rel_err(z[2 * b:2 * b + 2], ref) < tol, (N, b)


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


def test_trained_network_gain_on_heldout_geometry():
    """Train the field network on the GPU (solver-generated pairs on 16 random geometries,
    N = 32) and compare iterations to Res <= 1e-8 on a held-out geometry: the learned T_E against
    the paper's diagonal-block preconditioner (the method without the network) and against the
    classical field E0.  Eigenvalues agree to 1e-6 whatever the preconditioner."""
    from paper_2511_17107_amd import learned

    note("train learned field")
    net = kc.Net(seed=0)
    samples = learned.make_samples(32, range(16), log=lambda *a: None)
    l0 = learned.mean_loss(net, samples)
    learned.train(net, samples, steps=150, batch=4, lr=1e-3, log=lambda *a: None)
    l1 = learned.mean_loss(net, samples)
    assert l1 < l0
    wl = W.random_inclusions(32, 1000, nk=40, m=12)
    op = kc.Op(32, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints[[5, 15, 25, 35]])
    op.attach_net(net)
    out = {}
    for name, pc in (("diagonal", kc.KC_PRECOND_DIAG), ("transverse", kc.KC_PRECOND_TRANSVERSE),
                     ("learned", kc.KC_PRECOND_LEARNED)):
        note("solve held-out", name)
        eig, res, its, st = op.solve(12, tol=1e-8, guard=3, batch_k=4, precond=pc)
        assert st == 0 and res.max() <= 1e-8
        out[name] = (eig, its)
    for name in ("transverse", "learned"):
        assert np.max(np.abs(out[name][0] - out["diagonal"][0]) / out["diagonal"][0]) <= 1e-6
    it = {k: int(v[1].sum()) for k, v in out.items()}
    note("iterations (sum over 4 k-points)", it, "loss %.4f -> %.4f" % (l0, l1))
    assert it["learned"] < it["diagonal"]
