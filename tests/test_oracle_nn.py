"""Pins of the FP64 conv-net reference: direct definition on a delta, periodicity, central
finite differences for every gradient, Adam on a quadratic, BF16 round-to-nearest-even."""
import numpy as np
import pytest

from oracle import nn


def _params(rng, cin, ch, cout, scale=0.3):
    shp = [(ch, cin), (ch, ch), (cout, ch)]
    return [(scale * rng.standard_normal((o, i, 3, 3, 3)), 0.1 * rng.standard_normal(o)) for o, i in shp]


def test_conv_delta_response():
    """A unit impulse at the origin reproduces the flipped kernel around it (circularly)."""
    N = 5
    rng = np.random.default_rng(0)
    w = rng.standard_normal((2, 1, 3, 3, 3))
    x = np.zeros((1, N, N, N))
    x[0, 0, 0, 0] = 1.0
    y = nn.conv3d(x, w, np.zeros(2))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                # y[z] = w[d] x[z + d - 1] -> y at z = 1 - d
                z, yy, xx = (1 - dz) % N, (1 - dy) % N, (1 - dx) % N
                assert np.allclose(y[:, z, yy, xx], w[:, 0, dz, dy, dx])
    assert np.count_nonzero(np.abs(y).sum(axis=0)) == 27


def test_conv_translation_equivariance():
    N = 4
    rng = np.random.default_rng(1)
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    x = rng.standard_normal((2, N, N, N))
    y = nn.conv3d(x, w, b)
    ys = nn.conv3d(np.roll(x, (1, 2, 3), axis=(1, 2, 3)), w, b)
    assert np.allclose(ys, np.roll(y, (1, 2, 3), axis=(1, 2, 3)))


def test_gradients_finite_differences():
    """Central differences (step 1e-6) for inputs, every weight tensor and bias."""
    N = 4
    rng = np.random.default_rng(2)
    params = _params(rng, 3, 4, 2)
    x = rng.standard_normal((3, N, N, N))
    tgt = rng.standard_normal((2, N, N, N))

    def L(ps, xx):
        y, _ = nn.forward(ps, xx)
        return nn.loss(y, tgt)

    y, cache = nn.forward(params, x)
    grads, gx = nn.backward(params, x, cache, nn.loss_grad(y, tgt))
    h = 1e-6
    for li in range(3):
        for which in range(2):
            P = params[li][which]
            G = grads[li][which]
            for idx in [tuple(rng.integers(0, s) for s in P.shape) for _ in range(5)]:
                pp = [(w.copy(), b.copy()) for w, b in params]
                pm = [(w.copy(), b.copy()) for w, b in params]
                pp[li][which][idx] += h
                pm[li][which][idx] -= h
                fd = (L(pp, x) - L(pm, x)) / (2 * h)
                assert G[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    for idx in [tuple(rng.integers(0, s) for s in x.shape) for _ in range(5)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (L(params, xp) - L(params, xm)) / (2 * h)
        assert gx[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_adam_minimises_quadratic():
    p = np.array([3.0, -2.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 2001):
        p, m, v = nn.adam_step(p, 2 * p, m, v, t, lr=0.05)
    assert np.abs(p).max() < 1e-2


def test_bf16_round_to_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, -3.14159265, 65504.0, 1e-30],
                    dtype=np.float32)
    r = nn.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == np.float32(1.0 + 2 ** -7) or r[1] == 1.0  # tie between 1 and 1+2^-7: even -> 1.0
    assert r[1] == 1.0
    assert r[2] == np.float32(1.0 + 2 ** -7)   # above the tie
    assert r[3] == 1.0                          # below the tie
    assert abs(r[4] + 3.140625) < 1e-7          # -3.14159 -> -3.140625
    # all results have zero low 16 bits
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)
