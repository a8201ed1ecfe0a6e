"""The LOBPCG block kernels through the C ABI (kc_block_gram, kc_block_update) against the
oracle's definitions (oracle/block.py), element by element: small blocks with ragged row
counts and every block width class (the wide blocks of 65-96 columns included), and the full 128^3 shape of the benchmark (10 k-points,
16 bands + 4 guard) on sampled rows."""
import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W
from oracle import block

from gpu_util import note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _colscale(S):
    return np.linalg.norm(S, axis=2)  # (nb, nc)


@pytest.mark.parametrize("nb,nc,n", [(3, 60, 3 * 16 ** 3), (2, 13, 1007), (1, 64, 333), (4, 6, 16), (2, 63, 5),
                                     (2, 72, 1007), (1, 80, 333), (2, 96, 3 * 8 ** 3 + 3)])
def test_block_gram_matches_oracle(nb, nc, n):
    """AS = D S with a real diagonal D (a Hermitian operator, as the kernel requires)."""
    S = W.random_complex(11, (nb, nc, n))
    AS = np.random.default_rng(12).uniform(-2.0, 5.0, (nb, 1, n)) * S
    note("block_gram", nb, nc, n)
    GA, GB = kc.block_gram(to_dev(S), to_dev(AS))
    GA, GB = to_host(GA), to_host(GB)
    rA, rB = block.gram(S, AS)
    sS, sA = _colscale(S), _colscale(AS)
    # FP64 sums of n products (three real products per complex one): the error is a small
    # multiple of sqrt(n) eps |s_i| |a_j| (worst case n eps)
    assert np.max(np.abs(GA - rA) / (sS[:, :, None] * sA[:, None, :])) < 5e-13
    assert np.max(np.abs(GB - rB) / (sS[:, :, None] * sS[:, None, :])) < 5e-13


@pytest.mark.parametrize("nb,mb,n", [(3, 20, 3 * 16 ** 3), (2, 21, 1007), (2, 5, 1007), (1, 4, 48), (3, 1, 100),
                                     (2, 8, 3 * 8 ** 3 + 3), (1, 13, 17), (2, 22, 1007), (1, 24, 333),
                                     (2, 27, 3 * 8 ** 3 + 3), (1, 32, 17)])
def test_block_update_matches_oracle(nb, mb, n):
    """mb a multiple of 4 takes the uniform-offset path, the others the per-lane clamp; n not a
    multiple of 16 leaves a ragged last row block."""
    S = W.random_complex(21, (nb, 3 * mb, n))
    AS = W.random_complex(22, (nb, 3 * mb, n))
    C = W.random_complex(23, (nb, 3 * mb, 2 * mb))
    theta = np.random.default_rng(24).uniform(0.1, 2.0, (nb, mb))
    note("block_update", nb, mb, n)
    dS, dAS = to_dev(S), to_dev(AS)
    R, res, xn2 = kc.block_update(dS, dAS, to_dev(C), to_dev(theta))
    S1, AS1, R, res, xn2 = to_host(dS), to_host(dAS), to_host(R), to_host(res), to_host(xn2)
    rS, rAS, rR, rres, rxn2 = block.update(S, AS, C, theta)
    # each output entry is a 3mb-term FP64 sum (three real products per complex one): bound by
    # a small multiple of eps times the sum of |terms|
    bS = np.matmul(np.abs(np.transpose(C, (0, 2, 1))), np.abs(S))
    bA = np.matmul(np.abs(np.transpose(C, (0, 2, 1))), np.abs(AS))
    one = np.ones((nb, mb, n))  # W columns: compared exactly below
    scale_S = np.concatenate([bS[:, :mb], one, bS[:, mb:]], axis=1)
    scale_A = np.concatenate([bA[:, :mb], one, bA[:, mb:]], axis=1)
    assert np.max(np.abs(S1 - rS) / scale_S) < 5e-14
    assert np.max(np.abs(AS1 - rAS) / scale_A) < 5e-14
    assert np.array_equal(S1[:, mb:2 * mb], S[:, mb:2 * mb]) and np.array_equal(AS1[:, mb:2 * mb], AS[:, mb:2 * mb])
    scale_R = bA[:, :mb] + theta[:, :, None] * bS[:, :mb]
    assert np.max(np.abs(R - rR) / scale_R) < 5e-14
    assert np.max(np.abs(res - rres) / rres) < 1e-12
    assert np.max(np.abs(xn2 - rxn2) / rxn2) < 1e-12


def test_block_update_full_size_sampled():
    """The benchmark's shape: 128^3 (n = 6.3M rows), 10 k-points, 16 bands + 4 guard (60 input,
    40 output columns per block), inputs drawn on the device.  Sampled rows against the oracle
    (rows are independent), the norms against sums of the kernel's own outputs."""
    import torch

    nb, mb, n = 10, 20, 3 * 128 ** 3
    torch.cuda.empty_cache()
    g = torch.Generator(device="cuda")
    g.manual_seed(31)
    note("block_update full size: allocating", nb, mb, n)
    S = torch.randn((nb, 3 * mb, n), dtype=torch.complex128, device="cuda", generator=g)
    AS = torch.randn((nb, 3 * mb, n), dtype=torch.complex128, device="cuda", generator=g)
    C = W.random_complex(32, (nb, 3 * mb, 2 * mb)) / np.sqrt(3 * mb)
    theta = np.random.default_rng(33).uniform(0.1, 2.0, (nb, mb))
    rng = np.random.default_rng(34)
    rows = np.unique(np.concatenate([rng.integers(0, n, 3000), np.arange(16), np.arange(n - 16, n)]))
    ri = torch.from_numpy(rows).to("cuda")
    S0, AS0 = to_host(S[:, :, ri]), to_host(AS[:, :, ri])
    note("block_update full size: kernel")
    R, res, xn2 = kc.block_update(S, AS, to_dev(C), to_dev(theta))
    torch.cuda.synchronize()
    S1, AS1, R1 = to_host(S[:, :, ri]), to_host(AS[:, :, ri]), to_host(R[:, :, ri])
    rS, rAS, rR, _, _ = block.update(S0, AS0, C, theta)
    tol = 1e-13 * np.max(np.abs(rS))
    assert np.max(np.abs(S1 - rS)) < tol and np.max(np.abs(AS1 - rAS)) < tol
    assert np.max(np.abs(R1 - rR)) < 1e-13 * np.max(np.abs(rR))
    x2 = to_host(torch.sum(torch.abs(S[:, :mb]) ** 2, dim=2))
    r2 = to_host(torch.sum(torch.abs(R) ** 2, dim=2))
    assert np.max(np.abs(to_host(xn2) - x2) / x2) < 1e-12
    assert np.max(np.abs(to_host(res) - np.sqrt(r2 / x2)) / np.sqrt(r2 / x2)) < 1e-12
    del S, AS, R
    torch.cuda.empty_cache()
