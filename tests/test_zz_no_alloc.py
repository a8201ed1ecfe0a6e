"""kc_block_gram_noalloc (the entry point that allocates nothing; its partial sums live in a
static device array) against kc_block_gram, through the C ABI: two calls in a row, the second
smaller, every output entry written (outputs start as NaN)."""
import ctypes

import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W
from oracle import block

from gpu_util import note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _case(seed, nb, nc, n):
    S = W.random_complex(seed, (nb, nc, n))
    AS = np.random.default_rng(seed + 1).uniform(-2.0, 5.0, (nb, 1, n)) * S
    return S, AS


def _scaled_err(G, R, a, b):
    return float(np.max(np.abs(G - R) / (a[:, :, None] * b[:, None, :])))


@pytest.mark.parametrize("first,second", [((40, 60, 2 * 3 * 16 ** 3), (3, 13, 1007))])
def test_noalloc_gram_matches_block_gram(first, second):
    import torch

    for seed, (nb, nc, n) in [(31, first), (41, second)]:
        S, AS = _case(seed, nb, nc, n)
        dS, dAS = to_dev(S), to_dev(AS)
        note("block_gram_noalloc", nb, nc, n)
        GA = torch.full((nb, nc, nc), float("nan"), dtype=torch.complex128, device="cuda")
        GB = torch.full((nb, nc, nc), float("nan"), dtype=torch.complex128, device="cuda")
        kc.block_gram_noalloc(dS, dAS, GA, GB)
        GA, GB = to_host(GA), to_host(GB)
        note("block_gram", nb, nc, n)
        rA, rB = kc.block_gram(dS, dAS)
        rA, rB = to_host(rA), to_host(rB)
        sS, sA = np.linalg.norm(S, axis=2), np.linalg.norm(AS, axis=2)
        assert np.all(np.isfinite(GA)) and np.all(np.isfinite(GB))
        assert _scaled_err(GA, rA, sS, sA) < 5e-13
        assert _scaled_err(GB, rB, sS, sS) < 5e-13
        if n * nb * nc < 10 ** 6:
            oA, oB = block.gram(S, AS)
            assert _scaled_err(GA, oA, sS, sA) < 5e-13 and _scaled_err(GB, oB, sS, sS) < 5e-13


def test_noalloc_gram_rejects_sizes_beyond_the_array():
    L = kc.lib()
    fake = ctypes.c_void_p(1 << 40)  # never dereferenced: the size check fails first
    assert L.kc_block_gram_noalloc(410, 1000, 64, fake, fake, fake, fake, None) == 1
    assert b"KC_NOALLOC_SCRATCH_BYTES" in L.kc_last_error()
    assert L.kc_block_gram_noalloc(0, 1000, 64, None, None, None, None, None) == 0
