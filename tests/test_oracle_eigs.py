"""Pins of the oracle's eigensolve: closed forms, brute force and residual certificates."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import eigs, yee

from test_oracle_operator import s_of_p

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("k", [(0.3, 0.5, 0.7), (0.0, 0.0, 0.0), (math.pi, 0.0, 0.0)])
@pytest.mark.parametrize("method", ["dense", "shift_invert"])
def test_smallest_positive_homogeneous(k, method):
    """Closed form (Lemma 2.1, Prop 2.8) for eps^-1 = c I: the m smallest positive eigenvalues
    are the m smallest of {c s(p) (x2), gamma s(p)} minus the k = 0 zeros (Prop 2.5 (1))."""
    N = 6
    c = 1.0 / 13.0
    ids = np.ones((4, N ** 3), dtype=np.uint8)
    tab = W.eps_table([13.0 * np.eye(3)])
    g = yee.gamma_rule(k)
    s = s_of_p(N, k)
    ref = np.sort(np.concatenate([c * s, c * s, g * s]))
    ref = ref[ref > 1e-9][:12]
    Op = yee.compensated_operator(N, k, ids, tab, "crossdof")
    w = eigs.smallest_positive(Op, 12, method=method)
    assert np.allclose(w, ref, rtol=1e-10)


@pytest.mark.parametrize("scheme", ["trivial", "crossdof"])
def test_shift_invert_matches_brute_force(scheme):
    """Shift-invert Lanczos against the full dense spectrum (brute force) at N = 6."""
    wl = W.sphere_anisotropic(N=6, nk=3, m=8, scheme=scheme)
    for k in wl.kpoints:
        Op = yee.compensated_operator(wl.N, k, wl.ids, wl.table, scheme)
        full = eigs.all_eigenvalues(Op)
        full = full[full > 1e-10 * abs(full).max()][:8]
        w = eigs.smallest_positive(Op, 8, method="shift_invert")
        assert np.allclose(w, full, rtol=1e-11)


def test_residual_certificates():
    """Hermitian residual bound: each returned pair has ||Op v - lambda v|| <= 1e-9 ||Op||."""
    wl = W.sphere_anisotropic(N=8, nk=2, m=6)
    Op = yee.compensated_operator(wl.N, wl.kpoints[1], wl.ids, wl.table, "crossdof")
    w, V = eigs.smallest_positive(Op, 6, method="shift_invert", return_vectors=True)
    R = Op @ V - V * w[None, :]
    assert np.linalg.norm(R, axis=0).max() <= 1e-9 * eigs.op_norm_bound(Op)


@pytest.mark.slow
def test_sphere16_golden_reproducible():
    """The stored N=16 sphere eigenvalues (written by tests/golden/make_golden.py, which calls
    only the oracle) are reproduced by the oracle."""
    path = os.path.join(GOLDEN, "sphere16_iso.json")
    import json
    with open(path) as f:
        gold = json.load(f)
    wl = W.sphere_isotropic()
    Op = yee.compensated_operator(wl.N, wl.kpoints[0], wl.ids, wl.table, "crossdof")
    w = eigs.smallest_positive(Op, wl.m, method="shift_invert")
    assert np.allclose(w, gold["eigenvalues"], rtol=1e-12)
