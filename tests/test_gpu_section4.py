"""Section 4 experiments through the C ABI: the order-10 stencils against the frequency
differences Table 5 prints (grids up to 64^3, beyond the oracle's reach), the ill-conditioned
inclusion of the robustness experiment against the oracle's eigenvalues, and the Trivial /
CrossDoF difference of eq (4.6)."""
import json
import math
import os

import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W

from gpu_util import note

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Table 5 (smooth eps of eq (4.7), k = (pi, pi, pi), m = 5): differences of the first eight
# normalised frequencies omega / (2 pi) between h and 2h, columns h = 1/32 and h = 1/64.  (The
# header says omega^2; the values match the frequency reading, which the oracle pins at h = 1/32
# in test_oracle_highorder.py.)
TABLE5 = {32: [4.87e-09, 4.87e-09, 1.97e-08, 1.97e-08, 1.97e-08, 3.60e-08, 3.60e-08, 3.60e-08],
          64: [5.36e-12, 5.36e-12, 2.23e-11, 2.23e-11, 2.23e-11, 4.13e-11, 4.13e-11, 4.14e-11]}


def _smooth_freqs(N, m):
    wl = W.smooth_isotropic(N)
    op = kc.Op(N, kc.KC_EPS_DIAGONAL, wl.ids, wl.table, stencil_m=m)
    op.set_kpoints(wl.kpoints)
    note("smooth eps solve", N, m)
    eig, res, its, st = op.solve(8, tol=1e-8, guard=4, precond=kc.KC_PRECOND_TRANSVERSE)
    assert st == 0 and res.max() <= 1e-8
    return np.sqrt(eig[0]) / (2 * math.pi)


def test_table5_tenth_order_columns():
    """Order-10 stencils (m = 5): every band's frequency difference at h = 1/32 and h = 1/64 within
    3 % of the printed value (three significant digits), and the observed order near 10."""
    f = {N: _smooth_freqs(N, 5) for N in (16, 32, 64)}
    d32 = np.abs(f[32] - f[16])
    d64 = np.abs(f[64] - f[32])
    note("h=1/32", d32, "h=1/64", d64)
    assert np.allclose(d32, TABLE5[32], rtol=0.03), d32
    assert np.allclose(d64, TABLE5[64], rtol=0.03), d64
    order = np.log2(d32 / d64)
    assert np.all((order > 9.0) & (order < 10.5)), order


def test_second_order_converges_at_second_order():
    """The same case with the second-order Yee stencils: differences shrink by about 4 per halving
    of h (order 2), far above the order-10 values."""
    f = {N: _smooth_freqs(N, 1) for N in (16, 32, 64)}
    d32, d64 = np.abs(f[32] - f[16]), np.abs(f[64] - f[32])
    order = np.log2(d32 / d64)
    assert np.all((order > 1.8) & (order < 2.2)), order
    assert np.all(d64 > 1e3 * np.array(TABLE5[64]))


def _load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["illcond16", "illcond32"])
@pytest.mark.parametrize("prec", [kc.KC_PREC_FP64, kc.KC_PREC_FP32])
def test_ill_conditioned_inclusion_matches_oracle(name, prec):
    """Inverse permittivity U diag(1e-1, 1e-3, 1e-5) U^H in a sphere (condition number 1e4, the
    conditions of Props 3.8 / 3.10 not met), FP64 and the FP32-operator path (with the W-column
    Gram shortcut).  CrossDoF: Res <= 1e-8 and every band within 1e-6 of the oracle.  Trivial
    (which the paper reports to stagnate in this case, and whose lowest modes here sit far below
    CrossDoF's): every Ritz value within its residual of an oracle eigenvalue (the Hermitian
    bound |theta - lambda| <= |r| for a unit vector), and the residuals fall."""
    g = _load(name)
    wl = W.sphere_illconditioned(g["N"])
    for case in g["cases"]:
        op = kc.Op(wl.N, kc.SCHEMES[case["scheme"]], wl.ids, wl.table)
        op.set_kpoints(np.array([case["k"]]))
        note("ill-conditioned", name, case["scheme"], prec)
        eig, res, its, st = op.solve(10, tol=1e-8, guard=4, prec=prec, switch_tol=3e-4,
                                     precond=kc.KC_PRECOND_TRANSVERSE, maxit=400, check=False)
        ref = np.array(case["eigenvalues"])
        h, hp = op.residual_history(0)
        assert len(h) >= 1 and h[-1] < 1e-3 * h[0]
        if case["scheme"] == "crossdof":
            assert st == 0 and res.max() <= 1e-8, (its, res.max())
            assert np.max(np.abs(eig[0] - ref) / ref) <= 1e-6, (eig[0], ref)
        else:
            assert st in (0, kc.KC_ERR_NO_CONVERGENCE)
            assert np.all(np.abs(eig[0] - ref) <= 2 * res[0] + 1e-12), (eig[0], ref, res[0])


def test_trivial_and_crossdof_frequencies_close():
    """Eq (4.6): the two discretisations of Section 3 give frequencies that differ by little
    (Table 2 reports 1e-3 to 5e-3) on the anisotropic sphere at 32^3 over four k-points."""
    wl = W.sphere_anisotropic(N=32, nk=9, m=10)
    w = {}
    for scheme in ("trivial", "crossdof"):
        op = kc.Op(32, kc.SCHEMES[scheme], wl.ids, wl.table)
        op.set_kpoints(wl.kpoints[[1, 2, 4, 8]])
        note("scheme", scheme)
        eig, res, its, st = op.solve(10, tol=1e-8, guard=4, batch_k=4, precond=kc.KC_PRECOND_TRANSVERSE)
        assert st == 0
        w[scheme] = np.sqrt(eig)
    d = np.abs(w["trivial"] - w["crossdof"]) / w["crossdof"]
    assert 1e-6 < d.max() < 2e-2, d.max()


def test_unreachable_tolerance_stops_cleanly():
    """Order-10 stencils at 64^3 put the rounding floor of an FP64 application near 1e-9: asking
    for 1e-10 ends as KC_ERR_NO_CONVERGENCE after the stagnation window (200 iterations without
    progress), with the eigenvalues of the converged solve: the Rayleigh-Ritz steps whose Ritz
    values fall below the residual bound are rejected, so none is made of rounding noise."""
    N = 64
    wl = W.smooth_isotropic(N)
    op = kc.Op(N, kc.KC_EPS_DIAGONAL, wl.ids, wl.table, stencil_m=5)
    op.set_kpoints(wl.kpoints)
    note("unreachable tolerance")
    e1, r1, i1, s1 = op.solve(8, tol=1e-8, guard=4, precond=kc.KC_PRECOND_TRANSVERSE)
    e2, r2, i2, s2 = op.solve(8, tol=1e-10, guard=4, precond=kc.KC_PRECOND_TRANSVERSE, maxit=500, check=False)
    assert s1 == 0 and s2 == kc.KC_ERR_NO_CONVERGENCE
    assert np.max(np.abs(e2 - e1) / e1) < 1e-9, (e1, e2)
    assert i2[0] < 100  # stopped by the stagnation rule, not by maxit
