"""The transverse-projection preconditioner T_E and its training gradient (through the C ABI)
against the oracle's pseudo-inverse definition, and eigen-solves that use it against the
oracle's eigenvalues."""
import json
import os

import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W
from oracle import kspace

from gpu_util import note, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _op(N=16, nk=9):
    wl = W.sphere_anisotropic(N=N, nk=nk, m=6)
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints)
    return wl, op


@pytest.mark.parametrize("N", [16, 24])
@pytest.mark.parametrize("prec,tol", [(kc.KC_PREC_FP64, 1e-12), (kc.KC_PREC_FP32, 2e-6)])
def test_transverse_matches_oracle(N, prec, tol):
    """Classical field E0 = 1/(eps^-1)_cc, three k-points including Gamma, 2 vectors each.  The
    library stores the field in FP32, so the reference takes the same FP32-rounded field."""
    wl, op = _op(N)
    ks = [0, 1, 2]
    r = W.random_block(40 + N, 6, N)
    note("tp classical N=%d prec=%d" % (N, prec))
    z = to_host(op.precond_transverse(to_dev(r), ik0=0, vecs_per_k=2, prec=prec))
    E0 = kspace.edge_permittivity(wl.ids, wl.table).astype(np.float32).astype(np.float64)
    g = op.gamma()
    for b, ik in enumerate(ks):
        ref = kspace.transverse_precond_apply(N, wl.kpoints[ik], g[ik], E0, r[2 * b:2 * b + 2])
        assert rel_err(z[2 * b:2 * b + 2], ref) < tol, (N, ik)


@pytest.mark.parametrize("N,tol", [(32, 2e-6), (64, 3e-6), (96, 4e-6), (128, 5e-6)])
def test_transverse_plane_pass_large(N, tol):
    """FP32 with the classical field: the x-passes in the x-major layout around the yz-plane
    pass (a whole 128 x 128 plane in LDS at N = 128), one k-point off the symmetry lines and
    Gamma, two vectors each, against the oracle's pseudo-inverse definition."""
    wl = W.woodpile_gyrotropic(N=N, nk=60, m=16)
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    kp = np.array([wl.kpoints[0], wl.kpoints[23]])
    op.set_kpoints(kp)
    r = W.random_block(70 + N, 4, N)
    note("tp plane pass N=%d" % N)
    z = to_host(op.precond_transverse(to_dev(r), ik0=0, vecs_per_k=2, prec=kc.KC_PREC_FP32))
    E0 = kspace.edge_permittivity(wl.ids, wl.table).astype(np.float32).astype(np.float64)
    g = op.gamma()
    for b in range(2):
        ref = kspace.transverse_precond_apply(N, kp[b], g[b], E0, r[2 * b:2 * b + 2])
        assert rel_err(z[2 * b:2 * b + 2], ref) < tol, (N, b)


def test_transverse_field_per_kpoint():
    """A different positive field per k-point (device float32 [nk][3][N^3])."""
    N = 16
    wl, op = _op(N)
    rng = np.random.default_rng(3)
    E = rng.uniform(1.0, 14.0, size=(2, 3, N ** 3)).astype(np.float32)
    r = W.random_block(51, 4, N)
    note("tp field per k")
    z = to_host(op.precond_transverse(to_dev(r), ik0=3, vecs_per_k=2, efield=to_dev(E)))
    g = op.gamma()
    for b in range(2):
        ref = kspace.transverse_precond_apply(N, wl.kpoints[3 + b], g[3 + b], E[b].astype(np.float64),
                                              r[2 * b:2 * b + 2])
        assert rel_err(z[2 * b:2 * b + 2], ref) < 1e-12


def test_tp_grad_directional_derivative():
    """T_E is linear in E, so for any direction d: sum_{c,p} d g = sum_j w_j Re<e_j, (T_d - T_0) r_j>
    exactly (T_0 is the penalty part alone)."""
    import torch

    N = 16
    wl, op = _op(N)
    r = W.random_block(61, 4, N)
    e = W.random_block(62, 4, N)
    w = np.array([0.5, -1.0, 2.0, 0.25])
    note("tp grad")
    g = torch.zeros((2, 3, N ** 3), dtype=torch.float32, device="cuda")
    op.tp_grad(to_dev(r), to_dev(e), to_dev(w), g, ik0=4, vecs_per_k=2)
    g = to_host(g).astype(np.float64)
    gam = op.gamma()
    rng = np.random.default_rng(5)
    for trial in range(3):
        d = rng.standard_normal((2, 3, N ** 3))
        lhs = float(np.sum(d * g))
        rhs = 0.0
        for b in range(2):
            ik = 4 + b
            rb, eb = r[2 * b:2 * b + 2], e[2 * b:2 * b + 2]
            Td = kspace.transverse_precond_apply(N, wl.kpoints[ik], gam[ik], d[b], rb)
            T0 = kspace.transverse_precond_apply(N, wl.kpoints[ik], gam[ik], np.zeros((3, N ** 3)), rb)
            for j in range(2):
                rhs += w[2 * b + j] * float(np.vdot(eb[j], Td[j] - T0[j]).real)
        assert lhs == pytest.approx(rhs, rel=1e-5, abs=1e-9 * abs(rhs))


def _golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def test_solve_transverse_matches_oracle_and_converges_faster():
    g = _golden("sphere16_aniso")
    wl = W.sphere_anisotropic(N=16, nk=9, m=10)
    cases = [c for c in g["cases"] if c["scheme"] == "crossdof"]
    kpts = np.array([c["k"] for c in cases])
    op = kc.Op(16, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(kpts)
    note("solve transverse")
    e1, r1, i1, s1 = op.solve(10, tol=1e-8, batch_k=len(kpts), guard=2, precond=kc.KC_PRECOND_TRANSVERSE)
    e0, r0, i0, s0 = op.solve(10, tol=1e-8, batch_k=len(kpts), guard=2, precond=kc.KC_PRECOND_DIAG)
    assert s1 == 0 and r1.max() <= 1e-8
    for i, c in enumerate(cases):
        ref = np.array(c["eigenvalues"])
        assert np.max(np.abs(e1[i] - ref) / ref) <= 1e-6
    note("iterations diag", i0.tolist(), "transverse", i1.tolist())
    assert i1.sum() < i0.sum()


def test_solve_sphere32_mixed_transverse():
    """N = 32 anisotropic sphere (several FFT tiles per pencil), FP32 operator applications with
    the FP64 finish and T_E, against the oracle's shift-invert eigenvalues."""
    g = _golden("sphere32_aniso")
    wl = W.sphere_anisotropic(N=32, nk=9, m=g["m"])
    kpts = np.array([c["k"] for c in g["cases"]])
    op = kc.Op(32, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(kpts)
    note("solve sphere32 mixed transverse")
    eig, res, its, st = op.solve(g["m"], tol=1e-8, batch_k=len(kpts), guard=3, prec=kc.KC_PREC_FP32,
                                 switch_tol=1e-4, precond=kc.KC_PRECOND_TRANSVERSE)
    assert st == 0 and res.max() <= 1e-8
    for i, c in enumerate(g["cases"]):
        ref = np.array(c["eigenvalues"])
        assert np.max(np.abs(eig[i] - ref) / ref) <= 1e-6, (c["k"], eig[i], ref)


@pytest.mark.parametrize("m,guard", [(2, 1), (3, 1), (4, 1), (8, 0), (10, 3), (10, 6), (10, 11)])
@pytest.mark.parametrize("pc", [kc.KC_PRECOND_TRANSVERSE, kc.KC_PRECOND_DIAG])
def test_solve_block_sizes(m, guard, pc):
    """Block sizes mb = m + guard from 3 to 21: the update passes take whole groups of four
    columns when mb is a multiple of 4 and clamp per lane otherwise, and the fused update +
    residual pass (T_E) keeps 1 to 6 new X values per lane; every variant against the oracle's
    eigenvalues."""
    g = _golden("sphere16_aniso")
    wl = W.sphere_anisotropic(N=16, nk=9, m=10)
    cases = [c for c in g["cases"] if c["scheme"] == "crossdof"][:3]
    kpts = np.array([c["k"] for c in cases])
    op = kc.Op(16, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(kpts)
    note("solve m", m, "guard", guard, "precond", pc)
    eig, res, its, st = op.solve(m, tol=1e-8, batch_k=len(kpts), guard=guard, precond=pc)
    assert st == 0 and res.max() <= 1e-8
    for i, c in enumerate(cases):
        ref = np.array(c["eigenvalues"][:m])
        assert np.max(np.abs(eig[i] - ref) / ref) <= 1e-6, (m, guard, c["k"], eig[i], ref)
