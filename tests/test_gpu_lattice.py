"""General lattices through the coordinate transform (Section 2.2, eq (2.12)) on the HIP path,
against the oracle: operator applications (both discretisations, FP64 and FP32, second and
fourth order), the preconditioners, eigenvalues, the penalty spectrum's bottom, and the
free-photon spectrum of a homogeneous FCC crystal at 64^3."""
import math

import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W
from oracle import eigs, kspace, yee

from gpu_util import max_err, note, to_dev, to_host

pytestmark = pytest.mark.gpu
LATS = ["fcc", "bcc", "tric"]
KPTS = [(0.3, 0.5, 0.7), (0.0, 0.0, 0.0), (math.pi, 2 * math.pi, 0.0), (-1.2, 0.4, 2.1)]


def _case(lat, N, scheme):
    wl = W.lattice_sphere(lat, N, radius=0.22, eps=W.rotated_eps(np.random.default_rng(3), 4.0, 12.0),
                          scheme=scheme)
    return wl.ids, wl.table, W.LATTICES[lat]


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("N,scheme,m", [(8, "crossdof", 1), (12, "trivial", 1), (8, "crossdof", 2)])
def test_apply_matches_oracle(lat, N, scheme, m):
    ids, tab, L = _case(lat, N, scheme)
    op = kc.Op(N, kc.SCHEMES[scheme], ids, tab, lattice=L, stencil_m=m)
    op.set_kpoints(np.array(KPTS))
    x = W.random_block(20 + N, len(KPTS), N)
    note("lattice apply", lat, N, scheme, m)
    y64 = to_host(op.apply(to_dev(x), vecs_per_k=1))
    y32 = to_host(op.apply(to_dev(x), vecs_per_k=1, prec=kc.KC_PREC_FP32))
    for ik, k in enumerate(KPTS):
        Op = yee.compensated_operator(N, k, ids, tab, scheme, m=m, lattice=L)
        ref = kspace.kspace_apply(Op, x[ik:ik + 1], N)
        assert max_err(y64[ik:ik + 1], ref) < 1e-12, (k, max_err(y64[ik:ik + 1], ref))
        assert max_err(y32[ik:ik + 1], ref) < 3e-6


@pytest.mark.parametrize("lat", LATS)
def test_preconditioners_match_oracle(lat):
    N = 8
    ids, tab, L = _case(lat, N, "crossdof")
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, ids, tab, lattice=L)
    op.set_kpoints(np.array(KPTS))
    r = W.random_block(5, len(KPTS), N)
    note("lattice precond", lat)
    z = to_host(op.precond(to_dev(r), vecs_per_k=1))
    t = to_host(op.precond_transverse(to_dev(r), vecs_per_k=1))
    E = kspace.edge_permittivity(ids, tab).astype(np.float32).astype(np.float64)  # the library keeps E in FP32
    for ik, k in enumerate(KPTS):
        g = yee.gamma_rule(k)
        assert max_err(z[ik:ik + 1], kspace.precond_apply(N, k, g, r[ik:ik + 1], lattice=L)) < 1e-12
        assert max_err(t[ik:ik + 1], kspace.transverse_precond_apply(N, k, g, E, r[ik:ik + 1], lattice=L)) < 1e-12


@pytest.mark.parametrize("start", ["random", "plane_waves"])
@pytest.mark.parametrize("lat,N", [("fcc", 8), ("bcc", 8), ("tric", 12)])
def test_eigenvalues_match_oracle(lat, N, start):
    ids, tab, L = _case(lat, N, "crossdof")
    kp = np.array([KPTS[0], KPTS[2]])
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, ids, tab, lattice=L)
    op.set_kpoints(kp)
    note("lattice solve", lat, N, start)
    eig, res, its, st = op.solve(8, tol=1e-8, guard=3, batch_k=2, precond=kc.KC_PRECOND_TRANSVERSE,
                                 start=start)
    assert st == 0 and res.max() <= 1e-8
    for ik, k in enumerate(kp):
        Op = yee.compensated_operator(N, k, ids, tab, "crossdof", lattice=L)
        ref = eigs.smallest_positive(Op, 8, method="dense")
        assert np.max(np.abs(eig[ik] - ref) / ref) <= 1e-6, (lat, k, eig[ik], ref)


@pytest.mark.parametrize("lat", LATS)
def test_spurious_bound_on_lattices(lat):
    N = 6
    ids, tab, L = _case(lat, N, "trivial")
    kp = np.array([KPTS[0], KPTS[1], KPTS[3]])
    op = kc.Op(N, kc.KC_EPS_TRIVIAL, ids, tab, lattice=L)
    op.set_kpoints(kp)
    b, g = op.spurious_bound(), op.gamma()
    for ik, k in enumerate(kp):
        B = yee.div_matrix(N, k, 1, L).toarray()
        ev = np.linalg.eigvalsh(B.conj().T @ B)
        assert b[ik] == pytest.approx(g[ik] * ev[ev > 1e-9 * ev.max()].min(), rel=1e-10)


def test_fcc_homogeneous_free_photon_spectrum_n64():
    """Homogeneous FCC crystal at 64^3 through the bench's path (FP32 phase, T_E, guard columns):
    the 12 lowest eigenvalues are c s(p) (twice) from the oracle's order-2 lattice symbols."""
    N, c = 64, 1.0 / 4.0
    L = W.LATTICES["fcc"]
    ids = np.ones((4, N ** 3), dtype=np.uint8)
    tab = W.eps_table([4.0 * np.eye(3)])
    k = np.array([0.4, 2.3, 0.9])
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, ids, tab, lattice=L)
    op.set_kpoints(k[None])
    note("fcc free photon n64")
    eig, res, its, st = op.solve(12, tol=1e-8, guard=4, prec=kc.KC_PREC_FP32, switch_tol=3e-4,
                                 precond=kc.KC_PRECOND_TRANSVERSE)
    assert st == 0 and res.max() <= 1e-8
    K = kspace.symbols_3d(N, k, 1, L)
    s = np.sum(np.abs(K) ** 2, axis=0)
    g = yee.gamma_rule(k)
    ref = np.sort(np.concatenate([c * s, c * s, g * s]))[:12]
    assert np.max(np.abs(eig[0] - ref) / ref) <= 1e-6, (eig[0], ref)


def test_fcc_homogeneous_plane_wave_start_is_exact():
    """In a homogeneous isotropic medium the transverse plane waves are eigenvectors of the
    k-space operator (eq (2.30) with Lemma 2.4 (1)), so the plane-wave start built from the FCC
    lattice's symbols (eq (2.12)) must hold the 12 lowest eigenvectors already: the solve ends
    within a few iterations, at the free-photon values."""
    N, c = 32, 1.0 / 4.0
    L = W.LATTICES["fcc"]
    ids = np.ones((4, N ** 3), dtype=np.uint8)
    tab = W.eps_table([4.0 * np.eye(3)])
    k = np.array([0.4, 2.3, 0.9])
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, ids, tab, lattice=L)
    op.set_kpoints(k[None])
    note("fcc plane-wave start n32")
    eig, res, its, st = op.solve(12, tol=1e-8, guard=4, precond=kc.KC_PRECOND_TRANSVERSE, start="plane_waves")
    assert st == 0 and res.max() <= 1e-8
    K = kspace.symbols_3d(N, k, 1, L)
    s = np.sum(np.abs(K) ** 2, axis=0)
    ref = np.sort(np.concatenate([c * s, c * s, yee.gamma_rule(k) * s]))[:12]
    assert np.max(np.abs(eig[0] - ref) / ref) <= 1e-10, (eig[0], ref)
    assert its[0] <= 3, its
