"""The C-ABI boundary beyond the operator itself (through the binding): caller allocator,
validation and warning flags, real-space transforms, the spurious-mode bound."""
import math

import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W
from oracle import kspace, yee

from gpu_util import max_err, note, to_dev, to_host

pytestmark = pytest.mark.gpu


def _aniso(N):
    wl = W.sphere_anisotropic(N=N, nk=3, m=4)
    return wl.ids, wl.table


def test_rejected_kpoints_leave_the_handle_unchanged():
    """kc_set_kpoints checks every k and gamma before it changes the handle."""
    ids, tab = _aniso(8)
    op = kc.Op(8, kc.KC_EPS_CROSSDOF, ids, tab)
    good = np.array([[0.3, 0.2, 0.1], [1.0, 1.0, 1.0]])
    op.set_kpoints(good)
    g0 = op.gamma()
    bad_k = np.array([[0.1, 0.2, 0.3], [np.nan, 0.0, 0.0], [0.5, 0.5, 0.5]])
    for kk, gg in [(bad_k, None), (good[:1].repeat(3, 0), np.array([1.0, 0.0, 2.0])),
                   (good, np.array([1.0, np.inf]))]:
        with pytest.raises(kc.KcError) as e:
            op.set_kpoints(kk, gamma=gg)
        assert e.value.status == 1
        assert op.nk == 2 and np.array_equal(op.gamma(), g0)
    note("apply after rejected set_kpoints")
    x = W.random_block(3, 2, 8)
    y = to_host(op.apply(to_dev(x), vecs_per_k=1))
    for ik in range(2):
        ref = kspace.kspace_apply(yee.compensated_operator(8, good[ik], ids, tab, "crossdof"), x[ik:ik + 1], 8)
        assert max_err(y[ik:ik + 1], ref) < 1e-12


def test_k_outside_flag():
    ids, tab = _aniso(8)
    op = kc.Op(8, kc.KC_EPS_CROSSDOF, ids, tab)
    op.set_kpoints(np.array([[math.pi, math.pi, math.pi], [0.0, 0.0, 0.0], [3.2, 0.0, 0.0], [0.0, -3.5, 1.0]]))
    f = op.kpoint_flags()
    assert list(f & kc.KC_KFLAG_K_OUTSIDE) == [0, 0, 1, 1]


@pytest.mark.parametrize("m", [1, 3])
def test_spurious_bound_is_the_penalty_spectrum_minimum(m):
    """gamma * s_min equals gamma times the smallest positive eigenvalue of B^H B (the oracle's
    divergence, eq (2.7)); Lemma 2.4 (2): s_min = |k|^2 for k != 0 with second-order stencils."""
    N = 6
    ids, tab = _aniso(N)
    kp = np.array([[0.3, 0.5, 0.7], [0.0, 0.0, 0.0], [math.pi, 0.0, 0.0], [0.0, 1.1, -0.4]])
    op = kc.Op(N, kc.KC_EPS_TRIVIAL, ids, tab, stencil_m=m)
    op.set_kpoints(kp)
    b = op.spurious_bound()
    g = op.gamma()
    for ik, k in enumerate(kp):
        B = yee.div_matrix(N, k, m).toarray()
        ev = np.linalg.eigvalsh(B.conj().T @ B)
        smin = ev[ev > 1e-9 * ev.max()].min()
        assert b[ik] == pytest.approx(g[ik] * smin, rel=1e-10)
        if m == 1 and np.dot(k, k) > 0:
            assert b[ik] == pytest.approx(g[ik] * np.dot(k, k), rel=1e-12)


def test_spurious_risk_flag_after_solve():
    """With the rule of eq (2.26) the lowest bands stay below gamma s_min; with a tiny gamma the
    penalty term's eigenvalues gamma s(p) come first, and the flag reports it."""
    N = 8
    ids, tab = _aniso(N)
    k = np.array([[0.4, 0.2, 0.1]])
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, ids, tab)
    op.set_kpoints(k)
    note("solve: gamma rule")
    eig, res, its, st = op.solve(4, tol=1e-8, guard=2)
    assert st == 0 and not (op.kpoint_flags()[0] & kc.KC_KFLAG_SPURIOUS_RISK)
    assert eig[0, -1] < op.spurious_bound()[0]
    op.set_kpoints(k, gamma=np.array([0.05]))
    note("solve: tiny gamma")
    eig2, res2, its2, st2 = op.solve(4, tol=1e-8, guard=2)
    assert st2 == 0 and (op.kpoint_flags()[0] & kc.KC_KFLAG_SPURIOUS_RISK)
    # the smallest eigenvalue is then the penalty term's gamma |k|^2 (Prop 2.3)
    assert eig2[0, 0] == pytest.approx(0.05 * float(np.dot(k[0], k[0])), rel=1e-6)


def _gershgorin_from_oracle(N, ids, tab, sch):
    M = yee.eps_matrix(N, ids, tab, sch).tocsr()
    d = M.diagonal().real
    off = np.asarray(abs(M).sum(axis=1)).ravel() - np.abs(M.diagonal())
    return bool(np.all(d > off))


@pytest.mark.parametrize("scheme", ["trivial", "crossdof"])
def test_hpd_flag_matches_gershgorin_of_the_oracle_matrix(scheme):
    """KC_FLAG_HPD_UNPROVEN is set exactly when some row of the oracle's explicit M is not
    strictly diagonally dominant: on the anisotropic sphere, on the gyrotropic woodpile (whose
    tensor satisfies the conditions of Props 3.8 / 3.10) and on a strongly coupled tensor."""
    N = 8
    strong = np.array([[0.4, 0.25, 0.25], [0.25, 0.4, 0.25], [0.25, 0.25, 0.4]], dtype=complex)
    wp = W.woodpile_gyrotropic(N=N, nk=3, m=4)
    cases = [_aniso(N), (wp.ids, wp.table)]
    ids_s = W.sample_ids(N, [W.Sphere((0.5, 0.5, 0.5), 0.3, 1)])
    cases.append((ids_s, np.stack([np.eye(3, dtype=complex), strong])))
    seen = set()
    for ids, tab in cases:
        op = kc.Op(N, kc.SCHEMES[scheme], ids, tab)
        proven = _gershgorin_from_oracle(N, ids, tab, scheme)
        assert (op.flags() & kc.KC_FLAG_HPD_UNPROVEN == 0) == proven
        seen.add(proven)
    assert seen == {True, False}


@pytest.mark.parametrize("N", [6, 16, 32])
def test_real_space_transforms(N):
    """H = F3 x (N^{3/2} numpy ifftn per component) and back."""
    ids, tab = _aniso(N) if N <= 16 else (np.zeros((4, N ** 3), dtype=np.uint8), W.eps_table([]))
    op = kc.Op(N, kc.KC_EPS_TRIVIAL, ids, tab)
    x = W.random_block(5 + N, 3, N)
    note("real space", N)
    H = to_host(op.to_real_space(to_dev(x)))
    ref = kspace.F3(x, N)
    assert max_err(H, ref) < 1e-14 * math.log2(N) * 4
    xd = to_dev(x)
    op.to_real_space(xd, out=xd)
    op.to_kspace(xd, out=xd)
    assert max_err(to_host(xd), x) < 1e-14 * math.log2(N) * 4


def test_workspaces_come_from_the_torch_allocator():
    """The handle's device buffers are drawn from PyTorch's caching allocator (the default), and
    the hipMalloc variant gives the same results."""
    import torch

    N = 16
    ids, tab = _aniso(N)
    k = np.array([[0.3, 0.5, 0.7]])
    x = to_dev(W.random_block(1, 4, N))
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, ids, tab)
    op.set_kpoints(k)
    note("allocator: torch")
    y1 = op.apply(x)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - before - y1.numel() * 16
    # ids, tables and the two work buffers of 4 vectors at least
    assert grown >= 4 * N ** 3 + 2 * 4 * 3 * N ** 3 * 16
    op2 = kc.Op(N, kc.KC_EPS_CROSSDOF, ids, tab, allocator="hip")
    op2.set_kpoints(k)
    note("allocator: hip")
    y2 = op2.apply(x)
    assert torch.equal(y1, y2)
    op.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - before <= 2 * y1.numel() * 16
