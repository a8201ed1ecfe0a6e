"""Blocks of more than 21 columns per k-point (m + guard up to 32): the Gram products on the
96-column stage, the Rayleigh-Ritz with its matrices in global memory and the 96-row update
kernels, against the dense oracle eigenvalues, through kc_solve."""
import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W
from oracle import eigs, yee

from gpu_util import note

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,guard,precond", [(20, 2, kc.KC_PRECOND_DIAG), (24, 4, kc.KC_PRECOND_TRANSVERSE),
                                             (28, 4, kc.KC_PRECOND_TRANSVERSE), (30, 2, kc.KC_PRECOND_DIAG)])
def test_wide_blocks_match_dense_oracle(m, guard, precond):
    """Two k-points of the anisotropic sphere at N = 8 (CrossDoF), m bands with the guard columns
    taking the block to 22, 28 and 32 columns; every band within 1e-8 of the dense FP64
    eigenvalues, residuals at 1e-8."""
    N = 8
    wl = W.sphere_anisotropic(N=N, nk=9, m=m)
    kp = wl.kpoints[[2, 6]]
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(kp)
    g = op.gamma()
    note("wide block", m, guard, precond)
    eig, res, its, st = op.solve(m, tol=1e-8, guard=guard, batch_k=2, precond=precond, maxit=800)
    assert st == 0 and res.max() <= 1e-8, (its, res.max())
    for i in range(2):
        Op = yee.compensated_operator(N, kp[i], wl.ids, wl.table, "crossdof", gamma=g[i])
        ref = eigs.smallest_positive(Op, m, method="dense")
        assert np.max(np.abs(eig[i] - ref) / ref) <= 1e-8, (i, eig[i], ref)


def test_wide_block_mixed_precision_agrees_with_narrow():
    """The first 10 bands of a 22 + 4 column solve (FP32 phase, transverse preconditioner, fused
    update) equal those of a 10 + 2 column solve at N = 16."""
    N = 16
    wl = W.sphere_anisotropic(N=N, nk=9, m=10)
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints[[3]])
    note("wide mixed")
    e1, r1, i1, s1 = op.solve(10, tol=1e-8, guard=2, precond=kc.KC_PRECOND_TRANSVERSE, prec=kc.KC_PREC_FP32,
                              switch_tol=1e-4)
    e2, r2, i2, s2 = op.solve(22, tol=1e-8, guard=4, precond=kc.KC_PRECOND_TRANSVERSE, prec=kc.KC_PREC_FP32,
                              switch_tol=1e-4, maxit=800)
    assert s1 == 0 and s2 == 0
    assert np.max(np.abs(e2[0][:10] - e1[0]) / e1[0]) <= 1e-8
    assert np.all(np.diff(e2[0]) >= -1e-12)
