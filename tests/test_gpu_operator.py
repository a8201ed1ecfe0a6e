"""Parity of the HIP path (through the C ABI) against the CPU FP64 oracle: 3D DFT, operator
application and preconditioner, on seeded inputs at grids that span several tiles and
ragged shapes.  Every comparison is element-wise: max |gpu - ref| / max |ref|."""
import math

import numpy as np
import pytest

import paper_2511_17107_amd as kc
import workloads as W
from oracle import kspace, yee

from gpu_util import max_err, note, to_dev, to_host

pytestmark = pytest.mark.gpu

SMALL_N = [4, 6, 8, 12, 16]
KPTS = [(0.3, 0.5, 0.7), (0.0, 0.0, 0.0), (math.pi, math.pi, math.pi), (math.pi, 0.9, 0.0), (-1.2, 0.4, 2.1)]


# ---------------------------------------------------------------- 3D DFT
@pytest.mark.parametrize("N", [4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128])
@pytest.mark.parametrize("sign", [1, -1])
def test_fft3d_fp64(N, sign):
    import torch

    nvec = 3 if N <= 32 else 1
    note("fft3d fp64", N, sign)
    a = W.random_block(100 + N, nvec, N)[:, 0, :]
    x = to_dev(a)
    y = to_host(kc.kc_fft3d(x, sign, kc.KC_PREC_FP64))
    cube = a.reshape(nvec, N, N, N)
    if N <= 8:
        # direct DFT definition along each axis
        ref = cube
        for ax in (3, 2, 1):
            ref = np.moveaxis(kspace.direct_dft(np.moveaxis(ref, ax, -1), sign), -1, ax)
    else:
        ref = np.fft.fftn(cube, axes=(1, 2, 3)) if sign < 0 else np.fft.ifftn(cube, axes=(1, 2, 3)) * N ** 3
    ref = ref.reshape(nvec, -1)
    assert max_err(y, ref) < 1e-14 * math.log2(N) * 4
    # in place
    x2 = to_dev(a)
    kc.kc_fft3d(x2, sign, kc.KC_PREC_FP64, out=x2)
    assert max_err(to_host(x2), ref) < 1e-14 * math.log2(N) * 4
    del torch


@pytest.mark.parametrize("N", [6, 16, 96, 128])
def test_fft3d_fp32(N):
    import torch

    note("fft3d fp32", N)
    a = W.random_block(200 + N, 1, N)[:, 0, :]
    x = to_dev(a.astype(np.complex64))
    y = to_host(kc.kc_fft3d(x, -1, kc.KC_PREC_FP32))
    ref = np.fft.fftn(a.reshape(1, N, N, N), axes=(1, 2, 3)).reshape(1, -1)
    assert max_err(y, ref) < 3e-7 * math.log2(N)
    del torch


# ---------------------------------------------------------------- operator
def _case(N, scheme_name, seed=0):
    if scheme_name == "iso":
        wl = W.sphere_isotropic(N=N)
        return wl.ids, wl.table, "crossdof"
    if scheme_name == "gyro":
        # gyrotropic materials only ((eps^-1)_13 = (eps^-1)_23 = 0 everywhere: the stencil pass
        # drops the blocks (1,3) and (2,3)), two of them so that ids differ between point sets
        ids = W.sample_ids(N, [W.Sphere((0.5, 0.5, 0.5), 0.3, 1), W.Rod(2, (0.1, 0.2, 0.0), 0.17, 2)])
        tab = W.eps_table([W.gyrotropic_eps(12.0, 0.5, 10.0), W.gyrotropic_eps(7.0, -0.8, 4.0)])
        return ids, tab, "crossdof"
    wl = W.sphere_anisotropic(N=N, nk=2, m=4, seed=seed)
    # add a second inclusion with a gyrotropic tensor so all off-diagonals and complex
    # entries are exercised, and material ids differ between the point sets
    ids = W.sample_ids(N, [W.Sphere((0.5, 0.5, 0.5), 0.3, 1), W.Rod(2, (0.1, 0.2, 0.0), 0.17, 2)])
    tab = np.concatenate([wl.table, W.eps_table([W.gyrotropic_eps(12.0, 0.5, 10.0)])[1:]])
    return ids, tab, scheme_name


@pytest.mark.parametrize("N", SMALL_N)
@pytest.mark.parametrize("scheme", ["diagonal", "trivial", "crossdof", "iso", "gyro"])
def test_apply_fp64_matches_oracle(N, scheme):
    ids, tab, sch = _case(N, scheme)
    op = kc.Op(N, kc.SCHEMES[sch], ids, tab)
    op.set_kpoints(np.array(KPTS))
    nvec_per_k = 2
    x = W.random_block(7 + N, nvec_per_k * len(KPTS), N)
    note("apply fp64", N, scheme)
    y = to_host(op.apply(to_dev(x), ik0=0, vecs_per_k=nvec_per_k))
    for ik, k in enumerate(KPTS):
        Op = yee.compensated_operator(N, k, ids, tab, sch)
        ref = kspace.kspace_apply(Op, x[ik * nvec_per_k:(ik + 1) * nvec_per_k], N)
        err = max_err(y[ik * nvec_per_k:(ik + 1) * nvec_per_k], ref)
        assert err < 1e-12, (k, err)


@pytest.mark.parametrize("N", [8, 16])
@pytest.mark.parametrize("scheme", ["trivial", "crossdof", "gyro"])
def test_apply_fp32_close_to_oracle(N, scheme):
    ids, tab, sch = _case(N, scheme)
    op = kc.Op(N, kc.SCHEMES[sch], ids, tab)
    op.set_kpoints(np.array(KPTS[:2]))
    x = W.random_block(3, 4, N)
    note("apply fp32", N, scheme)
    y = to_host(op.apply(to_dev(x), vecs_per_k=2, prec=kc.KC_PREC_FP32))
    for ik, k in enumerate(KPTS[:2]):
        Op = yee.compensated_operator(N, k, ids, tab, sch)
        ref = kspace.kspace_apply(Op, x[2 * ik:2 * ik + 2], N)
        assert max_err(y[2 * ik:2 * ik + 2], ref) < 2e-6


@pytest.mark.parametrize("N", [4, 8, 16])
def test_precond_matches_oracle(N):
    ids, tab, sch = _case(N, "crossdof")
    op = kc.Op(N, kc.SCHEMES[sch], ids, tab)
    op.set_kpoints(np.array(KPTS))
    r = W.random_block(11, len(KPTS), N)
    note("precond", N)
    z = to_host(op.precond(to_dev(r), vecs_per_k=1))
    g = op.gamma()
    for ik, k in enumerate(KPTS):
        assert g[ik] == pytest.approx(yee.gamma_rule(k), rel=1e-15)
        ref = kspace.precond_apply(N, k, g[ik], r[ik:ik + 1])
        assert max_err(z[ik:ik + 1], ref) < 1e-13
    # in place
    rr = to_dev(r)
    op.precond(rr, vecs_per_k=1, out=rr)
    assert max_err(to_host(rr)[0:1], kspace.precond_apply(N, KPTS[0], g[0], r[0:1])) < 1e-13


@pytest.mark.parametrize("N", [32, 64, 128])
def test_apply_homogeneous_closed_form_large(N):
    """At full grid sizes: for a homogeneous anisotropic medium and the Trivial scheme,
    F3^H M F3 = eps1 per frequency, so Op_p = K_A eps1 K_A^H + gamma conj(K) K^T is a 3x3
    per-frequency map that the oracle symbols give independently of any FFT."""
    eps = W.gyrotropic_eps(12.0, 0.5, 10.0)
    ids = np.ones((4, N ** 3), dtype=np.uint8)
    tab = W.eps_table([eps])
    k = (0.4, -1.3, 2.2)
    op = kc.Op(N, kc.KC_EPS_TRIVIAL, ids, tab)
    op.set_kpoints(np.array([k]))
    x = W.random_block(5, 1, N)
    note("apply homogeneous", N)
    y = to_host(op.apply(to_dev(x)))[0]
    K = kspace.symbols_3d(N, k)
    v = K.conj()
    e1 = tab[1]
    e = -np.cross(v.T, x[0].T).T
    yy = np.cross(K.T, (e1 @ e).T).T + yee.gamma_rule(k) * v * (K * x[0]).sum(axis=0)[None, :]
    assert max_err(y, yy) < 1e-12


@pytest.mark.parametrize("N", [32, 64])
def test_apply_hermitian_positive(N):
    """Properties at any size: <u, Op w> = <Op u, w> and <u, Op u> > 0 for k != 0 (Prop 2.5)."""
    wl = W.sphere_anisotropic(N=N, nk=3, m=4)
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints[1:2])
    uw = W.random_block(9, 2, N)
    note("apply hermitian", N)
    out = to_host(op.apply(to_dev(uw)))
    a = np.vdot(uw[0], out[1])
    b = np.vdot(out[0], uw[1])
    assert abs(a - b) < 1e-12 * abs(a)
    assert np.vdot(uw[0], out[0]).real > 0


@pytest.mark.parametrize("scheme,prec,tol", [("crossdof", kc.KC_PREC_FP64, 1e-11), ("trivial", kc.KC_PREC_FP64, 1e-11),
                                             ("crossdof", kc.KC_PREC_FP32, 3e-6), ("gyro", kc.KC_PREC_FP64, 1e-11),
                                             ("gyro", kc.KC_PREC_FP32, 3e-6)])
def test_apply_n128_tiled_geometry_matches_scaled_oracle(scheme, prec, tol):
    """Full-size parity at N = 128, the benchmark's grid: with a geometry that repeats every 16
    cells and a field of the same period, the 128^3 operator at wave vector k equals 64 times the
    16^3 operator at k/8, tiled.  Every difference carries 1/h (h = 1/128 against 1/16), and the
    shifted 1D operators scale as (I - S)/h + i k (I + S)/2 = 8 [(I - S)/(1/16) + i (k/8)(I + S)/2];
    the averages of the CrossDoF scheme are index-based, so they do not change; gamma is set
    explicitly.  Compared element by element (max |diff| / max |ref|) over the whole 3 x 128^3
    real-space output."""
    n, N = 16, 128
    rep = N // n
    ids16, tab, sch = _case(n, scheme)
    ids = np.tile(ids16.reshape(4, n, n, n), (1, rep, rep, rep)).reshape(4, -1)
    k16 = np.array([0.4, -1.3, 2.2])
    g = 7.5
    op = kc.Op(N, kc.SCHEMES[sch], ids, tab)
    op.set_kpoints((rep * k16)[None], gamma=np.array([g]))
    H16 = W.random_block(21, 2, n)
    H = np.tile(H16.reshape(2, 3, n, n, n), (1, 1, rep, rep, rep)).reshape(2, 3, -1)
    x = kspace.F3H(H, N)
    note("apply n128 tiled", scheme, prec)
    y = to_host(op.apply(to_dev(x), prec=prec))
    Y = kspace.F3(y, N)
    Op16 = yee.compensated_operator(n, k16, ids16, tab, sch, gamma=g)
    ref16 = (Op16 @ H16.reshape(2, -1).T).T.reshape(2, 3, n, n, n) * rep ** 2
    ref = np.tile(ref16, (1, 1, rep, rep, rep)).reshape(2, 3, -1)
    assert max_err(Y, ref) < tol


def _oracle_apply_factored(N, k, ids, tab, sch, x, m=1):
    """y = F3^H (A M A^H + gamma B^H B) F3 x with the oracle's sparse factors of eqs (2.7),
    (3.3)-(3.8) applied one after the other (the product Op is never formed, which keeps large
    grids within the oracle's reach)."""
    A = yee.curl_matrix(N, k, m)
    B = yee.div_matrix(N, k, m)
    M = yee.eps_matrix(N, ids, tab, sch)
    g = yee.gamma_rule(k)
    H = kspace.F3(np.asarray(x, dtype=np.complex128), N).reshape(x.shape[0], -1).T
    Y = A @ (M @ (A.conj().T @ H)) + g * (B.conj().T @ (B @ H))
    return kspace.F3H(Y.T.reshape(x.shape), N)


@pytest.mark.parametrize("N,nk", [(24, 2), (48, 2), (96, 1)])
@pytest.mark.parametrize("scheme", ["trivial", "crossdof"])
def test_apply_radix3_grids_match_oracle(N, nk, scheme):
    """The radix-3 FFT plans (24 = 8 x 3, 48 = 16 x 3, 96 = 32 x 3) against the oracle's sparse
    factors, element by element over the whole output, FP64 and FP32."""
    ids, tab, sch = _case(N, scheme)
    op = kc.Op(N, kc.SCHEMES[sch], ids, tab)
    kp = np.array(KPTS[:nk])
    op.set_kpoints(kp)
    x = W.random_block(40 + N, nk, N)
    note("apply radix-3", N, scheme)
    y64 = to_host(op.apply(to_dev(x), vecs_per_k=1))
    y32 = to_host(op.apply(to_dev(x), vecs_per_k=1, prec=kc.KC_PREC_FP32))
    for ik in range(nk):
        ref = _oracle_apply_factored(N, kp[ik], ids, tab, sch, x[ik:ik + 1])
        assert max_err(y64[ik:ik + 1], ref) < 1e-12
        assert max_err(y32[ik:ik + 1], ref) < 3e-6


@pytest.mark.parametrize("m", [2, 3, 4, 5])
@pytest.mark.parametrize("N,scheme", [(8, "crossdof"), (12, "trivial"), (12, "crossdof")])
def test_apply_high_order_matches_oracle(m, N, scheme):
    """Order-2m curl and divergence stencils (eq (2.34), coefficients of eq (2.35)) against the
    oracle's wide circulants, FP64, several k-points including k = 0 and the zone corner."""
    ids, tab, sch = _case(N, scheme)
    op = kc.Op(N, kc.SCHEMES[sch], ids, tab, stencil_m=m)
    op.set_kpoints(np.array(KPTS))
    x = W.random_block(60 + m, len(KPTS), N)
    note("apply high order", m, N, scheme)
    y = to_host(op.apply(to_dev(x), vecs_per_k=1))
    for ik, k in enumerate(KPTS):
        Op = yee.compensated_operator(N, k, ids, tab, sch, m=m)
        assert max_err(y[ik:ik + 1], kspace.kspace_apply(Op, x[ik:ik + 1], N)) < 1e-12, (m, k)


@pytest.mark.parametrize("m", [3, 5])
def test_apply_high_order_homogeneous_n64(m):
    """At N = 64 with order-2m stencils: the homogeneous Trivial operator is the per-frequency
    3 x 3 map K_A eps1 K_A^H + gamma conj(K) K^T with the oracle's order-2m symbols."""
    N = 64
    eps = W.gyrotropic_eps(12.0, 0.5, 10.0)
    ids = np.ones((4, N ** 3), dtype=np.uint8)
    tab = W.eps_table([eps])
    k = (0.9, -0.2, 1.7)
    op = kc.Op(N, kc.KC_EPS_TRIVIAL, ids, tab, stencil_m=m)
    op.set_kpoints(np.array([k]))
    x = W.random_block(77, 1, N)
    note("apply high order homogeneous", m)
    y = to_host(op.apply(to_dev(x)))[0]
    K = kspace.symbols_3d(N, k, m)
    v = K.conj()
    e = -np.cross(v.T, x[0].T).T
    yy = np.cross(K.T, (tab[1] @ e).T).T + yee.gamma_rule(k) * v * (K * x[0]).sum(axis=0)[None, :]
    assert max_err(y, yy) < 1e-12
