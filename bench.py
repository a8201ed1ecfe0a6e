#!/usr/bin/env python3
"""Throughput benchmark: k-points per second to Res_j <= 1e-8 (eq (4.3)) for the simple-cubic
woodpile of four rod layers (rod width 0.25a) with gyrotropic permittivity
eps = [[12, 0.5i, 0], [-0.5i, 12, 0], [0, 0, 10]] at N = 128 (3 x 128^3 = 6.3M unknowns),
CrossDoF inverse permittivity, 16 bands, 60 k-points on Gamma-X-M-Gamma-R, FP32 operator
applications with FP64 orthogonalisation / Rayleigh-Ritz / residual checks.

One step = one kc_solve of a batch of k-points (default 10, interleaved along the 60-point
path so that consecutive steps walk the whole path; ~180 GB of HBM for the batch's blocks).  Inputs (geometry, tables, k-points)
are resident before the timed region; the solve allocates its block workspace once and
reuses it.  Prints one JSON line (see the keys below).

    python bench.py [--steps K] [--warmup W] [--kpb 10] [--guard 4] [--prec fp32|fp64]
                    [--precond transverse|diag] [--no-cpu-baseline]
    python bench.py --matvec-only | --update-only | --gram-only   (single kernels, for rocprofv3)

`roofline` is the fused block update + residual pass (the largest kernel of a step), timed live
at the solve's batch shape after the solve; `matvec` lists the operator passes, the roofline of
the whole application (pass-structure bytes, counter bytes and the boundary's bytes over its
time) and that of its longest pass.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch, from rocprofv3 FETCH_SIZE (x 2.0) and WRITE_SIZE (x 1.0), the factors
# read off a plain 1 GiB device copy in the same run: operator passes on 16 vectors at 128^3,
# FP32, keyed by pass and tile width (profiles/matvec_woodpile128_fp32_16vec.md; the stencil pass Zb
# as it runs on the woodpile, whose materials couple no z); the fused
# update keyed by N, k-points and block width (profiles/update_woodpile128_10k_20col.md).
MEASURED_TRAFFIC = {
    ("X1", 128, 16, "fp32", 4): 2.953e9, ("X1", 128, 16, "fp32", 8): 2.953e9, ("X1", 128, 16, "fp32", 16): 2.953e9,
    ("Y1", 128, 16, "fp32", 4): 4.027e9, ("Y1", 128, 16, "fp32", 8): 2.416e9, ("Y1", 128, 16, "fp32", 16): 1.611e9,
    ("Y1", 128, 16, "fp32", 32): 1.611e9,
    ("Za", 128, 16, "fp32", 4): 4.027e9, ("Za", 128, 16, "fp32", 8): 2.416e9, ("Za", 128, 16, "fp32", 16): 1.611e9,
    ("Za", 128, 16, "fp32", 32): 1.611e9,
    ("Zb", 128, 16, "fp32", 4): 1.777e9, ("Zb", 128, 16, "fp32", 8): 1.757e9, ("Zb", 128, 16, "fp32", 16): 1.755e9,
    ("Y2", 128, 16, "fp32", 4): 4.027e9, ("Y2", 128, 16, "fp32", 8): 2.416e9, ("Y2", 128, 16, "fp32", 16): 1.611e9,
    ("Y2", 128, 16, "fp32", 32): 1.611e9,
    ("X2", 128, 16, "fp32", 4): 2.953e9, ("X2", 128, 16, "fp32", 8): 2.953e9, ("X2", 128, 16, "fp32", 16): 2.954e9,
    ("update", 128, 10, 20): 221.51e9,
}
# tile-width slot of each CrossDoF operator pass in kc_tile_widths
PASS_SLOT = {"X1": 0, "Y1": 1, "Za": 2, "Zb": 3, "Y2": 5, "X2": 6}
FP64_MFMA_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--kpb", type=int, default=10, help="k-points per step (one batched solve)")
    ap.add_argument("--nk", type=int, default=60)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--m", type=int, default=16)
    ap.add_argument("--guard", type=int, default=4)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--switch-tol", type=float, default=3e-4)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=600)
    ap.add_argument("--precond", choices=["diag", "transverse"], default="transverse",
                    help="LOBPCG preconditioner: diagonal-block K_P^-1 or transverse-projection T_E")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--start", choices=["plane_waves", "random"], default="plane_waves",
                    help="start block of every solve: seeded random (preconditioned), or the k-point's lowest "
                         "transverse plane waves")
    ap.add_argument("--warm-start", action="store_true",
                    help="sweep the path: each timed step after the first starts its k-points from the "
                         "converged fields of the previous step's (their neighbours on the path)")
    ap.add_argument("--matvec-only", action="store_true",
                    help="only the operator application on one block (and a plain device copy of known "
                         "size, the reference for hardware byte counters); for profiling")
    ap.add_argument("--update-only", action="store_true",
                    help="only the fused block update (kc_block_update) at the solve's batch shape, three "
                         "launches, and the 1 GiB device copy; for profiling")
    ap.add_argument("--gram-only", action="store_true",
                    help="only the Gram products S^H AS, S^H S (kc_block_gram) at the solve's batch shape, "
                         "three launches; for profiling the MFMA counters")
    ap.add_argument("--workload", choices=["c4", "c2", "c3", "c5"], default="c4",
                    help="c4: the headline (128^3 woodpile); c2: 64^3 anisotropic sphere, 20 bands, 40 "
                         "k-points, FP64; c3: the same sphere, 16 bands, 120 k-points in two launch sets, "
                         "mixed precision against the FP64 path (per-band eigenvalue differences); c5: train "
                         "the learned preconditioner on 500 random geometries (32^3 and 64^3) and compare it at "
                         "96^3 (40 k-points) with the FP64 diagonal-preconditioned path")
    ap.add_argument("--c5-geoms", type=int, nargs=2, default=[400, 100],
                    help="training geometries at 32^3 and at 64^3 (c5)")
    ap.add_argument("--c5-steps", type=int, default=600)
    ap.add_argument("--c2-guard", type=int, default=4, help="guard columns of the c2 workload (20 bands)")
    ap.add_argument("--verbose", type=int, default=0)
    return ap.parse_args()


def pass_bytes(N, nvec, scheme_cross, tbytes):
    """Algorithmic bytes of each pencil pass of one operator application: what the pass must
    read and write once (complex128 input/output vectors, compute-precision intermediates,
    4-byte packed material ids, and the complex128 K.x per point that X1 hands to X2)."""
    n3 = N ** 3
    v64 = 16 * 3 * n3 * nvec
    vt = tbytes * 3 * n3 * nvec
    ids = 4 * n3 * nvec
    kx = 16 * n3 * nvec
    if scheme_cross:
        names = ["X1", "Y1", "Za", "Zb", "Y2", "X2"]
        b = [v64 + vt + kx, 2 * vt, 2 * vt, 2 * vt + ids, 2 * vt, vt + kx + v64]
    else:
        names = ["X1", "Y1", "Z", "Y2", "X2"]
        b = [v64 + vt + kx, 2 * vt, 2 * vt + ids, 2 * vt, vt + kx + v64]
    return names, b


def cpu_baseline(kpath):
    """The oracle (explicit sparse operator + shift-invert Lanczos) on the same woodpile geometry
    and k-path at the largest grid it solves in well under a minute (N = 16)."""
    ncpu = min(len(os.sched_getaffinity(0)), 16)
    os.environ["OPENBLAS_NUM_THREADS"] = str(ncpu)
    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(limits=ncpu)
    except Exception:
        pass
    import workloads as W
    from oracle import eigs, yee

    wl = W.woodpile_gyrotropic(N=16, nk=60, m=16)
    ks = [kpath[7]]
    t = time.time()
    for k in ks:
        Op = yee.compensated_operator(wl.N, k, wl.ids, wl.table, "crossdof")
        eigs.smallest_positive(Op, 16, method="shift_invert")
    dt = time.time() - t
    return {"value": len(ks) / dt, "unit": "k-points/s", "cores": ncpu, "kind": "oracle",
            "sample": "oracle shift-invert Lanczos on the explicit sparse operator, same woodpile/"
                      "gyrotropic geometry and k-path, N=16 (3*16^3 unknowns), 16 bands, 1 k-point "
                      "(%.1f s); the oracle cannot factor the N=128 operator" % dt}


def matvec_only(a, op, prec, dev):
    """Three operator applications on one block of a.m vectors, then three copies of a 1 GiB
    buffer (torch's copy kernel: 1 GiB read + 1 GiB written per launch)."""
    import torch

    x = torch.randn((a.m, 3, a.N ** 3), dtype=torch.complex128, device=dev)
    for r in range(3):
        y = op.apply(x, prec=prec)
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for r in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"matvec_vectors": a.m, "N": a.N, "copy_bytes_each_way": src.numel() * 8,
                      "checksum": float(y.abs().sum()) + float(dst[0])}), flush=True)


def update_block(a, dev):
    """Seeded inputs of the fused update at the solve's shape: blocks S, AS of kpb k-points x 3mb
    columns x 3N^3 rows, coefficients scaled so that repeated in-place updates keep the
    magnitudes, Ritz values in the woodpile's range."""
    import torch

    import workloads as W

    mb, nb, n = a.m + a.guard, a.kpb, 3 * a.N ** 3
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    S = torch.randn((nb, 3 * mb, n), dtype=torch.complex128, device=dev, generator=g)
    AS = torch.randn((nb, 3 * mb, n), dtype=torch.complex128, device=dev, generator=g)
    C = torch.from_numpy(W.random_complex(8, (nb, 3 * mb, 2 * mb)) / np.sqrt(6 * mb)).to(dev)
    theta = torch.from_numpy(np.random.default_rng(9).uniform(0.05, 0.5, (nb, mb))).to(dev)
    return S, AS, C, theta


def gram_only(a, dev):
    """Three Gram launches (GA = S^H AS, GB = S^H S over 3mb columns per k-point) at the solve's
    batch shape, with their HIP-event durations and the FP64 MFMA rate they imply."""
    import torch

    import paper_2511_17107_amd as kc

    mb, nb, n = a.m + a.guard, a.kpb, 3 * a.N ** 3
    S, AS, _, _ = update_block(a, dev)
    nc = 3 * mb
    GA = torch.empty((nb, nc, nc), dtype=torch.complex128, device=dev)
    GB = torch.empty_like(GA)
    work = torch.empty(kc.block_work_bytes(nb, n, nc), dtype=torch.uint8, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    for r in range(3):
        ev[2 * r].record()
        kc.block_gram(S, AS, GA, GB, work)
        ev[2 * r + 1].record()
    torch.cuda.synchronize()
    ms = [ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(3)]
    flops = 2 * nb * n * nc * nc * 8  # two nc x nc complex products over n rows (8 real flops per complex MAC)
    print(json.dumps({"gram_kpoints": nb, "columns": nc, "N": a.N, "ms": ms,
                      "tflops": flops / (min(ms) * 1e-3) / 1e12, "checksum": float(GB.abs().sum())}), flush=True)


def update_roofline(a, dev, reps=5):
    """The fused update + residual pass (the largest share of a solve step) timed live with HIP
    events on the stream it runs on, at the solve's batch shape."""
    import torch

    import paper_2511_17107_amd as kc

    mb, nb, n = a.m + a.guard, a.kpb, 3 * a.N ** 3
    S, AS, C, theta = update_block(a, dev)
    R = torch.empty((nb, mb, n), dtype=torch.complex128, device=dev)
    res = torch.empty((nb, mb), dtype=torch.float64, device=dev)
    xn2 = torch.empty_like(res)
    work = torch.empty(kc.block_work_bytes(nb, n, 3 * mb), dtype=torch.uint8, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * (reps + 1))]
    for r in range(reps + 1):
        ev[2 * r].record()
        kc.block_update(S, AS, C, theta, R, res, xn2, work)
        ev[2 * r + 1].record()
    torch.cuda.synchronize()
    ms = sum(ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(1, reps + 1)) / reps
    alg_bytes = nb * n * 11 * mb * 16          # read S, AS (3mb each); write X, P, AX, AP, R
    alg_flops = nb * n * 2 * (3 * mb) * (2 * mb) * 8  # two 3mb x 2mb complex products per row
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    del S, AS, R, work
    torch.cuda.empty_cache()
    return {"bound": "hbm", "kernel": "fused block update + residuals (k_update_res)",
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": MEASURED_TRAFFIC.get(("update", a.N, nb, mb)), "alg_bytes": alg_bytes,
            "ms_per_launch": ms, "alg_tflops": alg_flops / (ms * 1e-3) / 1e12,
            "mfma_frac": alg_flops / (ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS}


def update_only(a, dev):
    """Three fused updates at the solve's shape, then three copies of a 1 GiB buffer."""
    import torch

    import paper_2511_17107_amd as kc

    S, AS, C, theta = update_block(a, dev)
    for r in range(3):
        R, res, xn2 = kc.block_update(S, AS, C, theta)
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for r in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"update_kpoints": a.kpb, "mb": a.m + a.guard, "N": a.N,
                      "copy_bytes_each_way": src.numel() * 8, "res0": float(res[0, 0])}), flush=True)


def sphere64_run(a, dev):
    """The 64^3 anisotropic-sphere configurations (sphere r = 0.3a, eps = R diag(e) R^T with
    e_i ~ U[4,14], seed 0, CrossDoF, k-points uniform on Gamma-X-M-Gamma-R):
      c2: 20 bands (+ --c2-guard guard columns, default 4: a 24-column block, on the wide path of
          the block kernels), 40 k-points in one launch set, FP64 operator;
      c3: 16 bands (+4 guard), 120 k-points in two launch sets of 60, FP32 operator phase with FP64
          block algebra and finish, against the FP64 path on the same k-points (per-band relative
          eigenvalue differences) and the FP64 path one k-point at a time.
    Each solve is timed on its own (inputs resident, one untimed solve first for the tile tuner)."""
    import torch

    import paper_2511_17107_amd as kc
    import workloads as W

    c2 = a.workload == "c2"
    m, guard, nk, kpb = (20, a.c2_guard, 40, 40) if c2 else (16, 4, 120, 60)
    wl = W.sphere_anisotropic(N=64, nk=nk, m=m)
    op = kc.Op(64, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints)
    pc = kc.KC_PRECOND_TRANSVERSE

    def timed(prec, ik0, nkk, batch):
        torch.cuda.synchronize()
        t = time.perf_counter()
        eig, res, its, st = op.solve(m, ik0=ik0, nk=nkk, tol=a.tol, maxit=a.maxit, prec=prec, switch_tol=a.switch_tol,
                                     batch_k=batch, guard=guard, precond=pc)
        torch.cuda.synchronize()
        return time.perf_counter() - t, eig, res, its, st, op.last_solve_stats()

    for prec in (kc.KC_PREC_FP64, kc.KC_PREC_FP32):  # tile tuning, first-use allocations
        timed(prec, 0, 2, 2)
    out = {"workload": "sc64-sphere-aniso-crossdof (r=0.3, eps=R diag(e) R^T, e~U[4,14], seed 0), %d bands "
                       "(+%d guard), %d k-points G-X-M-G-R" % (m, guard, nk),
           "mode": a.workload, "N": 64, "bands": m, "kpoints": nk, "tol": a.tol, "preconditioner": "transverse",
           "unit": "k-points/s", "data": "synthetic"}
    runs = {}
    for name, prec in ([("fp64", kc.KC_PREC_FP64)] if c2 else [("mixed", kc.KC_PREC_FP32), ("fp64", kc.KC_PREC_FP64)]):
        T, E, R, I, S, ST = 0.0, [], [], [], [], np.zeros(8)
        for ik0 in range(0, nk, kpb):
            t, eig, res, its, st, stats = timed(prec, ik0, min(kpb, nk - ik0), kpb)
            T += t
            E.append(eig), R.append(res), I.append(its), S.append(st)
            ST += stats
        runs[name] = (np.concatenate(E), np.concatenate(R), np.concatenate(I))
        out[name] = {"value": nk / T, "seconds": T, "launch_sets": (nk + kpb - 1) // kpb, "batch_k": kpb,
                     "converged": all(st == 0 for st in S), "max_residual": float(np.concatenate(R).max()),
                     "iterations_mean": float(np.concatenate(I).mean()), "matvecs_fp64": float(ST[0]),
                     "matvecs_fp32": float(ST[1])}
    if not c2:
        e_m, e_d = runs["mixed"][0], runs["fp64"][0]
        rel = np.abs(e_m - e_d) / np.abs(e_d)
        out["band_rel_diff_mixed_vs_fp64"] = {"max": float(rel.max()),
                                              "per_band_max": [float(v) for v in rel.max(axis=0)]}
        # the FP64 path one k-point at a time, on every tenth k-point of the path
        sel = list(range(0, nk, 10))
        T = sum(timed(kc.KC_PREC_FP64, ik, 1, 1)[0] for ik in sel)
        out["fp64_sequential"] = {"value": len(sel) / T, "kpoints": len(sel), "batch_k": 1}
    out["eigenvalues_first_kpoints"] = [[float(v) for v in runs["fp64"][0][i]] for i in range(3)]
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU, a single MI355X; --gpus %d is not "
              "supported (k-points would shard across GPUs with no communication)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2511_17107_amd as kc
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.workload == "c5":
        from paper_2511_17107_amd import learned

        out = learned.c5(geoms32=a.c5_geoms[0], geoms64=a.c5_geoms[1], steps=a.c5_steps,
                         log=lambda *v: print(*v, file=sys.stderr, flush=True))
        print(json.dumps(out), flush=True)
        return
    if a.workload != "c4":
        sphere64_run(a, dev)
        return
    wl = W.woodpile_gyrotropic(N=a.N, nk=a.nk, m=a.m)
    op = kc.Op(wl.N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints)
    prec = kc.KC_PREC_FP32 if a.prec == "fp32" else kc.KC_PREC_FP64
    pc = kc.KC_PRECOND_TRANSVERSE if a.precond == "transverse" else kc.KC_PRECOND_DIAG
    nsteps_path = a.nk // a.kpb

    # k-points reordered so that batch s holds path points s, s + P, s + 2P, ... (P = nk/kpb):
    # consecutive steps walk the whole path, and each batch is a consecutive index range
    order = np.concatenate([[(s + j * nsteps_path) for j in range(a.kpb)] for s in range(nsteps_path)])
    op.set_kpoints(wl.kpoints[order])

    if a.matvec_only:
        matvec_only(a, op, prec, dev)
        return
    if a.update_only:
        update_only(a, dev)
        return
    if a.gram_only:
        gram_only(a, dev)
        return

    xbuf = None
    if a.warm_start:  # converged fields of the previous step (position j of batch s-1 is point s-1+jP)
        xbuf = [torch.empty((a.kpb, a.m, 3, a.N ** 3), dtype=torch.complex128, device=dev) for _ in range(2)]

    def run_step(step, x_init=None, x_out=None, tag="step"):
        ik0 = (step % nsteps_path) * a.kpb
        ts = time.perf_counter()
        eig, res, its, st = op.solve(a.m, ik0=ik0, nk=a.kpb, tol=a.tol, maxit=a.maxit, prec=prec,
                                     switch_tol=a.switch_tol, batch_k=a.kpb, guard=a.guard,
                                     verbose=a.verbose, check=True, precond=pc, X_out=x_out, x_init=x_init,
                                     start=a.start)
        # one progress line per solved batch (stderr; the result line is the only stdout line)
        print("%s %d: k-points %d..%d, iterations %d..%d (sum %d), max Res %.2e, %.3f s"
              % (tag, step, ik0, ik0 + a.kpb - 1, int(its.min()), int(its.max()), int(its.sum()),
                 float(res.max()), time.perf_counter() - ts), file=sys.stderr, flush=True)
        return ik0, eig, res, its, st, op.last_solve_stats()

    for w in range(a.warmup):
        run_step(nsteps_path - 1 - w, tag="warm-up")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for s in range(a.steps):
        if xbuf is None:
            results.append(run_step(s))
        else:
            warm = s > 0 and s % nsteps_path != 0
            results.append(run_step(s, x_init=xbuf[(s + 1) % 2] if warm else None, x_out=xbuf[s % 2]))
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    nkp = a.steps * a.kpb
    converged = all(r[4] == 0 for r in results)
    maxres = max(float(r[2].max()) for r in results)
    iters = [int(i) for r in results for i in r[3]]
    mv64 = sum(r[5][0] for r in results)
    mv32 = sum(r[5][1] for r in results)

    # per-pass roofline of the operator application on one block of 16 vectors
    x = torch.randn((a.m, 3, a.N ** 3), dtype=torch.complex128, device=dev)
    tbytes = 8 if prec == kc.KC_PREC_FP32 else 16
    names, pbytes = pass_bytes(a.N, a.m, True, tbytes)
    reps = 5
    acc = np.zeros(len(names))
    for r in range(reps + 1):
        _, ms = op.apply_timed(x, prec=prec)
        if r > 0:
            acc += ms
    ms = acc / reps
    gbs = [pb / (t * 1e-3) / 1e9 for pb, t in zip(pbytes, ms)]
    dom = int(np.argmax(ms))
    mv_time = float(ms.sum())
    alg_mv = (16 * 3 * a.N ** 3 * 2 + 4 * a.N ** 3) * a.m  # read x, write y, read ids
    tiles = {"fp32": op.tile_widths(kc.KC_PREC_FP32).tolist(), "fp64": op.tile_widths(kc.KC_PREC_FP64).tolist()}
    # the whole operator application (all passes of one kc_apply on a.m vectors): the pass
    # structure's algorithmic bytes, the counter-measured HBM bytes at the tuned widths (when the
    # profile covers them), and the boundary's bytes (read x, write y, read the ids) over its time
    traffic = [MEASURED_TRAFFIC.get((nm, a.N, a.m, a.prec, tiles[a.prec][PASS_SLOT[nm]])) for nm in names]
    tsum = None if any(t is None for t in traffic) else float(sum(traffic))
    alg_sum = float(sum(pbytes))
    sec = mv_time * 1e-3
    app_roofline = {"bound": "hbm", "kernel": "operator application (%d pencil passes)" % len(names),
                    "achieved": alg_sum / sec / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": alg_sum / sec / 1e9 / HBM_PEAK_GBS, "alg_bytes": alg_sum, "ms_per_launch": mv_time,
                    "traffic": tsum,
                    "traffic_GBps": None if tsum is None else tsum / sec / 1e9,
                    "traffic_frac": None if tsum is None else tsum / sec / 1e9 / HBM_PEAK_GBS,
                    "boundary_bytes": float(alg_mv), "boundary_GBps": alg_mv / sec / 1e9,
                    "boundary_frac": alg_mv / sec / 1e9 / HBM_PEAK_GBS}
    del x
    # the solver's block workspace (~180 GB at the default batch) goes with the handle, which
    # makes room for the update measurement's own blocks
    del op
    torch.cuda.empty_cache()
    upd = update_roofline(a, dev)

    out = {
        "metric": "k-points/s to rel. residual 1e-8 at n=128, 16 bands; matvec GB/s vs HBM peak",
        "value": nkp / T,
        "unit": "k-points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * T / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 operator / f64 block" if prec == kc.KC_PREC_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": "sc128-woodpile-gyrotropic-crossdof, 16 bands (+%d guard), "
                               "%d k-points/step of the 60-point G-X-M-G-R path" % (a.guard, a.kpb),
                   "N": a.N, "bands": a.m, "kpoints_per_step": a.kpb, "tol": a.tol,
                   "precision": a.prec, "preconditioner": a.precond,
                   "start": ("previous step's fields" if a.warm_start else
                             "lowest transverse plane waves" if a.start == "plane_waves" else "seeded random")},
        "converged": converged,
        "max_residual": maxres,
        "iterations": iters,
        "matvecs_fp64": mv64,
        "matvecs_fp32": mv32,
        "roofline": upd,
        "tile_widths": tiles,
        "matvec": {"passes": names, "ms": [round(float(t), 4) for t in ms],
                   "alg_GBps": [round(g, 1) for g in gbs], "nvec": a.m,
                   "ms_per_band": mv_time / a.m,
                   "effective_GBps": alg_mv / (mv_time * 1e-3) / 1e9,
                   "roofline": app_roofline,
                   "longest_pass": {"bound": "hbm", "kernel": "matvec pass " + names[dom],
                                    "achieved": gbs[dom], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": gbs[dom] / HBM_PEAK_GBS,
                                    "traffic": MEASURED_TRAFFIC.get(
                                        (names[dom], a.N, a.m, a.prec, tiles[a.prec][PASS_SLOT[names[dom]]])),
                                    "tile_width": tiles[a.prec][PASS_SLOT[names[dom]]],
                                    "alg_bytes": pbytes[dom]}},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl.kpoints)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
