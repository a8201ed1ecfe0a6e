"""Experiments of Section 4 run through the library (every eigen-solve is kc_solve on the GPU;
this module only sets up inputs and compares eigenvalues).

    python -m paper_2511_17107_amd.experiments highorder [--sizes 16 32 64] [--orders 1 5]
    python -m paper_2511_17107_amd.experiments robust [--N 128] [--bands 10]
    python -m paper_2511_17107_amd.experiments schemes [--geometry sphere64|woodpile128] [--nk 40]

highorder: the smooth permittivity of eq (4.7) at k = (pi, pi, pi) with order-2m stencils
    (Table 5): differences of the normalised frequencies omega / (2 pi) between successive grids
    and the observed order.
robust: an inclusion with the ill-conditioned inverse permittivity U diag(1e-1, 1e-3, 1e-5) U^H
    (Section 4, robustness under extreme cases) at k = (1/7, 3/5, 4/13) pi, both discretisations
    of Section 3, FP64 and the FP32-operator path: iterations, residual histories, eigenvalues.
schemes: the relative frequency differences of eq (4.6) between the Trivial and CrossDoF
    discretisations over a band path (Table 2), and the iterations of each (Table 6).
Each prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import _binding as kc

_SCHEMES = {"diagonal": kc.KC_EPS_DIAGONAL, "trivial": kc.KC_EPS_TRIVIAL, "crossdof": kc.KC_EPS_CROSSDOF}


def _solve(op, m, **kw):
    import torch

    torch.cuda.synchronize()
    t = time.perf_counter()
    eig, res, its, st = op.solve(m, check=False, **kw)
    torch.cuda.synchronize()
    return eig, res, its, st, time.perf_counter() - t


def highorder(sizes, orders, bands=8, tol=1e-8):
    import workloads as W

    out = {"experiment": "highorder", "k": "(pi, pi, pi)", "permittivity": "8.9 sin(2 pi (x+y+z)) + 13",
           "bands": bands, "tol": tol, "runs": {}}
    for m in orders:
        freqs = {}
        for N in sizes:
            wl = W.smooth_isotropic(N)
            op = kc.Op(N, kc.KC_EPS_DIAGONAL, wl.ids, wl.table, stencil_m=m)
            op.set_kpoints(wl.kpoints)
            eig, res, its, st, dt = _solve(op, bands, tol=tol, guard=4, precond=kc.KC_PRECOND_TRANSVERSE)
            freqs[N] = np.sqrt(eig[0]) / (2 * math.pi)
            out["runs"].setdefault(str(m), {})[str(N)] = {"status": int(st), "iterations": int(its[0]),
                                                           "max_residual": float(res.max()),
                                                           "eigenvalues": [float(v) for v in eig[0]]}
        diffs = {}
        for a, b in zip(sizes[:-1], sizes[1:]):
            diffs["h=1/%d" % b] = [float(v) for v in np.abs(freqs[b] - freqs[a])]
        out["runs"][str(m)]["freq_differences"] = diffs
        if len(sizes) >= 3:
            d1 = np.array(diffs["h=1/%d" % sizes[-2]])
            d2 = np.array(diffs["h=1/%d" % sizes[-1]])
            out["runs"][str(m)]["order_last"] = [float(v) for v in np.log2(d1 / d2)]
    return out


def robust(N, bands=10, seed=0, maxit=600, tol=1e-8):
    import workloads as W

    wl = W.sphere_illconditioned(N, seed=seed, m=bands)
    out = {"experiment": "robust", "N": N, "bands": bands, "tol": tol, "maxit": maxit,
           "k": [float(v) for v in wl.kpoints[0]],
           "inverse_permittivity_eigenvalues": [1e-1, 1e-3, 1e-5], "inclusion": "sphere r=0.25 at the cell centre",
           "runs": []}
    eigs = {}
    for scheme in ("trivial", "crossdof"):
        op = kc.Op(N, _SCHEMES[scheme], wl.ids, wl.table)
        op.set_kpoints(wl.kpoints)
        for prec, pc in ((kc.KC_PREC_FP64, kc.KC_PRECOND_TRANSVERSE), (kc.KC_PREC_FP32, kc.KC_PRECOND_TRANSVERSE),
                         (kc.KC_PREC_FP64, kc.KC_PRECOND_DIAG)):
            eig, res, its, st, dt = _solve(op, bands, tol=tol, guard=4, prec=prec, switch_tol=3e-4, precond=pc,
                                           maxit=maxit)
            h, hp = op.residual_history(0)
            step = max(1, len(h) // 40)
            out["runs"].append({"scheme": scheme, "prec": "fp64" if prec == kc.KC_PREC_FP64 else "fp32+fp64",
                                "precond": "transverse" if pc == kc.KC_PRECOND_TRANSVERSE else "diagonal",
                                "status": int(st), "iterations": int(its[0]), "seconds": dt,
                                "max_residual": float(res.max()), "hpd_unproven": bool(op.flags() & 1),
                                "eigenvalues": [float(v) for v in eig[0]],
                                "history_every": step, "history": [float(v) for v in h[::step]]})
            eigs[(scheme, prec, pc)] = eig[0]
    a = np.sqrt(eigs[("trivial", kc.KC_PREC_FP64, kc.KC_PRECOND_TRANSVERSE)])
    b = np.sqrt(eigs[("crossdof", kc.KC_PREC_FP64, kc.KC_PRECOND_TRANSVERSE)])
    out["domega_trivial_vs_crossdof"] = {"max": float(np.max(np.abs(a - b) / b)), "mean": float(np.mean(np.abs(a - b) / b))}
    return out


def schemes(geometry, nk, batch):
    import workloads as W

    if geometry == "sphere64":
        N, m, guard = 64, 16, 4
        make = lambda s: W.sphere_anisotropic(N=64, nk=nk, m=m, scheme=s)
    else:
        N, m, guard = 128, 16, 4
        make = lambda s: W.woodpile_gyrotropic(N=128, nk=nk, m=m, scheme=s)
    out = {"experiment": "schemes", "geometry": geometry, "N": N, "bands": m, "kpoints": nk, "tol": 1e-8,
           "prec": "fp32+fp64", "precond": "transverse", "runs": {}}
    w = {}
    for scheme in ("trivial", "crossdof"):
        wl = make(scheme)
        op = kc.Op(N, _SCHEMES[scheme], wl.ids, wl.table)
        op.set_kpoints(wl.kpoints)
        E, I, T, S, R = [], [], 0.0, [], []
        for ik0 in range(0, nk, batch):
            nb = min(batch, nk - ik0)
            eig, res, its, st, dt = _solve(op, m, ik0=ik0, nk=nb, batch_k=nb, guard=guard, prec=kc.KC_PREC_FP32,
                                           switch_tol=3e-4, precond=kc.KC_PRECOND_TRANSVERSE)
            E.append(eig), I.append(its), S.append(st), R.append(res)
            T += dt
        w[scheme] = np.sqrt(np.concatenate(E))
        its = np.concatenate(I)
        out["runs"][scheme] = {"status": [int(v) for v in S], "max_residual": float(np.concatenate(R).max()),
                               "iterations_mean": float(its.mean()), "iterations_std": float(its.std()),
                               "seconds": T, "hpd_unproven": bool(op.flags() & 1)}
    d = np.abs(w["trivial"] - w["crossdof"]) / np.abs(w["crossdof"])
    out["domega_max"] = float(d.max())
    out["domega_mean"] = float(d.mean())
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("highorder")
    a.add_argument("--sizes", type=int, nargs="+", default=[16, 32, 64])
    a.add_argument("--orders", type=int, nargs="+", default=[1, 2, 3, 4, 5])
    b = sub.add_parser("robust")
    b.add_argument("--N", type=int, default=128)
    b.add_argument("--bands", type=int, default=10)
    b.add_argument("--tol", type=float, default=1e-8)
    b.add_argument("--maxit", type=int, default=600)
    c = sub.add_parser("schemes")
    c.add_argument("--geometry", choices=["sphere64", "woodpile128"], default="sphere64")
    c.add_argument("--nk", type=int, default=40)
    c.add_argument("--batch", type=int, default=20)
    args = ap.parse_args(argv)
    import torch

    torch.cuda.set_device(0)
    if args.cmd == "highorder":
        out = highorder(args.sizes, args.orders)
    elif args.cmd == "robust":
        out = robust(args.N, args.bands, maxit=args.maxit, tol=args.tol)
    else:
        out = schemes(args.geometry, args.nk, args.batch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
