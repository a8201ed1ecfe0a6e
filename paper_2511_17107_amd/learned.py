"""Training and evaluation of the learned preconditioner.

The preconditioner is the transverse-projection operator T_E of kc_precond_transverse with a
field E predicted per cell by the convolution network from the dielectric structure and the wave
vector (kc_net_efield): E_c = E0_c exp(clamp(y_c, -3, 3)), E0_c = 1/(eps^-1)_cc at the c-edge
points.  Training pairs come from the solver itself on random dielectric geometries: for the
converged eigenpairs (x*, lambda) of one k-point, iterates x = x* + e with smooth perturbations
e orthogonal to the converged block give residuals r = Op x - theta x (theta the Rayleigh
quotient of x), and the target direction for each residual is c = Op^{-1} r (preconditioned CG
with the library's operator and T_E0; Op is Hermitian positive definite away from k = 0):
LOBPCG with the exact inverse as preconditioner converges at a rate set by the band gaps alone.
Rayleigh-Ritz fixes the scale of every direction, so the loss of one residual is the
scale-free misfit min_alpha |alpha T_E r - c|^2 / |c|^2 in the Op-norm (the norm in which
LOBPCG's convergence is measured; the Euclidean norm is an option), and its gradient with
respect to E (optimal alpha held fixed) is (2 alpha / |c|^2) Re(conj(G Op e) G r) with
G = F3 K_A^{+} and e = alpha T_E r - c (kc_tp_grad).  The chain rule through E = E0 exp(y) gives the gradient of the
network output, and the library's backward and Adam kernels update the weights.

    python -m paper_2511_17107_amd.learned train --out weights.npy [--geoms 32 --N 32]
    python -m paper_2511_17107_amd.learned eval --weights weights.npy [--N 96 --nk 8]

PyTorch here only holds device buffers (allocation, host-device copies, concatenation of the
network inputs and output gradients of a batch); the iterates, residuals, corrections (kc_pcg),
the loss and its gradient (kc_net_loss_grad), and every operator application, preconditioner,
FFT and network pass run in the library's kernels.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _torch():
    import torch

    return torch


def pcg(op, ik, r, tol=1e-7, maxit=400):
    """c = Op^{-1} r for a block r [nv][3][N^3] of k-point ik (kc_pcg: conjugate gradients with
    the library's FP64 operator, preconditioned with T_E of the classical field)."""
    c, its, ok = op.pcg(r, ik=ik, tol=tol, maxit=maxit)
    return c, its, ok


class Sample:
    """One geometry and k-point: its operator, network input, residuals and targets."""

    def __init__(self, op, feat, r, c, info):
        self.op, self.feat, self.r, self.c, self.info = op, feat, r, c, info


def make_samples(N, seeds, m=8, nk_path=40, amp=(0.02, 0.3), rng_seed=0, log=print):
    torch = _torch()
    import paper_2511_17107_amd as kc
    import workloads as W

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(rng_seed)
    n3 = N ** 3
    out = []
    for s in seeds:
        wl = W.random_inclusions(N, int(s), nk=nk_path, m=m)
        kidx = int(rng.integers(3, nk_path))  # a k-point of the path away from Gamma
        op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
        op.set_kpoints(wl.kpoints[kidx:kidx + 1])
        X = torch.zeros((m, 3, n3), dtype=torch.complex128, device=dev)
        eig, res, its, st = op.solve(m, tol=1e-7, guard=2, X_out=X, seed=int(s), precond=kc.KC_PRECOND_TRANSVERSE)
        op.release_workspaces()  # the training passes need only the operator's own buffers
        # iterates x = X + a e with smoothed noise e orthogonal to the converged block, and
        # their residuals (kc_perturbed_residuals); targets c = Op^{-1} r (kc_pcg)
        noise = torch.from_numpy(W.random_block(10_000 + int(s), m, N)).to(dev)
        a = rng.uniform(amp[0], amp[1], size=m)
        _, r = op.perturbed_residuals(X, noise, a)
        c, pits, ok = pcg(op, 0, r)
        feat = op.net_features(0, 1)
        op.release_workspaces()
        out.append(Sample(op, feat, r, c, {"seed": int(s), "k": kidx, "eig0": float(eig[0][0]), "iters": int(its[0]),
                                           "pcg_iters": pits, "pcg_converged": ok}))
        log("samples: geometry %d k=%d eig[0]=%.4f iters=%d pcg %d%s" % (s, kidx, eig[0][0], its[0], pits,
                                                                         "" if ok else " (not converged)"))
    return out


def sample_loss(net, smp, grad=False, loss_kind="energy", scale=1.0):
    """Mean scale-free misfit over the sample's residuals (kc_net_loss_grad); with grad, also
    scale times its gradient with respect to the network output (float32 [N^3][16]).

    energy:    min_alpha |alpha T_E r - c|_Op^2 / |c|_Op^2 = 1 - (z^H r)^2 / ((z^H Op z)(c^H r)),
               z = T_E r (the Op-norm, in which LOBPCG's convergence is measured)
    euclidean: min_alpha |alpha T_E r - c|^2 / |c|^2"""
    smp.op.attach_net(net)
    return smp.op.net_loss_grad(smp.r, smp.c, kind=loss_kind, grad=grad, scale=scale)


def train(net, samples, steps=400, batch=4, lr=1e-3, log=print, seed=0, loss_kind="energy"):
    """Adam on the mean sample loss; each step draws its batch from one grid size (the samples'
    network inputs are concatenated), cycling through the sizes present."""
    torch = _torch()
    groups = {}
    for i, smp in enumerate(samples):
        groups.setdefault(smp.op.N, []).append(i)
    sizes = sorted(groups)
    g = np.random.default_rng(seed)
    hist = []
    for it in range(steps):
        N = sizes[it % len(sizes)]
        pool = groups[N]
        idx = [pool[i] for i in g.choice(len(pool), size=min(batch, len(pool)), replace=False)]
        feats, gys, ls = [], [], []
        for i in idx:
            smp = samples[i]
            loss, gy = sample_loss(net, smp, grad=True, loss_kind=loss_kind, scale=1.0 / len(idx))
            ls.append(loss)
            feats.append(smp.feat)
            gys.append(gy)
        net.backward(torch.cat(feats).contiguous(), torch.stack(gys).contiguous(), N, host_grads=False)
        net.adam_step(lr * (0.5 ** (it / max(steps // 3, 1))))
        hist.append(float(np.mean(ls)))
        if it % 50 == 0 or it == steps - 1:
            log("train step %d loss %.4e" % (it, hist[-1]))
    return hist


def mean_loss(net, samples, loss_kind="energy"):
    out = []
    for smp in samples:
        smp.op.attach_net(net)
        out.append(sample_loss(net, smp, loss_kind=loss_kind)[0])
    return float(np.mean(out))


def evaluate(weights, N=96, nk=8, m=16, guard=4, seed=1000, log=print, batch_k=None, prec=None):
    """Iterations and time to Res <= 1e-8 with the diagonal-block, the classical
    transverse-projection and the learned preconditioner on a held-out random geometry."""
    torch = _torch()
    import paper_2511_17107_amd as kc
    import workloads as W

    prec = kc.KC_PREC_FP32 if prec is None else prec
    wl = W.random_inclusions(N, seed, nk=40, m=m)
    sel = np.linspace(1, 39, nk).round().astype(int)
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints[sel])
    net = kc.Net(seed=0)
    if weights is not None:
        net.set_params(np.load(weights))
    op.attach_net(net)
    out = {"N": N, "nk": nk, "m": m, "geometry_seed": seed}
    bk = batch_k or nk
    for name, pc in (("diagonal", kc.KC_PRECOND_DIAG), ("transverse", kc.KC_PRECOND_TRANSVERSE),
                     ("learned", kc.KC_PRECOND_LEARNED)):
        op.solve(m, nk=min(2, nk), tol=1e-8, guard=guard, batch_k=min(2, nk), precond=pc, prec=prec,
                 switch_tol=3e-4)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eig, res, its, st = op.solve(m, tol=1e-8, guard=guard, batch_k=bk, precond=pc, prec=prec, switch_tol=3e-4)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats = op.last_solve_stats()
        out[name] = {"seconds": dt, "kpoints_per_s": nk / dt, "iterations": its.tolist(), "status": int(st),
                     "max_res": float(res.max()), "eig": eig.tolist(), "kept": float(stats[4])}
        log("%s: %.2f s, iterations %s, status %d" % (name, dt, its.tolist(), st))
    e0 = np.array(out["diagonal"]["eig"])
    for name in ("transverse", "learned"):
        e1 = np.array(out[name]["eig"])
        out[name]["max_rel_eig_diff"] = float(np.max(np.abs(e1 - e0) / e0))
        out[name]["iteration_ratio"] = float(np.sum(out[name]["iterations"]) / np.sum(out["diagonal"]["iterations"]))
        out[name]["time_ratio"] = out[name]["seconds"] / out["diagonal"]["seconds"]
    return out


def c5(geoms32=400, geoms64=100, steps=600, nk=40, N=96, m=16, guard=4, batch_k=10, log=print):
    """The learned-preconditioner workload: train on solver-generated pairs of geoms32 random
    geometries at 32^3 and geoms64 at 64^3 (seeds 0.. of workloads.random_inclusions), then solve a
    held-out geometry (seed 1000) at N^3 over nk k-points of its path to Res <= 1e-8 with
      fp64_diagonal : FP64 operator, the diagonal-block preconditioner of eqs (2.31)-(2.32)
      fp32_diagonal : FP32 operator phase + FP64 finish, the same preconditioner
      fp32_transverse: FP32 phase, T_E with the classical field
      fp32_learned  : FP32 phase, T_E with the trained network's field
    all batched batch_k k-points per launch set; returns timings, iterations and eigenvalue
    differences against the FP64 run."""
    torch = _torch()
    import paper_2511_17107_amd as kc
    import workloads as W

    t0 = time.time()
    net = kc.Net(seed=0)
    cnt = [0]

    def every(msg):  # progress every 25 geometries
        cnt[0] += 1
        if cnt[0] % 25 == 0:
            log("c5 samples %d (%.0f s): %s" % (cnt[0], time.time() - t0, msg))

    samples = make_samples(32, range(geoms32), log=every)
    if geoms64:
        samples += make_samples(64, range(geoms64), rng_seed=7, log=every)
    held = make_samples(32, range(5000, 5008), rng_seed=1, log=every)
    t_samples = time.time() - t0
    l0 = mean_loss(net, held)
    hist = train(net, samples, steps=steps, log=log)
    l1 = mean_loss(net, held)
    t_train = time.time() - t0 - t_samples
    log("c5: %d samples in %.0f s, training %.0f s, held-out loss %.4f -> %.4f" % (len(samples), t_samples, t_train, l0, l1))
    for smp in samples + held:  # release the training handles before the large solves
        smp.op.close()
    del samples, held
    torch.cuda.empty_cache()
    wl = W.random_inclusions(N, 1000, nk=nk, m=m)
    op = kc.Op(N, kc.KC_EPS_CROSSDOF, wl.ids, wl.table)
    op.set_kpoints(wl.kpoints)
    op.attach_net(net)
    out = {"workload": "random inclusions (held-out seed 1000) at %d^3, %d bands (+%d guard), %d k-points of the "
                       "G-X-M-G-R path, %d per launch set" % (N, m, guard, nk, batch_k),
           "training": {"geometries_32": geoms32, "geometries_64": geoms64, "steps": steps,
                        "seconds_samples": t_samples, "seconds_training": t_train,
                        "heldout_loss_E0": l0, "heldout_loss_trained": l1}, "runs": {}}
    cfgs = [("fp64_diagonal", kc.KC_PREC_FP64, kc.KC_PRECOND_DIAG), ("fp32_diagonal", kc.KC_PREC_FP32, kc.KC_PRECOND_DIAG),
            ("fp32_transverse", kc.KC_PREC_FP32, kc.KC_PRECOND_TRANSVERSE),
            ("fp32_learned", kc.KC_PREC_FP32, kc.KC_PRECOND_LEARNED)]
    eig = {}
    for name, prec, pc in cfgs:
        op.solve(m, nk=2, batch_k=2, tol=1e-8, guard=guard, precond=pc, prec=prec, switch_tol=3e-4)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        E, I, S = [], [], []
        kept = 0.0
        for ik0 in range(0, nk, batch_k):
            nb = min(batch_k, nk - ik0)
            e, r, its, st = op.solve(m, ik0=ik0, nk=nb, batch_k=nb, tol=1e-8, guard=guard, precond=pc, prec=prec,
                                     switch_tol=3e-4, check=False)
            E.append(e), I.append(its), S.append(st)
            kept += op.last_solve_stats()[4]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        its = np.concatenate(I)
        eig[name] = np.concatenate(E)
        out["runs"][name] = {"seconds": dt, "kpoints_per_s": nk / dt, "iterations_mean": float(its.mean()),
                             "status": [int(v) for v in S], "learned_kept": kept if pc == kc.KC_PRECOND_LEARNED else None}
        log("c5 %s: %.2f s, %.1f iterations per k-point" % (name, dt, its.mean()))
    for name in out["runs"]:
        out["runs"][name]["max_rel_eig_diff_vs_fp64"] = float(np.max(np.abs(eig[name] - eig["fp64_diagonal"]) /
                                                                    eig["fp64_diagonal"]))
        out["runs"][name]["speedup_vs_fp64_diagonal"] = out["runs"]["fp64_diagonal"]["seconds"] / out["runs"][name]["seconds"]
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--N", type=int, default=32)
    t.add_argument("--geoms", type=int, default=32)
    t.add_argument("--holdout", type=int, default=8)
    t.add_argument("--steps", type=int, default=400)
    t.add_argument("--batch", type=int, default=4)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--loss", choices=["energy", "euclidean"], default="energy")
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=None)
    e.add_argument("--N", type=int, default=96)
    e.add_argument("--nk", type=int, default=8)
    e.add_argument("--json", default=None)
    a = ap.parse_args()
    import paper_2511_17107_amd as kc

    if a.cmd == "train":
        net = kc.Net(seed=a.seed)
        t0 = time.time()
        samples = make_samples(a.N, range(a.geoms))
        held = make_samples(a.N, range(5000, 5000 + a.holdout), rng_seed=1)
        l0_train, l0_held = mean_loss(net, samples, a.loss), mean_loss(net, held, a.loss)
        print("samples: %d + %d held out in %.1f s; loss with E0: train %.4e held-out %.4e"
              % (len(samples), len(held), time.time() - t0, l0_train, l0_held), flush=True)
        hist = train(net, samples, steps=a.steps, batch=a.batch, lr=a.lr, loss_kind=a.loss)
        np.save(a.out, net.get_params())
        l1_train, l1_held = mean_loss(net, samples, a.loss), mean_loss(net, held, a.loss)
        print(json.dumps({"samples": len(samples), "held_out": len(held), "loss_E0_train": l0_train,
                          "loss_E0_held": l0_held, "loss_train": l1_train, "loss_held": l1_held,
                          "steps": a.steps}), flush=True)
    else:
        out = evaluate(a.weights, N=a.N, nk=a.nk)
        s = json.dumps(out)
        print(s, flush=True)
        if a.json:
            with open(a.json, "w") as f:
                f.write(s)


if __name__ == "__main__":
    main()
