"""Writes the stored oracle eigenvalues under tests/golden/.

Calls only the oracle and the seeded input module: every value stored here is the oracle's.

    python tests/golden/make_golden.py            # all cases
    python tests/golden/make_golden.py NAME ...   # selected cases
"""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import eigs, yee  # noqa: E402


def case_sphere16_iso():
    wl = W.sphere_isotropic()
    return wl, [(wl.kpoints[0], "crossdof")]


def case_sphere16_aniso():
    wl = W.sphere_anisotropic(N=16, nk=9, m=10)
    # Gamma (k = 0), an interior point of Gamma-X, X, M, R
    sel = [0, 1, 2, 4, 8]
    return wl, [(wl.kpoints[i], s) for i in sel for s in ("crossdof", "trivial")]


def case_woodpile16_gyro():
    wl = W.woodpile_gyrotropic(N=16, nk=9, m=8)
    sel = [0, 3, 6]
    return wl, [(wl.kpoints[i], "crossdof") for i in sel]


def case_sphere32_aniso():
    wl = W.sphere_anisotropic(N=32, nk=9, m=12)
    sel = [2, 5]
    return wl, [(wl.kpoints[i], "crossdof") for i in sel]


CASES = {
    "sphere16_iso": case_sphere16_iso,
    "sphere16_aniso": case_sphere16_aniso,
    "woodpile16_gyro": case_woodpile16_gyro,
    "sphere32_aniso": case_sphere32_aniso,
}


def run(name):
    wl, items = CASES[name]()
    out = {"workload": wl.name, "N": wl.N, "m": wl.m, "cases": []}
    for k, scheme in items:
        t = time.time()
        Op = yee.compensated_operator(wl.N, k, wl.ids, wl.table, scheme)
        w, V = eigs.smallest_positive(Op, wl.m, method="shift_invert", return_vectors=True)
        res = np.linalg.norm(Op @ V - V * w[None, :], axis=0)
        out["cases"].append({"k": [float(v) for v in k], "scheme": scheme,
                             "gamma": yee.gamma_rule(k),
                             "eigenvalues": [float(v) for v in w],
                             "max_residual": float(res.max()),
                             "seconds": time.time() - t})
        print(name, scheme, k, w[:4], "%.1fs" % (time.time() - t), flush=True)
    if name == "sphere16_iso":
        out["eigenvalues"] = out["cases"][0]["eigenvalues"]
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for nm in names:
        run(nm)
