"""Writes calib_trajectory_7x7_256_q4096.json: the FP64 oracle's trajectory of
20 leave-one-out gradient steps (alpha 0.2, eps 1e-6; update of Sec. V-B) on
the 7x7-view, 256x256, 16-layer calibration workload, with a fresh subset of
4096 frequency bins per step (seeded), parameters rounded to float32 after
every step as the device stores them; the loss and gradient of every step are
kept too.  Calls only the oracle and the seeded
input generators.  Run from the repository root:

    python tests/golden/make_calib_trajectory.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), "..", ".."))
sys.path.insert(0, ROOT)

from oracle import fdl_oracle as O  # noqa: E402
from paper_1901_06919_amd import synth  # noqa: E402

STEPS, Q, SEED, ALPHA, EPS_G = 20, 4096, 505, 0.2, 1e-6
OUT = os.path.join(os.path.dirname(__file__), "calib_trajectory_7x7_256_q4096.json")


def main():
    spec, u0, d0 = synth.lf_7x7_256_calib()
    views = O.forward_views(spec.layers.astype(np.float64), spec.u, spec.d) + spec.noise
    b = O.rfft2(views.astype(np.float32)).astype(np.complex64).astype(np.complex128)
    H, W = spec.H, spec.W
    F = H * (W // 2 + 1)
    rng = np.random.default_rng(SEED)
    u, d = u0.astype(np.float64), d0.astype(np.float64)
    rec = {"workload": "7x7 views, 256x256, 16 layers (synth.lf_7x7_256_calib)", "steps": STEPS, "Q": Q,
           "seed": SEED, "alpha": ALPHA, "eps_g": EPS_G, "subset_sums": [], "loss": [], "grad_u": [], "grad_d": [],
           "u": [], "d": []}
    for step in range(STEPS):
        S = synth.frequency_subset(F, Q, rng)
        L, gu, gd = O.calib_loss_grad(b, u, d, H, W, spec.lam, spec.eps, spec.reg, O.LOSS_LOO, S)
        u, d = O.gd_step(u, d, gu, gd, ALPHA, EPS_G)
        u, d = u.astype(np.float32).astype(np.float64), d.astype(np.float32).astype(np.float64)
        rec["subset_sums"].append(int(np.sum(S.astype(np.int64))))
        rec["loss"].append(float(L))
        rec["grad_u"].append([float(x) for x in np.ravel(gu)])
        rec["grad_d"].append([float(x) for x in np.ravel(gd)])
        rec["u"].append([float(x) for x in u.ravel()])
        rec["d"].append([float(x) for x in d])
        print(f"step {step}: loss {L:.10e}", flush=True)
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
