"""Writes window400_lsqr.npz: the FP64 oracle's reconstructions of the window400 workload
(a standalone 64x64 problem at the 5 um step and 81x81-capped cone footprint of the 400x400
workload, depths +-80 um): plain Tikhonov LSQR (50 iterations) and the refinement schedule
(50 iterations + 2 residual-correction sweeps of 50), with the l2 weight rule.

Calls only the oracle and the seeded workload generators.  Takes ~15 minutes on 8 cores:

    python tests/golden/make_window400.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import model, operators, solvers  # noqa: E402


def problem(name="window400", seed=0):
    """Table, phantom and noisy signals of the workload, all from the oracle (FP64)."""
    cfg = W.config(name)
    g = cfg["grid"]
    H = model.build_table(cfg["sensor"], g)
    x0 = W.make_phantom(cfg, seed)
    clean = operators.forward(H, x0)
    sigma = np.max(np.abs(clean)) * 10 ** (-cfg["snr_db"] / 20)
    return cfg, H, x0, clean + sigma * W.unit_noise(cfg, seed)


def main():
    cfg, H, _, s = problem()
    g = cfg["grid"]
    shp_x, shp_s = (g["ny"], g["nx"], g["nz"]), (g["ny"], g["nx"], g["nt"])
    A = lambda v: operators.forward(H, v.reshape(shp_x)).ravel()
    AT = lambda u: operators.adjoint(H, u.reshape(shp_s)).ravel()
    so = cfg["solver"]
    lam = solvers.lam_l2(AT(s.ravel()))
    x_plain, _ = solvers.lsqr(A, AT, s.ravel(), damp=np.sqrt(lam), iters=so["iters"])
    print(f"plain LSQR done, lam {lam:.6e}", flush=True)
    x_ref = solvers.lsqr_refined(A, AT, s.ravel(), lam, so["iters"], so["sweeps"])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "window400_lsqr.npz")
    np.savez_compressed(out, lam=lam, s_norm=np.linalg.norm(s),
                        x_plain=x_plain.reshape(shp_x).astype(np.float32),
                        x_refined=x_ref.reshape(shp_x).astype(np.float32),
                        iters=so["iters"], sweeps=so["sweeps"])
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
