"""Writes the stored expected values for the full-size 3D cavity parity tests.

Calls only the FP64 oracle (oracle/) on the seeded workload description of
lbm_inputs; nothing here comes from the HIP path.  Run from the repository
root:  python tests/golden/make_golden.py  (about 45 minutes on 8 cores).

Output: tests/golden/cavity3d_d3q19_128_re1000.npz with
  steps        : the steps at which the sensor was evaluated (1000 .. 10000)
  block_max    : [len(steps), 16, 16, 16] L2-sensor block maxima
  flags        : same shape, int8 refine/keep/coarsen flags
  rho_mid_K, u_mid_K : rho and u on the plane z = 64 after step K, K = 5000
                 and K = 10000
  totals_K     : conservation totals (mass, momentum) after step K
  tau          : the relaxation time of the run
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lbm_inputs  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cavity3d_d3q19_128_re1000.npz")
SNAPSHOTS = (5000, 10000)


def main():
    w = lbm_inputs.cavity3d()
    tau = oracle.tau_from_reynolds(w.lid_speed, w.n_across, w.reynolds)
    G = oracle.Grid(q=19, n=w.n, bc=w.bc, wall_u=w.wall_u, tau=tau,
                    theta_refine=w.theta_refine, theta_coarsen=w.theta_coarsen)
    S = G.equilibrium_state()
    every = 1000
    out = {"tau": np.array(tau)}
    hist_all = []
    k = 0
    t0 = time.time()
    for K in SNAPSHOTS:
        S, hist = G.run(S, k, K - k, every)
        hist_all += hist
        k = K
        rho, u = G.macros(S)
        out[f"rho_mid_{K}"] = rho[64].copy()
        out[f"u_mid_{K}"] = u[:, 64].copy()
        out[f"totals_{K}"] = G.conservation(S)
        print(f"{K} oracle steps after {time.time() - t0:.0f} s", flush=True)
    out["steps"] = np.array([kk for kk, _, _ in hist_all])
    out["block_max"] = np.stack([b for _, b, _ in hist_all])
    out["flags"] = np.stack([f for _, _, f in hist_all])
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
