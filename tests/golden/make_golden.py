"""Writes the stored expected values for the full-size 3D cavity parity test.

Calls only the FP64 oracle (oracle/) on the seeded workload description of
lbm_inputs; nothing here comes from the HIP path.  Run from the repository
root:  python tests/golden/make_golden.py  (about 20 minutes on 8 cores).

Output: tests/golden/cavity3d_d3q19_128_re1000.npz with
  steps      : the steps at which the sensor was evaluated (1000 .. 5000)
  block_max  : [len(steps), 16, 16, 16] L2-sensor block maxima
  flags      : same shape, int8 refine/keep/coarsen flags
  rho_mid, u_mid : rho and u on the plane z = 64 after step 5000
  totals     : conservation totals (mass, momentum) after step 5000
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


def main():
    w = lbm_inputs.cavity3d()
    tau = oracle.tau_from_reynolds(w.lid_speed, w.n_across, w.reynolds)
    G = oracle.Grid(q=19, n=w.n, bc=w.bc, wall_u=w.wall_u, tau=tau,
                    theta_refine=w.theta_refine, theta_coarsen=w.theta_coarsen)
    S = G.equilibrium_state()
    every = 1000
    t0 = time.time()
    S, hist = G.run(S, 0, w.steps, every)
    print(f"{w.steps} oracle steps in {time.time() - t0:.0f} s", flush=True)
    rho, u = G.macros(S)
    np.savez_compressed(
        OUT,
        steps=np.array([k for k, _, _ in hist]),
        block_max=np.stack([b for _, b, _ in hist]),
        flags=np.stack([f for _, _, f in hist]),
        rho_mid=rho[64].copy(), u_mid=u[:, 64].copy(),
        totals=G.conservation(S),
        tau=np.array(tau))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
