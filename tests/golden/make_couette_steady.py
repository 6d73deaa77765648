"""Write the FP64 oracle's steady Couette state between no-slip walls to a golden file.

Runs only the oracle and the seeded input generator: gas at rest (rho = 1,
T = 1) between isothermal walls at T = 1, the wall at x = 1 moving at U = 0.5
along y, constant viscosity mu = 0.05, Pr = 0.71, f_mu = 0.16/N, from t = 0
to t = T_END on an N x 1 x 1 lattice (y and z are uniform).

usage: python tests/golden/make_couette_steady.py [N] [T_END]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import lbm  # noqa: E402


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 16
    t_end = float(sys.argv[2]) if len(sys.argv) > 2 else 30.0
    U, mu, f_mu = 0.5, 0.05, 0.16 / n
    prm = W.couette_params(n, U=U, T_L=1.0, T_R=1.0, mu=mu, f_mu=f_mu)
    sh = (1, 1, n)
    one, zero = np.ones(sh), np.zeros(sh)
    Q = W.conserved(one, zero, zero, zero, one, prm["gamma"])
    steps = int(round(t_end / prm["dt"]))
    t0 = time.time()
    Qn = lbm.moments(lbm.run(Q, prm, steps))
    rho, u, E, p, T = lbm.primitives(Qn, prm)
    out = dict(n=n, t_end=t_end, U=U, mu=mu, f_mu=f_mu, dt=prm["dt"], steps=steps,
               rho=rho[0, 0].tolist(), u_y=u[1, 0, 0].tolist(), p=p[0, 0].tolist(), T=T[0, 0].tolist(),
               oracle_seconds=round(time.time() - t0, 1))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"couette{n}_steady.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path, f"{steps} steps, {out['oracle_seconds']} s")


if __name__ == "__main__":
    main()
