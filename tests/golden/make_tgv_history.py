"""Write the FP64 oracle's Taylor-Green diagnostic history (Eq. (7)) to a golden file.

Runs only the oracle and the seeded input generator: the supersonic
Taylor-Green vortex (M0 1.25, Re 1600, Pr 0.71, mu ~ T^0.76) at N^3 from
t_c = 0 to t_c = T_END, recording E_k, eps_s, eps_d, mass and energy every
EVERY steps.

usage: python tests/golden/make_tgv_history.py [N] [T_END] [EVERY] [F_MU] [M0] [RE] [LAW] [PARTIAL]

The file name carries N, F_MU (if given), M0 and RE (if given), LAW (if not
the power law) and T_END (if not 20).

The defaults are the supersonic case; the subsonic verification case of
Section 3.2 is M0 0.5, Re 500 with F_MU 0.  LAW is the viscosity law:
"power" (mu ~ T^0.76, the default), "sutherland" or "const" (mu = 1/Re
everywhere).  With a temperature-dependent mu the declared stress flux
(mu_T/tau_R) Lambda(u) makes the system lose hyperbolicity at local Mach
numbers near 2, and the paper's background dissipation at 64^3 is not enough
to carry the run to t_c = 20; with constant mu it is.
"""
import json
import os
import sys
import time
import warnings

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import diagnostics, lbm  # noqa: E402


def main():
    warnings.simplefilter("ignore", RuntimeWarning)
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 64
    t_end = float(sys.argv[2]) if len(sys.argv) > 2 else 20.0
    every = int(sys.argv[3]) if len(sys.argv) > 3 else 10
    f_mu = float(sys.argv[4]) if len(sys.argv) > 4 else None
    M0 = float(sys.argv[5]) if len(sys.argv) > 5 else 1.25
    Re = float(sys.argv[6]) if len(sys.argv) > 6 else 1600.0
    law = sys.argv[7] if len(sys.argv) > 7 else "power"
    # PARTIAL > 0: also write the history so far every PARTIAL records
    partial = int(sys.argv[8]) if len(sys.argv) > 8 else 0
    case = W.tgv(n, f_mu=f_mu, M0=M0, Re=Re, law=law)
    prm = case.params
    steps = int(np.ceil(t_end / prm["dt"] / every)) * every
    tag = "" if f_mu is None else f"_fmu{f_mu:g}"
    if len(sys.argv) > 5:
        tag += f"_M{M0:g}_Re{Re:g}"
    if law != "power":
        tag += f"_{law}"
    if t_end != 20.0:
        tag += f"_t{t_end:g}"
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"tgv{n}{tag}_history.json")
    hist = dict(step=[], t=[], E_k=[], eps_s=[], eps_d=[], mass=[], energy=[])
    f = lbm.init_populations(case.Q0, prm)
    t0 = time.time()

    def write(last):
        # the history so far: a prefix of the run is itself a valid golden of
        # `last` steps, so a long run can be stopped and still leave one
        rec = dict(source="oracle.lbm FP64, oracle.diagnostics (Eq. (7), spectral derivatives)",
                   case=dict(n=n, M0=M0, Re=Re, Pr=0.71,
                             law={"power": "power 0.76", "sutherland": "Sutherland 0.4042", "const": "constant"}[law],
                             f_mu=prm["f_mu"], dt=prm["dt"], C_sigma=prm["C_sigma"], J_min=prm["J_min"],
                             omega_min=prm["omega_min"]),
                   every=every, steps=last, wall_seconds=round(time.time() - t0, 1), history=hist)
        with open(out + ".tmp", "w") as fh:
            json.dump(rec, fh)
        os.replace(out + ".tmp", out)

    for s in range(steps + 1):
        if s % every == 0:
            d = diagnostics.diagnostics(lbm.moments(f), prm)
            hist["step"].append(s)
            hist["t"].append(s * prm["dt"])
            for k in ("E_k", "eps_s", "eps_d", "mass", "energy"):
                hist[k].append(d[k])
            if not np.isfinite(d["E_k"]):
                break
            if s % (every * 20) == 0:
                print(f"step {s}/{steps} t_c {s * prm['dt']:.2f} E_k {d['E_k']:.5f} eps_d {d['eps_d']:.3e} "
                      f"({time.time() - t0:.0f} s)", flush=True)
            if partial and s > 0 and s % (every * partial) == 0:
                write(s)
        if s < steps:
            f = lbm.step(f, prm)
    write(hist["step"][-1])
    print("wrote", out)


if __name__ == "__main__":
    main()
