"""Taylor-Green runs on the GPU: Eq. (7) histories and shell spectra through the C ABI.

usage:
  python -m paper_2608_13437_amd.runs subsonic   [--n N] [--out PATH]
  python -m paper_2608_13437_amd.runs supersonic [--n N] [--f-mu F] [--t-end T] [--out PATH]
  python -m paper_2608_13437_amd.runs sweep      [--n N] [--f-mu F] [--C-sigma 10 20 40 80] [--out PATH]
  python -m paper_2608_13437_amd.runs gridstudy  [--n 192 256 320 384 512] [--out PATH]
  python -m paper_2608_13437_amd.runs couette    [--n 16 32 64 128] [--t-end T] [--out PATH]
  python -m paper_2608_13437_amd.runs becker     [--n 128 256 512 1024] [--t-end T] [--out PATH]

* subsonic: the shock-free verification case of Section 3.2 (Re 500, M0 0.5,
  f_mu 0) to t_c = 10.
* supersonic: the compressible case of Section 3.2 (Re 1600, M0 1.25, C_sigma 40,
  J_min 1e-2, omega_min 1.987) with the given f_mu.
* sweep: the supersonic case once per sensor slope C_sigma.
* gridstudy: the grid-convergence configurations of Section 3.2 (192^3 to
  512^3, C_sigma 20, each with its own f_mu and J_min).
* couette: steady compressible Couette flow between no-slip isothermal walls
  (one still, one moving at U = 0.5, Mach 0.42) at each resolution, against
  its closed form: u = U x/H and T = T_w + (mu U^2 / 2 kappa) (x/H)(1 - x/H)
  at uniform pressure, the steady state of Eq. (2) with constant viscosity.
* becker: the stationary Mach 2 viscous shock of Section 3.1 (n x 4 x 4,
  equilibrium ends) from its closed form to the steady state, with the
  10-90% density thickness against the closed form's.

Every Taylor-Green case takes --law (mu ~ T^0.76 by default, Sutherland, or
constant) and --storage.  Every step and every diagnostic runs in the HIP library; inputs come from the
seeded generators of ``workloads``.  A run that turns non-finite stops and
reports the time it happened.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

from . import Lattice  # noqa: E402

HISTORY_KEYS = ("E_k", "eps_s", "eps_d", "mass", "energy", "min_rho", "min_p", "sensor_fraction")


def tgv_run(n, *, t_end=None, steps=None, every=10, spectra_at=(), storage=W.STORAGE_FP32, slab=32, progress=0,
            placed=False, **tgv_kw):
    """Run the Taylor-Green vortex on an n^3 lattice to t_end (convective times; or
    for `steps` steps, a multiple of `every`), recording the FP64 diagnostics every
    `every` steps and the shell spectrum at the recorded steps nearest to each
    time in `spectra_at`.  progress > 0 prints a line every `progress` steps;
    placed puts the populations on the fastest of several probed allocations
    (Lattice.placed), which only changes the speed."""
    prm = W.tgv_params(n, storage=storage, **tgv_kw)
    L = Lattice.placed(prm) if placed else Lattice(prm)
    for z0 in range(0, n, slab):
        L.set_state(W.tgv_slab(prm, z0, min(n, z0 + slab)), z0=z0)
    dt = prm["dt"]
    if steps is None:
        steps = int(math.ceil(t_end / dt / every)) * every
    assert steps % every == 0
    want = {int(round(t / dt / every)) * every: t for t in spectra_at}
    hist = {"step": [], "t": []}
    hist.update({k: [] for k in HISTORY_KEYS})
    spectra = {}
    status, t0 = "ok", time.perf_counter()
    for s in range(0, steps + 1, every):
        E = L.spectrum().tolist() if s in want else None
        # the first of the next `every` updates also reduces the level it reads
        d = L.step_diagnostics(every, spectral=True) if s < steps else L.diagnostics(spectral=True)
        hist["step"].append(s)
        hist["t"].append(s * dt)
        for k in HISTORY_KEYS:
            hist[k].append(d[k])
        if d["nonfinite"]:
            status = f"non-finite at t_c = {s * dt:.3f}"
            break
        if E is not None:
            spectra[f"{s * dt:.4f}"] = E
        if progress and s % progress == 0:
            print(f"  n {n} step {s}/{steps} t_c {s * dt:.2f} E_k {d['E_k']:.5f} eps_s {d['eps_s']:.4e} "
                  f"eps_d {d['eps_d']:.4e} ({time.perf_counter() - t0:.0f} s)", flush=True)
    wall = time.perf_counter() - t0
    L.close()
    done = hist["step"][-1]
    case = dict(tgv_kw)
    case.update(n=n, dt=dt, storage=storage)
    case.update({k: prm[k] for k in ("f_mu", "C_sigma", "J_min", "omega_min", "mu0", "tau_R", "tau_q")})
    return dict(case=case, every=every, steps=done, status=status, wall_seconds=round(wall, 2),
                mlups_with_diagnostics=round(n ** 3 * done / wall / 1e6, 1) if wall > 0 else None,
                history=hist, spectra=spectra)


def couette_run(n, *, U=0.5, T_w=1.0, mu=0.05, f_mu=None, t_end=30.0, storage=W.STORAGE_FP32, ny=4, nz=4):
    """Couette flow from rest to t_end; errors of the final state against the closed
    form.  f_mu defaults to 0.16/n, so the background dissipation vanishes under
    refinement like the paper's resolution-dependent values."""
    import numpy as np
    f_mu = 0.16 / n if f_mu is None else f_mu
    prm = W.couette_params(n, ny, nz, U=U, T_L=T_w, T_R=T_w, mu=mu, f_mu=f_mu)
    prm["storage"] = storage
    L = Lattice(prm)
    sh = (nz, ny, n)
    one, zero = np.ones(sh), np.zeros(sh)
    L.set_state(W.conserved(one, zero, zero, zero, T_w * one, prm["gamma"]))
    steps = int(round(t_end / prm["dt"]))
    t0 = time.perf_counter()
    L.step(steps)
    P = L.primitives().mean(axis=(1, 2))
    wall = time.perf_counter() - t0
    L.step(100)
    change = float(np.abs(L.primitives().mean(axis=(1, 2)) - P).max())
    L.close()
    g = prm["gamma"]
    kappa = g * mu / ((g - 1.0) * prm["prandtl"])
    x = (np.arange(n) + 0.5) / n
    rise = mu * U * U / (2.0 * kappa)
    u_e, T_e = U * x, T_w + rise * x * (1.0 - x)
    return dict(n=n, f_mu=f_mu, dt=prm["dt"], steps=steps, wall_seconds=round(wall, 2),
                err_u=float(np.abs(P[2] - u_e).max() / U), err_T=float(np.abs(P[5] - T_e).max() / (rise / 4.0)),
                p_spread=float((P[4].max() - P[4].min()) / P[4].mean()), change_100_steps=change,
                u=P[2].tolist(), T=P[5].tolist())


def _crossing_width(x, rho, lo, hi, levels=(0.1, 0.9)):
    """Distance between the first crossings of two levels of a density jump from lo to hi."""
    import numpy as np
    xs = []
    for lev in levels:
        r = lo + lev * (hi - lo)
        i = int(np.nonzero(np.diff(np.sign(rho - r)) != 0)[0][0])
        xs.append(x[i] + (r - rho[i]) * (x[i + 1] - x[i]) / (rho[i + 1] - rho[i]))
    return abs(xs[1] - xs[0])


def becker_run(n, *, t_end=0.05, check_every=None, storage=W.STORAGE_FP32, ny=4, nz=4):
    """The stationary Becker shock (Mach 2, Pr 3/4, constant mu; equilibrium ends at
    the Rankine-Hugoniot states) on an n x ny x nz lattice from its closed-form
    profile to t_end.  Records the 10-90% density thickness every `check_every`
    steps (default: 20 records) against the closed form's, so the approach to
    the steady state can be read off; returns the final density profile (the
    y/z mean) with the records."""
    import numpy as np
    c = W.becker(n, ny, nz)
    prm = dict(c.params, storage=storage)
    L = Lattice(prm)
    L.set_state(c.Q0)
    x = c.meta["x"]
    (r1, u1, p1), (r2, u2, p2), _ = W.becker_states()
    xf = np.linspace(0.0, c.meta["L"], 20001)
    w_ex = _crossing_width(xf, W.becker_profile(xf, 0.5 * c.meta["L"])[0], r1, r2)
    steps = int(round(t_end / prm["dt"]))
    every = check_every or max(1, steps // 20)
    rec = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        L.step(k)
        done += k
        P = L.primitives().mean(axis=(1, 2))
        rec.append(dict(step=done, t=done * prm["dt"], excess=_crossing_width(x, P[0], r1, r2) / w_ex - 1.0))
    wall = time.perf_counter() - t0
    P = L.primitives().mean(axis=(1, 2))
    L.close()
    return dict(n=n, dt=prm["dt"], steps=steps, storage=storage, w_ex=w_ex, excess=rec[-1]["excess"],
                wall_seconds=round(wall, 3), us_per_step=round(wall / max(steps, 1) * 1e6, 2),
                records=rec, rho=P[0].tolist(), u=P[1].tolist(), p=P[4].tolist())


def eps_d_peaks(run, split=4.5):
    """The two dilatational-dissipation peaks of the supersonic run (Section 3.2
    places them near t_c = 2.5 and 6.5): the largest eps_d before and after
    t_c = split, their times, and the ratio early / late."""
    h = run["history"]
    early = [(e, t) for e, t in zip(h["eps_d"], h["t"]) if t <= split]
    late = [(e, t) for e, t in zip(h["eps_d"], h["t"]) if t > split]
    if not early or not late:
        return None
    (e1, t1), (e2, t2) = max(early), max(late)
    return dict(early=e1, t_early=t1, late=e2, t_late=t2, ratio=e1 / e2 if e2 > 0 else None)


def summary(run):
    h = run["history"]
    i = max(range(len(h["eps_s"])), key=lambda j: h["eps_s"][j])
    pk = eps_d_peaks(run)
    peaks = "" if pk is None else (f", eps_d peaks {pk['early']:.3e} at t_c {pk['t_early']:.2f} and "
                                   f"{pk['late']:.3e} at {pk['t_late']:.2f} (ratio {pk['ratio']:.3f})")
    return (f"n {run['case']['n']} {run['status']}: t_c {h['t'][-1]:.2f} ({run['steps']} steps), "
            f"peak eps_s {h['eps_s'][i]:.5e} at t_c {h['t'][i]:.2f}, max eps_d {max(h['eps_d']):.3e}{peaks}, "
            f"E_k end {h['E_k'][-1]:.5f}, {run['wall_seconds']} s")


# Grid-convergence configurations of Section 3.2 (Table "ctgv_conv", C_sigma = 20):
# (N, f_mu, J_min)
GRID_STUDY = ((192, 3e-2, 3e-3), (256, 1e-2, 3e-3), (320, 8e-3, 3e-3), (384, 1e-2, 3e-3), (512, 1e-2, 1e-2))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("case", choices=("subsonic", "supersonic", "sweep", "gridstudy", "couette", "becker"))
    ap.add_argument("--n", type=int, nargs="+", default=None)
    ap.add_argument("--f-mu", type=float, default=None)
    ap.add_argument("--C-sigma", type=float, nargs="+", default=[10.0, 20.0, 40.0, 80.0])
    ap.add_argument("--t-end", type=float, default=None)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--law", choices=("power", "sutherland", "const"), default="power",
                    help="viscosity law of the Taylor-Green runs (mu ~ T^0.76, Sutherland, or constant)")
    ap.add_argument("--storage", choices=("fp32", "fp16", "bf16"), default="fp32")
    ap.add_argument("--progress", type=int, default=1000, help="print a line every this many steps")
    ap.add_argument("--no-placement", action="store_true",
                    help="one plain allocation instead of the fastest of several probed ones")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    runs = []
    if a.case == "becker":
        for n in a.n or [128, 256, 512, 1024]:
            r = becker_run(n, t_end=a.t_end or 0.05)
            drift = abs(r["records"][-1]["excess"] - r["records"][-5]["excess"])
            print(f"becker n {n}: {r['steps']} steps, |w/w_ex - 1| {r['excess']:.4e} (change over the last "
                  f"20% of the run {drift:.1e}), {r['us_per_step']} us/step", flush=True)
            runs.append(r)
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(runs, fh)
        return
    if a.case == "couette":
        for n in a.n or [16, 32, 64, 128]:
            r = couette_run(n, t_end=a.t_end or 30.0, f_mu=a.f_mu)
            print(f"couette n {n}: {r['steps']} steps, max |u - u_e|/U {r['err_u']:.3e}, max |T - T_e|/rise "
                  f"{r['err_T']:.3e}, p spread {r['p_spread']:.2e}, change over 100 steps "
                  f"{r['change_100_steps']:.1e}, {r['wall_seconds']} s", flush=True)
            runs.append(r)
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(runs, fh)
        return
    n = (a.n or [128])[0]
    st = {"fp32": W.STORAGE_FP32, "fp16": W.STORAGE_FP16, "bf16": W.STORAGE_BF16}[a.storage]
    kw = dict(every=a.every, law=a.law, storage=st, progress=a.progress, placed=not a.no_placement)
    if a.case == "subsonic":
        runs.append(tgv_run(n, t_end=a.t_end or 10.0, spectra_at=(0.0, 5.0, 10.0),
                            M0=0.5, Re=500.0, f_mu=0.0 if a.f_mu is None else a.f_mu, **kw))
    elif a.case == "supersonic":
        runs.append(tgv_run(n, t_end=a.t_end or 20.0, spectra_at=(0.0, 2.5, 9.0, 20.0), f_mu=a.f_mu, **kw))
    elif a.case == "gridstudy":
        for (gn, f_mu, j_min) in GRID_STUDY:
            if a.n and gn not in a.n:
                continue
            runs.append(tgv_run(gn, t_end=a.t_end or 20.0, f_mu=f_mu, J_min=j_min, C_sigma=20.0, **kw))
    else:
        for cs in a.C_sigma:
            runs.append(tgv_run(n, t_end=a.t_end or 20.0, f_mu=a.f_mu, C_sigma=cs, **kw))
    for r in runs:
        r["eps_d_peaks"] = eps_d_peaks(r)
        print(summary(r), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(runs, fh)


if __name__ == "__main__":
    main()
