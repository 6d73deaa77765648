"""Brute-force per-cell, per-population FP64 version of the scheme, for tiny grids.

TEST INFRASTRUCTURE ONLY (see ``oracle.lbm``).

An independent second transcription of Eq. (2), Section 2.2 and Eqs. (3)-(6):
plain Python loops over cells and populations, an explicit neighbour table and
two buffers.  It imports nothing from ``oracle.lbm`` so that agreement between
the two is evidence about both.  Same readings as ``oracle.lbm``.
"""
from __future__ import annotations

import math

import numpy as np

VEL = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
WGT = [1 / 4, 1 / 8, 1 / 8, 1 / 8, 1 / 8, 1 / 8, 1 / 8]
BACK = [0, 2, 1, 4, 3, 6, 5]
# (a, b) of the six stress components k = 5..10
PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def _sidx(a, b):
    for j, (p, q) in enumerate(PAIRS):
        if (p, q) == (a, b) or (q, p) == (a, b):
            return 5 + j
    raise KeyError


def _mu(T, prm):
    th = T / prm["T_ref"]
    if prm["visc_law"] == 1:
        TS = prm["visc_param"]
        return prm["mu0"] * (1 + TS) * th ** 1.5 / (th + TS)
    if prm["visc_law"] == 2:
        return prm["mu0"] * th ** prm["visc_param"]
    return prm["mu0"]


def _cell_equilibrium(Qc, prm):
    """Equilibrium populations (14 x 7 list) of one cell's state vector."""
    g = prm["gamma"]
    lam = prm["dx"] / prm["dt"]
    rho = Qc[0]
    u = [Qc[1] / rho, Qc[2] / rho, Qc[3] / rho]
    E = Qc[4]
    p = (g - 1) * (E - 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2))
    T = p / rho
    mu = _mu(T, prm)
    visc = mu / prm["tau_R"]
    kap = g * prm["mu0"] / ((g - 1) * prm["prandtl"])
    heat = kap * (mu / prm["mu0"]) / prm["tau_q"]
    tau = [[Qc[_sidx(a, b)] for b in range(3)] for a in range(3)]
    q = [Qc[11], Qc[12], Qc[13]]
    # flux of component k along axis c
    F = [[0.0] * 3 for _ in range(14)]
    for c in range(3):
        F[0][c] = Qc[1 + c]
        for a in range(3):
            F[1 + a][c] = Qc[1 + a] * u[c] + (p if a == c else 0.0) - tau[a][c]
        tu = tau[c][0] * u[0] + tau[c][1] * u[1] + tau[c][2] * u[2]
        F[4][c] = (E + p) * u[c] - tu + q[c]
        for (a, b) in PAIRS:
            lam_abc = (u[a] if b == c else 0.0) + (u[b] if a == c else 0.0) - (2 / 3 * u[c] if a == b else 0.0)
            F[_sidx(a, b)][c] = tau[a][b] * u[c] - visc * lam_abc
        for a in range(3):
            F[11 + a][c] = q[a] * u[c] + (heat * T if a == c else 0.0)
    feq = [[0.0] * 7 for _ in range(14)]
    for k in range(14):
        for i in range(7):
            cf = VEL[i][0] * F[k][0] + VEL[i][1] * F[k][1] + VEL[i][2] * F[k][2]
            feq[k][i] = WGT[i] * (Qc[k] + cf / (0.25 * lam))
    return feq, rho, T, mu


def _collide_cell(fc, prm):
    """One cell: 14 x 7 populations in, 14 x 7 post-collision populations out."""
    Qc = [sum(fc[k][i] for i in range(7)) for k in range(14)]
    feq, rho, T, mu = _cell_equilibrium(Qc, prm)
    dt, dx = prm["dt"], prm["dx"]
    if prm.get("tau_base_override", 0.0) > 0:
        tb = prm["tau_base_override"]
    else:
        tb = 0.5 + 4 * prm["f_mu"] * (mu / rho) * dt / (dx * dx)
    om = 1.0 / tb
    if prm["C_sigma"] > 0:
        Dsum = 0.0
        for a in range(3):
            k = 5 + a
            n_plus = fc[k][1 + 2 * a] - feq[k][1 + 2 * a]
            n_minus = fc[k][2 + 2 * a] - feq[k][2 + 2 * a]
            n_rest = fc[k][0] - feq[k][0]
            Dsum += -(n_plus + n_minus - n_rest) / tb
        theta = -3 * prm["tau_R"] / (4 * mu) * Dsum
        s = max(0.0, -theta) / 0.5
        chi = min(1.0, prm["C_sigma"] * s) if s > prm["J_min"] else 0.0
        om = om - chi * max(0.0, om - prm["omega_min"])
    S = [0.0] * 14
    for k in range(5, 11):
        S[k] = -Qc[k] / prm["tau_R"]
    for k in range(11, 14):
        S[k] = -Qc[k] / prm["tau_q"]
    out = [[0.0] * 7 for _ in range(14)]
    for k in range(14):
        for i in range(7):
            out[k][i] = fc[k][i] - om * (fc[k][i] - feq[k][i]) + WGT[i] * dt * S[k]
    return out


def _noslip_return(Qc, prm, side, k, f_out):
    """Population of component k returning into a cell from the no-slip wall on
    its side 0 (x = 0) or 1 (x = nx dx), from the outgoing post-collision f_out
    and the cell's pre-collision state Qc.  Written out per component from the
    wall reading (a moving wall, isothermal at T_w > 0 or adiabatic): the
    momentum takes the wall's velocity and an adiabatic wall's q_x is zero (both
    anti-bounce-back); every other component returns with its normal flux at the
    wall: tau_xy, tau_xz: -visc(T*) u_w; q_x: heat(T_w) T_w; E: -(tau_xy u_wy +
    tau_xz u_wz) + q_x (the cell's q_x; zero on an adiabatic wall); the rest 0."""
    g = prm["gamma"]
    lam = prm["dx"] / prm["dt"]
    uw = [float(v) for v in prm["wall_u"][side]]
    Tw = float(prm["wall_T"][side])
    rho = Qc[0]
    u = [Qc[1] / rho, Qc[2] / rho, Qc[3] / rho]
    T = (g - 1) * (Qc[4] - 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)) / rho
    Tstar = Tw if Tw > 0 else T
    mu = _mu(Tstar, prm)
    visc = mu / prm["tau_R"]
    kap = g * prm["mu0"] / ((g - 1) * prm["prandtl"])
    heat = kap * (mu / prm["mu0"]) / prm["tau_q"]
    w = WGT[1]
    c_in = 1.0 if side == 0 else -1.0
    if k in (1, 2, 3):
        return -f_out + 2 * w * rho * uw[k - 1]
    if k == 11 and Tw <= 0:
        return -f_out
    if k == 4:
        Fx = -(Qc[8] * uw[1] + Qc[9] * uw[2]) + (Qc[11] if Tw > 0 else 0.0)
    elif k == 8:
        Fx = -visc * uw[1]
    elif k == 9:
        Fx = -visc * uw[2]
    elif k == 11:
        Fx = heat * Tstar
    else:
        Fx = 0.0
    return f_out + 2 * w * c_in * Fx / (0.25 * lam)


def run(Q0, prm, nsteps):
    """Brute-force run; Q0 (14, nz, ny, nx).  Returns f (14, 7, nz, ny, nx)."""
    nz, ny, nx = Q0.shape[1:]
    cells = [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx)]
    # explicit neighbour table: where population i of cell c goes
    dest = {}
    for (z, y, x) in cells:
        for i in range(7):
            cx, cy, cz = VEL[i]
            xd = x + cx
            dest[(z, y, x, i)] = ((z + cz) % nz, (y + cy) % ny, xd)   # xd checked below
    bc = prm.get("bc_x", 0)
    mirror = [1.0] * 14
    for k in (1, 8, 9, 11):
        mirror[k] = -1.0
    fl = fr = None
    if bc == 2:
        fl, _, _, _ = _cell_equilibrium(list(prm["Q_left"]), prm)
        fr, _, _, _ = _cell_equilibrium(list(prm["Q_right"]), prm)

    A = {}
    for (z, y, x) in cells:
        Qc = [float(Q0[k, z, y, x]) for k in range(14)]
        A[(z, y, x)] = _cell_equilibrium(Qc, prm)[0]
    for _ in range(nsteps):
        B = {c: [[None] * 7 for _ in range(14)] for c in cells}
        for c in cells:
            post = _collide_cell(A[c], prm)
            z, y, x = c
            for i in range(7):
                zd, yd, xd = dest[(z, y, x, i)]
                if 0 <= xd < nx:
                    for k in range(14):
                        B[(zd, yd, xd)][k][i] = post[k][i]
                elif bc == 0:
                    for k in range(14):
                        B[(zd, yd, xd % nx)][k][i] = post[k][i]
                elif bc == 1:
                    # the link hits the wall and returns reversed, with the mirror sign
                    for k in range(14):
                        B[(z, y, x)][k][BACK[i]] = mirror[k] * post[k][i]
                elif bc == 3:
                    Qc = [sum(A[c][k][j] for j in range(7)) for k in range(14)]
                    side = 0 if xd < 0 else 1
                    for k in range(14):
                        B[(z, y, x)][k][BACK[i]] = _noslip_return(Qc, prm, side, k, post[k][i])
                else:
                    pass  # leaves the domain
        if bc == 2:
            for (z, y, x) in cells:
                if x == 0:
                    for k in range(14):
                        B[(z, y, x)][k][1] = fl[k][1]
                if x == nx - 1:
                    for k in range(14):
                        B[(z, y, x)][k][2] = fr[k][2]
        A = B
    f = np.empty((14, 7, nz, ny, nx))
    for (z, y, x) in cells:
        for k in range(14):
            for i in range(7):
                f[k, i, z, y, x] = A[(z, y, x)][k][i]
    return f
