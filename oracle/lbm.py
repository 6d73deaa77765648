"""FP64 reference of the D3Q7 relaxed-flux compressible Navier-Stokes-Fourier scheme.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.

Plain NumPy, vectorised over cells, two arrays (pre- and post-collision), the
streaming done with ``np.roll``.  No reference shift, no compressed storage,
no in-place streaming: every step is written the way the paper states it.

Passages followed
-----------------
* Eq. (1)-(2), Section 2.1: the fourteen-component state Q = (rho, rho u, E,
  tau, q), the fluxes Phi and the sources S; ideal gas p = (gamma-1)(E -
  rho|u|^2/2), T = p/rho; Lambda(u) is the velocity tensor whose divergence is
  grad u + grad u^T - 2/3 (div u) I.  The listing of the declaration gives the
  temperature law mu_T, visc = mu_T/tau_R and heat = kappa (mu_T/mu)/tau_q.
* Section 2.2: one population set per component on D3Q7 (c_s^2 = 1/4), a
  linear equilibrium whose first moment is the flux, Q_k from the zeroth
  moment alone, BGK collide-and-stream with the source projected onto the
  lattice weights.
* Section 2.3, Eqs. (3)-(6): the one-sided local sensor s, the response chi,
  the blended rate omega_h and the baseline tau_base from f_mu.

Readings where the paper is silent (each listed in the design notes):
* The dilatation is recovered from the non-equilibrium of the three normal
  stress groups: per axis a, f^neq_{+a} + f^neq_{-a} - f^neq_0 of the tau_aa
  populations equals -tau_b dt d_a Phi_{tau_aa, a} to first order, and
  sum_a Phi_{tau_aa, a} carries -(4/3)(mu_T/tau_R) div u.
* The sensor divides by the baseline relaxation time and never raises the
  rate: omega_h = omega_b - chi * max(0, omega_b - omega_min).
* The source enters as w_i dt S_k with no half-step correction.
* One omega_h relaxes all 98 populations of a cell.
* No-slip walls (the paper's cases are periodic; it names wall boundaries
  generated from the declaration as the next step): the wall fixes the
  momentum, and q_x when adiabatic, by value; every other component returns
  with the declared normal flux at the wall state.

Pins (tests/test_oracle_pins.py; each checks against something other than
this code, so no function here is left with parity unpinned):
* equilibrium: its zeroth, first and second moments give Q, Phi and c_s^2 Q
  (closed forms of the lattice), and D3Q7's weights are isotropic.
* flux, viscosity, kappa: the characteristic speeds of the flux Jacobian
  equal the closed-form roots of the linearised system for constant,
  power-law and Sutherland viscosity; the Euler part converges to the exact
  Sod solution (star state equal to the textbook values), and the viscous and
  heat-flux parts to the closed-form Becker shock; Lambda's divergence is the
  deviatoric strain rate.
* source, collide: conservation to round-off and the exact decay of the
  summed stress and heat flux by (1 - dt/tau) per step.
* tau_base: a passive entropy mode diffuses at c_s^2 (tau_b - 1/2) dx^2/dt,
  and the added viscosity is f_mu mu/rho.
* dilatation, relaxation_rate: the estimate equals dt times the spectral
  divergence of a prescribed field; with C_sigma = 0 the rate is plain BGK.
* stream: brute force on 4^3 grids, fixed points, symmetry, the wall equal
  to the mirror-doubled periodic domain, y/z-uniform data equal to 1D.
* wall_state and the no-slip links: the loop transcription in oracle.brute,
  which writes each component's wall term out by hand, agrees with the
  declared flux evaluated at the wall state here; a still adiabatic wall equals the domain
  doubled with its point-inverted image; gas at rest, and gas moving with
  the walls, are fixed points; steady Couette flow is linear with
  tau_xy = mu U/H; steady conduction converges at second order to the
  linear temperature profile between the wall temperatures.

Array layout: f has shape (14, 7, nz, ny, nx); Q has shape (14, nz, ny, nx).
"""
from __future__ import annotations

import numpy as np

# D3Q7 (Section 2.2): rest, +x, -x, +y, -y, +z, -z.
C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.int64)
W = np.array([0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125])
CS2 = 0.25
OPP = np.array([0, 2, 1, 4, 3, 6, 5])

RHO, MX, MY, MZ, EN = 0, 1, 2, 3, 4
TXX, TYY, TZZ, TXY, TXZ, TYZ = 5, 6, 7, 8, 9, 10
QX, QY, QZ = 11, 12, 13
# component index of tau_ab
TAU = {(0, 0): TXX, (1, 1): TYY, (2, 2): TZZ,
       (0, 1): TXY, (1, 0): TXY, (0, 2): TXZ, (2, 0): TXZ, (1, 2): TYZ, (2, 1): TYZ}
TAU_PAIRS = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]

VISC_CONST, VISC_SUTHERLAND, VISC_POWER = 0, 1, 2
BC_PERIODIC, BC_WALL, BC_DIRICHLET, BC_NOSLIP = 0, 1, 2, 3

# Components odd under the reflection x -> -x: rho u_x, tau_xy, tau_xz, q_x.
SIGMA_X = np.ones(14)
SIGMA_X[[MX, TXY, TXZ, QX]] = -1.0


def kappa(prm):
    """Conductivity from the Prandtl number, c_p = gamma/(gamma-1) with R = 1."""
    g = prm["gamma"]
    return g * prm["mu0"] / ((g - 1.0) * prm["prandtl"])


def viscosity(T, prm):
    """mu_T of the declaration: constant, Sutherland (T_S in units of T_ref) or power law."""
    mu0 = prm["mu0"]
    th = T / prm["T_ref"]
    law = prm["visc_law"]
    if law == VISC_SUTHERLAND:
        TS = prm["visc_param"]
        return mu0 * (1.0 + TS) * th ** 1.5 / (th + TS)
    if law == VISC_POWER:
        return mu0 * th ** prm["visc_param"]
    return mu0 * np.ones_like(T)


def primitives(Q, prm):
    """rho, u (3, ...), E, p, T from the conserved state (ideal gas, Section 2.1)."""
    rho = Q[RHO]
    u = Q[MX:MZ + 1] / rho
    E = Q[EN]
    p = (prm["gamma"] - 1.0) * (E - 0.5 * rho * np.sum(u * u, axis=0))
    T = p / rho
    return rho, u, E, p, T


def stress_tensor(Q):
    return [[Q[TAU[(a, b)]] for b in range(3)] for a in range(3)]


def flux(Q, prm):
    """Phi_k (shape (14, 3, ...)) of Eq. (2), in the sign convention of Eq. (2)."""
    rho, u, E, p, T = primitives(Q, prm)
    muT = viscosity(T, prm)
    nu_R = muT / prm["tau_R"]                           # visc
    K_q = kappa(prm) * (muT / prm["mu0"]) / prm["tau_q"]  # heat
    tau = stress_tensor(Q)
    q = Q[QX:QZ + 1]
    Phi = np.zeros((14, 3) + Q.shape[1:], dtype=np.result_type(Q.dtype, np.float64))
    d = np.eye(3)
    for c in range(3):
        # mass: rho u
        Phi[RHO, c] = Q[MX + c]
        # momentum: rho u (x) u + p I - tau
        for a in range(3):
            Phi[MX + a, c] = Q[MX + a] * u[c] + p * d[a, c] - tau[a][c]
        # energy: (E + p) u - tau . u + q
        Phi[EN, c] = (E + p) * u[c] - sum(tau[c][b] * u[b] for b in range(3)) + q[c]
        # stress: tau (x) u - (mu_T/tau_R) Lambda(u)
        for (a, b) in TAU_PAIRS:
            Lam = u[a] * d[b, c] + u[b] * d[a, c] - (2.0 / 3.0) * d[a, b] * u[c]
            Phi[TAU[(a, b)], c] = tau[a][b] * u[c] - nu_R * Lam
        # heat flux: q (x) u + (kappa/tau_q) (mu_T/mu) T I
        for a in range(3):
            Phi[QX + a, c] = q[a] * u[c] + K_q * T * d[a, c]
    return Phi


def source(Q, prm):
    """S of Eq. (2): zero for rho, rho u, E; -tau/tau_R; -q/tau_q."""
    S = np.zeros_like(Q)
    S[TXX:TYZ + 1] = -Q[TXX:TYZ + 1] / prm["tau_R"]
    S[QX:QZ + 1] = -Q[QX:QZ + 1] / prm["tau_q"]
    return S


def lattice_speed(prm):
    return prm["dx"] / prm["dt"]


def equilibrium(Q, Phi, prm):
    """f^eq_{k,i} = w_i (Q_k + c_i . Phi_k / (c_s^2 lambda)), lambda = dx/dt (Section 2.2)."""
    lam = lattice_speed(prm)
    feq = np.empty((14, 7) + Q.shape[1:], dtype=np.result_type(Q.dtype, np.float64))
    for i in range(7):
        cphi = sum(C[i, a] * Phi[:, a] for a in range(3))
        feq[:, i] = W[i] * (Q + cphi / (CS2 * lam))
    return feq


def moments(f):
    """Q_k = sum_i f_{k,i}: the zeroth moment alone (Section 2.2)."""
    return f.sum(axis=1)


def tau_base(Q, prm):
    """Baseline relaxation time in time-step units, Eq. (6), with local mu_T/rho."""
    if prm.get("tau_base_override", 0.0) > 0.0:
        return np.full(Q.shape[1:], float(prm["tau_base_override"]))
    rho, u, E, p, T = primitives(Q, prm)
    muT = viscosity(T, prm)
    return 0.5 + 4.0 * prm["f_mu"] * (muT / rho) * prm["dt"] / prm["dx"] ** 2


def dilatation(f, feq, Q, prm):
    """Local estimate of dt * div u from the normal-stress non-equilibrium (Section 2.3)."""
    rho, u, E, p, T = primitives(Q, prm)
    muT = viscosity(T, prm)
    tb = tau_base(Q, prm)
    fneq = f - feq
    D = np.zeros(Q.shape[1:])
    for a in range(3):
        k = TAU[(a, a)]
        ip, im = 1 + 2 * a, 2 + 2 * a
        # ~ dt d_a Phi_{tau_aa, a}
        D += -(fneq[k, ip] + fneq[k, im] - fneq[k, 0]) / tb
    # sum_a Phi_{tau_aa,a} = ... - (4/3) (mu_T/tau_R) div u
    return -(3.0 * prm["tau_R"] / (4.0 * muT)) * D


def relaxation_rate(f, feq, Q, prm):
    """omega_h of Eqs. (3)-(5) per cell; also returns chi."""
    tb = tau_base(Q, prm)
    omega_b = 1.0 / tb
    Cs = prm["C_sigma"]
    if Cs <= 0.0:
        return omega_b, np.zeros_like(omega_b)
    theta = dilatation(f, feq, Q, prm)
    s = np.maximum(0.0, -theta) / np.sqrt(CS2)               # Eq. (3)
    chi = np.where(s > prm["J_min"], np.clip(Cs * s, 0.0, 1.0), 0.0)  # Eq. (4)
    omega_h = omega_b - chi * np.maximum(0.0, omega_b - prm["omega_min"])  # Eq. (5)
    return omega_h, chi


def collide(f, prm):
    """f* = f - omega_h (f - f^eq) + w_i dt S_k (Section 2.2)."""
    Q = moments(f)
    Phi = flux(Q, prm)
    feq = equilibrium(Q, Phi, prm)
    omega_h, _ = relaxation_rate(f, feq, Q, prm)
    S = source(Q, prm)
    fs = np.empty_like(f)
    for i in range(7):
        fs[:, i] = f[:, i] - omega_h * (f[:, i] - feq[:, i]) + W[i] * prm["dt"] * S
    return fs


def uniform_equilibrium(Qvec, prm):
    """f^eq (14, 7) of a uniform 14-vector state (used by the equilibrium inflow)."""
    Q = np.asarray(Qvec, dtype=np.float64).reshape(14, 1)
    return equilibrium(Q, flux(Q, prm), prm)[:, :, 0]


def wall_state(Qb, prm, side):
    """The state a no-slip wall imposes next to a boundary cell, and which components it fixes by value.

    The wall moves tangentially with u_w and is either isothermal (T_w > 0) or
    adiabatic (T_w = 0).  Its state keeps the cell's density, stress and heat
    flux, takes the wall's velocity and the wall's temperature (the cell's when
    adiabatic), and has no normal heat flux when adiabatic.  The wall fixes the
    momentum, and q_x when it is adiabatic; every other component, the energy
    included, takes its normal flux from the declared flux of Eq. (2) at this
    state, so an isothermal wall acts through K_q(T_w) T_w, the normal flux of q_x.
    """
    uw = np.asarray(prm["wall_u"][side], dtype=np.float64)
    Tw = float(prm["wall_T"][side])
    rho, u, E, p, T = primitives(Qb, prm)
    Tstar = np.full_like(T, Tw) if Tw > 0.0 else T
    Qw = np.array(Qb, dtype=np.float64, copy=True)
    for a in range(3):
        Qw[MX + a] = rho * uw[a]
    Qw[EN] = rho * Tstar / (prm["gamma"] - 1.0) + 0.5 * rho * float(uw @ uw)
    by_value = np.zeros(14, dtype=bool)
    by_value[[MX, MY, MZ]] = True
    if Tw <= 0.0:
        Qw[QX] = 0.0
        by_value[QX] = True
    return Qw, by_value


def stream(fs, prm, Q=None):
    """f_{k,i}(x + c_i) <- f*_{k,i}(x); periodic, or walls / equilibrium ends in x.

    Q: pre-collision moments of the step (needed by no-slip walls only)."""
    f = np.empty_like(fs)
    for i in range(7):
        # array axes (z, y, x)
        f[:, i] = np.roll(fs[:, i], shift=(C[i, 2], C[i, 1], C[i, 0]), axis=(1, 2, 3))
    bc = prm.get("bc_x", BC_PERIODIC)
    if bc == BC_NOSLIP:
        # the population leaving through a wall returns along the opposite
        # link: by value (anti-bounce-back) f_in = -f*_out + 2 w Q_w, by flux
        # (bounce-back) f_in = f*_out + 2 w c_in Phi_w,x / (c_s^2 lambda)
        lam = lattice_speed(prm)
        for side, (x, i_in, i_out, c_in) in enumerate(((0, 1, 2, 1.0), (-1, 2, 1, -1.0))):
            Qw, by_value = wall_state(Q[..., x], prm, side)
            Phw = flux(Qw, prm)[:, 0]
            for k in range(14):
                if by_value[k]:
                    f[k, i_in, :, :, x] = -fs[k, i_out, :, :, x] + 2.0 * W[1] * Qw[k]
                else:
                    f[k, i_in, :, :, x] = fs[k, i_out, :, :, x] + 2.0 * W[1] * c_in * Phw[k] / (CS2 * lam)
    elif bc == BC_WALL:
        # halfway bounce-back with the mirror sign of each component
        sig = SIGMA_X.reshape(14, 1, 1)
        f[:, 1, :, :, 0] = sig * fs[:, 2, :, :, 0]
        f[:, 2, :, :, -1] = sig * fs[:, 1, :, :, -1]
    elif bc == BC_DIRICHLET:
        fl = uniform_equilibrium(prm["Q_left"], prm)
        fr = uniform_equilibrium(prm["Q_right"], prm)
        f[:, 1, :, :, 0] = fl[:, 1].reshape(14, 1, 1)
        f[:, 2, :, :, -1] = fr[:, 2].reshape(14, 1, 1)
    return f


def step(f, prm):
    Q = moments(f) if prm.get("bc_x", BC_PERIODIC) == BC_NOSLIP else None
    return stream(collide(f, prm), prm, Q)


def init_populations(Q, prm):
    """Initial populations f = f^eq(Q)."""
    return equilibrium(Q, flux(Q, prm), prm)


def run(Q0, prm, nsteps, callback=None, every=0):
    f = init_populations(np.asarray(Q0, dtype=np.float64), prm)
    for n in range(nsteps):
        if callback is not None and every and n % every == 0:
            callback(n, f)
        f = step(f, prm)
    if callback is not None and every and nsteps % every == 0:
        callback(nsteps, f)
    return f
