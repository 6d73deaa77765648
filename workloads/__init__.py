"""Seeded synthetic inputs for the D3Q7 compressible Navier-Stokes-Fourier scheme.

This module is shared by the FP64 oracle tests and by the HIP path.  It holds
case parameters and initial macroscopic fields only: nothing of the lattice
Boltzmann update itself (equilibrium, flux, collision, streaming, sensor) is
computed here.  Initial conditions are given in primitive variables and
converted to the conserved fourteen-component state of Eq. (2):

    k = 0 rho, 1..3 rho*u, 4 E, 5..10 tau_xx,yy,zz,xy,xz,yz, 11..13 q_x,y,z

Fields are float64 arrays of shape (14, nz, ny, nx), x fastest.

The time step follows the acoustic Courant number of the parameter table
(Section 2.3, Table "Parameters"): dt = CFL * dx / a_ref.  a_ref is read here as
the largest characteristic speed of the relaxed fourteen-component system over
the initial field (see :func:`char_speed`), the bound that keeps the
sub-characteristic condition a_ref <= c_s * dx / dt satisfied for CFL <= 1/2.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NCOMP = 14
COMPONENT_NAMES = (
    "rho", "mx", "my", "mz", "E",
    "txx", "tyy", "tzz", "txy", "txz", "tyz",
    "qx", "qy", "qz",
)

VISC_CONST, VISC_SUTHERLAND, VISC_POWER = 0, 1, 2
BC_PERIODIC, BC_WALL, BC_DIRICHLET, BC_NOSLIP = 0, 1, 2, 3
STORAGE_FP32, STORAGE_FP16, STORAGE_BF16 = 0, 1, 2

# Largest characteristic speed |u*| + c*_R of the exact Sod Riemann solution
# (left (1, 0, 1), right (0.125, 0, 0.1), gamma = 1.4).  The tests recompute it
# from the oracle's exact Riemann solver.
SOD_A_REF = 2.191566


def default_params(nx: int, ny: int, nz: int) -> dict:
    """Parameter set with the field names of the C struct ``cnsf_params``."""
    return dict(
        nx=int(nx), ny=int(ny), nz=int(nz),
        dx=1.0, dt=0.1,
        gamma=1.4, mu0=1e-2, T_ref=1.0,
        visc_law=VISC_CONST, visc_param=0.0,
        prandtl=0.71,
        tau_R=0.5, tau_q=0.5,
        f_mu=0.0, tau_base_override=0.0,
        C_sigma=0.0, J_min=0.0, omega_min=1.0,
        bc_x=BC_PERIODIC,
        Q_left=[0.0] * NCOMP, Q_right=[0.0] * NCOMP,
        storage=STORAGE_FP32,
        Q_ref=[0.0] * NCOMP,
        storage_scale=[0.0] * NCOMP,
        a_ref=0.0,
        wall_u=[[0.0] * 3, [0.0] * 3], wall_T=[0.0, 0.0],
    )


@dataclasses.dataclass
class Case:
    name: str
    params: dict
    Q0: np.ndarray | None            # (14, nz, ny, nx) float64; None for slab-generated cases
    steps: int = 0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def shape(self):
        p = self.params
        return (p["nz"], p["ny"], p["nx"])

    @property
    def ncells(self):
        p = self.params
        return p["nx"] * p["ny"] * p["nz"]


# --------------------------------------------------------------------------
# primitive -> conserved (ideal gas, R = 1: E = p/(gamma-1) + rho|u|^2/2)
# --------------------------------------------------------------------------
def conserved(rho, u, v, w, p, gamma, tau=None, q=None):
    rho = np.asarray(rho, dtype=np.float64)
    shape = np.broadcast(rho, u, v, w, p).shape
    Q = np.zeros((NCOMP,) + shape)
    Q[0] = rho
    Q[1] = rho * u
    Q[2] = rho * v
    Q[3] = rho * w
    Q[4] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    if tau is not None:
        for j in range(6):
            Q[5 + j] = tau[j]
    if q is not None:
        for j in range(3):
            Q[11 + j] = q[j]
    return Q


def uniform_state(rho, u, p, gamma):
    """14-vector of a uniform state at rest in tau and q, velocity u = (ux, uy, uz)."""
    Q = conserved(np.float64(rho), u[0], u[1], u[2], p, gamma)
    return [float(x) for x in Q]


# --------------------------------------------------------------------------
# characteristic speed of the relaxed system (for the Courant number only)
# --------------------------------------------------------------------------
def _visc_ratio(T, T_ref, law, param):
    """mu(T)/mu0 for the three viscosity laws of the parameter struct."""
    th = T / T_ref
    if law == VISC_SUTHERLAND:
        return (1.0 + param) * th ** 1.5 / (th + param)
    if law == VISC_POWER:
        return th ** param
    return np.ones_like(th)


def _visc_log_slope(T, prm):
    """d ln mu / d ln T of the viscosity law."""
    law = prm["visc_law"]
    if law == VISC_SUTHERLAND:
        th = T / prm["T_ref"]
        return 1.5 - th / (th + prm["visc_param"])
    if law == VISC_POWER:
        return prm["visc_param"] * np.ones_like(T)
    return np.zeros_like(T)


def char_speed(rho, un, p, prm):
    """Largest characteristic speed along one axis of the relaxed system.

    Linearising Eq. (2) about a uniform state (rho, p) with tau = q = 0 and
    velocity un along the axis, the longitudinal subsystem (rho, rho*u_n, E,
    tau_nn, q_n) has speeds un +- s with

        s^4 - s^2 (a + c^2 + (gamma-1) b) + (gamma-1) b (a + p/rho) = 0,
        a = 4 mu_T / (3 rho tau_R),  b = kappa (mu_T/mu0) (1 + m) / (tau_q rho),
        c^2 = gamma p / rho,          kappa = gamma mu0 / ((gamma-1) Pr),
        m = d ln mu_T / d ln T,

    and the shear subsystem (rho*u_t, tau_nt) has un +- sqrt(mu_T/(rho tau_R)).
    The longitudinal root dominates.  Returns |un| + s (array-valued).
    """
    g = prm["gamma"]
    rho = np.asarray(rho, dtype=np.float64)
    T = p / rho
    muT = prm["mu0"] * _visc_ratio(T, prm["T_ref"], prm["visc_law"], prm["visc_param"])
    kappa = g * prm["mu0"] / ((g - 1.0) * prm["prandtl"])
    a = 4.0 * muT / (3.0 * rho * prm["tau_R"])
    # d(K_q T)/dT = K_q (1 + dln mu/dln T)
    b = kappa * (muT / prm["mu0"]) / (prm["tau_q"] * rho) * (1.0 + _visc_log_slope(T, prm))
    c2 = g * p / rho
    B = a + c2 + (g - 1.0) * b
    Cc = (g - 1.0) * b * (a + p / rho)
    s2 = 0.5 * (B + np.sqrt(np.maximum(B * B - 4.0 * Cc, 0.0)))
    return np.abs(un) + np.sqrt(s2)


# --------------------------------------------------------------------------
# random positive states (parity tests)
# --------------------------------------------------------------------------
def random_params(nx, ny, nz, *, sensor=True, seed=0):
    """Parameters for random-state parity cases: dx = 1, dt = 0.1 (lambda = 10)."""
    prm = default_params(nx, ny, nz)
    rng = np.random.default_rng(seed + 7919)
    prm.update(
        dx=1.0, dt=0.1,
        mu0=0.02, tau_R=0.5, tau_q=0.4, prandtl=0.71,
        visc_law=VISC_SUTHERLAND, visc_param=0.4042, T_ref=1.0,
        f_mu=2.0, tau_base_override=0.0,
    )
    if sensor:
        prm.update(C_sigma=30.0, J_min=2e-3, omega_min=1.0 + 0.3 * rng.random())
    prm["Q_ref"] = uniform_state(1.0, (0.0, 0.0, 0.0), 1.0, prm["gamma"])
    return prm


def random_state(nx, ny, nz, seed=0, *, amp=1.0, prm=None):
    """Positive random state: rho, p in [0.6, 1.4], |u| <= 0.3, small tau and q.

    Components are white noise per cell (maximal decorrelation, every cell a
    different sensor decision).  ``amp`` scales the perturbations.
    """
    if prm is None:
        prm = random_params(nx, ny, nz, seed=seed)
    rng = np.random.default_rng(seed)
    sh = (nz, ny, nx)
    rho = 1.0 + amp * 0.4 * (2 * rng.random(sh) - 1)
    p = 1.0 + amp * 0.4 * (2 * rng.random(sh) - 1)
    u, v, w = (amp * 0.3 * (2 * rng.random(sh) - 1) for _ in range(3))
    tau = [amp * 0.01 * (2 * rng.random(sh) - 1) for _ in range(6)]
    q = [amp * 0.01 * (2 * rng.random(sh) - 1) for _ in range(3)]
    return conserved(rho, u, v, w, p, prm["gamma"], tau, q)


def random_case(nx, ny, nz, seed=0, *, sensor=True, steps=20, amp=1.0):
    prm = random_params(nx, ny, nz, sensor=sensor, seed=seed)
    return Case(f"random{nx}x{ny}x{nz}_s{seed}", prm, random_state(nx, ny, nz, seed, amp=amp, prm=prm), steps)


def smooth_random_case(nx, ny, nz, seed=0, *, steps=100, modes=3, amp=0.2, sensor=True):
    """Smooth periodic random field: a few low Fourier modes per primitive."""
    prm = random_params(nx, ny, nz, sensor=sensor, seed=seed)
    rng = np.random.default_rng(seed + 101)
    z, y, x = np.meshgrid(*(2 * np.pi * np.arange(n) / n for n in (nz, ny, nx)), indexing="ij")

    def field():
        f = np.zeros((nz, ny, nx))
        for _ in range(modes):
            kx, ky, kz = rng.integers(0, 3, size=3)
            ph = rng.random(3) * 2 * np.pi
            f += (2 * rng.random() - 1) * np.cos(kx * x + ph[0]) * np.cos(ky * y + ph[1]) * np.cos(kz * z + ph[2])
        return f / modes

    rho = 1.0 + amp * field()
    p = 1.0 + amp * field()
    u, v, w = (amp * field() for _ in range(3))
    Q = conserved(rho, u, v, w, p, prm["gamma"])
    return Case(f"smooth{nx}x{ny}x{nz}_s{seed}", prm, Q, steps)


def tgv_wall_params(n, **kw):
    """The Taylor-Green parameters with no-slip x-walls: still and adiabatic at
    x = 0, isothermal at T_ref and moving at 0.5 along y at x = 2 pi."""
    prm = tgv_params(n, **kw)
    prm.update(bc_x=BC_NOSLIP, wall_u=[[0.0, 0.0, 0.0], [0.0, 0.5, 0.0]], wall_T=[0.0, prm["T_ref"]])
    return prm


def noslip_case(nx, ny, nz, seed=0, *, steps=100, amp=0.2, sensor=True,
                wall_u=((0.0, 0.1, -0.05), (0.0, 0.2, 0.1)), wall_T=(0.0, 1.1)):
    """Smooth random field between no-slip walls at x = 0 and x = nx dx.

    By default the wall at x = 0 is adiabatic and the one at x = nx dx
    isothermal, and both move tangentially, so every term of the wall rule
    is active."""
    c = smooth_random_case(nx, ny, nz, seed, steps=steps, amp=amp, sensor=sensor)
    prm = dict(c.params)
    prm.update(bc_x=BC_NOSLIP, wall_u=[list(map(float, w)) for w in wall_u], wall_T=[float(t) for t in wall_T])
    return Case(f"noslip{nx}x{ny}x{nz}_s{seed}", prm, c.Q0, steps)


def couette_params(n, ny=1, nz=1, *, U=0.02, T_L=1.0, T_R=1.0, mu=0.05, Pr=0.71, gamma=1.4,
                   f_mu=0.05, CFL=0.1):
    """Gas between no-slip isothermal walls at x = 0 (at rest, T_L) and x = 1 (moving
    with U along y, T_R); constant viscosity, dx = 1/n, tau_R = tau_q = 5 dt."""
    prm = default_params(n, ny, nz)
    dx = 1.0 / n
    prm.update(dx=dx, gamma=gamma, mu0=mu, T_ref=1.0, visc_law=VISC_CONST, prandtl=Pr, f_mu=f_mu,
               bc_x=BC_NOSLIP, wall_u=[[0.0, 0.0, 0.0], [0.0, float(U), 0.0]], wall_T=[float(T_L), float(T_R)])
    Tmax = max(T_L, T_R)
    dt = CFL * dx / (np.sqrt(gamma * Tmax) + abs(U))
    for _ in range(200):
        prm["tau_R"] = prm["tau_q"] = 5.0 * dt
        a = float(char_speed(1.0 / Tmax, abs(U), 1.0, prm))
        dt_new = CFL * dx / a
        if abs(dt_new - dt) < 1e-14 * dt:
            dt = dt_new
            break
        dt = 0.5 * (dt + dt_new)
    prm["dt"] = dt
    prm["tau_R"] = prm["tau_q"] = 5.0 * dt
    prm["a_ref"] = CFL * dx / dt
    return prm


# --------------------------------------------------------------------------
# Taylor-Green vortex (Section 3.2 and Eq. (7)); periodic [0, 2 pi)^3
# --------------------------------------------------------------------------
# Background dissipation f_mu of Section 3.2 per grid.  With a temperature-
# dependent viscosity the declared system loses hyperbolicity near local Mach 2,
# and at these values the 64^3, 256^3 and 512^3 runs turn non-finite near
# t_c = 5.7-7.5 (128^3 reaches t_c = 20); with constant viscosity (law="const")
# all of them reach t_c = 20.  The values are kept as the paper states them.
TGV_DEFAULT_FMU = {64: 1.8, 128: 0.9, 256: 1e-2, 384: 1e-2, 512: 1e-2}


def tgv_params(n, *, M0=1.25, Re=1600.0, Pr=0.71, gamma=1.4, law="power", f_mu=None,
               C_sigma=40.0, J_min=1e-2, omega_min=1.987, tau_R=5e-3, tau_q=5e-3,
               CFL=0.1, storage=STORAGE_FP32):
    """Supersonic Taylor-Green vortex parameters, rho0 = U0 = L = 1."""
    prm = default_params(n, n, n)
    U0 = 1.0
    c0 = U0 / M0
    T0 = c0 * c0 / gamma
    if f_mu is None:
        f_mu = TGV_DEFAULT_FMU.get(n, 115.2 / n if n <= 128 else 1e-2)
    if law == "power":
        visc_law, visc_param = VISC_POWER, 0.76
    elif law == "sutherland":
        visc_law, visc_param = VISC_SUTHERLAND, 0.4042
    else:
        visc_law, visc_param = VISC_CONST, 0.0
    prm.update(
        dx=2 * np.pi / n, gamma=gamma, mu0=1.0 / Re, T_ref=T0,
        visc_law=visc_law, visc_param=visc_param, prandtl=Pr,
        tau_R=tau_R, tau_q=tau_q, f_mu=f_mu, tau_base_override=0.0,
        C_sigma=C_sigma, J_min=J_min, omega_min=omega_min, storage=storage,
    )
    a_ref = tgv_a_ref(prm, M0)
    prm["a_ref"] = a_ref
    prm["dt"] = CFL * prm["dx"] / a_ref
    p0 = T0
    prm["Q_ref"] = uniform_state(1.0, (0.0, 0.0, 0.0), p0, gamma)
    return prm


def _tgv_primitives(x, y, z, T0, gamma):
    U0 = rho0 = 1.0
    p0 = rho0 * T0
    u = U0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -U0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = p0 + rho0 * U0 * U0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    rho = p / T0
    return rho, u, v, w, p


def tgv_a_ref(prm, M0, samples=64):
    """max over the initial field and the three axes of |u_n| + s (char_speed)."""
    n = samples
    g = 2 * np.pi * np.arange(n) / n
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    rho, u, v, w, p = _tgv_primitives(x, y, z, prm["T_ref"], prm["gamma"])
    a = max(float(np.max(char_speed(rho, c, p, prm))) for c in (u, v, w))
    return a


def tgv_slab(prm, z0, z1):
    """Conserved initial field of the Taylor-Green vortex for z in [z0, z1)."""
    n = prm["nx"]
    dx = prm["dx"]
    gx = dx * np.arange(n)
    gz = dx * np.arange(z0, z1)
    z, y, x = np.meshgrid(gz, dx * np.arange(prm["ny"]), gx, indexing="ij")
    rho, u, v, w, p = _tgv_primitives(x, y, z, prm["T_ref"], prm["gamma"])
    mu = prm["mu0"]   # uniform T0: mu(T0) = mu0 for every law
    U0 = 1.0
    # Newtonian stress mu (grad u + grad u^T) of the analytic field (div u = 0)
    txx = 2 * mu * U0 * np.cos(x) * np.cos(y) * np.cos(z)
    tyy = -2 * mu * U0 * np.cos(x) * np.cos(y) * np.cos(z)
    tzz = np.zeros_like(txx)
    txy = np.zeros_like(txx)
    txz = -mu * U0 * np.sin(x) * np.cos(y) * np.sin(z)
    tyz = mu * U0 * np.cos(x) * np.sin(y) * np.sin(z)
    zero = np.zeros_like(txx)
    return conserved(rho, u, v, w, p, prm["gamma"], (txx, tyy, tzz, txy, txz, tyz), (zero, zero, zero))


def tgv(n, *, steps=100, materialize=True, **kw):
    prm = tgv_params(n, **kw)
    Q0 = tgv_slab(prm, 0, n) if materialize else None
    M0 = kw.get("M0", 1.25)
    return Case(f"tgv{n}", prm, Q0, steps, meta=dict(M0=M0, t_conv=prm["dt"]))


# --------------------------------------------------------------------------
# Sod shock tube, 256 x 4 x 4, parity walls in x (Section 3.1)
# --------------------------------------------------------------------------
def sod(nx=256, ny=4, nz=4, *, steps=500, CFL=0.35, tau_base=0.55):
    prm = default_params(nx, ny, nz)
    dx = 1.0 / nx
    prm.update(
        dx=dx, gamma=1.4, mu0=1e-6, T_ref=1.0, visc_law=VISC_CONST, prandtl=0.71,
        tau_base_override=tau_base, f_mu=0.0,
        C_sigma=20.0, J_min=3e-3, omega_min=1.0,
        bc_x=BC_WALL,
    )
    prm["a_ref"] = SOD_A_REF
    prm["dt"] = CFL * dx / SOD_A_REF
    prm["tau_R"] = prm["tau_q"] = 5.0 * prm["dt"]
    xc = (np.arange(nx) + 0.5) * dx
    left = xc < 0.5
    rho1 = np.where(left, 1.0, 0.125)
    p1 = np.where(left, 1.0, 0.1)
    sh = (nz, ny, nx)
    rho = np.broadcast_to(rho1, sh).copy()
    p = np.broadcast_to(p1, sh).copy()
    z = np.zeros(sh)
    Q = conserved(rho, z, z, z, p, prm["gamma"])
    prm["Q_ref"] = uniform_state(0.5625, (0.0, 0.0, 0.0), 0.55, prm["gamma"])
    return Case(f"sod{nx}", prm, Q, steps, meta=dict(x=xc))


# --------------------------------------------------------------------------
# Becker stationary viscous shock, Pr = 3/4, constant mu (Section 3.1)
# --------------------------------------------------------------------------
BECKER = dict(gamma=1.4, M=2.0, rho1=1.0, c1=1.0, mu=2e-3, Pr=0.75, L=128.0 / 750.0)


def becker_states(gamma=1.4, M=2.0, rho1=1.0, c1=1.0):
    """Upstream and downstream (rho, u, p) of the Rankine-Hugoniot jump."""
    u1 = M * c1
    p1 = rho1 * c1 * c1 / gamma
    v2 = (gamma - 1.0) / (gamma + 1.0) + 2.0 / ((gamma + 1.0) * M * M)
    m = rho1 * u1
    u2 = v2 * u1
    rho2 = m / u2
    p2 = p1 + m * (u1 - u2)
    return (rho1, u1, p1), (rho2, u2, p2), v2


def becker_profile(x, x_mid, *, gamma=1.4, M=2.0, rho1=1.0, c1=1.0, mu=2e-3, Pr=0.75):
    """Closed-form Becker profile (constant mu, Pr = 3/4): rho, u, p, tau_xx, q_x.

    Total enthalpy is constant through the shock and v = u/u1 obeys
    x - x0 = l/(1-v2) [ln(1-v) - v2 ln(v-v2)],  l = 8 gamma mu / (3 (gamma+1) rho1 u1),
    with x0 placing v = (1+v2)/2 at x_mid.  tau_xx = 4/3 mu u', q_x = -kappa T'.
    """
    (r1, u1, p1), _, v2 = becker_states(gamma, M, rho1, c1)
    ell = 8.0 * gamma * mu / (3.0 * (gamma + 1.0) * r1 * u1)

    def X(v):
        return ell / (1.0 - v2) * (np.log(1.0 - v) - v2 * np.log(v - v2))

    vm = 0.5 * (1.0 + v2)
    x0 = x_mid - X(vm)
    x = np.asarray(x, dtype=np.float64)
    # invert the monotone relation x(v) by bisection on (v2, 1)
    lo = np.full(x.shape, v2 + 1e-15)
    hi = np.full(x.shape, 1.0 - 1e-15)
    target = x - x0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = X(mid) - target          # X decreasing in v
        hi = np.where(f < 0, mid, hi)
        lo = np.where(f < 0, lo, mid)
    v = 0.5 * (lo + hi)
    u = u1 * v
    rho = r1 / v
    H1 = gamma / (gamma - 1.0) * p1 / r1 + 0.5 * u1 * u1
    h = H1 - 0.5 * u * u
    p = rho * (gamma - 1.0) * h / gamma
    dvdx = (v - 1.0) * (v - v2) / (ell * v)
    du = u1 * dvdx
    tau_xx = 4.0 / 3.0 * mu * du
    q_x = mu * u * du / Pr     # -kappa T' with T = (gamma-1)/gamma h, kappa = gamma mu/((gamma-1) Pr)
    return rho, u, p, tau_xx, q_x


def becker(n, ny=4, nz=4, *, steps=1000, CFL=0.125, tau_base=0.0, f_mu=0.0):
    B = BECKER
    L = B["L"]
    prm = default_params(n, ny, nz)
    dx = L / n
    g = B["gamma"]
    prm.update(
        dx=dx, gamma=g, mu0=B["mu"], T_ref=1.0, visc_law=VISC_CONST, prandtl=B["Pr"],
        C_sigma=20.0, J_min=3e-3, omega_min=1.0, bc_x=BC_DIRICHLET,
    )
    # f_mu = 0 (omega_b = 2) by default: the only dissipation beyond the
    # declared mu is the sensor's, which fades under refinement.
    prm["f_mu"] = f_mu
    prm["tau_base_override"] = tau_base
    (r1, u1, p1), (r2, u2, p2), _ = becker_states(g, B["M"], B["rho1"], B["c1"])
    # dt = CFL dx / a_ref with tau_R = tau_q = 5 dt: fixed point in dt
    dt = CFL * dx / (u1 + B["c1"])
    for _ in range(200):
        prm["tau_R"] = prm["tau_q"] = 5.0 * dt
        a = max(float(char_speed(r1, u1, p1, prm)), float(char_speed(r2, u2, p2, prm)))
        dt_new = CFL * dx / a
        if abs(dt_new - dt) < 1e-14 * dt:
            dt = dt_new
            break
        dt = 0.5 * (dt + dt_new)
    prm["dt"] = dt
    prm["tau_R"] = prm["tau_q"] = 5.0 * dt
    prm["a_ref"] = CFL * dx / dt
    xc = (np.arange(n) + 0.5) * dx
    rho, u, p, txx, qx = becker_profile(xc, 0.5 * L, gamma=g, M=B["M"], rho1=B["rho1"], c1=B["c1"],
                                        mu=B["mu"], Pr=B["Pr"])
    sh = (nz, ny, n)
    bc = lambda a: np.broadcast_to(a, sh).copy()
    z = np.zeros(sh)
    Q = conserved(bc(rho), bc(u), z, z, bc(p), g, (bc(txx), z, z, z, z, z), (bc(qx), z, z))
    prm["Q_left"] = uniform_state(r1, (u1, 0.0, 0.0), p1, g)
    prm["Q_right"] = uniform_state(r2, (u2, 0.0, 0.0), p2, g)
    prm["Q_ref"] = uniform_state(0.5 * (r1 + r2), (0.0, 0.0, 0.0), 0.5 * (p1 + p2), g)
    return Case(f"becker{n}", prm, Q, steps, meta=dict(x=xc, L=L))


# --------------------------------------------------------------------------
# Batched Taylor-Green ensemble
# --------------------------------------------------------------------------
BATCH_EDGES = (32, 48, 64, 80, 96)


BATCH_M0_MAX = 1.25


def batch_ensemble(n_inst=64, seed=13437, *, storage=STORAGE_FP16, steps=2000, materialize=True):
    """Uneven Taylor-Green instances: edge from BATCH_EDGES, Mach number from U[0.5, 1.5].

    Draw order: for each instance its edge, then its Mach draw.  The Taylor-
    Green start has a negative pressure minimum p0 - 3/8 rho0 U0^2 above
    M0 = sqrt(8 / (3 gamma)) ~ 1.38, so the draw is mapped linearly onto
    [0.5, BATCH_M0_MAX], the paper's supersonic case being the ceiling.
    f_mu = 115.2 / N interpolates the 64^3 and 128^3 background values of
    Section 3.2.
    """
    rng = np.random.default_rng(seed)
    cases = []
    for j in range(n_inst):
        n = int(rng.choice(BATCH_EDGES))
        draw = float(rng.uniform(0.5, 1.5))
        M0 = 0.5 + (BATCH_M0_MAX - 0.5) * (draw - 0.5)
        prm = tgv_params(n, M0=M0, f_mu=115.2 / n, storage=storage)
        Q0 = tgv_slab(prm, 0, n) if materialize else None
        cases.append(Case(f"batch{j}_tgv{n}_M{M0:.3f}", prm, Q0, steps, meta=dict(M0=M0)))
    return cases
