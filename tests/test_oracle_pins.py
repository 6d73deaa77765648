"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it pins.  None of them compares the oracle with
itself: they use closed forms, invariants, an independent transcription of the
declared system, an independent brute-force loop version, exact solutions and
the paper's printed tables.
"""
import json
import os
import warnings

import numpy as np
import pytest
import sympy as sp

import workloads as W
from oracle import brute, characteristics, diagnostics, exact, lbm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
warnings.simplefilter("ignore", RuntimeWarning)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# --------------------------------------------------------------- P1 equilibrium
def test_equilibrium_moments_reproduce_state_and_flux():
    """Section 2.2: zeroth moment Q_k, first moment (times lambda) the flux, second c_s^2 Q_k I."""
    c = W.random_case(5, 4, 3, seed=3)
    prm = c.params
    Q = c.Q0
    Phi = lbm.flux(Q, prm)
    feq = lbm.equilibrium(Q, Phi, prm)
    lam = prm["dx"] / prm["dt"]
    m0 = feq.sum(axis=1)
    assert _rel(m0, Q) < 1e-14
    for a in range(3):
        m1 = lam * np.tensordot(lbm.C[:, a].astype(float), feq, axes=([0], [1]))
        assert _rel(m1, Phi[:, a]) < 1e-13
        for b in range(3):
            cc = (lbm.C[:, a] * lbm.C[:, b]).astype(float)
            m2 = np.tensordot(cc, feq, axes=([0], [1]))
            if a == b:
                assert _rel(m2, 0.25 * Q) < 1e-13
            else:
                assert np.max(np.abs(m2)) < 1e-15


def test_d3q7_weights_are_isotropic_with_cs2_quarter():
    """Section 2.2: D3Q7 with c_s^2 = 1/4 fixes w_0 = 1/4, w_{1..6} = 1/8."""
    assert abs(lbm.W.sum() - 1.0) < 1e-15
    for a in range(3):
        for b in range(3):
            s = np.sum(lbm.W * lbm.C[:, a] * lbm.C[:, b])
            assert abs(s - (0.25 if a == b else 0.0)) < 1e-15


# --------------------------------------------------------------- P2 flux vs the declaration
def _listing_flux_sympy():
    """Flux rows transcribed from the declaration listing (Section 2.1), in its own sign
    convention: the listing writes +tau in the momentum and energy fluxes and +visc*Lambda
    in the stress flux.  Returns a function of numbers."""
    rho, E, g, mu, kap, tR, tq, Tref = sp.symbols("rho E gamma mu kappa tau_R tau_q T_ref", real=True)
    m = sp.Matrix(sp.symbols("m0:3", real=True))
    tl = sp.symbols("tl0:6", real=True)
    qv = sp.Matrix(sp.symbols("q0:3", real=True))
    tauL = sp.Matrix([[tl[0], tl[3], tl[4]], [tl[3], tl[1], tl[5]], [tl[4], tl[5], tl[2]]])
    u = m / rho
    p = (g - 1) * (E - sp.Rational(1, 2) * rho * u.dot(u))
    T = p / rho
    TS = sp.Float(0.4042)
    muT = mu * (1 + TS) * (T / Tref) ** sp.Rational(3, 2) / (T / Tref + TS)
    visc = muT / tR
    heat = kap * (muT / mu) / tq
    I3 = sp.eye(3)
    F = {}
    F["rho"] = m
    F["rhou"] = m * u.T + p * I3 + tauL                          # rows a, columns c
    F["E"] = (E + p) * u + tauL * u + qv
    # Lambda: the velocity tensor whose divergence is the deviatoric strain rate
    lam3 = lambda a, b, c: (u[a] if b == c else 0) + (u[b] if a == c else 0) - (sp.Rational(2, 3) * u[c] if a == b else 0)
    F["tau"] = {(a, b, c): tauL[a, b] * u[c] + visc * lam3(a, b, c) for a in range(3) for b in range(3) for c in range(3)}
    F["q"] = qv * u.T + heat * T * I3
    syms = (rho, E, g, mu, kap, tR, tq, Tref) + tuple(m) + tl + tuple(qv)
    return syms, F


def test_flux_matches_declaration_listing():
    """Eq. (2) vs the listing: same system with tau_listing = -tau (P2)."""
    syms, F = _listing_flux_sympy()
    rng = np.random.default_rng(11)
    prm = W.default_params(1, 1, 1)
    prm.update(visc_law=W.VISC_SUTHERLAND, visc_param=0.4042, T_ref=0.8, mu0=0.03, prandtl=0.71,
               tau_R=0.3, tau_q=0.2, gamma=1.4)
    kap = lbm.kappa(prm)
    for trial in range(4):
        Q = W.random_state(1, 1, 1, seed=100 + trial)[:, 0, 0, 0]
        Phi = lbm.flux(Q.reshape(14, 1), prm)[:, :, 0]
        tau = Q[5:11]
        vals = dict(zip(syms, [Q[0], Q[4], prm["gamma"], prm["mu0"], kap, prm["tau_R"], prm["tau_q"], prm["T_ref"],
                               Q[1], Q[2], Q[3], *(-tau), Q[11], Q[12], Q[13]]))
        ev = lambda e: float(sp.N(e.subs(vals)))
        for c in range(3):
            assert abs(ev(F["rho"][c]) - Phi[0, c]) < 1e-13
            for a in range(3):
                assert abs(ev(F["rhou"][a, c]) - Phi[1 + a, c]) < 1e-12
                assert abs(ev(F["q"][a, c]) - Phi[11 + a, c]) < 1e-12
            assert abs(ev(F["E"][c]) - Phi[4, c]) < 1e-12
            for (a, b) in lbm.TAU_PAIRS:
                # tau = -tau_listing, so its flux is minus the listing's
                assert abs(-ev(F["tau"][(a, b, c)]) - Phi[lbm.TAU[(a, b)], c]) < 1e-12


def test_lambda_divergence_is_deviatoric_strain_rate():
    """Section 2.1: div of the stress flux at tau = 0, uniform T, is -(mu/tau_R)(grad u + grad u^T - 2/3 div u I)."""
    n = 16
    prm = W.default_params(n, n, n)
    prm.update(dx=2 * np.pi / n, visc_law=W.VISC_CONST, mu0=0.05, tau_R=0.25)
    g = prm["dx"] * np.arange(n)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    u = np.stack([np.sin(x) * np.cos(2 * y), 0.3 * np.cos(z) * np.sin(x), np.sin(y + z)])
    rho = np.ones_like(x)
    # uniform T: p = rho
    Q = W.conserved(rho, u[0], u[1], u[2], rho, prm["gamma"])
    Phi = lbm.flux(Q, prm)
    ax = {0: 2, 1: 1, 2: 0}
    d = lambda f, a: diagnostics.spectral_derivative(f, ax[a], prm["dx"])
    div_u = sum(d(u[a], a) for a in range(3))
    nu = prm["mu0"] / prm["tau_R"]
    for (a, b) in lbm.TAU_PAIRS:
        k = lbm.TAU[(a, b)]
        divPhi = sum(d(Phi[k, c], c) for c in range(3))
        target = -nu * (d(u[a], b) + d(u[b], a) - (2.0 / 3.0) * (a == b) * div_u)
        assert np.max(np.abs(divPhi - target)) < 1e-12


# --------------------------------------------------------------- P3 conservation
def test_conservation_and_exact_relaxation_decay():
    """Section 2.2 + Eq. (2) sources: rho, rho u, E conserved; sum tau, sum q decay by (1 - dt/tau)^n."""
    c = W.random_case(6, 5, 4, seed=5, sensor=True)
    prm = c.params
    f = lbm.init_populations(c.Q0, prm)
    Q0 = lbm.moments(f)
    n = 40
    fired = 0
    for _ in range(n):
        Q = lbm.moments(f)
        feq = lbm.equilibrium(Q, lbm.flux(Q, prm), prm)
        fired += int(np.sum(lbm.relaxation_rate(f, feq, Q, prm)[1] > 0))
        f = lbm.step(f, prm)
    Q = lbm.moments(f)
    assert fired > 0, "sensor never active"
    for k in range(5):
        s0, s1 = Q0[k].sum(), Q[k].sum()
        assert abs(s1 - s0) <= 1e-13 * max(abs(s0), np.abs(Q0[k]).sum())
    for k in range(5, 11):
        assert abs(Q[k].sum() - (1 - prm["dt"] / prm["tau_R"]) ** n * Q0[k].sum()) < 1e-13
    for k in range(11, 14):
        assert abs(Q[k].sum() - (1 - prm["dt"] / prm["tau_q"]) ** n * Q0[k].sum()) < 1e-13


# --------------------------------------------------------------- P4 fixed points
def test_uniform_moving_state_is_fixed_point():
    prm = W.random_params(4, 3, 5, sensor=True)
    Qv = W.uniform_state(0.9, (0.2, -0.1, 0.05), 1.1, prm["gamma"])
    Q = np.broadcast_to(np.array(Qv).reshape(14, 1, 1, 1), (14, 5, 3, 4)).copy()
    f = lbm.run(Q, prm, 10)
    assert _rel(lbm.moments(f), Q) < 1e-14


def test_gas_at_rest_between_parity_walls_is_fixed_point():
    prm = W.random_params(6, 2, 2, sensor=True)
    prm["bc_x"] = W.BC_WALL
    Qv = W.uniform_state(1.3, (0.0, 0.0, 0.0), 0.7, prm["gamma"])
    Q = np.broadcast_to(np.array(Qv).reshape(14, 1, 1, 1), (14, 2, 2, 6)).copy()
    f = lbm.run(Q, prm, 10)
    assert _rel(lbm.moments(f), Q) < 1e-14


def test_uniform_flow_through_equilibrium_ends_is_fixed_point():
    prm = W.random_params(6, 2, 2, sensor=True)
    prm["bc_x"] = W.BC_DIRICHLET
    Qv = W.uniform_state(1.1, (0.3, 0.0, 0.0), 0.9, prm["gamma"])
    prm["Q_left"] = prm["Q_right"] = Qv
    Q = np.broadcast_to(np.array(Qv).reshape(14, 1, 1, 1), (14, 2, 2, 6)).copy()
    f = lbm.run(Q, prm, 10)
    assert _rel(lbm.moments(f), Q) < 1e-14


# --------------------------------------------------------------- P5 symmetry
# relabelling of components and populations under x <-> y, and under x -> -x
SWAP_XY_COMP = [0, 2, 1, 3, 4, 6, 5, 7, 8, 10, 9, 12, 11, 13]
SWAP_XY_POP = [0, 3, 4, 1, 2, 5, 6]
REFL_X_POP = [0, 2, 1, 3, 4, 5, 6]


def test_axis_permutation_commutes_with_step():
    c = W.random_case(4, 4, 3, seed=8, sensor=True)
    prm = c.params
    f = lbm.init_populations(c.Q0, prm)
    for _ in range(3):
        f = lbm.step(f, prm)
    T = lambda g: np.swapaxes(g[SWAP_XY_COMP][:, SWAP_XY_POP], 3, 4)
    a = lbm.step(T(f), prm)
    b = T(lbm.step(f, prm))
    assert _rel(a, b) < 1e-14


def test_reflection_commutes_with_step():
    c = W.random_case(5, 3, 4, seed=9, sensor=True)
    prm = c.params
    f = lbm.init_populations(c.Q0, prm)
    for _ in range(2):
        f = lbm.step(f, prm)
    sig = lbm.SIGMA_X.reshape(14, 1, 1, 1, 1)
    # a reflected periodic lattice: x -> (-x) mod nx
    R = lambda g: sig * np.roll(g[:, REFL_X_POP][..., ::-1], 1, axis=4)
    a = lbm.step(R(f), prm)
    b = R(lbm.step(f, prm))
    assert _rel(a, b) < 1e-14


# --------------------------------------------------------------- P6 brute force
@pytest.mark.parametrize("sensor", [True, False])
def test_brute_force_4cubed_periodic(sensor):
    c = W.random_case(4, 4, 4, seed=21, sensor=sensor)
    n = 12
    fa = lbm.run(c.Q0, c.params, n)
    fb = brute.run(c.Q0, c.params, n)
    assert _rel(fa, fb) < 1e-12


@pytest.mark.parametrize("bc,wall_T", [(W.BC_WALL, None), (W.BC_DIRICHLET, None),
                                       (W.BC_NOSLIP, [0.0, 1.1]), (W.BC_NOSLIP, [1.2, 0.0])])
def test_brute_force_x_boundaries(bc, wall_T):
    """The vectorised oracle against the loop transcription; for no-slip walls the
    loop version writes each component's wall term out by hand, the vectorised
    one evaluates the declared flux at the wall state."""
    c = W.random_case(5, 3, 2, seed=22, sensor=True)
    prm = dict(c.params)
    prm["bc_x"] = bc
    prm["Q_left"] = W.uniform_state(1.2, (0.3, 0.0, 0.0), 1.1, prm["gamma"])
    prm["Q_right"] = W.uniform_state(0.8, (0.2, 0.1, 0.0), 0.9, prm["gamma"])
    prm["wall_u"] = [[0.0, 0.1, -0.2], [0.0, 0.05, 0.3]]
    prm["wall_T"] = wall_T or [0.0, 0.0]
    n = 10
    fa = lbm.run(c.Q0, prm, n)
    fb = brute.run(c.Q0, prm, n)
    assert _rel(fa, fb) < 1e-12


def test_wall_equals_mirrored_periodic_domain():
    """Parity walls: the wall-bounded run equals the mirror-doubled periodic run."""
    c = W.random_case(6, 3, 2, seed=23, sensor=True)
    prm = dict(c.params)
    prm["bc_x"] = W.BC_WALL
    sig = lbm.SIGMA_X.reshape(14, 1, 1, 1)
    Qd = np.concatenate([c.Q0, sig * c.Q0[..., ::-1]], axis=3)
    prd = dict(prm)
    prd["bc_x"] = W.BC_PERIODIC
    prd["nx"] = 12
    n = 15
    fa = lbm.moments(lbm.run(c.Q0, prm, n))
    fb = lbm.moments(lbm.run(Qd, prd, n))
    assert _rel(fa, fb[..., :6]) < 1e-13


# Point inversion x -> -x (1D data): vectors (rho u, q) change sign, scalars and
# the stress tensor do not.
PARITY_P = np.array([1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, -1, -1, -1], dtype=np.float64)


def test_noslip_still_adiabatic_wall_equals_inverted_doubled_domain():
    """A still, adiabatic no-slip wall: velocity and normal heat flux vanish at the
    wall, the mirror image of a point inversion.  On y,z-uniform data the wall
    run equals the periodic run of the domain doubled with its inverted image."""
    c = W.smooth_random_case(7, 1, 1, seed=31, sensor=True, amp=0.3)
    prm = dict(c.params)
    prm.update(bc_x=W.BC_NOSLIP, wall_u=[[0.0] * 3, [0.0] * 3], wall_T=[0.0, 0.0])
    Qd = np.concatenate([c.Q0, PARITY_P.reshape(14, 1, 1, 1) * c.Q0[..., ::-1]], axis=3)
    prd = dict(prm, bc_x=W.BC_PERIODIC, nx=14)
    n = 25
    fa = lbm.moments(lbm.run(c.Q0, prm, n))
    fb = lbm.moments(lbm.run(Qd, prd, n))
    assert _rel(fa, fb[..., :7]) < 1e-13


@pytest.mark.parametrize("wall_T", [(1.3, 1.3), (0.0, 0.0), (1.3, 0.0)])
def test_gas_at_rest_between_still_noslip_walls_is_fixed_point(wall_T):
    prm = W.random_params(6, 2, 2, sensor=True)
    prm.update(bc_x=W.BC_NOSLIP, wall_u=[[0.0] * 3, [0.0] * 3], wall_T=list(wall_T))
    Qv = W.uniform_state(0.9, (0.0, 0.0, 0.0), 0.9 * 1.3, prm["gamma"])   # T = 1.3
    Q = np.broadcast_to(np.array(Qv).reshape(14, 1, 1, 1), (14, 2, 2, 6)).copy()
    f = lbm.run(Q, prm, 10)
    assert _rel(lbm.moments(f), Q) < 1e-14


@pytest.mark.parametrize("wall_T", [(0.8, 0.8), (0.0, 0.8)])
def test_flow_moving_with_noslip_walls_is_fixed_point(wall_T):
    """Gas moving with both walls (the walls' velocity, the isothermal wall's
    temperature): the returning links carry the flow's own fluxes."""
    prm = W.random_params(6, 2, 2, sensor=True)
    uw = [0.0, 0.25, -0.15]
    prm.update(bc_x=W.BC_NOSLIP, wall_u=[uw, uw], wall_T=list(wall_T))
    Qv = W.uniform_state(1.25, tuple(uw), 1.25 * 0.8, prm["gamma"])          # T = 0.8
    Q = np.broadcast_to(np.array(Qv).reshape(14, 1, 1, 1), (14, 2, 2, 6)).copy()
    f = lbm.run(Q, prm, 10)
    assert _rel(lbm.moments(f), Q) < 1e-14


def test_low_mach_couette_flow_is_linear():
    """Steady Couette flow between a still and a moving isothermal wall: u_y = U x/H
    and tau_xy = mu U/H (closed form of the steady relaxed system with constant
    viscosity); at U = 0.02 the viscous heating changes rho by ~1e-5.  Mass is
    conserved to round-off."""
    n, U = 8, 0.02
    prm = W.couette_params(n, U=U, f_mu=0.01)
    x = (np.arange(n) + 0.5) / n
    sh = (1, 1, n)
    one, zero = np.ones(sh), np.zeros(sh)
    Q = W.conserved(one, zero, (U * x).reshape(sh), zero, one, prm["gamma"])
    f = lbm.run(Q, prm, int(round(4.0 / prm["dt"])))
    Qn = lbm.moments(f)
    rho, u, E, p, T = lbm.primitives(Qn, prm)
    assert np.abs(u[1, 0, 0] - U * x).max() < 1e-6 * U
    assert np.abs(Qn[lbm.TXY] / (prm["mu0"] * U) - 1.0).max() < 1e-5
    assert abs(Qn[0].sum() / Q[0].sum() - 1.0) < 1e-14


def test_steady_conduction_between_isothermal_walls_converges_second_order():
    """Gas at rest between walls at T = 1 and 1.2: the steady state has uniform p,
    q_x = -kappa dT/dx and T linear between the wall temperatures.  The error
    of the lattice solution falls by more than 3x per halving of dx."""
    err = []
    for n in (8, 16):
        prm = W.couette_params(n, U=0.0, T_L=1.0, T_R=1.2, f_mu=0.01)
        x = (np.arange(n) + 0.5) / n
        T_exact = 1.0 + 0.2 * x
        sh = (1, 1, n)
        zero = np.zeros(sh)
        Q = W.conserved((1.0 / T_exact).reshape(sh), zero, zero, zero, np.ones(sh), prm["gamma"])
        Qn = lbm.moments(lbm.run(Q, prm, int(round(6.0 / prm["dt"]))))
        T = lbm.primitives(Qn, prm)[4][0, 0]
        err.append(np.abs(T - T_exact).max())
    assert err[1] < 1e-3 and err[0] / err[1] > 3.0, err


def test_yz_uniform_data_equals_1d_run():
    c = W.sod(64, 3, 2, steps=0)
    c1 = W.sod(64, 1, 1, steps=0)
    fa = lbm.run(c.Q0, c.params, 30)
    fb = lbm.run(c1.Q0, c1.params, 30)
    assert np.array_equal(fa[..., 0:1, 0:1, :], fb)


# --------------------------------------------------------------- P7 sensor
def test_sensor_off_is_plain_bgk_rate():
    c = W.random_case(4, 3, 3, seed=4, sensor=False)
    prm = c.params
    f = lbm.init_populations(c.Q0, prm)
    f = lbm.step(f, prm)
    Q = lbm.moments(f)
    feq = lbm.equilibrium(Q, lbm.flux(Q, prm), prm)
    om, chi = lbm.relaxation_rate(f, feq, Q, prm)
    rho, u, E, p, T = lbm.primitives(Q, prm)
    mu = lbm.viscosity(T, prm)
    tb = 0.5 + 4 * prm["f_mu"] * mu / rho * prm["dt"] / prm["dx"] ** 2      # Eq. (6)
    assert np.all(chi == 0) and _rel(om, 1.0 / tb) < 1e-15


@pytest.mark.parametrize("tau_b", [0.7, 1.0])
def test_dilatation_estimate_matches_spectral_divergence(tau_b):
    """Section 2.3: the local recovery equals dt * div u of the macroscopic field (1D compression wave)."""
    n = 256
    prm = W.tgv_params(n)
    prm.update(ny=1, nz=1, tau_base_override=tau_b)
    x = prm["dx"] * np.arange(n)
    rho = np.ones((1, 1, n))
    u = 0.3 * np.sin(x)[None, None, :]
    z = np.zeros_like(rho)
    txx = (4 / 3) * prm["mu0"] * 0.3 * np.cos(x)[None, None, :]
    Q = W.conserved(rho, u, z, z, prm["T_ref"] * rho, prm["gamma"], (txx, -txx / 2, -txx / 2, z, z, z))
    f = lbm.run(Q, prm, 40)
    Q = lbm.moments(f)
    feq = lbm.equilibrium(Q, lbm.flux(Q, prm), prm)
    th = lbm.dilatation(f, feq, Q, prm)[0, 0]
    _, uu, _, _, _ = lbm.primitives(Q, prm)
    div = diagnostics.spectral_derivative(uu[0], 2, prm["dx"])[0, 0] * prm["dt"]
    assert np.max(np.abs(th - div)) < 0.01 * np.max(np.abs(div))
    # Eq. (3)-(4): s = max(0, -theta)/c_s and the clamp at 1/C_sigma
    prm2 = dict(prm, C_sigma=40.0, J_min=1e-4, omega_min=1.0)
    om, chi = lbm.relaxation_rate(f, feq, Q, prm2)
    s = np.maximum(0, -th) / 0.5
    expect = np.where(s > 1e-4, np.minimum(1, 40 * s), 0)
    assert np.array_equal(chi[0, 0], expect)


# --------------------------------------------------------------- P8 spectral diagnostics
def test_spectral_derivative_exact_for_trig():
    n = 24
    dx = 2 * np.pi / n
    x = dx * np.arange(n)
    f = np.sin(3 * x) + 0.5 * np.cos(7 * x)
    d = diagnostics.spectral_derivative(f, 0, dx)
    assert np.max(np.abs(d - (3 * np.cos(3 * x) - 3.5 * np.sin(7 * x)))) < 1e-13


def test_tgv_initial_diagnostics_closed_form():
    """Eq. (7) at t = 0: E_k = rho0 U0^2 / 8, eps_s = 3/4 mu0 U0^2, eps_d = 0 (solenoidal start)."""
    c = W.tgv(32)
    d = diagnostics.diagnostics(c.Q0, c.params)
    assert abs(d["E_k"] - 0.125) < 1e-14
    assert abs(d["eps_s"] - 0.75 * c.params["mu0"]) < 1e-15
    assert d["eps_d"] < 1e-28


def _field_state(n, u, v, w, rho=None, p=1.0):
    """Conserved state of a given velocity field on an n^3 periodic box (rho = 1, p = 1 by default)."""
    prm = W.default_params(n, n, n)
    rho = np.ones((n, n, n)) if rho is None else rho
    return W.conserved(rho, u, v, w, p * np.ones((n, n, n)), prm["gamma"]), prm


def test_shell_spectrum_single_modes_closed_form():
    """Section 3.2 spectra: a cosine mode of amplitude A and integer wavevector kappa
    puts A^2/4 (= <u^2>/2) in shell nint(|kappa|) and nothing elsewhere."""
    n = 12
    x = 2 * np.pi * np.arange(n) / n
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")
    zero = np.zeros((n, n, n))
    for (kx, ky, kz), shell in (((0, 3, 0), 3), ((1, 1, 0), 1), ((1, 1, 1), 2), ((2, 2, 1), 3), ((0, 0, 5), 5)):
        A = 0.3
        u = A * np.cos(kx * xx + ky * y + kz * z)
        Q, prm = _field_state(n, u, zero, zero)
        E = diagnostics.shell_spectrum(Q, prm)
        want = np.zeros_like(E)
        want[shell] = A * A / 4
        assert np.max(np.abs(E - want)) < 1e-15, (kx, ky, kz)


def test_shell_spectrum_tgv_start_and_parseval():
    """The Taylor-Green start has all its energy, <|u|^2>/2 = 1/8, at |kappa| = sqrt(3)
    (shell 2); on a random state the shells sum to <|u|^2>/2 computed in physical space."""
    c = W.tgv(16)
    E = diagnostics.shell_spectrum(c.Q0, c.params)
    assert len(E) == 1 + int(np.floor(np.sqrt(3) * 8 + 0.5))
    assert abs(E[2] - 0.125) < 1e-15 and np.sum(np.abs(E)) - E[2] < 1e-15
    rng = np.random.default_rng(3)
    n = 10
    u, v, w = (rng.normal(size=(n, n, n)) for _ in range(3))
    rho = 1.0 + 0.2 * rng.random((n, n, n))
    Q, prm = _field_state(n, u, v, w, rho=rho)
    E = diagnostics.shell_spectrum(Q, prm)
    assert abs(E.sum() - 0.5 * np.mean(u * u + v * v + w * w)) < 1e-13 * E.sum()
    assert np.all(E >= 0.0)


# --------------------------------------------------------------- P9 Sod
def test_exact_riemann_star_state_matches_textbook():
    g = json.load(open(os.path.join(GOLDEN, "sod_star_textbook.json")))
    st = exact.sod_star_states()
    for k in ("p_star", "u_star", "rho_star_L", "rho_star_R"):
        assert abs(st[k] - g[k]) < 0.6e-5
    assert abs(W.SOD_A_REF - st["a_max"]) < 1e-6


def test_sod_shock_thickness_and_l1_against_exact():
    """Section 3.1: captured Sod shock about 4.8 cells wide, w proportional to dx; L1(rho) as Table sod_conv."""
    tab = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))
    st = exact.sod_star_states()
    widths = {}
    for N in (375, 750):
        c = W.sod(N, 1, 1, tau_base=0.6)
        prm = c.params
        nst = int(round(0.2 / prm["dt"]))
        f = lbm.run(c.Q0, prm, nst)
        rho, u, E, p, T = lbm.primitives(lbm.moments(f), prm)
        t = nst * prm["dt"]
        x = c.meta["x"]
        re, _, _ = exact.sod_exact(x, t)
        xs = 0.5 + st["shock_speed"] * t
        sel = (x > xs - 0.04) & (x < xs + 0.04)
        widths[N] = exact.thickness(x[sel], rho[0, 0][sel], lo=0.125, hi=st["rho_star_R"]) / prm["dx"]
        if N == 750:
            L1 = exact.norms(rho[0, 0], re, prm["dx"])["L1"]
            assert L1 < 1.5 * tab["sod_L1_rho"]["750"]
    for N, w in widths.items():
        assert 3.5 < w < 6.5, widths
    assert abs(widths[375] - widths[750]) < 1.0     # fixed cell count: w ~ dx


def test_sod_bench_config_is_stable():
    c = W.sod(256, 1, 1)
    f = lbm.run(c.Q0, c.params, 500)
    Q = lbm.moments(f)
    rho, u, E, p, T = lbm.primitives(Q, c.params)
    assert np.all(np.isfinite(Q)) and rho.min() > 0.05 and p.min() > 0.0


# --------------------------------------------------------------- P10 Becker
def test_becker_closed_form_two_transcriptions_agree():
    L = W.BECKER["L"]
    x = np.linspace(0, L, 301)
    r1, u1, p1, _, _ = W.becker_profile(x, L / 2)
    r2, u2, p2 = exact.becker_exact(x, L / 2)
    assert np.max(np.abs(r1 - r2)) < 1e-9 and np.max(np.abs(p1 - p2)) < 1e-9
    # mass and momentum balance of the closed form (shock frame)
    (ra, ua, pa), (rb, ub, pb), _ = W.becker_states()
    assert abs(ra * ua - rb * ub) < 1e-14 and abs(ra * ua * ua + pa - rb * ub * ub - pb) < 1e-14


def test_becker_shock_converges_toward_closed_form():
    """Section 3.1: N = 128 holds a steady viscous shock near the Becker width."""
    wex = exact.becker_width()
    c = W.becker(128, 1, 1)
    prm = c.params
    f = lbm.run(c.Q0, prm, 6000)
    rho, u, E, p, T = lbm.primitives(lbm.moments(f), prm)
    w = exact.thickness(c.meta["x"], rho[0, 0], lo=1.0, hi=8.0 / 3.0)
    assert np.all(np.isfinite(rho))
    assert 0.0 < w / wex - 1.0 < 1.0
    # mass flux rho1 u1 = 2 carried through; the equilibrium ends hold it to a thin
    # boundary layer (they inject populations without a non-equilibrium part)
    mf = rho[0, 0] * u[0][0, 0]
    assert abs(mf[0] - 2.0) < 1e-2 and abs(mf[-1] - 2.0) < 1e-2
    assert abs(np.median(mf) - 2.0) < 2e-3


# --------------------------------------------------------------- P11 Eq. (6)
@pytest.mark.parametrize("tau_b", [0.6, 0.8, 1.2])
def test_entropy_mode_diffuses_at_lattice_rate(tau_b):
    """Eq. (6): the rate adds nu_num = c_s^2 (tau - 1/2) dx^2/dt; a passive entropy mode decays at it."""
    n = 64
    prm = W.default_params(n, 1, 1)
    prm.update(dx=1.0, dt=0.1, mu0=1e-12, tau_R=0.5, tau_q=0.5, tau_base_override=tau_b)
    x = np.arange(n)
    k = 2 * np.pi / n
    rho = 1 + 1e-4 * np.cos(k * x)[None, None, :]
    z = np.zeros_like(rho)
    f = lbm.run(W.conserved(rho, z, z, z, np.ones_like(rho), prm["gamma"]), prm, 50)
    a0 = np.abs(np.fft.rfft(lbm.moments(f)[0, 0, 0] - 1))[1]
    N = 300
    for _ in range(N):
        f = lbm.step(f, prm)
    a1 = np.abs(np.fft.rfft(lbm.moments(f)[0, 0, 0] - 1))[1]
    rate = -np.log(a1 / a0) / (N * prm["dt"])
    D = 0.25 * (tau_b - 0.5) * prm["dx"] ** 2 / prm["dt"]
    assert abs(rate / (D * k * k) - 1) < 0.01


def test_fmu_numerical_viscosity_is_fmu_mu_over_rho():
    """Eq. (6): tau_base with f_mu gives c_s^2 (tau - 1/2) dx^2/dt = f_mu mu/rho exactly."""
    prm = W.tgv_params(16)
    Q = W.tgv_slab(prm, 0, 16)
    tb = lbm.tau_base(Q, prm)
    rho, u, E, p, T = lbm.primitives(Q, prm)
    nu_num = 0.25 * (tb - 0.5) * prm["dx"] ** 2 / prm["dt"]
    assert _rel(nu_num, prm["f_mu"] * lbm.viscosity(T, prm) / rho) < 1e-13


# --------------------------------------------------------------- characteristic speeds (Courant number)
@pytest.mark.parametrize("law", ["const", "power", "sutherland"])
def test_closed_form_wave_speed_matches_flux_jacobian(law):
    prm = W.tgv_params(64, law=law)
    for (rho, un, p) in [(1.0, 0.0, 0.457), (0.18, 0.0, 0.082), (1.2, 0.7, 0.5), (0.5, -0.3, 0.2)]:
        Qv = W.uniform_state(rho, (un, 0.0, 0.0), p, prm["gamma"])
        num = characteristics.max_speed(Qv, prm, 0)
        cf = float(W.char_speed(rho, un, p, prm))
        tol = 1e-10 if (un == 0.0 or law == "const") else 0.03 * num
        assert abs(num - cf) < tol


def test_domain_of_dependence_crop_is_exact():
    """After n steps a cell depends only on the initial cube of half-width n: a periodic
    crop of half-width h + n reproduces the full run on its central (2h)^3 cells."""
    N, n, h = 32, 5, 3
    case = W.tgv(N)
    prm = case.params
    full = lbm.moments(lbm.run(case.Q0, prm, n))
    zc, yc, xc = 7, 30, 16
    H = h + n
    idx = lambda c: np.arange(c - H, c + H) % N
    crop = case.Q0[:, idx(zc)][:, :, idx(yc)][:, :, :, idx(xc)]
    out = lbm.moments(lbm.run(crop, dict(prm, nx=2 * H, ny=2 * H, nz=2 * H), n))
    a = out[:, n:n + 2 * h, n:n + 2 * h, n:n + 2 * h]
    b = full[:, idx(zc)[n:n + 2 * h]][:, :, idx(yc)[n:n + 2 * h]][:, :, :, idx(xc)[n:n + 2 * h]]
    assert np.array_equal(a, b)
