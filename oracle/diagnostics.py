"""FP64 reference of the volume-averaged diagnostics of Eq. (7).

TEST INFRASTRUCTURE ONLY (see ``oracle.lbm``).

Passages followed: Section 3.2, Eq. (7): kinetic energy E_k, solenoidal
dissipation eps_s = <mu_local |curl u|^2>/rho_ref and dilatational dissipation
eps_d = 4/3 <mu_local (div u)^2>/rho_ref, with curl and divergence evaluated
spectrally on the periodic box and mu_local applied per cell.

Readings: E_k = <rho |u|^2 / 2> / rho_ref (the paper names E_k without a
formula); mu_local follows the viscosity law of the run; the derivative of the
Nyquist mode of an even-length axis is taken as zero.
"""
from __future__ import annotations

import numpy as np

from . import lbm


def spectral_derivative(field, axis, dx):
    """d/dx along ``axis`` of a periodic field by the discrete Fourier transform."""
    n = field.shape[axis]
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=dx)
    if n % 2 == 0:
        k[n // 2] = 0.0
    F = np.fft.fft(field, axis=axis)
    shape = [1] * field.ndim
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * F, axis=axis))


def curl_div(u, dx):
    """(curl u (3, ...), div u) of u (3, nz, ny, nx); array axes are (z, y, x)."""
    ax = {0: 2, 1: 1, 2: 0}   # coordinate a -> array axis
    d = lambda comp, a: spectral_derivative(u[comp], ax[a], dx)
    wx = d(2, 1) - d(1, 2)
    wy = d(0, 2) - d(2, 0)
    wz = d(1, 0) - d(0, 1)
    div = d(0, 0) + d(1, 1) + d(2, 2)
    return np.stack([wx, wy, wz]), div


def diagnostics(Q, prm, rho_ref=1.0):
    """Conservation sums and Eq. (7) averages of a conserved field Q (14, nz, ny, nx)."""
    rho, u, E, p, T = lbm.primitives(Q, prm)
    muT = lbm.viscosity(T, prm)
    w, div = curl_div(u, prm["dx"])
    out = dict(
        mass=float(np.sum(rho)),
        momentum=[float(np.sum(Q[lbm.MX + a])) for a in range(3)],
        energy=float(np.sum(E)),
        E_k=float(np.mean(0.5 * rho * np.sum(u * u, axis=0)) / rho_ref),
        eps_s=float(np.mean(muT * np.sum(w * w, axis=0)) / rho_ref),
        eps_d=float(4.0 / 3.0 * np.mean(muT * div * div) / rho_ref),
        min_rho=float(np.min(rho)),
        min_p=float(np.min(p)),
        any_nonfinite=bool(not np.all(np.isfinite(Q))),
    )
    return out


def sensor_fraction(f, prm):
    """Fraction of cells whose sensor response chi is positive."""
    Q = lbm.moments(f)
    feq = lbm.equilibrium(Q, lbm.flux(Q, prm), prm)
    _, chi = lbm.relaxation_rate(f, feq, Q, prm)
    return float(np.mean(chi > 0.0))
