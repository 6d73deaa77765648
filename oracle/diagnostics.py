"""FP64 reference of the volume-averaged diagnostics of Eq. (7).

TEST INFRASTRUCTURE ONLY (see ``oracle.lbm``).

Passages followed: Section 3.2, Eq. (7): kinetic energy E_k, solenoidal
dissipation eps_s = <mu_local |curl u|^2>/rho_ref and dilatational dissipation
eps_d = 4/3 <mu_local (div u)^2>/rho_ref, with curl and divergence evaluated
spectrally on the periodic box and mu_local applied per cell.

Readings: E_k = <rho |u|^2 / 2> / rho_ref (the paper names E_k without a
formula); mu_local follows the viscosity law of the run; the derivative of the
Nyquist mode of an even-length axis is taken as zero.

Shell spectrum (Section 3.2, the velocity spectra of the Taylor-Green run):
shell-averaged, normalised so that its sum is <|u|^2>/2.  Readings: u is the
velocity rho u / rho (not density-weighted); wavenumbers are the integers of
the discrete Fourier transform on the cubic periodic box; a mode belongs to
shell k = nint(|kappa|) (never a tie: |kappa|^2 is an integer and (k + 1/2)^2
is not); every mode is counted, corners beyond N/2 included, so the sum is
exact by Parseval's identity.
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


def spectrum_shells(n):
    """Number of shells of an n^3 box: 1 + nint(sqrt(3) * (n // 2))."""
    m = n // 2
    return int(np.floor(np.sqrt(3.0 * m * m) + 0.5)) + 1


def shell_spectrum(Q, prm):
    """E(k) = 1/2 sum over modes with nint(|kappa|) = k of sum_c |u_hat_c(kappa)|^2,
    u_hat = (1/N^3) DFT of the velocity, on a cubic periodic box."""
    _, u, _, _, _ = lbm.primitives(Q, prm)
    nz, ny, nx = u.shape[1:]
    assert nx == ny == nz, "the shell spectrum is defined on a cubic box"
    n = nx
    m = np.fft.fftfreq(n, d=1.0 / n)
    k2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    shell = np.floor(np.sqrt(k2) + 0.5).astype(np.int64)
    e = sum(np.abs(np.fft.fftn(u[c])) ** 2 for c in range(3)) / float(n) ** 6 / 2.0
    return np.bincount(shell.ravel(), weights=e.ravel(), minlength=spectrum_shells(n))
