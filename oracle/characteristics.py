"""Characteristic speeds of the declared system from its flux Jacobian.

TEST INFRASTRUCTURE ONLY (see ``oracle.lbm``).

The Jacobian dPhi_{k,axis}/dQ_j of the Eq. (2) flux is taken by complex-step
differentiation of ``oracle.lbm.flux`` (exact to round-off for this analytic
flux), and its eigenvalues are the characteristic speeds along ``axis``.
"""
from __future__ import annotations

import numpy as np

from . import lbm


def flux_jacobian(Qvec, prm, axis=0, h=1e-30):
    Q0 = np.asarray(Qvec, dtype=np.complex128).reshape(14, 1)
    J = np.zeros((14, 14))
    for j in range(14):
        Q = Q0.copy()
        Q[j, 0] += 1j * h
        J[:, j] = np.imag(lbm.flux(Q, prm)[:, axis, 0]) / h
    return J


def max_speed(Qvec, prm, axis=0):
    return float(np.max(np.abs(np.linalg.eigvals(flux_jacobian(Qvec, prm, axis)))))
