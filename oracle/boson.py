"""Bosonic action and the full phonon log-weight (oracle; test infrastructure only).

Paper, SM Eq. (S2): the weight of a phonon configuration is
e^{-dtau S_Bose} det M_up det M_dn, with
S_Bose = Omega^2/2 sum X^2 + sum ((X_{l+1} - X_l)/dtau)^2, time periodic.

Readings:
  A1  build frame x = X - alpha with alpha = -lam/omega0^2: completing the square moves a
      linear term -lam*x into S_Bose (per site and slice; the constant is dropped) and the
      fermion chemical potential to 0 at half filling;
  A10 the kinetic prefactor c_kin multiplies sum ((x_{l+1}-x_l)/dtau)^2; the standard
      path-integral value for M = 1 is 1/2, the paper-literal value is 1 -- both sides
      take it as a parameter;
  A11 the bosonic factor is exp(-dtau * S_Bose) as printed.
"""

import numpy as np


def bosonic_action(x, lam, omega0, dtau, c_kin):
    """S_Bose in the build frame for x[Ltau, N] (time periodic)."""
    x = np.asarray(x, dtype=np.float64)
    pot = 0.5 * omega0 ** 2 * np.sum(x * x) - lam * np.sum(x)
    dx = np.roll(x, -1, axis=0) - x
    kin = c_kin * np.sum(dx * dx) / (dtau * dtau)
    return float(pot + kin)


def log_weight(logdet, x, lam, omega0, dtau, c_kin):
    """log w = -dtau S_Bose + 2 log|det M| (two identical spin determinants)."""
    return -dtau * bosonic_action(x, lam, omega0, dtau, c_kin) + 2.0 * logdet
