"""Training the effective model by multi-linear regression (oracle; test infrastructure
only).

Paper, main text ("the effective model is trained ...", Eq. 5) and SM Sec. III: the
coefficients of the effective model are obtained by a multi-linear regression of
-beta H_eff[X] onto ln w[X] over Monte Carlo configurations of the original model
(Table S1 lists one result).

Readings (listed in the design notes):
  A12 (as elsewhere) E_eff = +beta H_eff with weight exp(-E_eff).
  A39 regression.  Every term of E_eff is linear in its coefficient: E_eff(x) =
      sum_t J_t F_t(x) with the features F = (sum (x_{l+1}-x_l)^2, sum x^2, sum f4, sum f6,
      sum over bonds of each spatial range of x_i x_j, sum x_{i,l} x_{i,l+1}) in the order
      (Jk, J2, Jp, Jp6, Js0, Js1, Js2, Jt).  The fit is ordinary least squares of
      ln w(x) = E0 - sum_{t in mask} J_t F_t(x) over the configurations, the constant E0
      (the normalisation) included; terms outside the mask are zero.  Sum x^2, the time-
      kinetic sum and the temporal products are linearly dependent (sum (x_{l+1}-x_l)^2 =
      2 sum x^2 - 2 sum x_l x_{l+1}), so a mask may hold at most two of Jk, J2, Jt.
"""

import numpy as np

from .effective import _f4, _f6, _shift, BONDS

TERMS = ("Jk", "J2", "Jp", "Jp6", "Js0", "Js1", "Js2", "Jt")


def features(x, Lx, Ly, a):
    """F_t(x) for the 8 terms of E_eff (unit coefficients), in TERMS order."""
    x = np.asarray(x, dtype=np.float64)
    xn = np.roll(x, -1, axis=0)
    F = [np.sum((xn - x) ** 2), np.sum(x * x), np.sum(_f4(x, a)), np.sum(_f6(x, a))]
    for r in range(3):
        F.append(sum(float(np.sum(x * _shift(x, Lx, Ly, dx, dy))) for dx, dy in BONDS[r]))
    F.append(np.sum(x * xn))
    return np.array(F, dtype=np.float64)


def fit(F, logw, mask):
    """(E0, J[8]) minimising sum_c (logw_c - E0 + sum_t J_t F_ct)^2 over the masked terms
    (numpy lstsq on the design matrix [1, -F_mask])."""
    F = np.asarray(F, dtype=np.float64)
    cols = [t for t in range(len(TERMS)) if mask[t]]
    A = np.concatenate([np.ones((F.shape[0], 1)), -F[:, cols]], axis=1)
    c, *_ = np.linalg.lstsq(A, np.asarray(logw, dtype=np.float64), rcond=None)
    J = np.zeros(len(TERMS))
    J[cols] = c[1:]
    return float(c[0]), J
