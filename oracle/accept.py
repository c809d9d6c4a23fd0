"""SLMC cumulative-update acceptance (oracle; test infrastructure only).

Paper, Eq. (6): a configuration X' proposed by many effective-model moves is accepted
with probability min{1, [w(X')/w(X)] [w_eff(X)/w_eff(X')]}, where w is the exact weight
(SM Eq. S2: exp(-dtau S_Bose) (det M)^2) and w_eff = exp(-E_eff) (reading A12).

In logs: log r = log w(x') - log w(x) + E_eff(x') - E_eff(x); accept iff log u < log r,
u from Philox4x32-10 word 0 at counter (0xFFFFFFFF, 0xFFFFFFFF, proposal mod 2^32, chain)
with key (seed low, seed high).
"""

import numpy as np

from .boson import log_weight
from .effective import eff_energy
from .fermion import logdet_green
from .philox import philox4x32_10, uniform01


def cumulative_accept(E, Lx, Ly, dtau, lam, omega0, c_kin, n_s, eff, x_cur, x_prop,
                      logw_cur, eeff_cur, seed, proposal_idx, chain):
    """Returns (accepted, log_r, logw_prop, eeff_prop) for one chain."""
    ld, _, _ = logdet_green(E, x_prop, dtau, lam, n_s)
    logw_prop = log_weight(ld, x_prop, lam, omega0, dtau, c_kin)
    eeff_prop = eff_energy(x_prop, Lx, Ly, eff)
    log_r = (logw_prop - logw_cur) + (eeff_prop - eeff_cur)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    w = philox4x32_10((0xFFFFFFFF, 0xFFFFFFFF, proposal_idx & 0xFFFFFFFF, chain), key)
    u = float(uniform01(w[0]))
    return bool(np.log(u) < log_r), float(log_r), float(logw_prop), float(eeff_prop)
