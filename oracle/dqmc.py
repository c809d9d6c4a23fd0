"""DQMC comparison updates (oracle; test infrastructure only).

Paper, SM Sec. I (DQMC for the Holstein model): a local change of one phonon field
X_{i,l} multiplies one slice matrix by I + Delta(i, l), Delta with the single entry
Delta_ii = exp(-g dtau dX) - 1; the spin determinant ratio is R_sigma = 1 + (1 - G_ii)
Delta_ii (Eqs. S4, S5, both spins equal so R = R_sigma^2), and the Green's function is
updated in O(N^2) by the Sherman-Morrison formula (Eq. S6).  The block update reflects a
whole time column, X(i, tau) -> -X(i, tau) - 2g/Omega^2, accepted with the full weight
ratio (main text and SM Sec. I).

Readings (listed in the design notes):
  A36 factor order.  With B_l = e^{-dtau K} diag(v_l) (reading A4) the change at slice l
      is B_l -> B_l (I + Delta), on the right.  Rotating the product so that B_l comes
      last, the ratio needs G_{l-1} = [I + B_{l-1} .. B_0 B_{L-1} .. B_l]^{-1} (G after
      slice l-1, with G_{-1} = G_{L-1}) and takes the paper's form 1 + (1 - G_ii) Delta_ii;
      Sherman-Morrison then reads G' = G - (I - G) Delta G / R_sigma (the mirror of the
      printed G - G Delta (I - G) / R, which belongs to the factor order with the diagonal
      on the left).
  A37 local DQMC sweep.  Slices l = 0 .. L-1 in order; in each, sites i = 0 .. N-1 in order;
      move x -> x + delta (2 u1 - 1), accept iff log u2 < 2 log|R_sigma| - dtau dS_Bose
      (dS_Bose the change of the bosonic action of reading A1/A10 from the terms that touch
      (i, l)); u1, u2 = Philox4x32-10 words 0, 1 at counter (i + N l, 0xC0000000,
      sweep mod 2^32, chain), key (seed lo, seed hi).  G_{l-1} at the start of slice l is
      evaluated from its definition here (the library may propagate it between
      re-evaluations).
  A38 block update (build frame: x -> -x on the column, the reflection about the axis).
      Update u of a sweep: site floor(r N / 2^32), r = word 0 at counter (0xFFFFFFFB,
      0xFFFFFFFC, sweep n + u, chain); accept iff log u < log w(x') - log w(x), u = word 0
      at counter (0xFFFFFFFF, 0xFFFFFFFC, sweep n + u, chain), n updates per sweep.
"""

import numpy as np

from .boson import log_weight
from .fermion import logdet_green
from .measure import green_slices
from .philox import philox4x32_10, uniform01


def local_ratio(G, i, d):
    """R_sigma = 1 + (1 - G_ii) Delta_ii (SM Eq. S5)."""
    return 1.0 + (1.0 - G[i, i]) * d


def sherman_morrison(G, i, d):
    """G after Delta_ii = d at site i (SM Eq. S6 in the build factor order, reading A36)."""
    R = local_ratio(G, i, d)
    col = -G[:, i].copy()
    col[i] += 1.0                          # (I - G) e_i
    return G - np.outer(col, G[i, :]) * (d / R)


def bosonic_local_delta(x, i, l, xn, lam, omega0, dtau, c_kin):
    """S_Bose(x with x[l, i] -> xn) - S_Bose(x) from the terms touching (i, l)."""
    Lt = x.shape[0]
    xo, xp, xm = x[l, i], x[(l + 1) % Lt, i], x[(l - 1) % Lt, i]
    pot = 0.5 * omega0 ** 2 * (xn * xn - xo * xo) - lam * (xn - xo)
    kin = (xp - xn) ** 2 + (xn - xm) ** 2 - (xp - xo) ** 2 - (xo - xm) ** 2
    return pot + c_kin * kin / (dtau * dtau)


def _key(seed):
    return (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def local_sweep(E, x, dtau, lam, omega0, c_kin, n_s, delta, seed, sweep_idx, chain, margins=None):
    """One DQMC local sweep of one field, in place (reading A37).  Returns (accepted moves,
    G of the final field by definition).  `margins` collects |log u2 - log r|."""
    Lt, N = x.shape
    key = _key(seed)
    sw = sweep_idx & 0xFFFFFFFF
    acc = 0
    for l in range(Lt):
        G = green_slices(E, x, dtau, lam, n_s, slices=[(l - 1) % Lt])[0]
        for i in range(N):
            w = philox4x32_10((i + N * l, 0xC0000000, sw, chain), key)
            dx = delta * (2.0 * float(uniform01(w[0])) - 1.0)
            xn = x[l, i] + dx
            d = np.expm1(-dtau * lam * dx)
            R = local_ratio(G, i, d)
            log_r = 2.0 * np.log(abs(R)) - dtau * bosonic_local_delta(x, i, l, xn, lam, omega0, dtau, c_kin)
            lu = np.log(float(uniform01(w[1])))
            if margins is not None:
                margins.append(abs(lu - log_r))
            if lu < log_r:
                G = sherman_morrison(G, i, d)
                x[l, i] = xn
                acc += 1
    return acc, logdet_green(E, x, dtau, lam, n_s)[2]


def block_updates(E, x, logw, dtau, lam, omega0, c_kin, n_s, n_updates, seed, sweep_idx, chain,
                  margins=None):
    """n_updates column reflections of one field, in place (reading A38).  Returns
    (accepted count, log w of the final field)."""
    Lt, N = x.shape
    key = _key(seed)
    acc = 0
    for u in range(n_updates):
        ctr = (sweep_idx * n_updates + u) & 0xFFFFFFFF
        r = int(philox4x32_10((0xFFFFFFFB, 0xFFFFFFFC, ctr, chain), key)[0])
        s = (r * N) >> 32
        xp = x.copy()
        xp[:, s] = -xp[:, s]
        lwp = log_weight(logdet_green(E, xp, dtau, lam, n_s)[0], xp, lam, omega0, dtau, c_kin)
        lu = np.log(float(uniform01(philox4x32_10((0xFFFFFFFF, 0xFFFFFFFC, ctr, chain), key)[0])))
        if margins is not None:
            margins.append(abs(lu - (lwp - logw)))
        if lu < lwp - logw:
            x[:, :] = xp
            logw = lwp
            acc += 1
    return acc, logw
