"""Equal-time Green's function at every time slice and the CDW structure factor (oracle;
test infrastructure only).

Paper, SM Eq. (S3): G(l) = [I + B_l ... B_1 B_L ... B_{l+1}]^{-1}, the equal-time Green's
function at the time just after slice l (l = L gives the G of the weight).  Main text,
"Results": the CDW structure factor S_CDW = L^{-2} sum_ij (-1)^{i+j} (<n_i n_j> -
<n_i><n_j>), n_i the electron number on site i (both spins).

Readings (listed in the design notes):
  A7  G(l)[i, j] = <c_i c_j^dagger>; with the spec factor order (reading A4) the
      product is taken in the slice matrices E diag(v_l).
  A34 slice index.  Output slice l = 0 .. Ltau-1 is the paper's l + 1 (after the field's
      slice l), so slice Ltau-1 is the usual G.  It is evaluated by definition: the
      stabilized chain (oracle.fermion) of the field rotated so that its product is
      B_l ... B_0 B_{Ltau-1} ... B_{l+1}.
  A35 per-configuration estimators.  For a fixed phonon field the two spin species are
      independent and identical, and Wick's theorem gives <n_i>_x = 2 (1 - G_ii) and
      <n_i n_j>_x = <n_i>_x <n_j>_x + 2 (delta_ij - G_ji) G_ij.  The library returns per
      field and slice s_nn = N^-1 sum_ij (-1)^{i+j} <n_i n_j>_x and the staggered density
      m_st = N^-1 sum_i (-1)^i <n_i>_x, (-1)^i = (-1)^(ix+iy); the Monte Carlo estimate is
      S_CDW = mean(s_nn) - N mean(m_st)^2 (the second term is the N^-1 (sum_i (-1)^i
      <n_i>)^2 of the averaged densities; it vanishes at half filling).
"""

import numpy as np

from .fermion import logdet_green


def green_slices(E, x, dtau, lam, n_s, slices=None):
    """[G after slice l for l = 0 .. Ltau-1] (SM Eq. S3), each by the stabilized chain of
    the rotated field (reading A34); only the listed slices if `slices` is given."""
    Ltau = x.shape[0]
    out = []
    for l in (range(Ltau) if slices is None else slices):
        xr = np.roll(x, -(l + 1), axis=0)      # xr[k] = x[(k + l + 1) mod Ltau]
        out.append(logdet_green(E, xr, dtau, lam, n_s)[2])
    return np.array(out)


def stagger(Lx, Ly):
    """(-1)^(ix+iy) per site."""
    i = np.arange(Lx * Ly)
    return np.where(((i % Lx) + (i // Lx)) % 2 == 0, 1.0, -1.0)


def cdw_estimators(G, Lx, Ly):
    """(s_nn, m_st) of one equal-time Green's function (reading A35), by explicit sums."""
    N = Lx * Ly
    p = stagger(Lx, Ly)
    n = 2.0 * (1.0 - np.diag(G))
    s = 0.0
    for i in range(N):
        for j in range(N):
            nn = n[i] * n[j] + 2.0 * ((1.0 if i == j else 0.0) - G[j, i]) * G[i, j]
            s += p[i] * p[j] * nn
    return s / N, float(np.sum(p * n)) / N
