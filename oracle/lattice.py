"""Electron hopping matrix and its exponential (oracle; test infrastructure only).

Paper: the electronic part of the Holstein Hamiltonian, Eq. (2), is nearest-neighbour
hopping -t on an L x L square lattice with chemical potential mu; in the Trotter split
of SM Eq. (S1) each imaginary-time slice carries the whole exponential e^{-dtau K}
(no further checkerboard split, reading A5).  K is the N x N single-particle matrix of
H_el including -mu (reading A3: the phonon Hamiltonian enters only S_Bose).
"""

import numpy as np


def hopping_matrix(Lx, Ly, t, mu):
    """Single-particle matrix K of H_el, Eq. (2), periodic Lx x Ly lattice.

    Site index i = ix + Lx*iy.  Every site i contributes the bonds i -> i+x and
    i -> i+y, each adding -t to K[i,j] and K[j,i]; on a length-2 direction the two bonds
    of a pair land on the same matrix element, which then holds -2t (reading A6, the
    choice that keeps eps_k = -2t(cos kx + cos ky) - mu for every L >= 2).
    """
    if Lx < 2 or Ly < 2:
        raise ValueError("Lx and Ly must be >= 2")
    N = Lx * Ly
    K = np.zeros((N, N), dtype=np.float64)
    for iy in range(Ly):
        for ix in range(Lx):
            i = ix + Lx * iy
            for dx, dy in ((1, 0), (0, 1)):
                j = (ix + dx) % Lx + Lx * ((iy + dy) % Ly)
                K[i, j] -= t
                K[j, i] -= t
    K -= mu * np.eye(N)
    return K


def expk(K, dtau):
    """e^{-dtau K} for symmetric K through its eigen-decomposition (SM Eq. S1)."""
    e, Q = np.linalg.eigh(K)
    return (Q * np.exp(-dtau * e)[None, :]) @ Q.T
