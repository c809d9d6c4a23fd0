"""Independent reference computations that pin the oracle (test helpers).

None of these re-types the oracle's algorithm: the closed forms work in momentum space
and the brute force works in the 2^N-dimensional Fock space, so a dropped term, a wrong
sign, a transposed factor or a wrong slice order in the oracle shows up as a mismatch.
"""

import numpy as np
import scipy.linalg as sla


def momenta(Lx, Ly):
    kx = 2.0 * np.pi * np.arange(Lx) / Lx
    ky = 2.0 * np.pi * np.arange(Ly) / Ly
    KX, KY = np.meshgrid(kx, ky, indexing="xy")  # KX[iy, ix]
    return KX.ravel(), KY.ravel()


def band(Lx, Ly, t, mu):
    """eps_k = -2t (cos kx + cos ky) - mu (free electrons on the square lattice)."""
    kx, ky = momenta(Lx, Ly)
    return -2.0 * t * (np.cos(kx) + np.cos(ky)) - mu


def free_logdet(Lx, Ly, t, mu, beta, shift=0.0):
    """sum_k log(1 + exp(-beta eps_k - shift)): det(1 + e^{-beta K}) of free fermions,
    with a spatially uniform field contributing shift = dtau lam sum_l c_l."""
    e = band(Lx, Ly, t, mu)
    return float(np.sum(np.log1p(np.exp(-beta * e - shift))))


def free_green(Lx, Ly, t, mu, beta):
    """G_ij = N^-1 sum_k e^{i k (r_i - r_j)} / (1 + e^{-beta eps_k})."""
    kx, ky = momenta(Lx, Ly)
    e = -2.0 * t * (np.cos(kx) + np.cos(ky)) - mu
    N = Lx * Ly
    rx = np.arange(N) % Lx
    ry = np.arange(N) // Lx
    ph = np.exp(1j * (np.outer(rx, kx) + np.outer(ry, ky)))  # [i, k]
    occ = 1.0 / (1.0 + np.exp(-beta * e))
    G = (ph * occ[None, :]) @ ph.conj().T / N
    return G.real


def staggered_logdet(Lx, Ly, t, mu, dtau, lam, x0, Ltau):
    """Static staggered field x0 (-1)^(ix+iy): momenta k and k+(pi,pi) pair up, each
    pair's slice matrix has eigenvalues e^{dtau mu} e^{+-theta_k} with
    cosh theta_k = cosh(dtau lam x0) cosh(dtau eps0_k), eps0_k = -2t(cos kx + cos ky)."""
    kx, ky = momenta(Lx, Ly)
    e0 = -2.0 * t * (np.cos(kx) + np.cos(ky))
    th = np.arccosh(np.cosh(dtau * lam * x0) * np.cosh(dtau * e0))
    bm = Ltau * dtau * mu
    per_k = np.log(1.0 + 2.0 * np.exp(bm) * np.cosh(Ltau * th) + np.exp(2.0 * bm))
    return float(0.5 * np.sum(per_k))


# ---------------------------------------------------------------- Fock space brute force

def _annihilators(N):
    """Jordan-Wigner c_i on the 2^N occupation basis (state bit i = n_i)."""
    dim = 1 << N
    C = np.zeros((N, dim, dim))
    for s in range(dim):
        for i in range(N):
            if (s >> i) & 1:
                sgn = -1.0 if bin(s & ((1 << i) - 1)).count("1") % 2 else 1.0
                C[i, s ^ (1 << i), s] = sgn
    return C


def fock_logdet_green(K, x, dtau, lam):
    """Tr prod_l [e^{-dtau c^+ K c} e^{-dtau lam sum_i x_{i,l} n_i}] (slice l = 0
    rightmost) and G_ij = Tr[c_i c_j^+ prod] / Tr prod, by dense many-body matrices."""
    N = K.shape[0]
    C = _annihilators(N)
    Hk = np.einsum("ij,iab,jbc->ac", K, C.transpose(0, 2, 1), C)
    Ek = sla.expm(-dtau * Hk)
    dim = 1 << N
    occ = np.array([[(s >> i) & 1 for i in range(N)] for s in range(dim)], dtype=float)
    P = np.eye(dim)
    for l in range(x.shape[0]):
        d = np.exp(-dtau * lam * occ @ x[l])
        P = Ek @ (d[:, None] * P)
    Z = np.trace(P)
    G = np.empty((N, N))
    for i in range(N):
        for j in range(N):
            G[i, j] = np.trace(C[i] @ C[j].T @ P) / Z
    return float(np.log(abs(Z))), int(np.sign(Z)), G
