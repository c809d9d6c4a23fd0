"""Fermion weight of a phonon field (oracle; test infrastructure only).

Paper, SM Eq. (S2): integrating out the fermions leaves det M_up * det M_dn with
M = I + B_L ... B_1, and the two spin determinants are identical.  SM Eq. (S3): the
equal-time Green's function is G = [I + B_L ... B_1]^{-1} (taken at slice l = L).

Readings (listed in the design notes):
  A1  build frame x = X - alpha: the slice matrix carries diag(e^{-dtau*lam*x_l}) and the
      hopping matrix has mu = 0 at half filling;
  A4  factor order B_l = e^{-dtau K} diag(e^{-dtau lam x_l}) (the paper writes the two
      factors the other way round; log|det| is the same, G differs by a similarity
      with e^{-dtau K});
  A7  G[i,j] = <c_i c_j^dagger>, row i, column j;
  A8  the single-spin sign of det M is returned; the spin-summed weight uses 2 log|det|;
  A9  stabilization: column-pivoted QR every n_s slices, UDV accumulation, split of D at
      1 for the final solve; the last segment may be shorter.

Field layout: x[l, i], l = 0 .. Ltau-1, where l = 0 is the paper's slice 1 (the rightmost
factor B_1 of the product).
"""

import numpy as np
import scipy.linalg as sla


def slice_scales(x, dtau, lam):
    """v[l, i] = exp(-dtau * lam * x[l, i]): the diagonal of e^{-dtau H_int} per slice
    (SM Eq. S2 with H_int = g n X, coupling named lam here, reading A1)."""
    return np.exp(-dtau * lam * np.asarray(x, dtype=np.float64))


def udv_chain(E, v, n_s):
    """Stabilized product B_L ... B_1 = U diag(D) V with B_l = E diag(v[l]).

    Plain textbook form: start from U = I, D = 1, V = I.  For each block of n_s slices
    multiply the slices onto U, scale the columns by D, factor the result with a
    column-pivoted Householder QR (LAPACK dgeqp3 through scipy), keep |diag R| as the new
    D, Q as the new U, and fold D^{-1} R P^T into V.

    Returns (U, D, V, sign_det_U).
    """
    Ltau, N = v.shape
    U = np.eye(N)
    D = np.ones(N)
    V = np.eye(N)
    for k0 in range(0, Ltau, n_s):
        M = U.copy()
        for l in range(k0, min(k0 + n_s, Ltau)):
            M = E @ (v[l][:, None] * M)
        M = M * D[None, :]
        Q, R, p = sla.qr(M, pivoting=True)
        D = np.abs(np.diag(R))
        U = Q
        Rn = R / D[:, None]
        V = Rn[:, np.argsort(p)] @ V
    sign_u = np.linalg.slogdet(U)[0]
    return U, D, V, sign_u


def recombine(U, D, V, sign_u):
    """log|det(I + U D V)|, its sign and G = (I + U D V)^{-1}.

    With Db = max(D, 1) and Ds = min(D, 1) one has I + U D V = U Db X where
    X = Db^{-1} U^T + Ds V, so det = det U * prod Db * det X and G = X^{-1} Db^{-1} U^T.
    X is factored by LU with partial pivoting (LAPACK dgetrf through scipy).
    """
    Db = np.maximum(D, 1.0)
    Ds = np.minimum(D, 1.0)
    Ut_b = U.T / Db[:, None]
    X = Ut_b + Ds[:, None] * V
    lu, piv = sla.lu_factor(X)
    d = np.diag(lu)
    logdet = float(np.sum(np.log(Db)) + np.sum(np.log(np.abs(d))))
    n_swaps = int(np.count_nonzero(piv != np.arange(len(piv))))
    sign = sign_u * np.prod(np.sign(d)) * (-1.0) ** n_swaps
    G = sla.lu_solve((lu, piv), Ut_b)
    return logdet, int(sign), G


def logdet_green(E, x, dtau, lam, n_s):
    """Single-spin (log|det(I + B_L...B_1)|, sign, G) for one field x[Ltau, N]
    (SM Eqs. S2 and S3), stabilized every n_s slices."""
    v = slice_scales(x, dtau, lam)
    U, D, V, su = udv_chain(E, v, n_s)
    return recombine(U, D, V, su)


def logdet_green_direct(E, x, dtau, lam):
    """Unstabilized definition, for well-conditioned small cases only:
    A = B_L ... B_1 formed directly, then slogdet and inverse of I + A."""
    v = slice_scales(x, dtau, lam)
    N = E.shape[0]
    A = np.eye(N)
    for l in range(v.shape[0]):
        A = E @ (v[l][:, None] * A)
    M = np.eye(N) + A
    s, ld = np.linalg.slogdet(M)
    return float(ld), int(s), np.linalg.inv(M)
