"""Pins of the oracle's G at every time slice (SM Eq. S3) and of the CDW structure
factor's per-field estimators (main text, "Results"; reading A35).  CPU only.

G(l) is pinned by Fock-space traces with c_i c_j^dagger inserted between slices l and l+1
of the many-body product (no rotation of the field), by the free-fermion closed form, and
by the propagation identity G(l+1) = B_{l+1} G(l) B_{l+1}^{-1}.  The estimators are pinned
by a brute-force trace over the Fock space of BOTH spin species (dimension 4^N) with
n_i n_j inserted, which checks Wick's theorem and the spin sum at once."""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as o
import pins


def _slice_ops(K, x, dtau, lam, C):
    """Many-body slice operators e^{-dtau c^+ K c} e^{-dtau lam sum x n} for modes C."""
    Hk = np.einsum("ij,iab,jbc->ac", K, C.transpose(0, 2, 1), C)
    Ek = sla.expm(-dtau * Hk)
    nops = [C[i].T @ C[i] for i in range(C.shape[0])]
    out = []
    for l in range(x.shape[0]):
        d = sum(-dtau * lam * x[l, i] * np.diag(nops[i]) for i in range(len(nops)))
        out.append(Ek @ np.diag(np.exp(d)))
    return out


def _insert(ops, l, O):
    """Tr[B_{L-1} .. B_{l+1} O B_l .. B_0] / Tr[B_{L-1} .. B_0]."""
    dim = ops[0].shape[0]
    before = np.eye(dim)
    for k in range(l + 1):
        before = ops[k] @ before
    after = np.eye(dim)
    for k in range(l + 1, len(ops)):
        after = ops[k] @ after
    P = after @ before
    return np.trace(after @ O @ before) / np.trace(P)


@pytest.mark.parametrize("Lx,Ly,Ltau,lam,seed", [(2, 2, 6, 1.5, 1), (2, 3, 5, 2.0, 2)])
def test_green_slices_against_fock_space_insertion(Lx, Ly, Ltau, lam, seed):
    N = Lx * Ly
    K = o.hopping_matrix(Lx, Ly, 1.0, 0.2)
    x = np.random.default_rng(seed).normal(0.0, 1.3, size=(Ltau, N))
    C = pins._annihilators(N)
    ops = _slice_ops(K, x, 0.1, lam, C)
    Gs = o.green_slices(o.expk(K, 0.1), x, 0.1, lam, 2)
    for l in range(Ltau):
        Gf = np.array([[_insert(ops, l, C[i] @ C[j].T) for j in range(N)] for i in range(N)])
        assert np.max(np.abs(Gs[l] - Gf)) < 1e-11, l


def test_green_slices_free_fermions_are_the_closed_form_at_every_slice():
    Gs = o.green_slices(o.expk(o.hopping_matrix(4, 4, 1.0, 0.0), 0.1), np.zeros((20, 16)), 0.1, 1.5, 5)
    ref = pins.free_green(4, 4, 1.0, 0.0, 2.0)
    assert np.max(np.abs(Gs - ref[None])) < 1e-12


def test_green_slices_obey_the_propagation_identity():
    Lx, Ly, Ltau, lam, dtau = 4, 4, 24, 1.5, 0.1
    K = o.hopping_matrix(Lx, Ly, 1.0, 0.0)
    E, Einv = o.expk(K, dtau), o.expk(K, -dtau)
    x = np.random.default_rng(7).normal(size=(Ltau, 16))
    Gs = o.green_slices(E, x, dtau, lam, 6)
    for l in range(Ltau):
        ln = (l + 1) % Ltau
        v = np.exp(-dtau * lam * x[ln])
        prop = E @ (v[:, None] * Gs[l] / v[None, :]) @ Einv
        assert np.max(np.abs(prop - Gs[ln])) < 1e-10, l
    # the last slice is the G of the weight
    assert np.max(np.abs(Gs[-1] - o.logdet_green(E, x, dtau, lam, 6)[2])) < 1e-13


@pytest.mark.parametrize("Lx,Ly,Ltau,lam,seed", [(2, 2, 6, 1.5, 3), (2, 2, 4, 2.5, 4)])
def test_cdw_estimators_against_two_species_fock_space(Lx, Ly, Ltau, lam, seed):
    # modes 0..N-1 spin up, N..2N-1 spin down, the same hopping and field for both
    N = Lx * Ly
    K1 = o.hopping_matrix(Lx, Ly, 1.0, 0.3)
    K2 = np.kron(np.eye(2), K1)
    x = np.random.default_rng(seed).normal(0.0, 1.2, size=(Ltau, N))
    x2 = np.concatenate([x, x], axis=1)
    C = pins._annihilators(2 * N)
    ops = _slice_ops(K2, x2, 0.1, lam, C)
    nop = [C[i].T @ C[i] + C[i + N].T @ C[i + N] for i in range(N)]
    p = o.stagger(Lx, Ly)
    Gs = o.green_slices(o.expk(K1, 0.1), x, 0.1, lam, 2)
    for l in range(Ltau):
        ni = np.array([_insert(ops, l, nop[i]) for i in range(N)])
        nn = np.array([[_insert(ops, l, nop[i] @ nop[j]) for j in range(N)] for i in range(N)])
        s_ref = float(p @ nn @ p) / N
        m_ref = float(p @ ni) / N
        s, m = o.cdw_estimators(Gs[l], Lx, Ly)
        assert abs(s - s_ref) < 1e-10 and abs(m - m_ref) < 1e-11, (l, s, s_ref, m, m_ref)


def test_cdw_staggered_density_vanishes_at_half_filling_without_field():
    G = o.green_slices(o.expk(o.hopping_matrix(4, 4, 1.0, 0.0), 0.1), np.zeros((10, 16)), 0.1, 1.0, 5)[3]
    s, m = o.cdw_estimators(G, 4, 4)
    assert abs(m) < 1e-14
    assert s > 0.0
