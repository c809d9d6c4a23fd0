"""Pins of the oracle's bosonic weight, effective model, sweep, generator and accept
step (Eq. 4/S7, Eq. 6, SM Eq. S2).  CPU only."""

import os

import numpy as np
import pytest

import oracle as o
from oracle.effective import BONDS, EffModel, _shift

HERE = os.path.dirname(os.path.abspath(__file__))


def _E(Lx, Ly, t=1.0, mu=0.0, dtau=0.1):
    return o.expk(o.hopping_matrix(Lx, Ly, t, mu), dtau)


def _rand_eff(seed, js=(0.2, -0.1, 0.05), a=1.5):
    g = np.random.default_rng(seed)
    return EffModel(Jk=abs(g.normal()), J2=g.normal() * 0.3, Jp=abs(g.normal()) * 0.2,
                    Jp6=abs(g.normal()) * 0.01, a=a, Js=js, Jt=g.normal() * 0.2, delta=0.8)


# ------------------------------------------------------------------ P13 generator

def test_P13_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(h, 16) for h in r]
        out = o.philox4x32_10(v[0:4], v[4:6])
        assert [int(w) for w in out] == v[6:10]


def test_philox_vectorized_equals_scalar_and_uniform_is_open_interval():
    ctr = (np.arange(50, dtype=np.uint64), 7, 3, 11)
    vec = o.philox4x32_10(ctr, (123, 456))
    for j in range(50):
        sc = o.philox4x32_10((j, 7, 3, 11), (123, 456))
        assert all(int(vec[w][j]) == int(sc[w]) for w in range(4))
    u = o.uniform01(np.array([0, 0xFFFFFFFF], dtype=np.uint64))
    assert 0.0 < u[0] < u[1] < 1.0 and u[0] == 2.0 ** -33


# ------------------------------------------------------------------ bosonic action, P10, P11

def test_bosonic_action_by_explicit_double_loop():
    x = np.random.default_rng(1).normal(size=(6, 4))
    lam, w0, dt, ck = 1.3, 0.8, 0.1, 0.5
    s = 0.0
    for l in range(6):
        for i in range(4):
            s += 0.5 * w0 * w0 * x[l, i] ** 2 - lam * x[l, i]
            s += ck * ((x[(l + 1) % 6, i] - x[l, i]) / dt) ** 2
    assert abs(o.bosonic_action(x, lam, w0, dt, ck) - s) < 1e-12 * abs(s)


def test_bosonic_action_shift_of_frame():
    # S_Bose in the paper's frame, Omega^2/2 X^2 + c ((X'-X)/dtau)^2, with X = x + alpha,
    # alpha = -lam/omega0^2, equals the build-frame action up to a field-independent
    # constant (reading A1)
    lam, w0, dt, ck = 1.5, 1.0, 0.1, 0.5
    alpha = -lam / w0 ** 2
    g = np.random.default_rng(2)
    diffs = []
    for _ in range(3):
        x = g.normal(size=(8, 4))
        X = x + alpha
        paper = 0.5 * w0 ** 2 * np.sum(X * X) + ck * np.sum((np.roll(X, -1, 0) - X) ** 2) / dt ** 2
        diffs.append(paper - o.bosonic_action(x, lam, w0, dt, ck))
    assert np.ptp(diffs) < 1e-12


@pytest.mark.parametrize("Lx,Ly", [(4, 4), (6, 4)])
def test_P10_full_weight_is_Z2_even(Lx, Ly):
    E = _E(Lx, Ly)
    x = np.random.default_rng(3).normal(size=(20, Lx * Ly))
    lam, w0, dt, ck = 1.5, 1.0, 0.1, 0.5
    lw = o.log_weight(o.logdet_green(E, x, dt, lam, 5)[0], x, lam, w0, dt, ck)
    lwm = o.log_weight(o.logdet_green(E, -x, dt, lam, 5)[0], -x, lam, w0, dt, ck)
    assert abs(lw - lwm) < 1e-10 * abs(lw)


def test_P11_accept_limits():
    Lx = Ly = 4
    E = _E(Lx, Ly)
    lam, w0, dt, ck, n_s = 1.5, 1.0, 0.1, 0.5, 5
    g = np.random.default_rng(4)
    x = g.normal(size=(20, 16))
    eff = EffModel(**{k: v for k, v in dict(Jk=ck / dt, J2=dt * w0 ** 2 / 2).items()})
    ld = o.logdet_green(E, x, dt, lam, n_s)[0]
    lw = o.log_weight(ld, x, lam, w0, dt, ck)
    ee = o.eff_energy(x, Lx, Ly, eff)
    # identical proposal: log r = 0, always accepted
    acc, lr, _, _ = o.cumulative_accept(E, Lx, Ly, dt, lam, w0, ck, n_s, eff, x, x.copy(),
                                        lw, ee, 99, 5, 0)
    assert acc and abs(lr) < 1e-10
    # E_eff = symmetric bosonic part: log r = 2 (ld' - ld) + dtau lam sum(x' - x)
    xp = x + 0.3 * g.normal(size=x.shape)
    acc, lr, _, _ = o.cumulative_accept(E, Lx, Ly, dt, lam, w0, ck, n_s, eff, x, xp,
                                        lw, ee, 99, 5, 0)
    ldp = o.logdet_green(E, xp, dt, lam, n_s)[0]
    assert abs(lr - (2 * (ldp - ld) + dt * lam * np.sum(xp - x))) < 1e-9


def test_accept_decision_uses_philox_word():
    Lx = Ly = 4
    E = _E(Lx, Ly)
    x = np.random.default_rng(5).normal(size=(20, 16))
    eff = EffModel(Jk=0.1)
    ld = o.logdet_green(E, x, 0.1, 1.5, 5)[0]
    lw = o.log_weight(ld, x, 1.5, 1.0, 0.1, 0.5)
    ee = o.eff_energy(x, 4, 4, eff)
    xp = x + 0.2
    _, lr, _, _ = o.cumulative_accept(E, 4, 4, 0.1, 1.5, 1.0, 0.5, 5, eff, x, xp, lw, ee, 7, 3, 2)
    for seed, prop, ch in ((7, 3, 2), (8, 3, 2), (7, 4, 2), (7, 3, 1)):
        w = o.philox4x32_10((0xFFFFFFFF, 0xFFFFFFFF, prop, ch), (seed, 0))
        acc, lr2, _, _ = o.cumulative_accept(E, 4, 4, 0.1, 1.5, 1.0, 0.5, 5, eff, x, xp, lw, ee,
                                             seed, prop, ch)
        assert lr2 == lr
        assert acc == (np.log(float(o.uniform01(w[0]))) < lr)


# ------------------------------------------------------------------ P12 effective model

def test_eff_energy_by_explicit_loops():
    Lx, Ly, Lt = 4, 4, 6
    m = _rand_eff(6)
    x = np.random.default_rng(7).normal(size=(Lt, Lx * Ly))
    e = 0.0
    for l in range(Lt):
        for iy in range(Ly):
            for ix in range(Lx):
                i = ix + Lx * iy
                y = x[l, i]
                yn = x[(l + 1) % Lt, i]
                e += m.Jk * (yn - y) ** 2 + m.J2 * y * y + m.Jt * y * yn
                e += m.Jp * (y ** 4 / 4 - m.a ** 2 * y ** 2 / 2)
                e += m.Jp6 * (y ** 6 / 6 - m.a ** 2 * y ** 4 / 4)
                for r, bonds in enumerate(BONDS):
                    for dx, dy in bonds:
                        j = (ix + dx) % Lx + Lx * ((iy + dy) % Ly)
                        e += m.Js[r] * y * x[l, j]
    assert abs(o.eff_energy(x, Lx, Ly, m) - e) < 1e-11 * max(1, abs(e))


def test_P12_table_S1_double_wells_have_minima_at_alpha_mirror():
    # Table S1 coefficients (paper frame): J_p f4 + J_p' f6 with y = X - alpha has its
    # minima at y = +-|alpha|, i.e. X = 0 and X = 2 alpha (Fig. 1, atomic limit)
    vals = dict(l.split() for l in open(os.path.join(HERE, "golden", "table_s1.txt"))
                if l.strip() and not l.startswith("#"))
    Jp, Jp6, alpha = float(vals["Jp"]), float(vals["Jp6"]), float(vals["alpha"])
    X = np.linspace(-10, 2, 120001)
    y = X - alpha
    f = Jp * (y ** 4 / 4 - alpha ** 2 * y ** 2 / 2) + Jp6 * (y ** 6 / 6 - alpha ** 2 * y ** 4 / 4)
    core = (X > -9) & (X < 1)
    Xc, fc = X[core], f[core]
    left = Xc[np.argmin(np.where(Xc < alpha, fc, np.inf))]
    right = Xc[np.argmin(np.where(Xc > alpha, fc, np.inf))]
    assert abs(left - 2 * alpha) < 1e-3 and abs(right - 0.0) < 1e-3
    # each function alone: derivative zero at y = +-|alpha| and y = 0
    for fn in (lambda y: y ** 3 - alpha ** 2 * y, lambda y: y ** 5 - alpha ** 2 * y ** 3):
        for y0 in (alpha, -alpha, 0.0):
            assert abs(fn(y0)) < 1e-12


def test_P12_Z2_and_lattice_invariance_of_eff_energy():
    Lx = Ly = 4
    m = _rand_eff(8)
    x = np.random.default_rng(9).normal(size=(6, 16))
    e = o.eff_energy(x, Lx, Ly, m)
    assert abs(o.eff_energy(-x, Lx, Ly, m) - e) < 1e-12 * abs(e)
    i = np.arange(16)
    ix, iy = i % 4, i // 4
    for gx, gy in ((ix + 1, iy), (-iy, ix), (-ix, iy), (iy, ix)):
        g = (gx % 4) + 4 * (gy % 4)
        assert abs(o.eff_energy(x[:, g], Lx, Ly, m) - e) < 1e-12 * abs(e)
    assert abs(o.eff_energy(np.roll(x, 2, 0), Lx, Ly, m) - e) < 1e-12 * abs(e)
    assert abs(o.eff_energy(x[::-1], Lx, Ly, m) - e) < 1e-12 * abs(e)


@pytest.mark.parametrize("Lx,Ly,Lt", [(4, 4, 6), (8, 4, 4), (4, 8, 2)])
def test_P12_local_delta_equals_global_difference(Lx, Ly, Lt):
    m = _rand_eff(10)
    g = np.random.default_rng(11)
    x = g.normal(size=(Lt, Lx * Ly))
    e0 = o.eff_energy(x, Lx, Ly, m)
    for _ in range(20):
        i, l = int(g.integers(Lx * Ly)), int(g.integers(Lt))
        xn = x[l, i] + g.normal()
        de = o.eff_local_delta(x, Lx, Ly, m, i, l, xn)
        x2 = x.copy()
        x2[l, i] = xn
        assert abs(de - (o.eff_energy(x2, Lx, Ly, m) - e0)) < 1e-11 * max(1, abs(e0))


def test_colouring_has_no_coupled_pair_inside_a_phase():
    for js, L in (((0.1, 0.0, 0.0), 4), ((0.1, 0.2, 0.0), 6), ((0.1, 0.2, 0.3), 8),
                  ((0.1, 0.2, 0.3), 12), ((0.0, 0.0, 0.3), 6)):
        m = EffModel(Jk=1.0, Js=js, Jt=0.1)
        mod, ph, P = o.colouring(L, L, 4, m)
        assert P == 2 * mod * mod
        N = L * L
        for l in range(4):
            for i in range(N):
                ix, iy = i % L, i // L
                nb = [((l + 1) % 4, i), ((l - 1) % 4, i)]
                for r in range(3):
                    if js[r]:
                        for dx, dy in BONDS[r]:
                            for s in (1, -1):
                                nb.append((l, (ix + s * dx) % L + L * ((iy + s * dy) % L)))
                assert all(ph[ll, j] != ph[l, i] for ll, j in nb)


def test_colouring_rejects_incompatible_lattices():
    with pytest.raises(ValueError):
        o.colouring(4, 4, 5, EffModel(Jk=1.0))                       # odd Ltau
    with pytest.raises(ValueError):
        o.colouring(10, 10, 4, EffModel(Jk=1.0, Js=(0.1, 0.1, 0.1)))  # neither 4 nor 3 divides


def test_sweep_result_does_not_depend_on_order_inside_a_phase():
    # the decomposition is valid iff shuffling the site order inside each phase gives
    # bit-identical fields (updates of one phase touch no other site of that phase)
    Lx = Ly = 4
    Lt = 4
    m = _rand_eff(12)
    x0 = np.random.default_rng(13).normal(size=(Lt, 16))
    xa = x0.copy()
    na = o.sweep(xa, Lx, Ly, m, 2, 77, 3, 1)
    # same moves applied with a per-phase shuffled order
    from oracle.effective import eff_local_delta
    _, ph, P = o.colouring(Lx, Ly, Lt, m)
    coin = int(o.philox4x32_10((0xFFFFFFFF, 0xFFFFFFFE, 3, 1), (77, 0))[0])
    order = list(range(P)) if coin < 2 ** 31 else list(range(P - 1, -1, -1))
    rng = np.random.default_rng(14)
    xb = x0.copy()
    nb = 0
    for s in range(2):
        for p in order:
            sites = [(i + 16 * l, i, l) for l in range(Lt) for i in range(16) if ph[l, i] == p]
            rng.shuffle(sites)
            for site, i, l in sites:
                w = o.philox4x32_10((site, s, 3, 1), (77, 0))
                u1, u2 = float(o.uniform01(w[0])), float(o.uniform01(w[1]))
                xn = xb[l, i] + m.delta * (2 * u1 - 1)
                if np.log(u2) < -eff_local_delta(xb, Lx, Ly, m, i, l, xn):
                    xb[l, i] = xn
                    nb += 1
    assert na == nb and np.array_equal(xa, xb)
    assert 0 < na < 2 * Lt * 16


@pytest.mark.slow
def test_P12_gaussian_model_moments():
    # quadratic E_eff = x^T A x / 2 with A positive definite has the Gaussian stationary
    # law N(0, A^{-1}); the sweep must sample it (checked on <x_i^2> and <x_i x_j>)
    Lx, Ly, Lt = 2, 2, 4
    m = EffModel(Jk=0.6, J2=0.4, Js=(0.15, 0.0, 0.0), delta=1.6)
    N = Lx * Ly
    n = Lt * N
    A = np.zeros((n, n))
    for a in range(n):                     # Hessian of E_eff by finite structure
        ea = np.zeros(n); ea[a] = 1
        for b in range(n):
            eb = np.zeros(n); eb[b] = 1
            A[a, b] = (o.eff_energy((ea + eb).reshape(Lt, N), Lx, Ly, m)
                       - o.eff_energy(ea.reshape(Lt, N), Lx, Ly, m)
                       - o.eff_energy(eb.reshape(Lt, N), Lx, Ly, m))
    C = np.linalg.inv(A)
    x = np.zeros((Lt, N))
    samples = []
    for prop in range(12000):
        o.sweep(x, Lx, Ly, m, 1, 2024, prop, 0)
        if prop >= 200:
            samples.append(x.ravel().copy())
    S = np.array(samples)
    emp = S.T @ S / len(S)
    # statistical bars ~3.5 sigma (12k correlated sweeps); a wrong sign of the coupling
    # would move the off-diagonal moment by ~0.8 in these units
    assert abs(np.mean(np.diag(emp)) / np.mean(np.diag(C)) - 1) < 0.07
    assert abs(emp[0, 1] + emp[1, 0] - 2 * C[0, 1]) < 0.2 * np.mean(np.diag(C))
