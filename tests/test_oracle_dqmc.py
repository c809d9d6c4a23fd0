"""Pins of the oracle's DQMC comparison updates (SM Sec. I, Eqs. S4-S6; readings
A36-A38).  CPU only.

The local ratio and the Sherman-Morrison update are checked against two independent
evaluations of the definition (log-determinants and G of the changed field), at every
slice, with the printed left-perturbation form shown to fail in the build factor order;
the local bosonic change against the global action; the local sweep's accept rule by a
Gaussian moment test with the fermions switched off; the block update's accept rule by
its acceptance frequency per site."""

import numpy as np
import pytest

import oracle as o
from oracle.dqmc import bosonic_local_delta, local_ratio, sherman_morrison, local_sweep, block_updates
from oracle.measure import green_slices


def _setup(Lx=4, Ly=4, Ltau=12, seed=1, mu=0.1):
    K = o.hopping_matrix(Lx, Ly, 1.0, mu)
    return o.expk(K, 0.1), np.random.default_rng(seed).normal(size=(Ltau, Lx * Ly))


@pytest.mark.parametrize("l,i,dx", [(0, 3, 0.7), (5, 10, -1.1), (11, 0, 0.4), (7, 15, 2.0)])
def test_local_ratio_is_the_determinant_ratio(l, i, dx):
    E, x = _setup()
    lam, dtau = 1.5, 0.1
    G = green_slices(E, x, dtau, lam, 4, slices=[(l - 1) % 12])[0]
    d = np.expm1(-dtau * lam * dx)
    xp = x.copy()
    xp[l, i] += dx
    ld0, s0, _ = o.logdet_green(E, x, dtau, lam, 4)
    ld1, s1, _ = o.logdet_green(E, xp, dtau, lam, 4)
    R = local_ratio(G, i, d)
    assert abs(np.log(abs(R)) - (ld1 - ld0)) < 1e-11
    assert np.sign(R) == s0 * s1
    # the G after slice l (not l - 1) does not give it
    Gw = green_slices(E, x, dtau, lam, 4, slices=[l])[0]
    assert abs(np.log(abs(local_ratio(Gw, i, d))) - (ld1 - ld0)) > 1e-6


@pytest.mark.parametrize("l,i,dx", [(0, 3, 0.7), (6, 9, -1.3), (11, 14, 0.9)])
def test_sherman_morrison_gives_the_changed_fields_green_function(l, i, dx):
    E, x = _setup(seed=2)
    lam, dtau = 1.5, 0.1
    G = green_slices(E, x, dtau, lam, 4, slices=[(l - 1) % 12])[0]
    d = np.expm1(-dtau * lam * dx)
    xp = x.copy()
    xp[l, i] += dx
    ref = green_slices(E, xp, dtau, lam, 4, slices=[(l - 1) % 12])[0]
    assert np.max(np.abs(sherman_morrison(G, i, d) - ref)) < 1e-11
    # the printed left-perturbation form G - G Delta (I - G) / R belongs to the other
    # factor order and misses here
    col = np.eye(16)[i] - G[i, :]
    wrong = G - np.outer(G[:, i], col) * d / local_ratio(G, i, d)
    assert np.max(np.abs(wrong - ref)) > 1e-6


def test_bosonic_local_delta_is_the_global_difference():
    _, x = _setup(seed=3)
    for (i, l, xn) in ((2, 0, 1.3), (7, 11, -0.4), (15, 5, 2.2)):
        xp = x.copy()
        xp[l, i] = xn
        g = o.bosonic_action(xp, 1.5, 1.0, 0.1, 0.5) - o.bosonic_action(x, 1.5, 1.0, 0.1, 0.5)
        assert abs(bosonic_local_delta(x, i, l, xn, 1.5, 1.0, 0.1, 0.5) - g) < 1e-9 * max(1.0, abs(g))


def test_local_sweep_samples_the_free_phonon_gaussian_without_coupling():
    # lam = 0: R_sigma = 1, the sweep samples exp(-dtau S_Bose), a Gaussian per site with
    # precision dtau omega0^2 I + (2 c_kin / dtau) (periodic 1-D Laplacian) over the slices
    Lx, Ly, Lt, dtau, w0, ck = 2, 2, 6, 0.1, 1.0, 0.5
    E = o.expk(o.hopping_matrix(Lx, Ly, 1.0, 0.0), dtau)
    lap = 2.0 * np.eye(Lt) - np.roll(np.eye(Lt), 1, axis=0) - np.roll(np.eye(Lt), -1, axis=0)
    cov = np.linalg.inv(dtau * w0 ** 2 * np.eye(Lt) + (2.0 * ck / dtau) * lap)
    x = np.zeros((Lt, 4))
    samples = []
    for sw in range(700):
        local_sweep(E, x, dtau, 0.0, w0, ck, 3, 2.5, 31, sw, 0)
        if sw >= 100:
            samples.append(x.copy())
    s = np.array(samples)
    var = float(np.mean(s ** 2))
    # effective sample size is well below 2400: a 15 % bar on the variance
    assert abs(var - cov[0, 0]) < 0.15 * cov[0, 0], (var, cov[0, 0])
    c1 = float(np.mean(s[:, :-1] * s[:, 1:]))
    assert abs(c1 - cov[0, 1]) < 0.15 * cov[0, 0]


def test_block_update_accepts_with_the_weight_ratio():
    # the same field again and again: the acceptance frequency of a reflection of column s
    # is min(1, w(x^s) / w(x))
    Lx, Ly, Lt, dtau, lam = 2, 2, 40, 0.1, 2.0
    E = o.expk(o.hopping_matrix(Lx, Ly, 1.0, 0.0), dtau)
    x0 = np.random.default_rng(3).normal(0.0, 1.0, size=(Lt, 4))
    x0[:, 1] *= -1.0
    x0[:, 2] *= -1.0
    lw0 = o.log_weight(o.logdet_green(E, x0, dtau, lam, 3)[0], x0, lam, 1.0, dtau, 0.5)
    expect = []
    for s in range(4):
        xp = x0.copy()
        xp[:, s] = -xp[:, s]
        lw = o.log_weight(o.logdet_green(E, xp, dtau, lam, 3)[0], xp, lam, 1.0, dtau, 0.5)
        expect.append(min(1.0, np.exp(lw - lw0)))
    hit = np.zeros(4)
    tot = np.zeros(4)
    from oracle.philox import philox4x32_10
    for sw in range(1200):
        x = x0.copy()
        acc, _ = block_updates(E, x, lw0, dtau, lam, 1.0, 0.5, 3, 1, 5, sw, 2)
        r = int(philox4x32_10((0xFFFFFFFB, 0xFFFFFFFC, sw, 2), (5, 0))[0])
        s = (r * 4) >> 32
        tot[s] += 1
        hit[s] += acc
        assert acc == 0 or np.array_equal(x[:, s], -x0[:, s])
    assert np.all(tot > 200)
    for s in range(4):
        p = expect[s]
        assert abs(hit[s] / tot[s] - p) <= 4.0 * np.sqrt(p * (1 - p) / tot[s]) + 1e-9, (s, hit[s] / tot[s], p)
    assert min(expect) < 0.9
