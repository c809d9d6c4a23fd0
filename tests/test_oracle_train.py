"""Pins of the oracle's effective-model regression (Eq. 5, SM Sec. III; reading A39).  CPU
only: the features reproduce the pinned effective energy term by term, the regression
recovers known coefficients exactly from noise-free targets, satisfies the normal
equations with noise, and finds the bosonic action's own coefficients when the target is
-dtau S_Bose of fields with no linear term."""

import numpy as np
import pytest

import oracle as o
from oracle.effective import EffModel, eff_energy
from oracle.train import features, fit, TERMS


def _J(model):
    return np.array([model.Jk, model.J2, model.Jp, model.Jp6, model.Js[0], model.Js[1], model.Js[2], model.Jt])


@pytest.mark.parametrize("Lx,Ly,Ltau", [(4, 4, 6), (6, 4, 8), (2, 3, 4)])
def test_features_reproduce_the_effective_energy(Lx, Ly, Ltau):
    rng = np.random.default_rng(Lx + Ly + Ltau)
    for _ in range(4):
        m = EffModel(*rng.normal(size=4), a=1.3, Js=tuple(rng.normal(size=3)), Jt=rng.normal())
        x = rng.normal(size=(Ltau, Lx * Ly))
        F = features(x, Lx, Ly, m.a)
        assert abs(_J(m) @ F - eff_energy(x, Lx, Ly, m)) < 1e-12 * max(1.0, np.abs(F).sum())
        # and each feature alone is the energy of that unit term
        for t in range(8):
            unit = np.zeros(8)
            unit[t] = 1.0
            mt = EffModel(Jk=unit[0], J2=unit[1], Jp=unit[2], Jp6=unit[3], a=m.a, Js=tuple(unit[4:7]), Jt=unit[7])
            assert abs(F[t] - eff_energy(x, Lx, Ly, mt)) < 1e-12 * max(1.0, abs(F[t]))


def test_fit_recovers_known_coefficients_from_exact_targets():
    rng = np.random.default_rng(5)
    Lx, Ly, Lt = 4, 4, 8
    mask = [1, 0, 1, 1, 1, 1, 0, 1]
    J = np.array([0.7, 0.0, 0.05, -0.002, 0.11, -0.03, 0.0, 0.2])
    xs = [rng.normal(0.0, 1.2, size=(Lt, Lx * Ly)) for _ in range(60)]
    F = np.array([features(x, Lx, Ly, 1.1) for x in xs])
    y = 3.5 - F @ J
    E0, Jf = fit(F, y, mask)
    assert abs(E0 - 3.5) < 1e-8
    assert np.max(np.abs(Jf - J)) < 1e-10
    assert np.all(Jf[[t for t in range(8) if not mask[t]]] == 0.0)


def test_fit_satisfies_the_normal_equations_with_noise():
    rng = np.random.default_rng(6)
    xs = [rng.normal(size=(6, 16)) for _ in range(40)]
    F = np.array([features(x, 4, 4, 1.0) for x in xs])
    y = rng.normal(size=40) * 5.0
    mask = [1, 1, 1, 0, 1, 0, 0, 0]
    E0, J = fit(F, y, mask)
    cols = [t for t in range(8) if mask[t]]
    A = np.concatenate([np.ones((40, 1)), -F[:, cols]], axis=1)
    r = y - A @ np.concatenate([[E0], J[cols]])
    assert np.max(np.abs(A.T @ r)) < 1e-8 * np.max(np.abs(A.T @ y))


def test_fit_of_the_bosonic_action_returns_its_coefficients():
    # -dtau S_Bose = -(dtau omega0^2 / 2) sum x^2 - (c_kin / dtau) sum (dx)^2 + dtau lam sum x:
    # at lam = 0 the regression on (Jk, J2) must return J2 = dtau omega0^2 / 2, Jk = c_kin / dtau
    rng = np.random.default_rng(7)
    xs = [rng.normal(size=(10, 9)) for _ in range(30)]
    y = np.array([-0.1 * o.bosonic_action(x, 0.0, 1.3, 0.1, 0.5) for x in xs])
    F = np.array([features(x, 3, 3, 1.0) for x in xs])
    E0, J = fit(F, y, [1, 1, 0, 0, 0, 0, 0, 0])
    assert abs(J[0] - 0.5 / 0.1) < 1e-10 and abs(J[1] - 0.1 * 1.3 ** 2 / 2) < 1e-12 and abs(E0) < 1e-9
