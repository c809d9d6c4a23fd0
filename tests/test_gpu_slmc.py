"""GPU parity of the SLMC proposal and acceptance: effective energy (Eq. 4), checkerboard
Metropolis sweeps of the effective model (SM Sec. III, local updates), the full log-weight
(SM Eq. S2) and the cumulative-update acceptance (Eq. 6), through the C ABI, against the
oracle on the same seeded inputs.

Bars: energies and log-weights to 1e-12 / 1e-11 relative; sweep fields to 1e-12 absolute
with identical per-chain accept counts (a decision can only differ on an exact tie of
log u against -dE, which has probability ~1e-13 per site); accept decisions identical."""

import numpy as np
import pytest

import oracle
from oracle.effective import EffModel
from synth import gen, eff_coefficients, physical_eff

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1802_06177_amd as slmc  # noqa: E402

DEV = "cuda:0"

FULL = dict(Jk=0.31, J2=0.12, Jp=0.21, Jp6=0.05, a=1.5, Js=(0.11, -0.06, 0.03), Jt=0.07, delta=0.7)
NN_ONLY = dict(Jk=0.4, J2=0.2, Jp=0.15, Jp6=0.0, a=1.2, Js=(0.2, 0.1, 0.0), Jt=0.0, delta=0.9)


def _md(Lx, Ly, Ltau, n_s=10, lam=1.5):
    return dict(Lx=Lx, Ly=Ly, Ltau=Ltau, n_s=n_s, t=1.0, mu=0.0, dtau=0.1, lam=lam,
                omega0=1.0, c_kin=0.5)


def _pair(d):
    d = dict(d)
    return EffModel(**{**d, "Js": tuple(d["Js"])}), slmc.eff_model(**d)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _E(md):
    return oracle.expk(oracle.hopping_matrix(md["Lx"], md["Ly"], md["t"], md["mu"]), md["dtau"])


# ------------------------------------------------------------------------- energy

@pytest.mark.parametrize("Lx,Ly,Ltau,coef", [(4, 4, 8, "full"), (6, 6, 10, "full"),
                                             (12, 12, 120, "seeded"), (16, 16, 160, "full"),
                                             (8, 4, 6, "nn")])
def test_eff_energy_matches_oracle(Lx, Ly, Ltau, coef):
    print("case: energy %dx%dx%d %s" % (Lx, Ly, Ltau, coef), flush=True)
    d = {"full": FULL, "nn": NN_ONLY, "seeded": eff_coefficients(3, 0, 1.5, delta=0.5)}[coef]
    om, em = _pair(d)
    m = slmc.model(Lx, Ly, Ltau, 1)
    g = gen(201, Lx * 1000 + Ltau)
    xs = g.normal(0.0, 1.2, size=(5, Ltau, Lx * Ly))
    e = slmc.eff_energy(m, em, _dev(xs)).cpu().numpy()
    for c in range(len(xs)):
        ref = oracle.eff_energy(xs[c], Lx, Ly, om)
        assert abs(e[c] - ref) <= 1e-12 * max(1.0, abs(ref)), (c, e[c], ref)


# ------------------------------------------------------------------------- sweeps

def _coins(seed, prop, chains):
    from oracle.philox import philox4x32_10
    key = (seed & 0xFFFFFFFF, seed >> 32)
    return [int(philox4x32_10((0xFFFFFFFF, 0xFFFFFFFE, prop & 0xFFFFFFFF, c), key)[0]) < 2 ** 31
            for c in range(chains)]


@pytest.mark.parametrize("Lx,Ly,Ltau,coef,n_sw,chains", [
    (4, 4, 8, "full", 3, 6),        # colouring modulus 4, field in LDS
    (6, 6, 10, "full", 2, 4),       # modulus 3
    (8, 4, 6, "nn", 2, 4),          # modulus 2 (no third-neighbour coupling)
    (16, 16, 80, "full", 1, 2),     # 160 KB field: updated in place in global memory
    (12, 12, 120, "seeded", 1, 2),  # the 12x12 workload shape
])
def test_sweep_matches_oracle(Lx, Ly, Ltau, coef, n_sw, chains):
    print("case: sweep %dx%dx%d %s sweeps=%d chains=%d" % (Lx, Ly, Ltau, coef, n_sw, chains),
          flush=True)
    d = {"full": FULL, "nn": NN_ONLY, "seeded": eff_coefficients(3, 0, 1.5, delta=0.8)}[coef]
    om, em = _pair(d)
    m = slmc.model(Lx, Ly, Ltau, 1)
    seed = (0x9E3779B97F4A7C15 + Lx) & ((1 << 64) - 1)
    prop = (5 << 32) + 17 + Ltau          # only the low 32 bits enter the counter
    g = gen(202, Lx * 1000 + Ltau)
    xs = g.normal(0.0, 1.0, size=(chains, Ltau, Lx * Ly))
    xg = _dev(xs)
    nacc = slmc.eff_sweep(m, em, xg, n_sw, seed, prop).cpu().numpy()
    xg = xg.cpu().numpy()
    for c in range(chains):
        xo = xs[c].copy()
        acc = oracle.sweep(xo, Lx, Ly, om, n_sw, seed, prop, c)
        assert int(nacc[c]) == acc, (c, int(nacc[c]), acc)
        assert 0 < acc < n_sw * Lx * Ly * Ltau
        assert np.max(np.abs(xg[c] - xo)) <= 1e-12


def test_sweep_uses_both_phase_orders():
    # the coin picks the forward or the reversed phase order per (proposal, chain); the
    # sweep test above covers both directions on its chains
    c = _coins((0x9E3779B97F4A7C15 + 4) & ((1 << 64) - 1), (5 << 32) + 25, 6)
    assert any(c) and not all(c)


def test_sweep_zero_sweeps_is_identity_and_counts_zero():
    om, em = _pair(FULL)
    m = slmc.model(4, 4, 8, 1)
    xs = gen(203, 0).normal(size=(2, 8, 16))
    xg = _dev(xs)
    nacc = slmc.eff_sweep(m, em, xg, 0, 1, 2).cpu().numpy()
    assert np.array_equal(xg.cpu().numpy(), xs) and np.all(nacc == 0)


# ------------------------------------------------------------------------- weight + accept

@pytest.mark.parametrize("Lx,Ltau,n_s", [(4, 40, 10), (8, 80, 10)])
def test_log_weight_matches_oracle(Lx, Ltau, n_s):
    md = _md(Lx, Lx, Ltau, n_s)
    m = slmc.model_from_dict(md)
    E = _E(md)
    xs = gen(204, Lx).normal(0.0, 1.0, size=(4, Ltau, Lx * Lx))
    lw = slmc.log_weight(m, _dev(xs)).cpu().numpy()
    for c in range(len(xs)):
        ld = oracle.logdet_green(E, xs[c], md["dtau"], md["lam"], n_s)[0]
        ref = oracle.log_weight(ld, xs[c], md["lam"], md["omega0"], md["dtau"], md["c_kin"])
        assert abs(lw[c] - ref) <= 1e-11 * abs(ref), (c, lw[c], ref)


def test_cumulative_accept_matches_oracle_12x12():
    # 12x12, Ltau = 120, n_s = 10; proposals at several distances from the current field so
    # that both decisions occur
    md = _md(12, 12, 120, 10)
    m = slmc.model_from_dict(md)
    om, em = _pair(eff_coefficients(3, 0, 1.5, delta=0.5))
    E = _E(md)
    g = gen(205, 0)
    eps = [1e-3, 3e-3, 1e-2, 3e-1]
    xc = g.normal(0.0, 1.0, size=(4, 120, 144))
    xp = xc + np.array(eps)[:, None, None] * g.normal(size=xc.shape)
    seed, prop = 77, 3
    ref = []
    lw0, ee0 = np.empty(4), np.empty(4)
    for c in range(4):
        ld = oracle.logdet_green(E, xc[c], 0.1, 1.5, 10)[0]
        lw0[c] = oracle.log_weight(ld, xc[c], 1.5, 1.0, 0.1, 0.5)
        ee0[c] = oracle.eff_energy(xc[c], 12, 12, om)
        ref.append(oracle.cumulative_accept(E, 12, 12, 0.1, 1.5, 1.0, 0.5, 10, om, xc[c], xp[c],
                                            lw0[c], ee0[c], seed, prop, c))
    decisions = [r[0] for r in ref]
    assert any(decisions) and not all(decisions), decisions
    xg, lwg, eeg = _dev(xc), _dev(lw0), _dev(ee0)
    G = torch.empty((4, 144, 144), dtype=torch.float64, device=DEV)
    acc, lr = slmc.cumulative_accept(m, em, xg, _dev(xp), lwg, eeg, seed, prop, G_prop=G)
    acc, lr = acc.cpu().numpy(), lr.cpu().numpy()
    xg, lwg, eeg, G = xg.cpu().numpy(), lwg.cpu().numpy(), eeg.cpu().numpy(), G.cpu().numpy()
    for c in range(4):
        a, log_r, lwp, eep = ref[c]
        assert bool(acc[c]) == a
        assert abs(lr[c] - log_r) <= 1e-11 * (abs(lwp) + abs(lw0[c])), (c, lr[c], log_r)
        if a:
            assert np.array_equal(xg[c], xp[c])
            assert abs(lwg[c] - lwp) <= 1e-11 * abs(lwp) and abs(eeg[c] - eep) <= 1e-11 * abs(eep)
        else:
            assert np.array_equal(xg[c], xc[c]) and lwg[c] == lw0[c] and eeg[c] == ee0[c]
        rG = oracle.logdet_green(E, xp[c], 0.1, 1.5, 10)[2]
        assert np.max(np.abs(G[c] - rG)) <= 1e-9


def test_slmc_chain_two_proposals_12x12():
    # full proposal loop on the 12x12 workload shape: copy, one sweep of the effective
    # model, cumulative accept -- twice, GPU against the oracle, fields compared at the end
    md = _md(12, 12, 120, 10)
    m = slmc.model_from_dict(md)
    om, em = _pair(physical_eff(0.1, 1.0, 0.5, delta=0.3))
    E = _E(md)
    chains, seed = 2, 4242
    xs = gen(206, 0).normal(0.0, 0.3, size=(chains, 120, 144))
    xo = xs.copy()
    lwo, eeo = np.empty(chains), np.empty(chains)
    for c in range(chains):
        ld = oracle.logdet_green(E, xo[c], 0.1, 1.5, 10)[0]
        lwo[c] = oracle.log_weight(ld, xo[c], 1.5, 1.0, 0.1, 0.5)
        eeo[c] = oracle.eff_energy(xo[c], 12, 12, om)
    xg, lwg, eeg = _dev(xs), _dev(lwo), _dev(eeo)
    xpg = torch.empty_like(xg)
    for k in range(2):
        xpg.copy_(xg)
        slmc.eff_sweep(m, em, xpg, 1, seed, k)
        acc, _ = slmc.cumulative_accept(m, em, xg, xpg, lwg, eeg, seed, k)
        acc = acc.cpu().numpy()
        for c in range(chains):
            xp = xo[c].copy()
            oracle.sweep(xp, 12, 12, om, 1, seed, k, c)
            a, _, lwp, eep = oracle.cumulative_accept(E, 12, 12, 0.1, 1.5, 1.0, 0.5, 10, om, xo[c], xp,
                                                      lwo[c], eeo[c], seed, k, c)
            assert bool(acc[c]) == a, (k, c)
            if a:
                xo[c], lwo[c], eeo[c] = xp, lwp, eep
    assert np.max(np.abs(xg.cpu().numpy() - xo)) <= 1e-12
    assert np.allclose(lwg.cpu().numpy(), lwo, rtol=1e-11, atol=0)
