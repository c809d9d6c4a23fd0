"""GPU parity of the DQMC comparison updates (SM Sec. I, Eqs. S4-S6): local sweeps with
Sherman-Morrison updates and column block updates, through the C ABI, against the oracle
(which evaluates G after slice l-1 from its definition at every slice) on the same fields
and Philox streams.

Bars (T6): a decision can differ only where |log u - log r_oracle| <= 1e-8; such near-ties
are counted and the fixed seeds here have none, so accept counts are equal and the fields
agree within 1e-13 (a move x + delta (2u - 1) may be one fused multiply-add on the GPU;
a block update is an exact negation, bit for bit).  The final G (evaluated by the
stabilized chain) meets the FP64 bar 1e-9; cached log weights 1e-11 relative."""

import numpy as np
import pytest

import oracle
from synth import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1802_06177_amd as slmc  # noqa: E402

DEV = "cuda:0"


def _md(Lx, Ly, Ltau, n_s, lam=1.5, mu=0.0):
    return dict(Lx=Lx, Ly=Ly, Ltau=Ltau, n_s=n_s, t=1.0, mu=mu, dtau=0.1, lam=lam, omega0=1.0, c_kin=0.5)


def _E(md):
    return oracle.expk(oracle.hopping_matrix(md["Lx"], md["Ly"], md["t"], md["mu"]), md["dtau"])


@pytest.mark.parametrize("Lx,Ly,Ltau,n_s,n_rec,delta,chains", [
    (4, 4, 12, 4, 1, 1.0, 3),      # G evaluated at every slice
    (4, 4, 12, 4, 3, 1.0, 3),      # propagated between evaluations
    (2, 3, 10, 5, 10, 1.5, 2),     # propagated through the whole sweep
    (8, 8, 40, 10, 10, 0.8, 2),
    # above N = 64 the delayed updates: 32 kept (a flush after every 32 accepts and at the
    # end of each slice), 16 at N = 272 where 32 do not fit in LDS
    (10, 10, 8, 4, 4, 0.8, 1),
    (16, 16, 4, 2, 4, 0.8, 1),
    (17, 16, 2, 1, 2, 0.8, 1),
    (21, 21, 2, 1, 2, 0.8, 1),     # the largest lattice (N = 441, LDS rows padded to 448)
])
def test_local_sweep_matches_oracle(Lx, Ly, Ltau, n_s, n_rec, delta, chains):
    md = _md(Lx, Ly, Ltau, n_s, mu=0.05)
    print("case: dqmc sweep %dx%d Ltau=%d n_rec=%d" % (Lx, Ly, Ltau, n_rec), flush=True)
    m = slmc.model_from_dict(md)
    xs = gen(501, Lx * 100 + Ltau + n_rec).normal(0.0, 1.0, size=(chains, Ltau, Lx * Ly))
    xg = torch.tensor(xs, dtype=torch.float64, device=DEV)
    seed, sw = 4321 + Lx, 7
    nacc, st, G = slmc.dqmc_sweep(m, xg, delta, n_rec, seed, sw, want_g=True)
    nacc, st, G, xg = nacc.cpu().numpy(), st.cpu().numpy(), G.cpu().numpy(), xg.cpu().numpy()
    assert np.all(st == 0)
    E = _E(md)
    for c in range(chains):
        xo = xs[c].copy()
        margins = []
        acc, Go = oracle.local_sweep(E, xo, md["dtau"], md["lam"], md["omega0"], md["c_kin"], n_s, delta,
                                     seed, sw, c, margins=margins)
        ties = int(np.sum(np.asarray(margins) <= 1e-8))
        print("  chain %d: accepted %d (oracle %d) of %d, near-ties %d, min margin %.2e" %
              (c, nacc[c], acc, len(margins), ties, min(margins)), flush=True)
        assert ties == 0
        assert int(nacc[c]) == acc and 0 < acc < Ltau * Lx * Ly
        assert np.max(np.abs(xg[c] - xo)) <= 1e-13
        assert np.max(np.abs(G[c] - Go)) <= 1e-9


def test_block_updates_match_oracle():
    md = _md(4, 4, 20, 5, lam=2.0)
    m = slmc.model_from_dict(md)
    E = _E(md)
    xs = gen(502, 0).normal(0.0, 1.0, size=(5, 20, 16))
    lw = np.array([oracle.log_weight(oracle.logdet_green(E, xs[c], 0.1, 2.0, 5)[0], xs[c], 2.0, 1.0, 0.1, 0.5)
                   for c in range(5)])
    xg = torch.tensor(xs, dtype=torch.float64, device=DEV)
    lwg = torch.tensor(lw, dtype=torch.float64, device=DEV)
    seed, sw, nu = 99, 3, 4
    nacc, st = slmc.dqmc_block(m, xg, lwg, nu, seed, sw)
    nacc, st, xg, lwg = nacc.cpu().numpy(), st.cpu().numpy(), xg.cpu().numpy(), lwg.cpu().numpy()
    assert np.all(st == 0)
    tot = 0
    for c in range(5):
        xo = xs[c].copy()
        margins = []
        acc, lwo = oracle.block_updates(E, xo, lw[c], 0.1, 2.0, 1.0, 0.5, 5, nu, seed, sw, c, margins=margins)
        assert int(np.sum(np.asarray(margins) <= 1e-8)) == 0
        assert int(nacc[c]) == acc
        assert np.array_equal(xg[c], xo)
        assert abs(lwg[c] - lwo) <= 1e-11 * abs(lwo)
        tot += acc
    assert 0 < tot < 5 * nu


def test_dqmc_sweep_int8x5_evaluations():
    # the evaluations of G may use the mixed path: decisions as the FP64 oracle's
    md = _md(4, 4, 12, 4)
    m = slmc.model_from_dict(md)
    xs = gen(503, 0).normal(0.0, 1.0, size=(2, 12, 16))
    xg = torch.tensor(xs, dtype=torch.float64, device=DEV)
    nacc, st, G = slmc.dqmc_sweep(m, xg, 1.0, 4, 11, 2, opt=slmc.options("int8x5", 1), want_g=True)
    nacc, G, xg = nacc.cpu().numpy(), G.cpu().numpy(), xg.cpu().numpy()
    E = _E(md)
    for c in range(2):
        xo = xs[c].copy()
        margins = []
        acc, Go = oracle.local_sweep(E, xo, 0.1, 1.5, 1.0, 0.5, 4, 1.0, 11, 2, c, margins=margins)
        assert int(np.sum(np.asarray(margins) <= 1e-6)) == 0
        assert int(nacc[c]) == acc and np.max(np.abs(xg[c] - xo)) <= 1e-13
        assert np.max(np.abs(G[c] - Go)) <= 1e-6
