"""Pins of the oracle's modified Wolff cluster update (SM Sec. IV, Eq. S8; readings
A25, A31-A33).  CPU only.

The pins do not re-type the oracle's bond rule: detailed balance is checked by brute-force
enumeration of every open/closed pattern of the bonds on tiny lattices (the cluster
probabilities of the state and of its reflected state must stand in the ratio of their
effective weights, which holds only for the right bond probability and a complete bond
set), the oracle's random cluster growth is checked against those enumerated
probabilities by sampling, and the energy change of a reflection is checked against the
bonds that cross the cluster's boundary."""

import numpy as np
import pytest

import oracle
from oracle.effective import EffModel, eff_energy
from oracle.wolff import bonds, bond_energy, bond_probability, cluster, reflect, wolff, propose
from oracle.effective import sweep


def _components(N, edges, mask):
    """Component label of every site in the graph of the bonds whose bit is set."""
    parent = list(range(N))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for k, (i, j) in enumerate(edges):
        if (mask >> k) & 1:
            ri, rj = find(i), find(j)
            if ri != rj:
                parent[ri] = rj
    return [find(a) for a in range(N)]


def _cluster_table(N, edges):
    """For every open-bond pattern and seed site: the cluster of the seed as a bit mask."""
    nb = len(edges)
    tab = np.zeros((1 << nb, N), dtype=np.int64)
    for mask in range(1 << nb):
        lab = _components(N, edges, mask)
        for s in range(N):
            tab[mask, s] = sum(1 << a for a in range(N) if lab[a] == lab[s])
    return tab


def _cluster_probs(x, Lx, Ly, m, tab, bl, prob=bond_probability):
    """P(cluster C | x) for every cluster mask C, seed uniform over the sites."""
    N = Lx * Ly
    nb = len(bl)
    p = np.array([prob(bond_energy(x, i, j, J)) for _, i, j, J in bl])
    bits = (np.arange(1 << nb)[:, None] >> np.arange(nb)[None, :]) & 1
    with np.errstate(divide="ignore"):
        lw = np.where(bits == 1, np.log(p)[None, :], np.log1p(-p)[None, :]).sum(axis=1)
    w = np.exp(lw)
    probs = {}
    for s in range(N):
        for C, ww in zip(tab[:, s], w):
            if ww > 0.0:
                probs[int(C)] = probs.get(int(C), 0.0) + ww / N
    return probs


def _sites(C, N):
    return [a for a in range(N) if (C >> a) & 1]


CASES = [
    (2, 2, 3, EffModel(Jk=0.3, J2=0.1, Jp=0.2, a=1.0, Js=(0.45, 0.0, 0.0), Jt=0.05)),
    (2, 2, 2, EffModel(Jk=0.2, J2=0.1, Jp=0.1, Jp6=0.02, a=1.2, Js=(0.3, -0.25, 0.0))),
    (3, 2, 2, EffModel(Jk=0.4, J2=0.2, Js=(0.35, 0.0, 0.0), Jt=0.1)),
]


@pytest.mark.parametrize("Lx,Ly,Ltau,m", CASES)
def test_wolff_exact_detailed_balance_by_enumeration(Lx, Ly, Ltau, m):
    # P(C | x) exp(-E(x)) = P(C | x') exp(-E(x')) with x' = x reflected on C, for every
    # cluster C that can be formed (SM Sec. IV: acceptance one)
    N = Lx * Ly
    bl = bonds(Lx, Ly, m)
    tab = _cluster_table(N, [(i, j) for _, i, j, _ in bl])
    rng = np.random.default_rng(11 + Lx + 10 * Ltau)
    for trial in range(3):
        x = rng.normal(0.0, 1.2, size=(Ltau, N))
        px = _cluster_probs(x, Lx, Ly, m, tab, bl)
        assert abs(sum(px.values()) - 1.0) < 1e-12
        checked = 0
        for C, pc in px.items():
            xr = x.copy()
            reflect(xr, _sites(C, N))
            pr = _cluster_probs(xr, Lx, Ly, m, tab, bl).get(C, 0.0)
            lhs = pc * np.exp(-eff_energy(x, Lx, Ly, m))
            rhs = pr * np.exp(-eff_energy(xr, Lx, Ly, m))
            assert abs(lhs - rhs) <= 1e-12 * max(lhs, rhs), (C, lhs, rhs)
            checked += 1
        assert checked >= 3


def test_wolff_detailed_balance_fails_for_a_wrong_bond_rule():
    # the enumeration is sharp: with the Ising-style rule 1 - exp(-2|e|) (any sign) the
    # same check fails
    Lx, Ly, Ltau, m = CASES[0]
    N = Lx * Ly
    bl = bonds(Lx, Ly, m)
    tab = _cluster_table(N, [(i, j) for _, i, j, _ in bl])
    x = np.random.default_rng(5).normal(0.0, 1.2, size=(Ltau, N))

    def ising(e):
        return float(-np.expm1(-2.0 * abs(e)))
    bad = 0
    px = _cluster_probs(x, Lx, Ly, m, tab, bl, ising)
    for C, pc in px.items():
        xr = x.copy()
        reflect(xr, _sites(C, N))
        pr = _cluster_probs(xr, Lx, Ly, m, tab, bl, ising).get(C, 0.0)
        lhs = pc * np.exp(-eff_energy(x, Lx, Ly, m))
        rhs = pr * np.exp(-eff_energy(xr, Lx, Ly, m))
        bad += abs(lhs - rhs) > 1e-6 * max(lhs, rhs)
    assert bad > 0


def test_wolff_cluster_growth_samples_the_enumerated_distribution():
    # the oracle's random clusters (Philox bond draws, seed draw, growth) against the exact
    # cluster distribution of the same state
    Lx, Ly, Ltau, m = CASES[1]
    N = Lx * Ly
    bl = bonds(Lx, Ly, m)
    tab = _cluster_table(N, [(i, j) for _, i, j, _ in bl])
    x = np.random.default_rng(21).normal(0.0, 1.0, size=(Ltau, N))
    px = _cluster_probs(x, Lx, Ly, m, tab, bl)
    K = 3000
    counts = {}
    for k in range(K):
        sites, s0 = cluster(x, Lx, Ly, m, 977, k, 3, 0)
        assert s0 in sites
        C = sum(1 << a for a in sites)
        counts[C] = counts.get(C, 0) + 1
    assert set(counts) <= set(px)
    for C, pc in px.items():
        n = counts.get(C, 0)
        sd = np.sqrt(K * pc * (1.0 - pc)) + 1.0
        assert abs(n - K * pc) <= 5.0 * sd, (C, n, K * pc)


@pytest.mark.parametrize("Lx,Ly", [(4, 4), (6, 4), (4, 2)])
def test_reflection_energy_change_is_twice_the_boundary_bonds(Lx, Ly):
    m = EffModel(Jk=0.31, J2=0.12, Jp=0.21, Jp6=0.05, a=1.5, Js=(0.11, -0.06, 0.03), Jt=0.07)
    N = Lx * Ly
    rng = np.random.default_rng(Lx * 7 + Ly)
    x = rng.normal(0.0, 1.0, size=(6, N))
    for _ in range(4):
        C = set(rng.choice(N, size=rng.integers(1, N), replace=False).tolist())
        xr = x.copy()
        reflect(xr, sorted(C))
        # the boundary bonds, listed here from E_eff's own bond rule (every site's offsets
        # (1,0),(0,1) / (1,1),(1,-1) / (2,0),(0,2) with Js[0] / Js[1] / Js[2])
        d = 0.0
        for i in range(N):
            ix, iy = i % Lx, i // Lx
            for r, offs in enumerate((((1, 0), (0, 1)), ((1, 1), (1, -1)), ((2, 0), (0, 2)))):
                for dx, dy in offs:
                    j = (ix + dx) % Lx + Lx * ((iy + dy) % Ly)
                    if (i in C) != (j in C):
                        d += -2.0 * m.Js[r] * float(x[:, i] @ x[:, j])
        dE = eff_energy(xr, Lx, Ly, m) - eff_energy(x, Lx, Ly, m)
        assert abs(dE - d) <= 1e-12 * max(1.0, abs(d))
        reflect(xr, sorted(C))
        assert np.array_equal(xr, x)


def test_bonds_skip_self_terms_and_keep_parallel_ones():
    m = EffModel(Js=(0.1, 0.2, 0.3))
    bl = bonds(2, 4, m)
    assert all(i != j for _, i, j, _ in bl)
    # on a length-2 ring the (1,0) offset of sites 0 and 1 gives two bonds between them
    assert sum(1 for _, i, j, _ in bl if {i, j} == {0, 1}) >= 2
    # the (2,0) offset on a length-2 ring is a self term: no bond of type 4
    assert not any(b % 6 == 4 for b, _, _, _ in bl)


def test_propose_orders_sweeps_and_clusters_by_the_coin():
    m = EffModel(Jk=0.3, J2=0.2, Jp=0.1, a=1.0, Js=(0.25, 0.1, 0.0), delta=0.8)
    Lx, Ly, Ltau = 4, 4, 6
    x0 = np.random.default_rng(3).normal(size=(Ltau, Lx * Ly))
    seen = set()
    for prop in range(8):
        from oracle.philox import philox4x32_10
        coin = int(philox4x32_10((0xFFFFFFFF, 0xFFFFFFFE, prop, 1), (77, 0))[0]) < 2 ** 31
        seen.add(coin)
        x = x0.copy()
        acc, sizes = propose(x, Lx, Ly, m, 1, 2, 77, prop, 1)
        y = x0.copy()
        if coin:
            a2 = sweep(y, Lx, Ly, m, 1, 77, prop, 1)
            s2 = wolff(y, Lx, Ly, m, 2, 77, prop, 1)
        else:
            s2 = wolff(y, Lx, Ly, m, 2, 77, prop, 1)
            a2 = sweep(y, Lx, Ly, m, 1, 77, prop, 1)
        assert np.array_equal(x, y) and acc == a2 and sizes == s2
    assert seen == {True, False}
