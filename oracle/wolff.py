"""Modified Wolff cluster update of the symmetric effective model (oracle; test
infrastructure only).

Paper, SM Sec. IV (Wolff update of the effective Hamiltonian): clusters are grown in the
spatial plane only, each site taking its whole imaginary-time column along, with a bond
probability built from the spatial coupling summed over the column (SM Eq. S8); all
fields of the cluster are then reflected about the symmetry axis.  The effective model is
even under that global reflection, so the move is accepted with probability one.  The
cumulative proposal combines these cluster moves with the local sweeps (the section's last
paragraph).

Readings (listed in the design notes):
  A25 bond probability.  With E_eff of Eq. 4 read as +beta H_eff (reading A12, weight
      exp(-E_eff)), a spatial bond term J sum_tau x_i,tau x_j,tau of E_eff has the bond
      energy e_ij = J sum_tau x_i x_j (build frame: axis at x = 0).  Reflecting a cluster
      that holds i but not j turns e_ij into -e_ij, so the probability of adding j is
      p_ij = 1 - exp(min(0, 2 e_ij)), the continuous-spin (Hasenbusch / Wolff embedding)
      form; the printed exponent carries a dtau and no min, taken as a different
      normalisation of the same coupling.
  A31 bonds.  Every spatial bond term of the effective model is a cluster bond: from each
      site i the offsets (1,0),(0,1) with Js[0], (1,1),(1,-1) with Js[1], (2,0),(0,2) with
      Js[2] (the paper's model has the nearest-neighbour term only; with the further
      terms of the workload, leaving any of them out would make the reflection change
      E_eff).  A term whose two ends are the same site (a length-2 or length-4 ring with
      the (2,0) offset) is even under the reflection and is no bond.  Parallel terms
      between the same two sites are separate bonds with separate draws.
  A32 random numbers.  Philox4x32-10, key (seed low, seed high).  Bond b = 6 i + t
      (t = 0..5 over the six offsets above) of cluster w of a proposal: counter
      (b, 0x80000000 + w, proposal mod 2^32, chain), word 0 -> u; the bond is open iff
      e_ij < 0 and u < -expm1(2 e_ij).  Seed site of cluster w: counter (0xFFFFFFFD,
      0x80000000 + w, proposal, chain), word 0 -> r, seed = floor(r N / 2^32).
      The cluster is the connected component of the seed in the graph of open bonds (the
      same set as the sequential growth that tests each bond once).
  A33 cumulative proposal.  The per-proposal coin of the local sweep (reading A17) also
      orders the cluster moves: forward: n_sweeps sweeps in forward phase order, then
      n_clusters cluster moves; reverse: n_clusters cluster moves, then the sweeps in
      reverse phase order.  Each cluster move and each colour phase satisfies detailed
      balance with exp(-E_eff), so the equal mixture of the two orders is reversible and
      the acceptance of Eq. 6 stays exact.
"""

import numpy as np

from .effective import sweep
from .philox import philox4x32_10, uniform01

OFFSETS = ((1, 0), (0, 1), (1, 1), (1, -1), (2, 0), (0, 2))   # bond type t -> offset
RANGE = (0, 0, 1, 1, 2, 2)                                   # bond type t -> Js index


def bonds(Lx, Ly, m):
    """Cluster bonds of the effective model: list of (bond index 6 i + t, i, j, J)."""
    out = []
    for i in range(Lx * Ly):
        ix, iy = i % Lx, i // Lx
        for t, (dx, dy) in enumerate(OFFSETS):
            J = m.Js[RANGE[t]]
            if J == 0.0:
                continue
            j = (ix + dx) % Lx + Lx * ((iy + dy) % Ly)
            if j != i:
                out.append((6 * i + t, i, j, J))
    return out


def bond_energy(x, i, j, J):
    """e_ij = J sum_tau x[tau, i] x[tau, j] (the bond's share of E_eff)."""
    return J * float(np.dot(x[:, i], x[:, j]))


def bond_probability(e):
    """p = 1 - exp(min(0, 2 e)) (reading A25)."""
    return float(-np.expm1(2.0 * e)) if e < 0.0 else 0.0


def _key(seed):
    return (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def cluster(x, Lx, Ly, m, seed, proposal_idx, chain, w, margins=None):
    """Sites of cluster w of a proposal (sorted list) and its seed site.  If `margins` is a
    list, |u - p| of every bond with p > 0 is appended (for counting near-ties)."""
    N = Lx * Ly
    key = _key(seed)
    pr = proposal_idx & 0xFFFFFFFF
    r = int(philox4x32_10((0xFFFFFFFD, 0x80000000 + w, pr, chain), key)[0])
    s0 = (r * N) >> 32
    nbr = [[] for _ in range(N)]
    for b, i, j, J in bonds(Lx, Ly, m):
        p = bond_probability(bond_energy(x, i, j, J))
        if p <= 0.0:
            continue
        u = float(uniform01(philox4x32_10((b, 0x80000000 + w, pr, chain), key)[0]))
        if margins is not None:
            margins.append(abs(u - p))
        if u < p:
            nbr[i].append(j)
            nbr[j].append(i)
    seen = {s0}
    todo = [s0]
    while todo:
        i = todo.pop()
        for j in nbr[i]:
            if j not in seen:
                seen.add(j)
                todo.append(j)
    return sorted(seen), s0


def reflect(x, sites):
    """x[:, i] -> -x[:, i] for every site of the cluster (axis at 0), in place."""
    for i in sites:
        x[:, i] = -x[:, i]


def wolff(x, Lx, Ly, m, n_clusters, seed, proposal_idx, chain, margins=None):
    """n_clusters cluster moves of one chain, in place; returns the cluster sizes."""
    sizes = []
    for w in range(n_clusters):
        sites, _ = cluster(x, Lx, Ly, m, seed, proposal_idx, chain, w, margins)
        reflect(x, sites)
        sizes.append(len(sites))
    return sizes


def propose(x, Lx, Ly, m, n_sweeps, n_clusters, seed, proposal_idx, chain, margins=None):
    """The cumulative proposal of one chain, in place (reading A33): local sweeps and
    cluster moves in the order the proposal's coin picks.  Returns (accepted local moves,
    cluster sizes)."""
    key = _key(seed)
    coin = int(philox4x32_10((0xFFFFFFFF, 0xFFFFFFFE, proposal_idx & 0xFFFFFFFF, chain), key)[0])
    if coin < 2 ** 31:
        acc = sweep(x, Lx, Ly, m, n_sweeps, seed, proposal_idx, chain, margins)
        sizes = wolff(x, Lx, Ly, m, n_clusters, seed, proposal_idx, chain, margins)
    else:
        sizes = wolff(x, Lx, Ly, m, n_clusters, seed, proposal_idx, chain, margins)
        acc = sweep(x, Lx, Ly, m, n_sweeps, seed, proposal_idx, chain, margins)
    return acc, sizes
