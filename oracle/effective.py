"""Symmetric effective boson model and its local Metropolis sweep (oracle; test
infrastructure only).

Paper, Eq. (4) (= SM Eq. S7): the effective model is a polynomial in the phonon field
with a time-kinetic term J_k, two symmetric double-well functions
    f4(y) = y^4/4 - alpha^2 y^2/2,   f6(y) = y^6/6 - alpha^2 y^4/4   (Fig. 1, SM Sec. III),
with y = X - alpha, spatial nearest-neighbour products J_nn and temporal
nearest-neighbour products J'_nn; it is invariant under the mirror y -> -y.  The
simulation proposes moves with cheap local updates on this model (main text, "SLMC";
SM Sec. IV, last paragraph).

Build frame and readings:
  A1  y = x (axis at 0); the wells sit at +-a with a = lam/omega0^2;
  A12 the printed coefficients are those of +beta H_eff = E_eff and the weight is
      exp(-E_eff) (the printed minus sign in front of beta H_eff is taken as garbled);
  A14 the workload adds an on-site x^2 term (J2) and spatial couplings out to the third
      neighbour: Js[0] for offsets (1,0),(0,1); Js[1] for (1,1),(1,-1); Js[2] for
      (2,0),(0,2); every bond is counted once, from the site it starts at;
  A16 checkerboard colouring: spatial colour (ix mod m) + m (iy mod m) with m = 2 when the
      spatial range is at most the diagonal neighbour, m = 4 (else 3) with third
      neighbours, m | Lx and m | Ly required; temporal colour l mod 2 (Ltau even);
      phase p = spatial colour + m^2 * temporal colour, P = 2 m^2 phases;
  A17 per proposal a coin picks the forward (0..P-1) or the reverse (P-1..0) phase order
      for all its sweeps, which makes the proposal reversible;
  A19 a move is x -> x + delta (2 u1 - 1) accepted when log u2 < -dE.

Random numbers: Philox4x32-10 with key (seed low 32 bits, seed high 32 bits) and
counter (site = i + N l, sweep index, proposal index mod 2^32, chain) -> words 0, 1;
coin: counter (0xFFFFFFFF, 0xFFFFFFFE, proposal, chain) word 0, forward iff < 2^31.
"""

from dataclasses import dataclass, field

import numpy as np

from .philox import philox4x32_10, uniform01

BONDS = (((1, 0), (0, 1)), ((1, 1), (1, -1)), ((2, 0), (0, 2)))


@dataclass
class EffModel:
    Jk: float = 0.0
    J2: float = 0.0
    Jp: float = 0.0
    Jp6: float = 0.0
    a: float = 0.0
    Js: tuple = (0.0, 0.0, 0.0)
    Jt: float = 0.0
    delta: float = 0.5


def _f4(y, a):
    return 0.25 * y ** 4 - 0.5 * a * a * y ** 2


def _f6(y, a):
    return y ** 6 / 6.0 - 0.25 * a * a * y ** 4


def _shift(x, Lx, Ly, dx, dy):
    """s[l, i] = x[l, i + (dx, dy)] on the periodic lattice."""
    Ltau = x.shape[0]
    g = x.reshape(Ltau, Ly, Lx)
    g = np.roll(g, shift=(-dy, -dx), axis=(1, 2))
    return g.reshape(Ltau, Lx * Ly)


def eff_energy(x, Lx, Ly, m):
    """E_eff[x] of Eq. (4) in the build frame (reading A12: the weight is exp(-E_eff))."""
    x = np.asarray(x, dtype=np.float64)
    xn = np.roll(x, -1, axis=0)
    e = m.Jk * np.sum((xn - x) ** 2)
    e += m.J2 * np.sum(x * x)
    e += m.Jp * np.sum(_f4(x, m.a))
    e += m.Jp6 * np.sum(_f6(x, m.a))
    for r in range(3):
        if m.Js[r] != 0.0:
            for dx, dy in BONDS[r]:
                e += m.Js[r] * np.sum(x * _shift(x, Lx, Ly, dx, dy))
    e += m.Jt * np.sum(x * xn)
    return float(e)


def _site(ix, iy, Lx, Ly):
    return (ix % Lx) + Lx * (iy % Ly)


def eff_local_delta(x, Lx, Ly, m, i, l, xnew):
    """E_eff(x with x[l,i] -> xnew) - E_eff(x), from the terms that touch (i, l)."""
    Ltau = x.shape[0]
    xo = x[l, i]
    xp = x[(l + 1) % Ltau, i]
    xm = x[(l - 1) % Ltau, i]
    d = xnew - xo
    de = m.Jk * ((xp - xnew) ** 2 - (xp - xo) ** 2 + (xnew - xm) ** 2 - (xo - xm) ** 2)
    de += m.J2 * (xnew * xnew - xo * xo)
    de += m.Jp * (_f4(xnew, m.a) - _f4(xo, m.a))
    de += m.Jp6 * (_f6(xnew, m.a) - _f6(xo, m.a))
    ix, iy = i % Lx, i // Lx
    for r in range(3):
        if m.Js[r] != 0.0:
            s = 0.0
            for dx, dy in BONDS[r]:
                s += x[l, _site(ix + dx, iy + dy, Lx, Ly)] + x[l, _site(ix - dx, iy - dy, Lx, Ly)]
            de += m.Js[r] * d * s
    de += m.Jt * d * (xp + xm)
    return float(de)


def colouring(Lx, Ly, Ltau, m):
    """(mod, phase[l, i], P) of the checkerboard decomposition (reading A16)."""
    if Ltau % 2:
        raise ValueError("Ltau must be even for the temporal colouring")
    rng = 3 if m.Js[2] != 0.0 else (2 if m.Js[1] != 0.0 else (1 if m.Js[0] != 0.0 else 0))
    if rng == 0:
        cands = (1,)
    elif rng <= 2:
        cands = (2, 3)
    else:
        cands = (4, 3)
    mod = next((c for c in cands if Lx % c == 0 and Ly % c == 0), None)
    if mod is None:
        raise ValueError("no colouring modulus divides the lattice")
    ph = np.zeros((Ltau, Lx * Ly), dtype=np.int64)
    for l in range(Ltau):
        for i in range(Lx * Ly):
            ix, iy = i % Lx, i // Lx
            ph[l, i] = (ix % mod) + mod * (iy % mod) + mod * mod * (l % 2)
    return mod, ph, 2 * mod * mod


def sweep(x, Lx, Ly, m, n_sweeps, seed, proposal_idx, chain, margins=None):
    """n_sweeps checkerboard Metropolis sweeps of one chain, in place (SM Sec. IV, last
    paragraph: local updates over the space-time lattice).  Sites are visited one at a
    time, phase by phase, in increasing site order inside a phase.  Returns the number of
    accepted moves.  If `margins` is a list, the decision margin log u2 + dE of every
    visited site is appended to it (for counting near-ties; it changes nothing else)."""
    Ltau, N = x.shape
    _, ph, P = colouring(Lx, Ly, Ltau, m)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    pr = proposal_idx & 0xFFFFFFFF
    coin = int(philox4x32_10((0xFFFFFFFF, 0xFFFFFFFE, pr, chain), key)[0])
    order = list(range(P)) if coin < 2 ** 31 else list(range(P - 1, -1, -1))
    members = [[] for _ in range(P)]
    for l in range(Ltau):
        for i in range(N):
            members[ph[l, i]].append((i + N * l, i, l))
    for p in members:
        p.sort()
    acc = 0
    for s in range(n_sweeps):
        for p in order:
            for site, i, l in members[p]:
                w = philox4x32_10((site, s, pr, chain), key)
                u1 = float(uniform01(w[0]))
                u2 = float(uniform01(w[1]))
                xn = x[l, i] + m.delta * (2.0 * u1 - 1.0)
                de = eff_local_delta(x, Lx, Ly, m, i, l, xn)
                if margins is not None:
                    margins.append(float(np.log(u2) + de))
                if np.log(u2) < -de:
                    x[l, i] = xn
                    acc += 1
    return acc
