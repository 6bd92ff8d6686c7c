"""Exact enumeration of the periodic 2x2x2 Ising lattice -- TEST INFRASTRUCTURE ONLY.

Everything here is computed from the Hamiltonian (eq. 1) by brute force over
the 2^8 states, independently of the rate table of the C oracle:

* site i = x + 2 (y + 2 z); the neighbour of i along axis e is i with bit e of
  its coordinates toggled, and each of the 6 neighbour slots counts, so every
  distinct pair appears twice in B = sum_i sum_e s_i s_(i+e) (multiplicity).
* the flip energy change of site s is E(state with s flipped) - E(state).
* Glauber rate 1 / (1 + exp(beta dE)), Metropolis min(1, exp(-beta dE)).

Closed forms returned:
* ``boltzmann``  -- exp(-beta E) / Z: the stationary law of the serial BKL
  dynamics, and of the spkMC cycle when R_max spans all octants.
* ``spkmc_active`` -- the stationary law of the spkMC cycle with R_max taken
  over the active octant only: with one domain of eight single-site octants the
  drawn site always fires, so the jump chain is the uniform walk on the 8-cube
  and the mean holding time in a state is (1/64) sum_s 1/r_s; the time-weighted
  law is proportional to sum_s 1/r_s(state).
"""
import math

import numpy as np


def coords(i):
    return i & 1, (i >> 1) & 1, (i >> 2) & 1


def spins_of(state):
    return np.array([1 if (state >> i) & 1 else -1 for i in range(8)], dtype=np.int64)


def energy(sp, J, H):
    B = 0
    for i in range(8):
        for e in range(3):
            B += sp[i] * sp[i ^ (1 << e)]
    M = int(sp.sum())
    return -J * B - H * M, M, B


def flip_rate(dE, beta, rates):
    if rates == 0:
        return 1.0 / (1.0 + math.exp(beta * dE))
    return 1.0 if dE <= 0 else math.exp(-beta * dE)


def tables(J, H, T, rates=0):
    beta = 1.0 / T
    E = np.zeros(256)
    M = np.zeros(256)
    w_boltz = np.zeros(256)
    w_active = np.zeros(256)
    for st in range(256):
        sp = spins_of(st)
        e0, m0, _ = energy(sp, J, H)
        E[st] = e0
        M[st] = m0
        inv = 0.0
        for s in range(8):
            sp2 = sp.copy()
            sp2[s] = -sp2[s]
            e1, _, _ = energy(sp2, J, H)
            inv += 1.0 / flip_rate(e1 - e0, beta, rates)
        w_active[st] = inv
    w_boltz = np.exp(-beta * (E - E.min()))
    return E, M, w_boltz / w_boltz.sum(), w_active / w_active.sum()


def averages(J, H, T, rates=0):
    """Exact <E>, <|M|>, <M^2> under both stationary laws."""
    E, M, pb, pa = tables(J, H, T, rates)
    out = {}
    for name, p in (("boltzmann", pb), ("spkmc_active", pa)):
        out[name] = {"E": float(p @ E), "absM": float(p @ np.abs(M)), "M2": float(p @ M ** 2),
                     "p": p}
    return out


def cycle_law(J, H, T, rates=0, colours=8, scope=0):
    """Exact time-weighted stationary law of the spkMC cycle on the periodic
    2x2x2 lattice with domain edge 2 (one domain, eight single-site octants).

    A cycle draws a colour uniformly: one site (8 colours) or the four sites of
    one parity of x + y + z (2 colours, never neighbours of one another).  Every
    active site fires independently with probability r_s / R, where R is the
    largest rate among the active sites (scope 0), among all eight sites
    (scope 1), or the largest rate any site can have (scope 2: the largest
    single-flip rate over every state of the lattice).  The cycle lasts
    Exp(1) / (S R) with S the number of colours.  The jump chain's stationary
    law, weighted by the mean cycle length in each state, is the law of the
    state at a random time."""
    beta = 1.0 / T
    E = np.zeros(256)
    rate = np.zeros((256, 8))
    for st in range(256):
        sp = spins_of(st)
        e0, _, _ = energy(sp, J, H)
        E[st] = e0
        for s in range(8):
            sp2 = sp.copy()
            sp2[s] = -sp2[s]
            e1, _, _ = energy(sp2, J, H)
            rate[st, s] = flip_rate(e1 - e0, beta, rates)
    rbound = rate.max()
    if colours == 8:
        groups = [[s] for s in range(8)]
    else:
        groups = [[s for s in range(8) if bin(s).count("1") % 2 == c] for c in (0, 1)]
    P = np.zeros((256, 256))
    hold = np.zeros(256)
    for st in range(256):
        for grp in groups:
            if scope == 0:
                R = max(rate[st, s] for s in grp)
            elif scope == 1:
                R = rate[st].max()
            else:
                R = rbound
            hold[st] += (1.0 / len(groups)) / (colours * R)
            probs = [rate[st, s] / R for s in grp]
            for mask in range(1 << len(grp)):
                pr = 1.0
                nxt = st
                for b, s in enumerate(grp):
                    if (mask >> b) & 1:
                        pr *= probs[b]
                        nxt ^= 1 << s
                    else:
                        pr *= 1.0 - probs[b]
                P[st, nxt] += pr / len(groups)
    w, v = np.linalg.eig(P.T)
    pi = np.real(v[:, np.argmin(np.abs(w - 1.0))])
    pi = pi / pi.sum()
    pt = pi * hold
    return pt / pt.sum()
