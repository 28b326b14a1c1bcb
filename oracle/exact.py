"""Exact references for tiny replica lattices.  TEST INFRASTRUCTURE ONLY.

Only tests/ may import this module.  Everything is FP64 numpy, written from
the paper's definitions, and independent of both the C oracle
(ee_oracle.c) and the HIP path:

* ``log_z_bruteforce``  -- log Z_n(l) (or at a ramp position m) by summing
  exp(-H/T) over every configuration (Sec. 3, replica Hamiltonian).
* ``log_z_transfer``    -- the same by a transfer matrix along Euclidean
  time, with the cut between t=0 and t=1 (Sec. 3, Fig. "cut along the links
  of the dual lattice").
* ``log_z_kaufman``     -- the textbook closed form of the 2D Ising torus
  (Kaufman 1949), used to pin the two above: Z_n(0) = Z^n (no glued link)
  and, when every column is glued, the n replicas form one torus of time
  extent n*Lt.
* ``exact_protocol``    -- exact propagation of the joint distribution of
  (configuration, integer work) through the non-equilibrium protocol with
  exact Metropolis kernels (App. A: work on phi_k, then a transition at
  lambda_{k+1}; the discretised average of exp(-W)).  Jarzynski's equality
  must hold for every N when the start is the equilibrium distribution.

Conventions (same reading of the paper as the C oracle): the +t bond of
(r,0,y,x) goes to ((r+1)%n,1,y,x) for x<l, is ramped for x==l (intra weight
N-m, inter weight m, in units of beta/N) and stays in replica r otherwise.
The whole-region protocol (Sec. 3) ramps the bonds of every x < l instead and
glues none.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BULK, INTRA, INTER = 0, 1, 2


@dataclass(frozen=True)
class Lattice:
    dim: int
    lt: int
    lx: int
    ly: int
    n: int
    l: int  # noqa: E741  (paper notation: size of region A)

    @property
    def nsites(self) -> int:
        return self.n * self.lt * self.ly * self.lx

    def index(self, r: int, t: int, y: int, x: int) -> int:
        return ((r * self.lt + t) * self.ly + y) * self.lx + x


def bonds(lat: Lattice, glued_upto: int | None = None, ramp: bool = True, whole: bool = False):
    """Bond list [(a, b, kind, y)] of the replica lattice (y: the row of the bond).

    ``glued_upto`` overrides l for the glued columns x < glued_upto; with
    ``ramp=False`` no column is ramped (a pure geometry A(glued_upto)).
    ``whole=True``: the columns x < l are all ramped and none is glued.
    """
    if whole:
        out = []
        for r in range(lat.n):
            for t in range(lat.lt):
                for y in range(lat.ly):
                    for x in range(lat.lx):
                        s = lat.index(r, t, y, x)
                        out.append((s, lat.index(r, t, y, (x + 1) % lat.lx), BULK, y))
                        if lat.dim == 3:
                            out.append((s, lat.index(r, t, (y + 1) % lat.ly, x), BULK, y))
                        if t == 0 and x < lat.l:
                            out.append((s, lat.index(r, 1, y, x), INTRA, y))
                            out.append((s, lat.index((r + 1) % lat.n, 1, y, x), INTER, y))
                        else:
                            out.append((s, lat.index(r, (t + 1) % lat.lt, y, x), BULK, y))
        return out
    l = lat.l if glued_upto is None else glued_upto
    out = []
    for r in range(lat.n):
        for t in range(lat.lt):
            for y in range(lat.ly):
                for x in range(lat.lx):
                    s = lat.index(r, t, y, x)
                    out.append((s, lat.index(r, t, y, (x + 1) % lat.lx), BULK, y))
                    if lat.dim == 3:
                        out.append((s, lat.index(r, t, (y + 1) % lat.ly, x), BULK, y))
                    if t == 0 and x < l:
                        out.append((s, lat.index((r + 1) % lat.n, 1, y, x), BULK, y))
                    elif t == 0 and x == l and ramp:
                        out.append((s, lat.index(r, 1, y, x), INTRA, y))
                        out.append((s, lat.index((r + 1) % lat.n, 1, y, x), INTER, y))
                    else:
                        out.append((s, lat.index(r, (t + 1) % lat.lt, y, x), BULK, y))
    return out


def weights(kinds: np.ndarray, N: int, m: int) -> np.ndarray:
    w = np.full(kinds.shape, float(N))
    w[kinds == INTRA] = N - m
    w[kinds == INTER] = m
    return w


def _all_spins(nsites: int) -> np.ndarray:
    states = np.arange(1 << nsites, dtype=np.int64)
    bits = (states[:, None] >> np.arange(nsites)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8)  # bit 1 -> spin +1


def log_z_bruteforce(lat: Lattice, beta: float, N: int = 1, m: int = 0,
                     glued_upto: int | None = None, ramp: bool = True) -> float:
    """log sum_sigma exp(-H/T), H/T = -(beta/N) sum_b w_b s_a s_b."""
    if lat.nsites > 22:
        raise ValueError("brute force limited to 22 spins")
    b = bonds(lat, glued_upto, ramp)
    a = np.array([x[0] for x in b])
    c = np.array([x[1] for x in b])
    w = weights(np.array([x[2] for x in b]), N, m)
    S = _all_spins(lat.nsites).astype(np.float64)
    e = (S[:, a] * S[:, c]) @ w * (beta / N)  # -H/T
    mx = e.max()
    return float(mx + math.log(np.exp(e - mx).sum()))


def log_z_transfer(lat: Lattice, beta: float, N: int = 1, m: int = 0,
                   glued_upto: int | None = None, ramp: bool = True) -> float:
    """Transfer matrix along t.  A plane state holds the n*Ly*Lx spins of one
    time slice of every replica; T_t[a, b] = exp(in-plane couplings of a +
    couplings between plane t (state a) and plane t+1 (state b))."""
    l = lat.l if glued_upto is None else glued_upto
    P = lat.n * lat.ly * lat.lx
    if P > 13:
        raise ValueError("plane too large for the transfer matrix")
    S = _all_spins(P).astype(np.float64)  # [state, p], p = (r*Ly + y)*Lx + x

    def p_of(r, y, x):
        return (r * lat.ly + y) * lat.lx + x

    # in-plane bonds: +x and (3D) +y, coupling beta
    e_plane = np.zeros(1 << P)
    for r in range(lat.n):
        for y in range(lat.ly):
            for x in range(lat.lx):
                e_plane += S[:, p_of(r, y, x)] * S[:, p_of(r, y, (x + 1) % lat.lx)]
                if lat.dim == 3:
                    e_plane += S[:, p_of(r, y, x)] * S[:, p_of(r, (y + 1) % lat.ly, x)]
    e_plane *= beta

    # plain time links: same replica, coupling beta
    same = np.zeros((P, P))
    for p in range(P):
        same[p, p] = 1.0
    # cut links between t=0 (lower) and t=1 (upper)
    cut = np.zeros((P, P))
    for r in range(lat.n):
        for y in range(lat.ly):
            for x in range(lat.lx):
                lo = p_of(r, y, x)
                if x < l:
                    cut[lo, p_of((r + 1) % lat.n, y, x)] += 1.0
                elif x == l and ramp:
                    cut[lo, p_of(r, y, x)] += (N - m) / N
                    cut[lo, p_of((r + 1) % lat.n, y, x)] += m / N
                else:
                    cut[lo, p_of(r, y, x)] += 1.0

    def tmat(coup):
        # exponent[a, b] = e_plane[a] + beta * sum_{p,q} coup[p,q] s_a[p] s_b[q]
        ex = e_plane[:, None] + beta * (S @ coup @ S.T)
        return ex

    ex_bulk = tmat(same)
    ex_cut = tmat(cut)
    # Tr(T_cut T_bulk^(Lt-1)) with running log scale
    shift_b = ex_bulk.max()
    Tb = np.exp(ex_bulk - shift_b)
    shift_c = ex_cut.max()
    M = np.exp(ex_cut - shift_c)
    log_scale = shift_c
    for _ in range(lat.lt - 1):
        M = M @ Tb
        s = M.max()
        M /= s
        log_scale += shift_b + math.log(s)
    return float(log_scale + math.log(np.trace(M)))


def log_z_kaufman(rows: int, cols: int, K: float) -> float:
    """Exact log Z of the 2D Ising model on a rows x cols torus, coupling K
    (Kaufman, Phys. Rev. 76 (1949) 1232)."""
    def gamma(k):
        if k == 0:
            return 2.0 * K + math.log(math.tanh(K))
        c = math.cosh(2 * K) / math.tanh(2 * K) - math.cos(math.pi * k / cols)
        return math.acosh(c)

    g_odd = [gamma(2 * r + 1) for r in range(cols)]
    g_even = [gamma(2 * r) for r in range(cols)]
    # the four products, in log form with explicit signs
    terms = []
    for gs, fn in ((g_odd, "cosh"), (g_odd, "sinh"), (g_even, "cosh"), (g_even, "sinh")):
        lg, sign = 0.0, 1.0
        for g in gs:
            v = rows * g / 2.0
            if fn == "cosh":
                lg += math.log(2 * math.cosh(v))
            else:
                sv = 2 * math.sinh(v)
                if sv == 0.0:
                    lg, sign = -math.inf, 0.0
                    break
                lg += math.log(abs(sv))
                sign *= math.copysign(1.0, sv)
        terms.append((lg, sign))
    mx = max(t[0] for t in terms if t[1] != 0.0)
    tot = sum(s * math.exp(lg - mx) for lg, s in terms if s != 0.0)
    return (rows * cols / 2.0) * math.log(2 * math.sinh(2 * K)) - math.log(2.0) + mx + math.log(tot)


# ---------------------------------------------------------------------------
# Exact propagation of the protocol
# ---------------------------------------------------------------------------

def _site_coords(lat: Lattice):
    out = []
    for r in range(lat.n):
        for t in range(lat.lt):
            for y in range(lat.ly):
                for x in range(lat.lx):
                    out.append((r, t, y, x))
    return out


def exact_protocol(lat: Lattice, beta: float, N: int, start: str = "equilibrium",
                   n_therm: int = 0, reverse: bool = False, subsets: bool = False, whole: bool = False):
    """Exact distribution of the integer work I over trajectories.

    start='equilibrium': phi_0 ~ pi at the starting ramp position.
    start='hot': every spin +-1 with probability 1/2, then n_therm exact
    Metropolis sweeps at the starting ramp position.

    Each protocol step k: I += D_k(phi_k) where D_k is minus the change of the
    integer energy (units of beta/N) when the ramp moves to its next position,
    then one sweep (colour 0, then colour 1, single-site Metropolis kernels
    with acceptance min(1, exp(-Delta H/T))) at the new position.

    subsets=True is protocol 2 of App. B: the Ly rows of the ramped column
    move one after the other, row y during steps [y S, (y+1) S), S = N/Ly,
    with weights in units of beta/S (W = -(beta/S) I).

    whole=True is the whole-region protocol of Sec. 3: the cut links of every
    x < l move together, from n decoupled replicas to A(l).

    Returns (values, probs): the support of I and its probabilities.
    """
    ns = lat.nsites
    if ns > 20:
        raise ValueError("exact propagation limited to 20 spins")
    b = bonds(lat, whole=whole)
    ba = np.array([x[0] for x in b])
    bb = np.array([x[1] for x in b])
    bk = np.array([x[2] for x in b])
    by = np.array([x[3] for x in b])
    S = _all_spins(ns).astype(np.int64)
    nstates = 1 << ns
    pair = S[:, ba] * S[:, bb]  # [state, bond]
    if subsets and N % lat.ly:
        raise ValueError("protocol 2 needs N divisible by Ly")
    unit = N // lat.ly if subsets else N  # weights in units of beta/unit

    def wvec(pos):
        m = np.clip(pos - by * unit, 0, unit) if subsets else np.full(by.shape, pos)
        w = np.full(bk.shape, unit, dtype=np.int64)
        w[bk == INTRA] = (unit - m)[bk == INTRA]
        w[bk == INTER] = m[bk == INTER]
        return w

    def energy_units(m):
        return -(pair @ wvec(m))  # H/T = (beta/unit) * energy_units

    def m_of(k):  # ramp position after step k (k=-1: start)
        return N - (k + 1) if reverse else k + 1

    coords = _site_coords(lat)
    colour = np.array([(t + y + x) & 1 for (_, t, y, x) in coords])
    idx = np.arange(nstates)

    def sweep(P, m):
        E = energy_units(m).astype(np.float64)
        for c in (0, 1):
            for i in np.nonzero(colour == c)[0]:
                flipped = idx ^ (1 << int(i))
                dE = (E[flipped] - E) * (beta / unit)
                acc = np.minimum(1.0, np.exp(-dE))  # acceptance from each state
                # P has shape [nI, nstates]
                P = P * (1.0 - acc)[None, :] + (P * acc[None, :])[:, flipped]
        return P

    m0 = m_of(-1)
    # bound on |D_k|: two per ramped (replica, row, column) that moves in one step
    Dmax = 2 * lat.n * (1 if subsets else lat.ly) * (lat.l if whole else 1)
    nI = 2 * Dmax * N + 1
    off = Dmax * N
    P = np.zeros((nI, nstates))
    if start == "equilibrium":
        e = -energy_units(m0) * (beta / unit)
        p = np.exp(e - e.max())
        P[off] = p / p.sum()
    elif start == "hot":
        P[off] = 1.0 / nstates
        for _ in range(n_therm):
            P = sweep(P, m0)
    else:
        raise ValueError(start)
    for k in range(N):
        mk, mk1 = m_of(k - 1), m_of(k)
        D = -(energy_units(mk1) - energy_units(mk))  # integer, per state
        Q = np.zeros_like(P)
        for d in np.unique(D):
            sel = D == d
            if d >= 0:
                Q[d:, sel] += P[: nI - d, sel]
            else:
                Q[: nI + d, sel] += P[-d:, sel]
        P = sweep(Q, mk1)
    probs = P.sum(axis=1)
    vals = np.arange(nI) - off
    keep = probs > 0
    return vals[keep], probs[keep]


def jarzynski_average(vals: np.ndarray, probs: np.ndarray, beta: float, N: int) -> float:
    """<exp(-W)> with W = -(beta/N) I."""
    return float(np.sum(probs * np.exp(beta * vals / N)))
