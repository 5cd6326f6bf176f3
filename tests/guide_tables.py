"""Guide tables for tests: eg[u] over 13-site bond neighbourhoods u (site b-6
in bit 0, the bond's own sites in bits 6 and 7), zero where the bond is not an
allowed hop.  Built from definitions or from exact diagonalisation."""
import numpy as np

from oracle import ed


def allowed(u):
    return ((u >> 6) & 1) != ((u >> 7) & 1)


def constant_table(value=1 << 16):
    t = np.zeros(8192, np.uint32)
    for u in range(8192):
        if allowed(u):
            t[u] = value
    return t


def random_table(seed, lo=1 << 15, hi=1 << 17):
    rng = np.random.default_rng(seed)
    t = np.zeros(8192, np.uint32)
    for u in range(8192):
        if allowed(u):
            t[u] = rng.integers(lo, hi)
    return t


def window13(bits, L, b):
    """Neighbourhood of bond b in a configuration given as an int (bit i = site i)."""
    u = 0
    for o in range(13):
        site = (b - 6 + o) % L
        u |= ((bits >> site) & 1) << o
    return u


def guided_generator(L, N, s, table):
    """Generator of the guided dynamics: hop across allowed bond b at rate
    e^{-s} table[u_b] 2^-16."""
    states = ed.basis(L, N)
    index = {c: k for k, c in enumerate(states)}
    n = len(states)
    Wg = np.zeros((n, n))
    for k, c in enumerate(states):
        for b in range(L):
            b2 = (b + 1) % L
            if ((c >> b) & 1) != ((c >> b2) & 1):
                rate = np.exp(-s) * float(table[window13(c, L, b)]) * 2.0**-16
                Wg[index[c ^ (1 << b) ^ (1 << b2)], k] += rate
                Wg[k, k] -= rate
    return Wg


def doob_table(L, N, s):
    """eg = 2^16 v(C after the hop)/v(C) with v the dominant eigenvector of the
    tilted generator; representable exactly (up to rounding) when L <= 13,
    since the neighbourhood then covers the whole ring."""
    assert L <= 13
    _, v = ed.dominant(L, N, s)
    states = ed.basis(L, N)
    index = {c: k for k, c in enumerate(states)}
    t = np.zeros(8192, np.uint32)
    for c in states:
        for b in range(L):
            b2 = (b + 1) % L
            if ((c >> b) & 1) != ((c >> b2) & 1):
                c2 = c ^ (1 << b) ^ (1 << b2)
                t[window13(c, L, b)] = int(round(2.0**16 * v[index[c2]] / v[index[c]]))
    return t
