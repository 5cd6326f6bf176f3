"""Test infrastructure: exact diagonalisation of the tilted SSEP generator.

For a periodic ring of L sites with N particles, the configurations are the
C(L, N) L-bit words with N set bits (bit i = occupancy of site i).  The tilted
generator of the activity K (arXiv:1711.05095, Sec. 2.1 eqs. psi-z, psi-mean;
Sec. 3.1) is

    W_s[C', C] = e^{-s} * (number of bonds whose hop takes C to C'),
    W_s[C, C]  = -r(C),

with r(C) the number of bonds (i, i+1 mod L) whose sites differ.  It is
symmetric, so

    psi(s)        = largest eigenvalue of W_s,
    -psi'(s)      = e^{-s} v^T T v / v^T v   (Hellmann-Feynman; T = hop part),
    Z(s, t)       = q0^T exp(W_s t) 1,  q0 uniform over configurations,

and the cloning estimator's large-population limit at finite t_obs is
(1/t_obs) ln Z(s, t_obs).
"""
from functools import lru_cache
from math import comb

import numpy as np
import scipy.linalg


@lru_cache(maxsize=None)
def basis(L, N):
    """Sorted L-bit words with N set bits."""
    out = [c for c in range(1 << L) if bin(c).count("1") == N]
    assert len(out) == comb(L, N)
    return tuple(out)


def escape_rate(c, L):
    return sum(((c >> i) & 1) != ((c >> ((i + 1) % L)) & 1) for i in range(L))


@lru_cache(maxsize=None)
def _hop_and_rate(L, N):
    states = basis(L, N)
    index = {c: k for k, c in enumerate(states)}
    n = len(states)
    T = np.zeros((n, n))
    r = np.zeros(n)
    for k, c in enumerate(states):
        for i in range(L):
            j = (i + 1) % L
            if ((c >> i) & 1) != ((c >> j) & 1):
                T[index[c ^ (1 << i) ^ (1 << j)], k] += 1.0
                r[k] += 1.0
    return T, r


def generator(L, N, s):
    """W_s as a dense matrix over basis(L, N)."""
    T, r = _hop_and_rate(L, N)
    return np.exp(-s) * T - np.diag(r)


def scgf(L, N, s):
    """psi(s): the largest eigenvalue of W_s."""
    return float(np.linalg.eigvalsh(generator(L, N, s))[-1])


def dominant(L, N, s):
    """(psi, v) with v the positive normalised dominant eigenvector."""
    w, V = np.linalg.eigh(generator(L, N, s))
    v = V[:, -1]
    v = v * np.sign(v.sum())
    return float(w[-1]), v


def activity(L, N, s):
    """-psi'(s) = lim <K_t / t>_s by Hellmann-Feynman."""
    T, _ = _hop_and_rate(L, N)
    _, v = dominant(L, N, s)
    return float(np.exp(-s) * (v @ T @ v) / (v @ v))


def partition(L, N, s, t):
    """Z(s, t) = <e^{-s K_t}>_0 from a uniform start, by the matrix exponential."""
    n = len(basis(L, N))
    q0 = np.full(n, 1.0 / n)
    return float(q0 @ scipy.linalg.expm(generator(L, N, s) * t) @ np.ones(n))


def partition_spectral(L, N, s, t):
    """Z(s, t) by the spectral sum over all eigenpairs (a second route)."""
    w, V = np.linalg.eigh(generator(L, N, s))
    n = len(w)
    q0 = np.full(n, 1.0 / n)
    return float(np.sum(np.exp(w * t) * (q0 @ V) * (V.T @ np.ones(n))))


def finite_time_scgf(L, N, s, t):
    """(1/t) ln Z(s, t): what psi-hat estimates at t_obs = t as Nc -> infinity.
    Evaluated as psi + (1/t) ln(q0^T e^{(W_s - psi) t} 1) so that it does not
    underflow at long times."""
    psi = scgf(L, N, s)
    n = len(basis(L, N))
    q0 = np.full(n, 1.0 / n)
    shifted = generator(L, N, s) - psi * np.eye(n)
    return float(psi + np.log(q0 @ scipy.linalg.expm(shifted * t) @ np.ones(n)) / t)


def one_interval_weight(L, N, s, dt, c0):
    """E[Upsilon over one interval | start in configuration c0] = (e^{W_s dt} 1)(c0)."""
    states = basis(L, N)
    n = len(states)
    row = scipy.linalg.expm(generator(L, N, s).T * dt)  # (e^{W^T dt})[c0, :] = e^{W dt}[:, c0]
    k0 = states.index(c0)
    return float(row[k0] @ np.ones(n))


def transition_law(L, N, rate_scale, dt, c0):
    """Law of the configuration after time dt of the (unbiased) SSEP with all
    rates multiplied by rate_scale, started from c0: column c0 of
    exp(rate_scale * W_0 * dt)."""
    states = basis(L, N)
    P = scipy.linalg.expm(generator(L, N, 0.0) * rate_scale * dt)
    return P[:, states.index(c0)]
