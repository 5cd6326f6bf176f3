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


def _shifted(L, N, s):
    """(psi, W_s - psi I): the generator shifted so that exp stays O(1) at long times."""
    psi = scgf(L, N, s)
    return psi, generator(L, N, s) - psi * np.eye(len(basis(L, N)))


def ln_partition(L, N, s, t):
    """ln Z(s, t) from a uniform start (t >= 0)."""
    if t == 0:
        return 0.0
    psi, A = _shifted(L, N, s)
    n = len(basis(L, N))
    return float(psi * t + np.log(np.full(n, 1.0 / n) @ scipy.linalg.expm(A * t) @ np.ones(n)))


def interval_log_limit(L, N, s, dt, M):
    """The large-population limit of the per-interval log of the cloning
    algorithm: the population after the cloning stage of interval beta - 1 has
    the law q0^T e^{W_s (beta-1) dt} (normalised), so ln of its mean cloning
    factor over interval beta tends to ln Z(s, beta dt) - ln Z(s, (beta-1) dt),
    beta = 1..M (eq. Z-ups)."""
    lz = [ln_partition(L, N, s, b * dt) for b in range(M + 1)]
    return np.diff(np.array(lz))


def _integral_expm(A, t):
    """int_0^t exp(A u) du, from the exponential of [[A, I], [0, 0]] t."""
    n = A.shape[0]
    B = np.zeros((2 * n, 2 * n))
    B[:n, :n] = A
    B[:n, n:] = np.eye(n)
    return scipy.linalg.expm(B * t)[:n, n:]


def interval_mean_hops(L, N, s, dt, M, modified=True):
    """The large-population limit of the population mean of K^beta before the
    cloning stage of interval beta = 1..M: the population starts the interval
    with the law p of interval_log_limit and runs the SSEP with all rates
    times e^{-s} (modified dynamics, Sec. 3.2) or unscaled (direct weights);
    a clone in C makes hops at rate c r(C) (c = e^{-s} or 1), so its expected
    hops are c (int_0^dt e^{c W_0 u} du r)(C)."""
    T, r = _hop_and_rate(L, N)
    n = len(r)
    c = np.exp(-s) if modified else 1.0
    W0 = T - np.diag(r)
    # generator acts on columns (W[C', C]); a function of the end point f
    # evolves as e^{W^T u} f, and W_0 is symmetric
    h = c * (_integral_expm(c * W0, dt) @ r)
    psi, A = _shifted(L, N, s)
    step = scipy.linalg.expm(A * dt)          # columns: from, rows: to
    p = np.full(n, 1.0 / n)
    out = np.empty(M)
    for b in range(M):
        out[b] = (p @ h) / p.sum()
        p = step @ p
        p = p / p.sum()
    return out


def activity_after(L, N, s, t_b, t):
    """The large-population limit of k-hat with the first t_b of t left out:
    the hops in (t_b, t] along the ancestral lines, per site and unit time,
    -d/ds2 ln Z(s1, s2) / (L (t - t_b)) at s1 = s2 = s, where
    Z(s1, s2) = q0^T e^{W_{s1} t_b} e^{W_{s2} (t - t_b)} 1 tilts the two parts
    of the trajectory apart (the Frechet derivative of the exponential gives
    d/ds2 exactly: dW/ds = -e^{-s} T).  t_b = 0 gives -d/ds ln Z(s, t)/(L t)."""
    T, _ = _hop_and_rate(L, N)
    n = T.shape[0]
    psi, A = _shifted(L, N, s)
    tau = t - t_b
    E2, dE2 = scipy.linalg.expm_frechet(A * tau, -np.exp(-s) * T * tau)
    q = np.full(n, 1.0 / n) @ scipy.linalg.expm(A * t_b)
    one = np.ones(n)
    Z = q @ E2 @ one
    dZ = q @ dE2 @ one
    return float(-dZ / Z / (L * tau))
