"""Seeded synthetic inputs and the named workloads.

This module holds no arithmetic of the method: it only generates parameter
sets and random starting populations from explicit seeds, so that the GPU
library and the test oracle can be fed identical inputs.  The workloads
follow the paper's SSEP runs (half filling, scaled bias lambda = s L^2
around lambda_c = 2 pi^2, cloning intervals and observation times of its
runs scaled to the sizes below; arXiv:1711.05095 Secs. 3.3, 4.3, 5, 6).
"""
import numpy as np

# Workload "L=10 parity": CPU-checkable against exact diagonalisation.
SMALL = dict(L=10, N=5, s_values=[round(-0.4 + 0.1 * i, 10) for i in range(9)], Nc=1000,
             dt=0.1, t_obs=100.0, seed0=1000)

# Workload "L=100 transition sweep": 32 scaled biases from -10 to +20.
SWEEP = dict(L=100, N=50, lambdas=[-10.0 + 30.0 * i / 31.0 for i in range(32)],
             Nc_values=[10_000, 100_000], dt=0.5, t_obs=2000.0, seed0=2000)

# Workload "L=400 large": bit-packed 400-site states, 1e6 clones.
LARGE = dict(L=400, N=200, lambdas=[0.0, 10.0, 20.0], Nc=1_000_000, dt=1.0, t_obs=1.0e4,
             seed0=5000)

# Workload "guide": L=100 near the transition.
GUIDE = dict(L=100, N=50, lambdas=[5.0, 10.0, 15.0, 20.0], Nc_train=100_000, Nc_guided=10_000,
             Nc_reference=1_000_000, dt=0.5, t_obs=2000.0, seed0=4000)


def s_of_lambda(lam, L):
    """The paper's scaled bias lambda = s L^2 (eq. def-lambda), inverted."""
    return lam / float(L * L)


def batched_instances(n=64, seed=3000):
    """Uneven batch: L uniform in {20, 40, ..., 200}, N = L/2, lambda uniform
    in [-10, 20], Nc log-uniform in [1e3, 1e5]; dt = 0.5, t_obs = 1000."""
    rng = np.random.Generator(np.random.Philox(seed))
    out = []
    for i in range(n):
        L = int(20 * rng.integers(1, 11))
        lam = float(rng.uniform(-10.0, 20.0))
        Nc = int(10 ** rng.uniform(3.0, 5.0))
        out.append(dict(L=L, N=L // 2, s=s_of_lambda(lam, L), lam=lam, Nc=Nc, dt=0.5,
                        t_obs=1000.0, seed=seed + 1 + i, instance=i))
    return out


def random_population(L, N, Nc, seed):
    """Nc independent uniform N-subsets of L sites: uint8 [Nc, L]."""
    rng = np.random.default_rng(seed)
    occ = np.zeros((Nc, L), np.uint8)
    if N == 0:
        return occ
    keys = rng.random((Nc, L))
    idx = np.argpartition(keys, N - 1, axis=1)[:, :N] if N < L else np.tile(np.arange(L), (Nc, 1))
    np.put_along_axis(occ, idx, 1, axis=1)
    return occ


def random_counts(Nc, seed, high=1000):
    """Accumulated hop counts to carry with a population: uint64 [Nc]."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, high, Nc).astype(np.uint64)


def random_log_weights(Nc, seed, spread=1.0, zeros=0.0):
    """Log cloning factors with a given spread; a fraction `zeros` of the
    clones get a weight 1e-300 times smaller than the rest (never chosen)."""
    rng = np.random.default_rng(seed)
    ell = rng.normal(0.0, spread, Nc)
    if zeros > 0:
        mask = rng.random(Nc) < zeros
        ell[mask] -= 700.0
    return ell


def guide_theta0(seed):
    """Initial parameters of the guide network (flat float32, layout of
    include/pd_guide.h): weights uniform in +-1/sqrt(fan-in), the last layer
    scaled by 0.1 so that the untrained guide is close to flat; biases 0."""
    rng = np.random.default_rng(seed)
    th = np.zeros(5506, np.float32)
    th[0:160] = rng.uniform(-1, 1, 160) / np.sqrt(5.0)
    th[192:5312] = rng.uniform(-1, 1, 5120) / np.sqrt(160.0)
    th[5344:5504] = rng.uniform(-1, 1, 160) / np.sqrt(160.0) * 0.1
    return th
