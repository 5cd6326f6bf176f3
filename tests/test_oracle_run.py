"""Pins of the oracle's whole algorithm (Sec. 2.3, eq. psihat, eq. khat).

  * unbiasedness: for ANY population size, E[prod_beta (1/Nc) sum_i Ups_i^beta]
    = Z(s, t) exactly (the identity behind eq. Z-ups with unbiased selection),
    so the mean of exp(t psi-hat) over many independent runs must match the
    exact-diagonalisation Z within its standard error, for [eq] and [iid],
    modified and direct weights; the same holds for the product over the
    first b intervals of the per-interval log, against Z(s, b dt);
  * s = 0 with modified dynamics: every weight is exactly 1, [eq] is the
    identity, psi-hat is exactly 0 (Sec. 4.3);
  * N = 1: r = 2 always, psi-hat = 2(e^{-s} - 1) up to rounding;
  * at s = 0, k-hat estimates 2N(L-N)/((L-1)L);
  * at the L = 10 workload, psi-hat over seeds sits within 3 sigma of the
    finite-time target (1/t_obs) ln Z(s, t_obs) from exact diagonalisation.
"""
import numpy as np
import pytest

import oracle
from oracle import ed
from paper_1711_05095_amd import inputs


@pytest.mark.parametrize("mode", [oracle.MODIFIED, oracle.DIRECT])
def test_zero_bias_exact(mode):
    o = oracle.Oracle(10, 5, 0.0, 500, 0.1, M=50, seed=3, mode=mode)
    r = o.run(per_interval=True)
    assert r["psi"] == 0.0 and np.all(r["lbeta"] == 0.0)


def test_single_particle():
    s = 0.3
    r = oracle.Oracle(10, 1, s, 300, 0.1, M=100, seed=4).run()
    assert r["psi"] == pytest.approx(2 * (np.exp(-s) - 1), abs=1e-12)


def test_zero_bias_activity():
    L, N = 10, 5
    ks = [oracle.Oracle(L, N, 0.0, 1000, 0.1, M=200, seed=100 + i).run()["k_hat"]
          for i in range(8)]
    exact = 2.0 * N * (L - N) / ((L - 1) * L)
    assert abs(np.mean(ks) - exact) < 4 * np.std(ks) / np.sqrt(len(ks)) + 1e-3


@pytest.mark.parametrize("Nc,s,mode,sel,runs", [
    (1, 0.5, oracle.MODIFIED, oracle.SEL_EQ, 40000),
    (2, -0.5, oracle.DIRECT, oracle.SEL_EQ, 30000),
    (8, -0.5, oracle.MODIFIED, oracle.SEL_EQ, 20000),
    (8, 0.5, oracle.MODIFIED, oracle.SEL_IID, 20000),
    (8, 0.5, oracle.DIRECT, oracle.SEL_EQ, 20000),
])
def test_unbiased_partition_function(Nc, s, mode, sel, runs):
    """Also interval by interval: the product of the first b per-interval
    means, exp(lbeta_1 + ... + lbeta_b), is unbiased for Z(s, b dt) for every
    b, so the per-interval log is pinned at s != 0 too."""
    L, N, dt, M = 6, 3, 0.25, 4
    t = M * dt
    vals = np.empty(runs)
    prefix = np.empty((runs, M))
    for i in range(runs):
        r = oracle.Oracle(L, N, s, Nc, dt, M=M, seed=10_000 + i, mode=mode,
                          selection=sel).run(per_interval=True)
        vals[i] = np.exp(t * r["psi"])
        prefix[i] = np.exp(np.cumsum(r["lbeta"]))
    Z = ed.partition(L, N, s, t)
    se = vals.std() / np.sqrt(runs)
    assert abs(vals.mean() - Z) < 5 * se, (vals.mean(), Z, se)
    for b in range(1, M + 1):
        Zb = ed.partition(L, N, s, b * dt)
        seb = prefix[:, b - 1].std() / np.sqrt(runs)
        assert abs(prefix[:, b - 1].mean() - Zb) < 5 * seb, (b, prefix[:, b - 1].mean(), Zb, seb)


@pytest.mark.parametrize("s", [-0.4, 0.2, 0.4])
def test_small_workload_matches_ed(s):
    w = inputs.SMALL
    M = int(round(w["t_obs"] / w["dt"]))
    psis = []
    for r in range(8):
        o = oracle.Oracle(w["L"], w["N"], s, w["Nc"], w["dt"], M=M, seed=w["seed0"] + r)
        psis.append(o.run()["psi"])
    target = ed.finite_time_scgf(w["L"], w["N"], s, w["t_obs"])
    sigma = np.std(psis, ddof=1)
    assert abs(np.mean(psis) - target) < 3 * sigma / np.sqrt(len(psis)) + 2e-4, (
        np.mean(psis), target, sigma)
