"""Pins of the oracle's guided dynamics (eqs. modpdef, upsdef of Sec. 2.2).

  * with a constant table the guide is the modified dynamics, so at s = 0
    every weight is exactly 1 and psi-hat is exactly 0;
  * the configuration after one interval follows column C0 of exp(W' t), W'
    the generator of the guided rates (pins the proposal rate and the
    thinning that takes a proposal with probability eg / eg_max);
  * the mean cloning factor over one interval is (e^{W_s dt} 1)(C0) for any
    table (pins the compensating weight);
  * E[e^{t psi-hat}] = Z(s, t) for any table and any population size;
  * with the exact Doob table (built from the dominant eigenvector) the
    weights barely fluctuate: psi-hat varies over seeds far less than with
    the plain method, and sits on (1/t) ln Z.
"""
import numpy as np
import pytest
import scipy.linalg
from scipy import stats

import oracle
from guide_tables import constant_table, doob_table, guided_generator, random_table
from oracle import ed

G = oracle.GUIDED


def test_constant_table_zero_bias_exact():
    r = oracle.Oracle(10, 5, 0.0, 300, 0.1, M=30, seed=2, mode=G, guide=constant_table()).run(
        per_interval=True)
    assert r["psi"] == 0.0 and np.all(r["lbeta"] == 0.0)


@pytest.mark.parametrize("s", [0.5, -0.4])
def test_guided_transition_law(s):
    L, N, dt, Nc = 6, 3, 0.4, 60000
    table = random_table(7)
    c0 = 0b000111
    o = oracle.Oracle(L, N, s, Nc, dt, seed=5, mode=G, guide=table)
    occ = np.tile(np.array([(c0 >> i) & 1 for i in range(L)], np.uint8), (Nc, 1))
    o.step(1, occ, np.zeros(Nc, np.uint64))
    P = scipy.linalg.expm(guided_generator(L, N, s, table) * dt)
    states = ed.basis(L, N)
    law = P[:, states.index(c0)]
    codes = (occ.astype(np.int64) << np.arange(L)).sum(axis=1)
    counts = np.array([np.count_nonzero(codes == c) for c in states])
    chi2 = ((counts - law * Nc) ** 2 / (law * Nc)).sum()
    assert chi2 < stats.chi2.ppf(1 - 1e-6, len(states) - 1)


@pytest.mark.parametrize("s,seed", [(0.4, 1), (-0.3, 2)])
def test_guided_one_interval_mean_weight(s, seed):
    L, N, dt, Nc = 6, 3, 0.5, 200000
    c0 = 0b010101
    o = oracle.Oracle(L, N, s, Nc, dt, seed=seed, mode=G, guide=random_table(seed))
    occ = np.tile(np.array([(c0 >> i) & 1 for i in range(L)], np.uint8), (Nc, 1))
    _, _, ell = o.step(2, occ, np.zeros(Nc, np.uint64))
    ups = np.exp(ell)
    exact = ed.one_interval_weight(L, N, s, dt, c0)
    assert abs(ups.mean() - exact) < 5 * ups.std() / np.sqrt(Nc)


@pytest.mark.parametrize("Nc,s,runs", [(1, 0.5, 30000), (4, -0.5, 20000)])
def test_guided_unbiased_partition_function(Nc, s, runs):
    L, N, dt, M = 6, 3, 0.25, 4
    table = random_table(11)
    vals = np.empty(runs)
    for i in range(runs):
        r = oracle.Oracle(L, N, s, Nc, dt, M=M, seed=50_000 + i, mode=G, guide=table).run()
        vals[i] = np.exp(M * dt * r["psi"])
    Z = ed.partition(L, N, s, M * dt)
    assert abs(vals.mean() - Z) < 5 * vals.std() / np.sqrt(runs), (vals.mean(), Z)


def test_exact_doob_guide_single_clone():
    """With the exact Doob guide a single clone's weight telescopes to
    e^{psi t} v(C_0)/v(C_t): every run gives psi within ln(v_max/v_min)/t,
    while a single clone of the plain method estimates the typical (s = 0)
    activity instead."""
    L, N, s, dt, M, R = 10, 5, 0.3, 0.5, 120, 12
    t = M * dt
    table = doob_table(L, N, s)
    psi, v = ed.dominant(L, N, s)
    bound = np.log(v.max() / v.min()) / t + 1e-3   # + table rounding
    guided = [oracle.Oracle(L, N, s, 1, dt, M=M, seed=700 + i, mode=G, guide=table).run()["psi"]
              for i in range(R)]
    assert np.all(np.abs(np.array(guided) - psi) <= bound), (guided, psi, bound)
    plain = [oracle.Oracle(L, N, s, 1, dt, M=M, seed=700 + i).run()["psi"] for i in range(R)]
    assert abs(np.mean(plain) - psi) > 5 * bound
