"""Pins of the oracle's per-interval log, its transient-excluded estimators
and its ancestral lines.

What fixes each expected value (none of it is the oracle's own formula):
  * per interval, as Nc grows, ln((1/Nc) sum_i Ups_i^beta) tends to
    ln Z(s, beta dt) - ln Z(s, (beta-1) dt) (the population after the cloning
    stage of interval beta - 1 has the law q0^T e^{W_s (beta-1) dt}, eq. Z-ups),
    and the population mean of K^beta before cloning to the hops the SSEP
    with rates e^{-s} makes from that law -- both from exact diagonalisation;
  * at s = 0 the uniform law is stationary: every interval's mean K^beta has
    expectation dt 2N(L-N)/(L-1) (the s = 0 activity);
  * with one particle every clone has r = 2 at all times, so with modified
    weights every ln Ups^beta is -2(1 - e^{-s}) dt exactly, selection is the
    identity, and each clone's hops are a Poisson process of rate 2 e^{-s}:
    k_hat_burn has expectation 2 e^{-s}/L over any window;
  * psi_burn tends to (ln Z(s, t) - ln Z(s, t_b)) / (t - t_b) and k_hat_burn
    to -d/ds2 ln Z(s1, s2) / (L (t - t_b)) with the trajectory's parts before
    and after t_b tilted by s1 and s2 (exact diagonalisation and the Frechet
    derivative of the matrix exponential);
  * the population laws of Sec. 2.4 (eq. Opave): for long times the clones
    after the last cloning stage are distributed as v / sum v and their
    ancestors at an earlier time, far from both ends, as v^2 / sum v^2, v the
    dominant eigenvector of the symmetric tilted generator.  Tested on the
    classes of configurations that rotations and reflections of the ring map
    into each other (v is constant on each), across independent runs.

The statistical pins allow for the O(1/Nc) bias of the cloning estimators.
"""
import numpy as np
import pytest

import oracle
from oracle import ed


def runs(L, N, s, Nc, dt, M, seeds, burn_in=0, mode=oracle.MODIFIED):
    out = []
    for r in seeds:
        o = oracle.Oracle(L, N, s, Nc, dt, M=M, seed=r, mode=mode, burn_in=burn_in)
        out.append(o.run(per_interval=True))
    return out


@pytest.mark.parametrize("s", [0.4, -0.3])
def test_interval_log_and_activity_match_ed(s):
    L, N, Nc, dt, M, R = 10, 5, 2000, 0.1, 60, 12
    rs = runs(L, N, s, Nc, dt, M, range(100, 100 + R))
    lb = np.array([r["lbeta"] for r in rs])
    mk = np.array([r["mean_kb"] for r in rs])
    want_l = ed.interval_log_limit(L, N, s, dt, M)
    want_k = ed.interval_mean_hops(L, N, s, dt, M)
    se_l = lb.std(0, ddof=1) / np.sqrt(R)
    se_k = mk.std(0, ddof=1) / np.sqrt(R)
    z_l = np.abs(lb.mean(0) - want_l) / (se_l + 1e-5)
    z_k = np.abs(mk.mean(0) - want_k) / (se_k + 1e-5)
    assert z_l.max() < 5.0, (z_l.max(), np.argmax(z_l))
    assert z_k.max() < 5.0, (z_k.max(), np.argmax(z_k))
    # the transient is resolved: the first and last intervals differ by many s.e.
    assert abs(want_k[0] - want_k[-1]) > 4 * (se_k[0] + se_k[-1])


def test_zero_bias_activity_every_interval():
    L, N, Nc, dt, M, R = 10, 5, 1000, 0.2, 40, 8
    rs = runs(L, N, 0.0, Nc, dt, M, range(300, 300 + R))
    mk = np.array([r["mean_kb"] for r in rs])
    want = dt * 2.0 * N * (L - N) / (L - 1)
    se = mk.std(0, ddof=1) / np.sqrt(R)
    assert np.max(np.abs(mk.mean(0) - want) / se) < 5.0
    assert abs(mk.mean() - want) < 5 * mk.mean(1).std(ddof=1) / np.sqrt(R)
    assert all(np.all(r["lbeta"] == 0.0) for r in rs)


@pytest.mark.parametrize("mode", [oracle.MODIFIED, oracle.DIRECT])
def test_single_particle_window(mode):
    """N = 1: every interval alike; the window beyond burn_in is two intervals
    of dt = 1, so counting one interval too many or too few moves k_hat_burn
    by 50%."""
    L, s, Nc, dt, M, burn = 10, 0.3, 10_000, 1.0, 12, 10
    r = oracle.Oracle(L, 1, s, Nc, dt, M=M, seed=7, mode=mode, burn_in=burn).run(
        per_interval=True)
    if mode == oracle.MODIFIED:
        assert np.allclose(r["lbeta"], -2.0 * (1.0 - np.exp(-s)) * dt, rtol=1e-13, atol=0)
        assert r["psi_burn"] == pytest.approx(-2.0 * (1.0 - np.exp(-s)), rel=1e-13)
    want = 2.0 * np.exp(-s) / L
    # Poisson count: mean Nc 2 e^{-s} (t - t_b); allow 6 s.e. plus the O(1/Nc) bias
    se = want / np.sqrt(Nc * 2.0 * np.exp(-s) * (M - burn) * dt)
    assert abs(r["k_hat_burn"] - want) < 6 * se + 1e-4, (r["k_hat_burn"], want, se)


def test_burn_in_psi_short_window_matches_ed():
    """psi_burn over the three intervals after t_b = 10 (dt = 0.1)."""
    L, N, s, Nc, dt, burn, M, R = 10, 5, 0.4, 1000, 0.1, 100, 103, 16
    rs = runs(L, N, s, Nc, dt, M, range(400, 400 + R), burn_in=burn)
    pb = np.array([r["psi_burn"] for r in rs])
    t, tb = M * dt, burn * dt
    want = (ed.ln_partition(L, N, s, t) - ed.ln_partition(L, N, s, tb)) / (t - tb)
    se = pb.std(ddof=1) / np.sqrt(R)
    assert abs(pb.mean() - want) < 4 * se + 1e-3, (pb.mean(), want, se)


def test_burn_in_estimators_long_window_match_ed():
    """At the L = 10 workload (t_obs = 100) with the first 10 time units left
    out: psi_burn and k_hat_burn against their large-population limits, which
    differ from those of psi-hat and k-hat (the transient of Sec. 5.1)."""
    L, N, s, Nc, dt, burn, M, R = 10, 5, 0.4, 1000, 0.1, 100, 1000, 20
    rs = runs(L, N, s, Nc, dt, M, range(500, 500 + R), burn_in=burn)
    t, tb = M * dt, burn * dt
    pb = np.array([r["psi_burn"] for r in rs])
    kb = np.array([r["k_hat_burn"] for r in rs])
    kf = np.array([r["k_hat"] for r in rs])
    want_p = (ed.ln_partition(L, N, s, t) - ed.ln_partition(L, N, s, tb)) / (t - tb)
    want_k = ed.activity_after(L, N, s, tb, t)
    want_kf = ed.activity_after(L, N, s, 0.0, t)
    se_p = pb.std(ddof=1) / np.sqrt(R)
    se_k = kb.std(ddof=1) / np.sqrt(R)
    assert abs(pb.mean() - want_p) < 4 * se_p + 2e-4, (pb.mean(), want_p, se_p)
    assert abs(kb.mean() - want_k) < 4 * se_k + 2e-4, (kb.mean(), want_k, se_k)
    assert abs(kf.mean() - want_kf) < 4 * kf.std(ddof=1) / np.sqrt(R) + 2e-4
    # the pin can tell psi_burn from psi-hat
    assert abs(want_p - ed.finite_time_scgf(L, N, s, t)) > 5 * se_p + 2e-4


def test_burn_in_activity_short_run_matches_ed():
    """k_hat_burn over (2, 12] against its limit, which lies 4% below that of
    k-hat over (0, 12]: the first two time units from the uniform start are
    more active than the rest."""
    L, N, s, Nc, dt, burn, M, R = 10, 5, 0.4, 2000, 0.1, 20, 120, 40
    rs = runs(L, N, s, Nc, dt, M, range(700, 700 + R), burn_in=burn)
    kb = np.array([r["k_hat_burn"] for r in rs])
    want = ed.activity_after(L, N, s, burn * dt, M * dt)
    other = ed.activity_after(L, N, s, 0.0, M * dt)
    se = kb.std(ddof=1) / np.sqrt(R)
    assert abs(kb.mean() - want) < 4 * se + 2e-4, (kb.mean(), want, se)
    assert abs(kb.mean() - other) > 5 * se


def _orbit_classes(L, N):
    """Class of every configuration of ed.basis(L, N) under the rotations and
    reflections of the ring."""
    states = ed.basis(L, N)
    full = (1 << L) - 1

    def canon(c):
        best = c
        for x in (c, int(format(c, "0%db" % L)[::-1], 2)):
            for k in range(L):
                best = min(best, ((x >> k) | (x << (L - k))) & full)
        return best
    keys = sorted({canon(c) for c in states})
    return np.array([keys.index(canon(c)) for c in states]), len(keys)


@pytest.mark.parametrize("s", [0.4, -0.4])
def test_population_laws(s):
    L, N, Nc, dt, M, beta0, R = 10, 5, 1000, 0.1, 200, 100, 40
    cls, ncls = _orbit_classes(L, N)
    index = {c: k for k, c in enumerate(ed.basis(L, N))}
    _, v = ed.dominant(L, N, s)
    p_end = np.bincount(cls, weights=v / v.sum(), minlength=ncls)
    p_ave = np.bincount(cls, weights=v * v / (v * v).sum(), minlength=ncls)

    def classes(occ):
        words = (occ.astype(np.int64) << np.arange(L)).sum(1)
        return cls[[index[int(w)] for w in words]]
    f_end, f_anc = [], []
    for r in range(R):
        occ0, occ1, org = oracle.Oracle(L, N, s, Nc, dt, M=M, seed=600 + r).run_lineage(beta0)
        f_end.append(np.bincount(classes(occ1), minlength=ncls) / Nc)
        f_anc.append(np.bincount(classes(occ0)[org], minlength=ncls) / Nc)
    for f, want, other in ((np.array(f_end), p_end, p_ave), (np.array(f_anc), p_ave, p_end)):
        m = f.mean(0)
        # across-run s.e., floored at the multinomial s.e. of R independent populations
        se = np.maximum(f.std(0, ddof=1) / np.sqrt(R), np.sqrt(want * (1 - want) / (R * Nc)))
        assert np.max(np.abs(m - want) / se) < 4.5, np.max(np.abs(m - want) / se)
        assert np.max(np.abs(m - other) / se) > 8.0      # v and v^2 are told apart
