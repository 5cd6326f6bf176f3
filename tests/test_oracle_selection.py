"""Pins of the oracle's cloning stage ([eq] and [iid] selection, Sec. 4.1).

Independent of the oracle's floating-point code:
  * exact rational arithmetic (fractions.Fraction) locates the interval of the
    cumulative line that holds each point (the definition in eq. alpha-Ups and
    the number-line picture of Fig. Key); only points within rounding of an
    interval end may differ;
  * a systematic-resampling property: clone k gets floor or ceil of
    Nc Ups_k / Ups_T copies, and the counts sum to Nc;
  * the selection requirement (mean copies = Nc Ups_k / Ups_T), by averaging
    over a fine grid of offsets d, or over many iid draws;
  * equal weights give the identity map for every d (Sec. 4.3: at s = 0 the
    [eq] method deletes no clone), even for offsets at the ends of (0, 1).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1711_05095_amd import inputs


def _exact_ends(ell):
    """Interval ends y_k in units of the spacing, as exact rationals, from the
    weights exp(ell - max) rounded to doubles."""
    w = np.exp(np.asarray(ell) - np.max(ell))
    acc = Fraction(0)
    C = []
    for x in w:
        acc += Fraction(float(x))
        C.append(acc)
    T = C[-1]
    n = len(w)
    return [c * n / T for c in C]


def _check_against_exact(anc, ends, points):
    n = len(ends)
    ambiguous = 0
    for j, pt in enumerate(points):
        pt = Fraction(pt)
        k = int(anc[j])
        lo = ends[k - 1] if k > 0 else Fraction(0)
        hi = ends[k] if k < n - 1 else Fraction(10**30)
        if lo <= pt < hi:
            continue
        # allowed only when the point sits within rounding of an interval end
        near = min(abs(pt - lo), abs(pt - ends[min(k, n - 1)]))
        assert near <= Fraction(1, 10**9) * max(1, abs(pt)), (j, k, float(pt))
        ambiguous += 1
    return ambiguous


@pytest.mark.parametrize("seed,spread,zeros", [(1, 0.5, 0.0), (2, 3.0, 0.0), (3, 1.0, 0.3)])
@pytest.mark.parametrize("d", [0.5, 2.0**-53, 1 - 2.0**-53, 0.123456789])
def test_eq_matches_exact_intervals(seed, spread, zeros, d):
    Nc = 257
    ell = inputs.random_log_weights(Nc, seed, spread, zeros)
    anc, lm = oracle.select(ell, d=d)
    assert np.all(np.diff(anc) >= 0)
    ends = _exact_ends(ell)
    amb = _check_against_exact(anc, ends, [j + Fraction(d) for j in range(Nc)])
    assert amb <= 2
    w = np.exp(ell - ell.max())
    assert lm == pytest.approx(ell.max() + np.log(w.sum() / Nc), rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("seed", range(5))
def test_eq_offspring_floor_or_ceil(seed):
    Nc = 1000
    ell = inputs.random_log_weights(Nc, seed, 1.5, 0.1)
    d = np.random.default_rng(seed).random()
    anc, _ = oracle.select(ell, d=d)
    counts = np.bincount(anc, minlength=Nc)
    assert counts.sum() == Nc
    w = np.exp(ell - ell.max())
    mean = Nc * w / w.sum()
    assert np.all(counts >= np.floor(mean - 1e-9)) and np.all(counts <= np.ceil(mean + 1e-9))


def test_eq_unbiased_over_offset():
    Nc = 50
    ell = inputs.random_log_weights(Nc, 17, 2.0)
    grid = (np.arange(4000) + 0.5) / 4000
    tot = np.zeros(Nc)
    for d in grid:
        anc, _ = oracle.select(ell, d=d)
        tot += np.bincount(anc, minlength=Nc)
    w = np.exp(ell - ell.max())
    # a grid of G offsets reproduces the mean to within 1/G per interval end
    assert np.allclose(tot / len(grid), Nc * w / w.sum(), atol=2.0 / len(grid))


@pytest.mark.parametrize("Nc", [1, 2, 1000, 1_000_000])
@pytest.mark.parametrize("d", [2.0**-53, 0.5, 1 - 2.0**-53])
def test_equal_weights_identity(Nc, d):
    for value in (0.0, -0.0, -3.25):
        anc, lm = oracle.select(np.full(Nc, value), d=d)
        assert np.array_equal(anc, np.arange(Nc, dtype=np.int32))
        assert lm == value


def test_iid_matches_exact_intervals_and_is_unbiased():
    Nc = 200
    ell = inputs.random_log_weights(Nc, 4, 1.0, 0.2)
    rng = np.random.default_rng(5)
    ends = _exact_ends(ell)
    w = np.exp(ell - ell.max())
    tot = np.zeros(Nc)
    R = 3000
    for r in range(R):
        pts = rng.random(Nc) * Nc
        anc, _ = oracle.select(ell, points=pts)
        if r < 3:
            assert _check_against_exact(anc, ends, [Fraction(float(p)) for p in pts]) <= 2
        tot += np.bincount(anc, minlength=Nc)
    mean = Nc * w / w.sum()
    se = np.sqrt(mean * (1 - w / w.sum()) / R)
    assert np.all(np.abs(tot / R - mean) <= 6 * se + 1e-12)


def test_resample_pulls_state_and_count():
    L, N, Nc = 12, 5, 300
    o = oracle.Oracle(L, N, 0.3, Nc, 0.5, seed=12)
    occ = inputs.random_population(L, N, Nc, 2)
    K = inputs.random_counts(Nc, 3)
    ell = inputs.random_log_weights(Nc, 4, 1.0)
    occ2, K2, anc, lm = o.resample(7, occ, K, ell)
    assert np.array_equal(occ2, occ[anc]) and np.array_equal(K2, K[anc])
    anc_ref, lm_ref = oracle.select(ell, d=o.eq_offset(7))
    assert np.array_equal(anc, anc_ref) and lm == lm_ref
    d = o.eq_offset(7)
    assert 0.0 < d < 1.0
    assert o.eq_offset(8) != d
