"""Pins of the observable definitions (closed forms, exact enumeration)."""
import itertools
from math import comb

import numpy as np
import pytest

from oracle import observables as ob


def test_zero_mode_is_n_squared_over_l():
    occ = np.zeros((3, 12), np.uint8)
    occ[0, :5] = 1
    occ[1, ::3] = 1
    occ[2, [0, 7]] = 1
    assert np.allclose(ob.density_mode(occ, 0), [25 / 12, 16 / 12, 4 / 12])


@pytest.mark.parametrize("L,N,n", [(10, 5, 1), (11, 3, 2), (12, 6, 5)])
def test_uniform_average_closed_form(L, N, n):
    """Average over all C(L, N) configurations: N (L - N) / (L (L - 1)) for
    n != 0 mod L (the pair correlation of a uniform N-subset is -1/(L-1))."""
    rows = []
    for S in itertools.combinations(range(L), N):
        r = np.zeros(L, np.uint8)
        r[list(S)] = 1
        rows.append(r)
    occ = np.array(rows)
    assert len(occ) == comb(L, N)
    assert ob.density_mode(occ, n).mean() == pytest.approx(N * (L - N) / (L * (L - 1)), rel=1e-12)


@pytest.mark.parametrize("L,N,n,shift", [(20, 7, 1, 0), (50, 25, 1, 13), (33, 10, 3, 5)])
def test_compact_cluster_closed_form(L, N, n, shift):
    occ = np.zeros((1, L), np.uint8)
    occ[0, [(shift + i) % L for i in range(N)]] = 1
    want = (np.sin(np.pi * n * N / L) / np.sin(np.pi * n / L)) ** 2 / L
    assert ob.density_mode(occ, n)[0] == pytest.approx(want, rel=1e-12)


def test_means():
    v = np.array([1.0, 2.0, 4.0, 8.0])
    assert ob.population_mean(v) == 3.75
    assert ob.ancestral_mean(v, [0, 0, 3, 3]) == 4.5
    assert ob.ancestral_mean(v, [0, 1, 2, 3]) == 3.75


def test_histogram_unit_bins_of_integers():
    """Integers 0..99 in bins of width 1 starting at -0.5: one count each;
    bins past the data stay empty."""
    counts = ob.histogram(np.arange(100.0), -0.5, 1.0, 120)
    assert counts.dtype == np.uint64
    assert np.array_equal(counts[:100], np.ones(100, np.uint64)) and counts[100:].sum() == 0


def test_histogram_edges_and_exclusions():
    """A value at lo falls in bin 0, one at lo + nbins * width is out, as are
    values below lo and NaN; a bin holds its lower edge, not its upper."""
    v = [2.0, 2.25, 2.5, 2.75, 3.0 - 1e-12, 3.0, 1.9999, float("nan"), 2.5 - 1e-12]
    counts = ob.histogram(v, 2.0, 0.25, 4)
    assert counts.tolist() == [1, 2, 1, 2]


def test_histogram_matches_numpy_away_from_edges():
    """Random values (none within 1e-9 of an edge) binned as numpy's
    histogram bins them, and the counts sum to the values in range."""
    rng = np.random.default_rng(3)
    v = rng.normal(0.3, 1.1, 20000)
    lo, width, nb = -2.0, 0.125, 40
    t = (v - lo) / width
    v = v[np.abs(t - np.round(t)) > 1e-9]
    counts = ob.histogram(v, lo, width, nb)
    ref, _ = np.histogram(v, bins=nb, range=(lo, lo + nb * width))
    assert np.array_equal(counts, ref.astype(np.uint64))
    assert counts.sum() == np.count_nonzero((v >= lo) & (v < lo + nb * width))


def test_histogram_through_origins_counts_descendants():
    """Ancestral form: a value recorded per slot, taken at each clone's origin:
    the histogram weighs each ancestor by its descendant count."""
    values = np.array([0.5, 1.5, 2.5, 3.5])
    origin = np.array([0, 0, 0, 2, 2, 3])
    counts = ob.histogram(values, 0.0, 1.0, 4, origin=origin)
    assert counts.tolist() == [3, 0, 2, 1]
