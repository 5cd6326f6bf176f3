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
