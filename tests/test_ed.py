"""Pins of the exact-diagonalisation checker against closed forms.

Each test fixes a value the mathematics determines without diagonalising:
  * N = 1: the lone particle is a rate-2 random walk, K ~ Poisson(2t), so
    Z = exp(2t(e^{-s} - 1)) and psi = 2(e^{-s} - 1) exactly;
  * s = 0: W_0 is a stochastic generator, psi(0) = 0, Z(0, t) = 1;
  * psi'(0) = -(mean activity) = -2N(L-N)/(L-1) for the uniform steady state
    at fixed N (arXiv:1711.05095 Sec. 3.1 gives the large-L form 2L rho(1-rho));
  * particle-hole symmetry psi(L, N) = psi(L, L-N);
  * Hellmann-Feynman -psi' agrees with a finite difference of psi;
  * the two routes to Z (matrix exponential, spectral sum) agree;
  * L = 2, N = 1: two distinct bonds join the two sites, so the hop rate is 2.
"""
import math

import numpy as np
import pytest

from oracle import ed


@pytest.mark.parametrize("L", [3, 5, 10])
@pytest.mark.parametrize("s", [-0.4, 0.0, 0.3])
def test_single_particle_closed_form(L, s):
    assert ed.scgf(L, 1, s) == pytest.approx(2.0 * (math.exp(-s) - 1.0), abs=1e-12)
    assert ed.scgf(L, L - 1, s) == pytest.approx(2.0 * (math.exp(-s) - 1.0), abs=1e-12)
    t = 3.0
    assert ed.partition(L, 1, s, t) == pytest.approx(math.exp(2 * t * (math.exp(-s) - 1)),
                                                     rel=1e-10)


def test_two_sites_two_bonds():
    # L = 2, N = 1: both ring bonds join sites 0 and 1, total hop rate 2.
    assert ed.scgf(2, 1, 0.3) == pytest.approx(2.0 * (math.exp(-0.3) - 1.0), abs=1e-12)


@pytest.mark.parametrize("L,N", [(6, 3), (10, 5), (9, 4)])
def test_zero_bias(L, N):
    assert abs(ed.scgf(L, N, 0.0)) < 1e-12
    assert ed.partition(L, N, 0.0, 7.0) == pytest.approx(1.0, abs=1e-12)
    assert ed.activity(L, N, 0.0) == pytest.approx(2.0 * N * (L - N) / (L - 1), rel=1e-12)


@pytest.mark.parametrize("L,N,s", [(10, 5, 0.2), (8, 3, -0.3), (12, 4, 0.1)])
def test_hellmann_feynman_vs_finite_difference(L, N, s):
    h = 1e-5
    fd = -(ed.scgf(L, N, s + h) - ed.scgf(L, N, s - h)) / (2 * h)
    assert ed.activity(L, N, s) == pytest.approx(fd, rel=1e-7)


def test_particle_hole_symmetry():
    for s in (-0.2, 0.2):
        assert ed.scgf(12, 4, s) == pytest.approx(ed.scgf(12, 8, s), abs=1e-12)


@pytest.mark.parametrize("s,t", [(0.4, 1.0), (-0.3, 5.0), (0.1, 20.0)])
def test_partition_two_routes(s, t):
    assert ed.partition(8, 4, s, t) == pytest.approx(ed.partition_spectral(8, 4, s, t),
                                                     rel=1e-9)


def test_finite_time_approaches_scgf():
    # (1/t) ln Z -> psi with a 1/t correction: the gap closes as t grows.
    s = 0.3
    psi = ed.scgf(10, 5, s)
    gaps = [abs(ed.finite_time_scgf(10, 5, s, t) - psi) for t in (10.0, 100.0, 1000.0)]
    assert gaps[0] > gaps[1] > gaps[2]
    assert gaps[2] < 1e-3


def test_dominant_vector_positive():
    _, v = ed.dominant(8, 4, 0.3)
    assert np.all(v > 0)
