"""Test infrastructure: plain definitions of the observables of Secs. 2.4 and
3.3 that the library computes over a population.

  * density_mode: |delta rho_n|^2 with delta rho_n = L^{-1/2} sum over the
    occupied sites X of exp(-2 pi i n X / L) (eq. fourdens), per
    configuration;
  * population_mean: the average over the current clones (the end-time
    distribution p_end of Sec. 2.4);
  * ancestral_mean: the average over the current clones of a value recorded
    for their ancestors at an earlier time (the ancestral distribution p_ave
    of Sec. 2.4, eq. Opave), given each clone's origin slot.
"""
import numpy as np


def density_mode(occ, n):
    """|delta rho_n|^2 for each row of occ (uint8 [B, L])."""
    occ = np.asarray(occ)
    L = occ.shape[1]
    phase = np.exp(-2j * np.pi * n * np.arange(L) / L)
    rho = (occ * phase[None, :]).sum(axis=1) / np.sqrt(L)
    return np.abs(rho) ** 2


def population_mean(values):
    return float(np.mean(np.asarray(values, np.float64)))


def ancestral_mean(values_at_origin, origin):
    """(1/Nc) sum_j values[origin[j]]."""
    v = np.asarray(values_at_origin, np.float64)
    return float(np.mean(v[np.asarray(origin)]))
