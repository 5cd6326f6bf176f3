"""Test infrastructure: plain definitions of the observables of Secs. 2.4 and
3.3 that the library computes over a population.

  * density_mode: |delta rho_n|^2 with delta rho_n = L^{-1/2} sum over the
    occupied sites X of exp(-2 pi i n X / L) (eq. fourdens), per
    configuration;
  * population_mean: the average over the current clones (the end-time
    distribution p_end of Sec. 2.4);
  * ancestral_mean: the average over the current clones of a value recorded
    for their ancestors at an earlier time (the ancestral distribution p_ave
    of Sec. 2.4, eq. Opave), given each clone's origin slot;
  * histogram: counts of a per-clone quantity in equal bins, over the current
    clones (p_end) or over their ancestors (p_ave), as the distributions of
    Sec. 2.4 are shown (the activity distributions of Sec. 5).
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


def histogram(values, lo, width, nbins, origin=None):
    """counts[b] = #{j : floor((v_j - lo) / width) = b}, b = 0..nbins-1, with
    v_j = values[j], or values[origin[j]] when origins are given; values whose
    (v - lo) / width lies outside [0, nbins), and NaN, are not counted.  The
    bin is decided by one FP64 subtraction and one FP64 division, then the
    floor."""
    v = np.asarray(values, np.float64)
    if origin is not None:
        v = v[np.asarray(origin)]
    t = (v - np.float64(lo)) / np.float64(width)
    keep = (t >= 0) & (t < nbins)
    return np.bincount(np.floor(t[keep]).astype(np.int64), minlength=nbins).astype(np.uint64)
