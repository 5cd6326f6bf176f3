"""Conversions between the oracle's byte-per-site occupancies and the library's
bit-packed state words (site i = bit i%64 of word i//64; word w of clone j at
[w, j]).  Layout only."""
import numpy as np


def pack(occ):
    """uint8 [Nc, L] -> uint64 [W, Nc]."""
    Nc, L = occ.shape
    W = (L + 63) // 64
    out = np.zeros((W, Nc), np.uint64)
    for i in range(L):
        out[i // 64] |= occ[:, i].astype(np.uint64) << np.uint64(i % 64)
    return out


def unpack(words, L):
    """uint64 [W, Nc] -> uint8 [Nc, L]."""
    W, Nc = words.shape
    occ = np.zeros((Nc, L), np.uint8)
    for i in range(L):
        occ[:, i] = ((words[i // 64] >> np.uint64(i % 64)) & np.uint64(1)).astype(np.uint8)
    return occ
