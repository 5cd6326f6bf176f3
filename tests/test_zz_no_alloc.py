"""The allocation-free conditional distillation (pdg_bond_table_cond_noalloc)
against the workspace entry point (pdg_bond_table_cond), through the C ABI,
on two calls in a row, the second with a smaller sample (and a different L),
and once without G (the uniform-context table then lives in the library's
scratch too).

Both run the same kernels; the per-neighbourhood sums are accumulated with
atomics in an order that can change from run to run, so G agrees to 1e-12
(as the workspace entry point agrees with the FP64 reference), the counts
exactly, and the integer table exactly except where 2^16 e^G lies within
rounding of a half-integer.
"""
import numpy as np
import pytest
import torch

from oracle import guide_net as ref
from paper_1711_05095_amd import guide_net as gn
from paper_1711_05095_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gn.lib()


def _states(occ):
    n, L = occ.shape
    W = (L + 63) // 64
    words = np.zeros((W, n), np.uint64)
    for i in range(L):
        words[i // 64] |= occ[:, i].astype(np.uint64) << np.uint64(i % 64)
    return torch.from_numpy(words.view(np.int64)).cuda()


def _tables(window, states, L, min_count, gmax, noalloc, with_G=True):
    eg = torch.full((gn.PDG_WINDOWS,), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((gn.PDG_WINDOWS,), -1, dtype=torch.int32, device="cuda")
    G = torch.full((gn.PDG_WINDOWS,), np.nan, dtype=torch.float64, device="cuda") if with_G \
        else None
    if noalloc:
        gn.bond_table_cond_noalloc(window, states, L, min_count, gmax, eg, G, cnt)
    else:
        gn.bond_table_cond(window, states, L, min_count, gmax, eg, G, cnt)
    torch.cuda.synchronize()
    return (eg.cpu().numpy().view(np.uint32), None if G is None else G.cpu().numpy(),
            cnt.cpu().numpy())


def _same(a, b, gmax, G_ref):
    eg_a, G_a, c_a = a
    eg_b, G_b, c_b = b
    assert np.array_equal(c_a, c_b)
    if G_a is not None and G_b is not None:
        assert np.allclose(G_a, G_b, rtol=1e-12, atol=1e-12)
    x = 65536.0 * np.exp(np.clip(G_ref, -gmax, gmax))
    tie = np.abs(x - np.floor(x) - 0.5) < 1e-6
    assert np.array_equal(eg_a[~tie], eg_b[~tie])


def test_noalloc_equals_workspace_entry_point():
    th = ref.init_theta(41)
    th[ref.OFF_W3:ref.OFF_B3] *= 30
    H = torch.from_numpy(ref.window_table(th).astype(np.float32)).cuda()
    gmax = 1.0
    cases = [(100, 50, 3000, 2), (40, 20, 300, 1)]     # the second call smaller
    for L, N, n, min_count in cases:
        print(f"noalloc L={L} n={n} min_count={min_count}", flush=True)
        occ = inputs.random_population(L, N, n, seed=L + n)
        st = _states(occ)
        want = _tables(H, st, L, min_count, gmax, noalloc=False)
        got = _tables(H, st, L, min_count, gmax, noalloc=True)
        _same(want, got, gmax, want[1])
        assert np.sum(want[2] >= min_count) > 100     # the data branch is exercised
        # without G: the uniform-context table is kept in the library's scratch
        got2 = _tables(H, st, L, min_count, gmax, noalloc=True, with_G=False)
        _same(want, got2, gmax, want[1])
    # argument checks come before any device work
    with pytest.raises(Exception):
        gn.bond_table_cond_noalloc(H, _states(inputs.random_population(20, 10, 10, seed=1)), 20, 1,
                                   gmax, torch.empty(gn.PDG_WINDOWS, dtype=torch.int32,
                                                     device="cuda"))
