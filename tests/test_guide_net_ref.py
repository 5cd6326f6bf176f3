"""Pins of the FP64 reference of the guide network.

  * the analytic gradient equals central finite differences of the loss;
  * f(C) is the sum over sites of the window table h (the circular network
    and its 13-site window evaluation are two independent computations);
  * f is invariant under rotations of the ring;
  * a network with zero weights gives f = L b3;
  * the distilled bond table equals, for L = 13 rings, the exact log-ratio
    f(C after the hop) - f(C) averaged over the outer sites (brute force);
  * the option that rounds h1 to bf16 before layer 2 changes nothing when h1
    is exactly representable, and otherwise moves f by the first-order effect
    of the roundings (to second order).
"""
import numpy as np
import pytest

from oracle import guide_net as gn
from paper_1711_05095_amd import inputs


def test_gradient_matches_finite_differences():
    th = gn.init_theta(1)
    th[gn.OFF_W3:gn.OFF_B3] *= 10
    occ = inputs.random_population(20, 9, 3, seed=2)
    n = np.array([0.0, 2.0, 1.0])
    g = gn.grad(th, occ, n)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(gn.PARAMS, 60, replace=False), [gn.OFF_B3, gn.OFF_C0]])
    h = 1e-6
    for i in idx:
        e = np.zeros(gn.PARAMS)
        e[i] = h
        fd = (gn.loss(th + e, occ, n) - gn.loss(th - e, occ, n)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9), i


@pytest.mark.parametrize("L", [13, 20, 37])
def test_f_is_sum_of_window_table(L):
    th = gn.init_theta(4)
    H = gn.window_table(th)
    occ = inputs.random_population(L, L // 2, 5, seed=L)
    f, _ = gn.forward(th, occ)
    for b in range(5):
        bits = sum(int(v) << i for i, v in enumerate(occ[b]))
        wsum = sum(H[sum(((bits >> ((c + o - 6) % L)) & 1) << o for o in range(13))]
                   for c in range(L))
        assert f[b] == pytest.approx(wsum, rel=1e-12, abs=1e-12)


def test_rotation_invariance_and_zero_net():
    th = gn.init_theta(5)
    occ = inputs.random_population(30, 14, 4, seed=6)
    f0, _ = gn.forward(th, occ)
    f1, _ = gn.forward(th, np.roll(occ, 7, axis=1))
    assert np.allclose(f0, f1, rtol=1e-12)
    z = np.zeros(gn.PARAMS)
    z[gn.OFF_B3] = 0.25
    f, _ = gn.forward(z, occ)
    assert np.allclose(f, 30 * 0.25)


def test_distilled_table_is_the_average_log_ratio():
    """The 14-window difference of the table for one outer context equals the
    brute-force f(C after the hop) - f(C) on a ring long enough not to wrap,
    and the bond table is the average of that over all 8192 outer contexts."""
    th = gn.init_theta(7)
    H = gn.window_table(th)
    eg, G = gn.distill(H, gmax=50.0)
    rng = np.random.default_rng(8)
    for _ in range(4):
        u = int(rng.integers(0, 8192))
        if ((u >> 6) & 1) == ((u >> 7) & 1):
            u ^= 1 << 7
        diffs = []
        for ctx in list(rng.integers(0, 8192, 3)) + [0, 8191]:
            s0 = (int(ctx) & 0x3F) | (u << 6) | ((int(ctx) >> 6) << 19)
            d = sum(H[((s0 ^ (3 << 12)) >> o) & 0x1FFF] - H[(s0 >> o) & 0x1FFF]
                    for o in range(14))
            occ = np.array([[(s0 >> i) & 1 for i in range(40)]], np.uint8)  # sites 26..39 empty
            f0, _ = gn.forward(th, occ)
            occ[0, 12], occ[0, 13] = occ[0, 13], occ[0, 12]
            f1, _ = gn.forward(th, occ)
            assert d == pytest.approx(f1[0] - f0[0], rel=1e-10, abs=1e-10)
            diffs.append(d)
        allctx = np.arange(8192)
        s0 = (allctx & 0x3F) | (u << 6) | ((allctx >> 6) << 19)
        full = sum(H[((s0 ^ (3 << 12)) >> o) & 0x1FFF] - H[(s0 >> o) & 0x1FFF] for o in range(14))
        assert G[u] == pytest.approx(full.mean(), rel=1e-12, abs=1e-12)
        assert eg[u] == int(np.rint(65536.0 * np.exp(G[u])))
    assert np.all(eg[[u for u in range(8192) if ((u >> 6) & 1) == ((u >> 7) & 1)]] == 0)


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.1415926])
    r = gn.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0078125   # ties to even, then up
    assert abs(r[3] - x[3]) <= 2 ** -8 * abs(x[3])


def test_bond_deltas_are_exact_log_ratios():
    """On rings of L >= 26 sites the 14-window difference is the net's exact
    f(C after the hop) - f(C), checked by running the whole circular network
    on both configurations."""
    th = gn.init_theta(9)
    th[gn.OFF_W3:gn.OFF_B3] *= 10
    H = gn.window_table(th)
    for L in (26, 31):
        occ = inputs.random_population(L, L // 2, 3, seed=L)
        u, d = gn.bond_deltas(H, occ)
        k = 0
        for i in range(3):
            f0, _ = gn.forward(th, occ[i:i + 1])
            for b in range(L):
                b2 = (b + 1) % L
                if occ[i, b] == occ[i, b2]:
                    continue
                c = occ[i:i + 1].copy()
                c[0, b], c[0, b2] = c[0, b2], c[0, b]
                f1, _ = gn.forward(th, c)
                assert d[k] == pytest.approx(f1[0] - f0[0], rel=1e-9, abs=1e-9)
                want_u = sum(int(occ[i, (b - 6 + o) % L]) << o for o in range(13))
                assert u[k] == want_u
                k += 1
        assert k == len(d)


def test_conditional_table_is_the_mean_per_neighbourhood():
    """G[u] is the plain mean of the deltas sharing u where u is seen at least
    min_count times, and the uniform-context value elsewhere."""
    th = gn.init_theta(10)
    th[gn.OFF_W3:gn.OFF_B3] *= 10
    H = gn.window_table(th)
    occ = inputs.random_population(40, 20, 30, seed=11)
    eg, G, cnt = gn.distill_conditional(H, occ, gmax=0.3, min_count=2)
    u, d = gn.bond_deltas(H, occ)
    groups = {}
    for a, b in zip(u, d):
        groups.setdefault(int(a), []).append(b)
    _, G_uni = gn.distill(H, 0.3)
    assert sum(len(v) for v in groups.values()) == cnt.sum() == len(d)
    for v in range(8192):
        if ((v >> 6) & 1) == ((v >> 7) & 1):
            assert eg[v] == 0 and G[v] == 0.0 and v not in groups
            continue
        if len(groups.get(v, [])) >= 2:
            assert G[v] == pytest.approx(np.mean(groups[v]), rel=1e-12, abs=1e-15)
        else:
            assert G[v] == G_uni[v]
        assert eg[v] == int(np.rint(65536.0 * np.exp(np.clip(G[v], -0.3, 0.3))))


def test_h1_rounding_option():
    occ = inputs.random_population(24, 11, 6, seed=4)
    th = gn.init_theta(5)
    # h1 = tanh(b1) = 0.5 exactly representable: W1 = 0, b1 = atanh(0.5)
    t0 = th.copy()
    t0[gn.OFF_W1:gn.OFF_B1] = 0.0
    t0[gn.OFF_B1:gn.OFF_W2] = np.arctanh(0.5)
    f0, A0 = gn.forward(t0, occ)
    assert np.all(A0["h1"] == 0.5)
    f0r, _ = gn.forward(t0, occ, h1_bf16=True)
    assert np.array_equal(f0, f0r)
    # general weights: f(rounded) - f = sum_j (bf16(h1) - h1) df/dh1 + O(u^2)
    P = gn.unpack(th)
    f, A = gn.forward(th, occ)
    fr, _ = gn.forward(th, occ, h1_bf16=True)
    g_z2 = gn._conv_T(np.ones((6, 1, 24)), P["W3"][None]) * (1 - A["h2"] ** 2)
    dh1 = gn._conv_T(g_z2, P["W2"])
    lin = ((gn.bf16(A["h1"]) - A["h1"]) * dh1).sum(axis=(1, 2))
    assert np.all(np.abs(fr - f) > 0)
    assert np.allclose(fr - f, lin, rtol=0.05, atol=1e-9)
