"""Parity of the guide network's HIP kernels (through the C ABI in
include/pd_guide.h) with the FP64 reference oracle/guide_net.py.

Tolerances follow from the arithmetic: the weights are rounded to bfloat16 on
both sides (the reference is given the rounded weights), and the GPU rounds
the layer-1 activations h1 to bfloat16 as they enter the matrix cores
(relative error eps, |eps| <= u = 2^-8) and accumulates in float32.  h1 at a
position depends only on the 5-site window of inputs around it, so positions
with the same window share one value and one rounding error per channel: to
first order f changes by sum over windows w and channels c of
eps_wc G_wc, G_wc = sum over the positions j with window w of
h1_cj df/dh1_cj.  With the eps_wc independent and uniform its standard
deviation is
    sigma_f = (u / sqrt 3) * || G ||_2
which the reference computes from its own activations and adjoint.  (Taking
one independent error per position instead underestimates sigma_f by up to
sqrt(L/32) and fails at L = 512 for right answers.)  Each f must agree to
6 sigma_f (plus 1e-4 for float32 rounding elsewhere); the worst-case bound
(all errors aligned) is far looser and would not separate a right answer
from a wrong one.  Sharper: against the reference evaluated with h1 rounded
to bf16 where layer 2 reads it (oracle option h1_bf16), every f must agree
to 1e-4 (1 + |f|) plus the effect of the h1 roundings that float32 can
decide either way: the entries of the 32 x 32 table h1[window][channel]
within 2e-6 of a bf16 rounding boundary, each flip moving h1 by one bf16 ulp
and f by that times the summed df/dh1 of the window's positions (such a flip
moves every configuration, as all of them hold every common window).  The window table is held to the
same rule with its own sigma.  Gradients pass through bf16-rounded dz2 and h1
(the W2 gradient), dz2 (the h1 adjoint) and dz1 (the W1 gradient, whose other
factor, the input +-1, is exact): each parameter group must agree to 1e-2 in
2-norm and 2e-2 of its largest entry; a CPU emulation of this rounding model
gives at most 1.2e-3 on these cases.  Adam and the bond table
are float32 / float64 elementwise and agree to rounding.
"""
import numpy as np
import pytest
import torch

from layout import pack
from oracle import guide_net as ref
from paper_1711_05095_amd import guide_net as gn
from paper_1711_05095_amd import inputs

pytestmark = pytest.mark.gpu

GROUPS = [("W1", ref.OFF_W1, ref.OFF_B1), ("b1", ref.OFF_B1, ref.OFF_W2),
          ("W2", ref.OFF_W2, ref.OFF_B2), ("b2", ref.OFF_B2, ref.OFF_W3),
          ("W3", ref.OFF_W3, ref.OFF_B3), ("b3", ref.OFF_B3, ref.OFF_C0),
          ("c0", ref.OFF_C0, ref.PARAMS)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gn.lib()


def theta_for(seed, w3_scale=10.0):
    th = ref.init_theta(seed)
    th[ref.OFF_W3:ref.OFF_B3] *= w3_scale
    th[ref.OFF_B1:ref.OFF_W2] = np.random.default_rng(seed + 100).uniform(-0.3, 0.3, 32)
    th[ref.OFF_B2:ref.OFF_W3] = np.random.default_rng(seed + 101).uniform(-0.3, 0.3, 32)
    th[ref.OFF_B3] = 0.01
    th[ref.OFF_C0] = -0.2
    return th.astype(np.float32)


def dev(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def states_dev(occ):
    return dev(pack(occ).view(np.int64))


U = 2.0 ** -8          # unit roundoff of bfloat16 (8 significant bits)
DELTA = 2e-6           # bound on |h1 (float32 on the GPU) - h1 (float64)|


def _grouped_sigma(prod, win):
    """(u / sqrt 3) * || G ||_2 per configuration, G[w, c] = sum of prod[c, j]
    over the positions j whose input window is w: h1 (and so its rounding
    error) depends only on the 5-site window, so positions that share a window
    share their error.  prod: [n, 32, P] (h1 * df/dh1), win: [n, P] in 0..31."""
    onehot = (win[:, :, None] == np.arange(32)[None, None, :]).astype(np.float64)
    G = np.einsum("bcp,bpw->bwc", prod, onehot)
    return U / np.sqrt(3) * np.sqrt((G ** 2).sum(axis=(1, 2)))


def _forward_model(th64, occ):
    """Per configuration: sigma_f of the rounding model, and the most f can move
    by flips of the h1 roundings that float32 can decide either way: the
    entries of the 32 x 32 table h1[window][channel] within DELTA of a bf16
    rounding boundary, each flip moving h1 by one bf16 ulp and f by that times
    the sum of df/dh1 over the positions with that window."""
    tb = ref.bf16_weights(th64)
    P = ref.unpack(tb)
    _, A = ref.forward(tb, occ)
    n, L = occ.shape
    g_z2 = ref._conv_T(np.ones((n, 1, L)), P["W3"][None]) * (1 - A["h2"] ** 2)
    dh1 = ref._conv_T(g_z2, P["W2"])                               # df/dh1
    win = sum(np.roll(occ.astype(np.int64), -(k - 2), axis=1) << k for k in range(5))
    onehot = (win[:, :, None] == np.arange(32)[None, None, :]).astype(np.float64)
    G = np.einsum("bcp,bpw->bwc", A["h1"] * dh1, onehot)
    sigma = U / np.sqrt(3) * np.sqrt((G ** 2).sum(axis=(1, 2)))
    # the table of h1 by window (a_k = 2 bit_k(w) - 1 for sites j-2 .. j+2)
    a = 2.0 * ((np.arange(32)[:, None] >> np.arange(5)) & 1) - 1.0
    h1w = np.tanh(a @ P["W1"].T + P["b1"][None, :])                # [window, channel]
    e = np.floor(np.log2(np.maximum(np.abs(h1w), 1e-300)))
    off = np.abs(h1w - ref.bf16(h1w))
    amb = (np.abs(off - 2.0 ** (e - 8)) <= DELTA) | (np.abs(off - 2.0 ** (e - 9)) <= DELTA)
    ulp = 2.0 ** (e - 7)
    D = np.einsum("bcp,bpw->bwc", dh1, onehot)                      # [b, window, channel]
    flips = np.einsum("bwc,wc->b", np.abs(D), np.where(amb, ulp, 0.0))
    return sigma, flips


def forward_bound(th64, occ):
    """6 sigma_f + 1e-4: tolerance of f_gpu - f per configuration."""
    return 6 * _forward_model(th64, occ)[0] + 1e-4


def window_bound(tb):
    """6 sigma + 1e-4 per window of the table (same rule, valid convolutions)."""
    P = ref.unpack(tb)
    w = np.arange(8192)
    bits = (w[:, None] >> np.arange(13)) & 1
    a = 2.0 * bits - 1.0
    h1 = np.tanh(np.einsum("ck,bkp->bcp", P["W1"], np.stack([a[:, k:k + 9] for k in range(5)], 1))
                 + P["b1"][None, :, None])                          # [8192, 32, 9]
    x = np.stack([h1[:, :, k:k + 5] for k in range(5)], axis=2)    # [b, c', k, p]
    h2 = np.tanh(np.einsum("dck,bckp->bdp", P["W2"], x) + P["b2"][None, :, None])
    dz2 = P["W3"][None] * (1 - h2 ** 2)                             # [b, c, p]
    dh1 = np.zeros_like(h1)
    for k in range(5):
        dh1[:, :, k:k + 5] += np.einsum("dck,bdp->bcp", P["W2"][:, :, k:k + 1], dz2)
    win = sum(bits[:, k:k + 9] << k for k in range(5))              # [8192, 9]
    return 6 * _grouped_sigma(h1 * dh1, win) + 1e-4


@pytest.mark.parametrize("L,n", [(5, 200), (13, 300), (37, 1000), (64, 300), (100, 1000),
                                 (200, 257), (288, 120), (512, 70)])
def test_forward_matches_reference(L, n):
    th = theta_for(L)
    occ = inputs.random_population(L, L // 2, n, seed=L + 1)
    f = torch.empty(n, dtype=torch.float32, device="cuda")
    gn.forward(dev(th), states_dev(occ), L, f)
    torch.cuda.synchronize()
    th64 = th.astype(np.float64)
    tb = ref.bf16_weights(th64)
    got = f.cpu().numpy().astype(np.float64)
    # the FP64 net: the GPU differs by the bf16 rounding of h1, within 6 sigma
    want, _ = ref.forward(tb, occ)
    sigma, flips = _forward_model(th64, occ)
    bound = 6 * sigma + 1e-4
    err = np.abs(got - want)
    assert np.all(err <= bound), (L, float(np.max(err / bound)), float(np.max(err)))
    # the same net with h1 rounded to bf16 where layer 2 reads it: what remains
    # is float32 accumulation and the flips of the h1 roundings that float32
    # decides either way
    want_r, _ = ref.forward(tb, occ, h1_bf16=True)
    d = np.abs(got - want_r)
    tight = 1e-4 * (1 + np.abs(want_r))
    assert np.all(d <= tight + flips), (L, float(np.max(d / (tight + flips))), float(np.max(d)))
    # the net varies across configurations far beyond the tight tolerance
    assert np.std(want) > 20 * np.max(tight)


def test_forward_equivariance_on_gpu():
    """f is invariant under rotations of the ring: every per-site value is the
    same product in the same order, only the float32 sum over sites runs in
    another order (a difference of order 1e-6 here)."""
    L = 64
    th = theta_for(3)
    occ = inputs.random_population(L, 20, 64, seed=4)
    rot = np.roll(occ, 17, axis=1)
    f0 = torch.empty(64, dtype=torch.float32, device="cuda")
    f1 = torch.empty_like(f0)
    gn.forward(dev(th), states_dev(occ), L, f0)
    gn.forward(dev(th), states_dev(rot), L, f1)
    torch.cuda.synchronize()
    assert np.max(np.abs(f0.cpu().numpy() - f1.cpu().numpy())) <= 1e-4


def test_column_slices_of_a_wider_array():
    """A column slice (leading dimension > n) gives bit-identical results."""
    L, n, a, b = 100, 700, 123, 456
    th = dev(theta_for(5))
    occ = inputs.random_population(L, 50, n, seed=6)
    full = states_dev(occ)
    f_full = torch.empty(n, dtype=torch.float32, device="cuda")
    f_cut = torch.empty(b - a, dtype=torch.float32, device="cuda")
    gn.forward(th, full, L, f_full)
    gn.forward(th, full[:, a:b], L, f_cut)
    counts = dev(np.random.default_rng(7).poisson(1.0, n).astype(np.float32))
    work = torch.empty(gn.workspace_bytes(n), dtype=torch.uint8, device="cuda")
    g_cut = torch.empty(gn.PDG_PARAMS, dtype=torch.float32, device="cuda")
    g_copy = torch.empty_like(g_cut)
    gn.loss_grad(th, full[:, a:b], counts[a:b], L, g_cut, None, work)
    gn.loss_grad(th, full[:, a:b].contiguous(), counts[a:b].contiguous(), L, g_copy, None, work)
    torch.cuda.synchronize()
    assert torch.equal(f_cut, f_full[a:b])
    assert torch.equal(g_cut, g_copy)


# L = 288 runs 3 waves per block (L = 512: 1), so one wave builds two of the
# four layer-1 table tiles.  Its parameters make e^(f + c0) small against the
# counts, as at the other sizes here: where e^(f + c0) dominates (L = 232 and
# 296 with these parameters), delta carries the shift of f that the bf16
# rounding of h1 makes (up to ~1e-2 at these L, inside the forward bound) and
# every gradient group moves by that fraction, 0.9-1.3%, against the 1e-2 below
@pytest.mark.parametrize("L,n", [(5, 150), (13, 200), (64, 300), (100, 900), (288, 80),
                                 (512, 70)])
def test_loss_and_gradient_match_reference(L, n):
    th = theta_for(L + 7)
    occ = inputs.random_population(L, L // 2, n, seed=L + 2)
    counts = np.random.default_rng(L).poisson(1.5, n).astype(np.float32)
    work = torch.empty(gn.workspace_bytes(n), dtype=torch.uint8, device="cuda")
    grad = torch.empty(gn.PDG_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    gn.loss_grad(dev(th), states_dev(occ), dev(counts), L, grad, loss, work)
    torch.cuda.synchronize()
    th64 = th.astype(np.float64)
    tb = ref.bf16_weights(th64)
    cnt = counts.astype(np.float64)
    want_g = ref.grad(tb, occ, cnt)
    want_l = ref.loss(tb, occ, cnt)
    got_g = grad.cpu().numpy().astype(np.float64)
    got_l = float(loss.item())
    # the loss moves with f through exp(f + c0): to first order by
    # mean((e^z - count) df), with |df| within the forward bound
    f, _ = ref.forward(tb, occ)
    ez = np.exp(f + ref.unpack(tb)["c0"])
    sigma, _ = _forward_model(th64, occ)
    fb = 6 * sigma + 1e-4
    assert abs(got_l - want_l) <= np.mean(np.abs(ez - cnt) * fb + ez * fb ** 2) + 1e-4 * abs(want_l)
    # and sharply: the training pass's f is the forward pass's (checked above
    # against both references), so its loss is the loss of pdg_forward's f
    fgpu = torch.empty(n, dtype=torch.float32, device="cuda")
    gn.forward(dev(th), states_dev(occ), L, fgpu)
    torch.cuda.synchronize()
    zg = fgpu.cpu().numpy().astype(np.float64) + float(th[ref.OFF_C0])
    lg = float(np.mean(np.exp(zg) - cnt * zg))
    assert abs(got_l - lg) <= 1e-5 * (abs(lg) + 1), (got_l, lg)
    for name, a, b in GROUPS:
        d = got_g[a:b] - want_g[a:b]
        nrm = np.linalg.norm(want_g[a:b])
        assert np.linalg.norm(d) <= 1e-2 * nrm + 1e-7, (name, np.linalg.norm(d), nrm)
        assert np.max(np.abs(d)) <= 2e-2 * np.max(np.abs(want_g[a:b])) + 1e-7, name


def test_gradient_is_additive_over_batches():
    """Gradient of the mean loss over 2n samples = mean of the gradients over
    its two halves: the per-block partial sums and their reduction cover every
    sample exactly once.  n is a power of two so that the 1/n inside dz2
    scales without changing its bfloat16 rounding; what remains is float32
    summation order."""
    L, n = 40, 1024
    th = theta_for(11)
    occ = inputs.random_population(L, 20, 2 * n, seed=12)
    counts = np.random.default_rng(13).poisson(1.0, 2 * n).astype(np.float32)
    out = []
    for sl in (slice(0, 2 * n), slice(0, n), slice(n, 2 * n)):
        o = occ[sl]
        m = o.shape[0]
        work = torch.empty(gn.workspace_bytes(m), dtype=torch.uint8, device="cuda")
        g = torch.empty(gn.PDG_PARAMS, dtype=torch.float32, device="cuda")
        gn.loss_grad(dev(th), states_dev(o), dev(counts[sl]), L, g, None, work)
        torch.cuda.synchronize()
        out.append(g.cpu().numpy().astype(np.float64))
    comb = (out[1] + out[2]) / 2
    assert np.allclose(out[0], comb, rtol=1e-4, atol=1e-5 * np.max(np.abs(out[0])))


def test_train_epoch_equals_gradient_and_adam_steps():
    """pdg_train_epoch (minibatches enqueued by the library, reduction fused
    with Adam) gives the same parameters, moments and summed loss, bit for
    bit, as pdg_loss_grad + pdg_adam called per minibatch, including a short
    last minibatch and a nonzero starting step."""
    L, n, batch, step0, lr = 37, 2500, 1024, 5, 3e-3
    th = theta_for(21)
    occ = inputs.random_population(L, 15, n, seed=22)
    counts = np.random.default_rng(23).poisson(1.2, n).astype(np.float32)
    S, C = states_dev(occ), dev(counts)
    rng = np.random.default_rng(24)
    m0 = (rng.standard_normal(gn.PDG_PARAMS) * 1e-3).astype(np.float32)
    v0 = (rng.random(gn.PDG_PARAMS) * 1e-6).astype(np.float32)
    work = torch.empty(gn.workspace_bytes(batch), dtype=torch.uint8, device="cuda")

    t1, m1, v1 = dev(th), dev(m0), dev(v0)
    total = torch.zeros(1, dtype=torch.float64, device="cuda")
    k = gn.train_epoch(t1, m1, v1, S, C, L, batch, step0, lr, total, work)
    assert k == 3

    t2, m2, v2 = dev(th), dev(m0), dev(v0)
    grad = torch.empty(gn.PDG_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    want = 0.0
    for i, a in enumerate(range(0, n, batch)):
        b = min(n, a + batch)
        gn.loss_grad(t2, S[:, a:b], C[a:b], L, grad, loss, work)
        gn.adam(t2, m2, v2, grad, step0 + i + 1, lr)
        torch.cuda.synchronize()
        want += float(loss.item())
    torch.cuda.synchronize()
    assert torch.equal(t1, t2) and torch.equal(m1, m2) and torch.equal(v1, v2)
    assert float(total.item()) == want
    assert not torch.equal(t1, dev(th))


def test_adam_matches_reference():
    rng = np.random.default_rng(5)
    th = rng.normal(size=gn.PDG_PARAMS).astype(np.float32)
    m = np.zeros(gn.PDG_PARAMS, np.float32)
    v = np.zeros(gn.PDG_PARAMS, np.float32)
    t_th, t_m, t_v = dev(th), dev(m), dev(v)
    want = (th.astype(np.float64), m.astype(np.float64), v.astype(np.float64))
    for step in range(1, 4):
        g = rng.normal(size=gn.PDG_PARAMS).astype(np.float32)
        gn.adam(t_th, t_m, t_v, dev(g), step, 1e-2)
        want = ref.adam(want[0], want[1], want[2], g.astype(np.float64), step, 1e-2)
    torch.cuda.synchronize()
    assert np.allclose(t_th.cpu().numpy(), want[0], rtol=1e-5, atol=1e-6)
    assert np.allclose(t_m.cpu().numpy(), want[1], rtol=1e-5, atol=1e-7)
    assert np.allclose(t_v.cpu().numpy(), want[2], rtol=1e-5, atol=1e-8)


def test_window_table_matches_reference():
    th = theta_for(21)
    table = torch.empty(gn.PDG_WINDOWS, dtype=torch.float32, device="cuda")
    gn.window_table(dev(th), table)
    torch.cuda.synchronize()
    th64 = th.astype(np.float64)
    tb = ref.bf16_weights(th64)
    H = ref.window_table(tb)
    got = table.cpu().numpy().astype(np.float64)
    bound = window_bound(tb)
    err = np.abs(got - H)
    assert np.all(err <= bound), (float(np.max(err / bound)), float(np.max(err)))
    assert np.std(H) > 20 * np.max(bound)


@pytest.mark.parametrize("gmax", [gn.PDG_MAX_GMAX, 0.05])
def test_bond_table_matches_reference(gmax):
    th = ref.init_theta(31)
    th[ref.OFF_W3:ref.OFF_B3] *= 30
    H = ref.window_table(th).astype(np.float32)
    eg = torch.empty(gn.PDG_WINDOWS, dtype=torch.int32, device="cuda")
    G = torch.empty(gn.PDG_WINDOWS, dtype=torch.float64, device="cuda")
    gn.bond_table(dev(H), gmax, eg, G)
    torch.cuda.synchronize()
    want_eg, want_G = ref.distill(H.astype(np.float64), gmax)
    got_G = G.cpu().numpy()
    got_eg = eg.cpu().numpy().view(np.uint32)
    assert np.allclose(got_G, want_G, rtol=1e-12, atol=1e-12)
    hop = ((np.arange(8192) >> 6) ^ (np.arange(8192) >> 7)) & 1
    assert np.all(got_eg[hop == 0] == 0)
    # rint ties aside, the integer table is identical
    x = 65536.0 * np.exp(np.clip(want_G, -gmax, gmax))
    tie = np.abs(x - np.floor(x) - 0.5) < 1e-6
    assert np.array_equal(got_eg[~tie], want_eg[~tie])
    if gmax < 1:
        assert np.sum(np.abs(want_G[hop == 1]) > gmax) > 100   # the clip is exercised
    assert got_eg[hop == 1].max() <= 1024 * got_eg[hop == 1].min()


@pytest.mark.parametrize("L,n,min_count", [(40, 300, 1), (100, 120, 3)])
def test_conditional_bond_table_matches_reference(L, n, min_count):
    th = ref.init_theta(41)
    th[ref.OFF_W3:ref.OFF_B3] *= 30
    H = ref.window_table(th).astype(np.float32)
    occ = inputs.random_population(L, L // 2, n, seed=L + 3)
    gmax = 1.0
    eg = torch.empty(gn.PDG_WINDOWS, dtype=torch.int32, device="cuda")
    G = torch.empty(gn.PDG_WINDOWS, dtype=torch.float64, device="cuda")
    cnt = torch.empty(gn.PDG_WINDOWS, dtype=torch.int32, device="cuda")
    gn.bond_table_cond(dev(H), states_dev(occ), L, min_count, gmax, eg, G, cnt)
    torch.cuda.synchronize()
    want_eg, want_G, want_cnt = ref.distill_conditional(H.astype(np.float64), occ, gmax, min_count)
    assert np.array_equal(cnt.cpu().numpy(), want_cnt)          # integer: exact
    assert np.allclose(G.cpu().numpy(), want_G, rtol=1e-12, atol=1e-12)
    got_eg = eg.cpu().numpy().view(np.uint32)
    x = 65536.0 * np.exp(np.clip(want_G, -gmax, gmax))
    tie = np.abs(x - np.floor(x) - 0.5) < 1e-6
    assert np.array_equal(got_eg[~tie], want_eg[~tie])
    assert np.sum(want_cnt >= min_count) > 100                  # the data branch is exercised
