"""Test infrastructure: FP64 reference of the learned guide.

The guide predicts ln v(C), v the dominant eigenvector of the tilted
generator, whose ratios across a hop are the optimal control (Doob
transform) of the modified dynamics in Sec. 2.2; a clone's expected number
of descendants after a long lag is proportional to v(C) (the p_end / p_ave
discussion of Sec. 2.4), which is what the training data measure.

Network (parameters theta, flat, PARAMS entries):
    a_j   = 2 n_j - 1                                   (occupancy as +-1)
    h1    = tanh(b1[c] + sum_k W1[c,k] a_{j+k-2})        32 channels, kernel 5
    h2    = tanh(b2[c] + sum_{c',k} W2[c,c',k] h1[c',j+k-2])
    o_j   = b3 + sum_{c',k} W3[c',k] h2[c',j+k-2]
    f(C)  = sum_j o_j                                    (indices mod L)
so f(C) = sum_j h(window_j) with h a function of the 13 sites j-6..j+6.
Poisson regression on descendant counts n:  loss = mean(exp(f+c0) - n (f+c0)).
"""
import numpy as np

CH, KS = 32, 5
OFF_W1 = 0
OFF_B1 = OFF_W1 + CH * KS
OFF_W2 = OFF_B1 + CH
OFF_B2 = OFF_W2 + CH * CH * KS
OFF_W3 = OFF_B2 + CH
OFF_B3 = OFF_W3 + CH * KS
OFF_C0 = OFF_B3 + 1
PARAMS = OFF_C0 + 1


def unpack(theta):
    t = np.asarray(theta, np.float64)
    return dict(W1=t[OFF_W1:OFF_B1].reshape(CH, KS), b1=t[OFF_B1:OFF_W2],
                W2=t[OFF_W2:OFF_B2].reshape(CH, CH, KS), b2=t[OFF_B2:OFF_W3],
                W3=t[OFF_W3:OFF_B3].reshape(CH, KS), b3=t[OFF_B3], c0=t[OFF_C0])


def init_theta(seed):
    """Small random initial parameters (uniform, fan-in scaled)."""
    rng = np.random.default_rng(seed)
    th = np.zeros(PARAMS)
    th[OFF_W1:OFF_B1] = rng.uniform(-1, 1, CH * KS) / np.sqrt(KS)
    th[OFF_W2:OFF_B2] = rng.uniform(-1, 1, CH * CH * KS) / np.sqrt(CH * KS)
    th[OFF_W3:OFF_B3] = rng.uniform(-1, 1, CH * KS) / np.sqrt(CH * KS) * 0.1
    return th


def bf16(x):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_weights(theta):
    """theta with the weight matrices rounded to bfloat16 (biases kept)."""
    t = np.array(theta, np.float64)
    for a, b in ((OFF_W1, OFF_B1), (OFF_W2, OFF_B2), (OFF_W3, OFF_B3)):
        t[a:b] = bf16(t[a:b])
    return t


def _conv(x, W):
    """Circular conv: out[b, c, j] = sum_{c', k} W[c, c', k] x[b, c', j + k - 2]."""
    out = np.zeros((x.shape[0], W.shape[0], x.shape[2]))
    for k in range(KS):
        out += np.einsum("dc,bcj->bdj", W[:, :, k], np.roll(x, -(k - 2), axis=2))
    return out


def forward(theta, occ, h1_bf16=False):
    """f for each configuration in occ (uint8 [B, L]); also the activations.
    h1_bf16: layer 2 reads h1 rounded to bfloat16 (a precision model of
    bf16 matrix operands; the returned h1 is the unrounded one)."""
    P = unpack(theta)
    a = (2.0 * occ.astype(np.float64) - 1.0)[:, None, :]
    h1 = np.tanh(_conv(a, P["W1"][:, None, :]) + P["b1"][None, :, None])
    h2 = np.tanh(_conv(bf16(h1) if h1_bf16 else h1, P["W2"]) + P["b2"][None, :, None])
    o = _conv(h2, P["W3"][None, :, :])[:, 0, :] + P["b3"]
    return o.sum(axis=1), dict(a=a, h1=h1, h2=h2)


def loss(theta, occ, n, h1_bf16=False):
    f, _ = forward(theta, occ, h1_bf16)
    z = f + unpack(theta)["c0"]
    return float(np.mean(np.exp(z) - n * z))


def _conv_T(g, W):
    """Adjoint of _conv with respect to its input."""
    out = np.zeros((g.shape[0], W.shape[1], g.shape[2]))
    for k in range(KS):
        out += np.roll(np.einsum("dc,bdj->bcj", W[:, :, k], g), (k - 2), axis=2)
    return out


def _conv_W(g, x):
    """Gradient of sum(g * _conv(x, W)) with respect to W."""
    return np.stack([np.einsum("bdj,bcj->dc", g, np.roll(x, -(k - 2), axis=2))
                     for k in range(KS)], axis=2)


def grad(theta, occ, n):
    """Analytic gradient of loss(theta, occ, n)."""
    P = unpack(theta)
    f, A = forward(theta, occ)
    B = occ.shape[0]
    delta = (np.exp(f + P["c0"]) - n) / B                        # d loss / d f
    L = occ.shape[1]
    g_o = np.broadcast_to(delta[:, None, None], (B, 1, L))
    g = np.zeros(PARAMS)
    g[OFF_W3:OFF_B3] = _conv_W(g_o, A["h2"])[0].ravel()
    g[OFF_B3] = float(np.sum(delta) * L)
    g_h2 = _conv_T(g_o, P["W3"][None, :, :])
    g_z2 = g_h2 * (1 - A["h2"] ** 2)
    g[OFF_W2:OFF_B2] = _conv_W(g_z2, A["h1"]).ravel()
    g[OFF_B2:OFF_W3] = g_z2.sum(axis=(0, 2))
    g_h1 = _conv_T(g_z2, P["W2"])
    g_z1 = g_h1 * (1 - A["h1"] ** 2)
    g[OFF_W1:OFF_B1] = _conv_W(g_z1, A["a"])[:, 0, :].ravel()
    g[OFF_B1:OFF_W2] = g_z1.sum(axis=(0, 2))
    g[OFF_C0] = float(np.sum(delta))
    return g


def window_table(theta):
    """h(w) for every 13-site window w (site c-6 in bit 0 ... c+6 in bit 12):
    the net evaluated on the window alone (valid convolutions 13 -> 9 -> 5 -> 1)."""
    P = unpack(theta)
    w = np.arange(8192)
    a = (2.0 * ((w[:, None] >> np.arange(13)) & 1) - 1.0)             # [8192, 13]
    h1 = np.tanh(np.stack([P["b1"][c] + sum(P["W1"][c, k] * a[:, k:k + 9] for k in range(KS))
                           for c in range(CH)], axis=1))              # [8192, 32, 9]
    h2 = np.tanh(np.einsum("dck,bckp->bdp", P["W2"],
                           np.stack([h1[:, :, k:k + 5] for k in range(KS)], axis=2))
                 + P["b2"][None, :, None])                            # [8192, 32, 5]
    return P["b3"] + np.einsum("ck,bck->b", P["W3"], h2)


def distill(H, gmax):
    """Bond table from the window table: for an allowed neighbourhood u of bond
    b (sites b-6..b+6), the log-ratio f(C after the hop) - f(C) averaged over
    the 13 outer sites b-12..b-7, b+7..b+13 taken uniform; then
    eg[u] = round(2^16 exp(clip(G, -gmax, gmax))), 0 for non-hop u."""
    H = np.asarray(H, np.float64)
    ctx = np.arange(8192)
    lo = ctx & 0x3F
    hi = ctx >> 6
    eg = np.zeros(8192, np.uint32)
    G = np.zeros(8192)
    for u in range(8192):
        if ((u >> 6) & 1) == ((u >> 7) & 1):
            continue
        s0 = lo | (u << 6) | (hi << 19)
        s1 = s0 ^ (3 << 12)
        d = np.zeros(8192)
        for o in range(14):
            d += H[(s1 >> o) & 0x1FFF] - H[(s0 >> o) & 0x1FFF]
        G[u] = d.mean()
        eg[u] = int(np.rint(65536.0 * np.exp(np.clip(G[u], -gmax, gmax))))
    return eg, G


def adam(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bond_deltas(H, occ):
    """For every configuration in occ (uint8 [B, L], L >= 26) and every bond
    (b, b+1) whose sites differ: the neighbourhood u of the bond (site b-6 in
    bit 0 ... b+6 in bit 12) and d = f(C after the hop) - f(C), computed as
    the 14 windows holding b or b+1 after minus before (the other windows do
    not change).  Returns (u int64 [m], d float64 [m]) in (sample, bond) order."""
    H = np.asarray(H, np.float64)
    B, L = occ.shape
    assert L >= 26
    us, ds = [], []
    for i in range(B):
        for b in range(L):
            if occ[i, b] == occ[i, (b + 1) % L]:
                continue
            w0 = 0
            for k in range(26):
                w0 |= int(occ[i, (b - 12 + k) % L]) << k
            w1 = w0 ^ (3 << 12)
            d = 0.0
            for o in range(14):
                d += H[(w1 >> o) & 0x1FFF] - H[(w0 >> o) & 0x1FFF]
            us.append((w0 >> 6) & 0x1FFF)
            ds.append(d)
    return np.array(us, np.int64), np.array(ds)


def distill_conditional(H, occ, gmax, min_count):
    """Bond table conditioned on data: G[u] = mean of d over the (sample,
    bond) pairs of occ with neighbourhood u (bond_deltas) where u occurs at
    least min_count times, else the uniform-context average of distill();
    eg = round(2^16 exp(clip(G, -gmax, gmax))), 0 for non-hop u.  Also
    returns the counts."""
    _, G = distill(H, gmax)
    u, d = bond_deltas(H, occ)
    cnt = np.bincount(u, minlength=8192)
    sm = np.bincount(u, weights=d, minlength=8192)
    seen = cnt >= max(min_count, 1)
    G = np.where(seen, sm / np.maximum(cnt, 1), G)
    eg = np.zeros(8192, np.uint32)
    hop = ((np.arange(8192) >> 6) ^ (np.arange(8192) >> 7)) & 1
    for v in np.nonzero(hop)[0]:
        eg[v] = int(np.rint(65536.0 * np.exp(np.clip(G[v], -gmax, gmax))))
    G = np.where(hop == 1, G, 0.0)
    return eg, G, cnt
