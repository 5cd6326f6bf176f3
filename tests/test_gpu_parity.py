"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer results (occupancies, hop counts, accumulated K, ancestor maps) must be
bit-identical for identical Philox counters; floating-point results (the
integral of r dt, ln Upsilon, psi-hat) agree to 1e-12 relative per interval
and 1e-9 relative on a whole run.  The only allowed integer difference is a
selection decided by a point within rounding (1e-9 of the spacing) of an
interval end, which the tests certify case by case (the GPU sums the weights
in a tiled order, the oracle sequentially).
"""
import numpy as np
import pytest
import torch

import oracle
from layout import pack, unpack
from oracle import ed
from paper_1711_05095_amd import inputs, pd

pytestmark = pytest.mark.gpu

MOD, DIR = pd.PD_W_MODIFIED, pd.PD_W_DIRECT


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pd.lib()  # raises if the library is not built


def make(L, N, s, Nc, dt, M=1, seed=0, mode=MOD, sel=pd.PD_SEL_EQ, instance=0, log_cycles=0,
         burn_in=0):
    p = pd.make_params(L, N, s, Nc, M * dt, dt, seed=seed, selection=sel, weight_mode=mode,
                       instance=instance, log_cycles=log_cycles, burn_in=burn_in)
    o = oracle.Oracle(L, N, s, Nc, dt, M=M, seed=seed, instance=instance, mode=mode,
                      selection=sel, burn_in=burn_in)
    return p, o


def check_selection(anc_gpu, ell, d, what):
    """GPU ancestor map == oracle selection on the same log-weights, except at
    certified near-ties."""
    anc_o, lm = oracle.select(ell, d=d)
    diff = np.nonzero(anc_gpu != anc_o)[0]
    if diff.size:
        w = np.exp(ell - ell.max())
        y = np.cumsum(w) * len(ell) / w.sum()
        for j in diff:
            near = np.min(np.abs(y - (j + d)))
            assert near < 1e-9 * max(1.0, j), (what, j, anc_gpu[j], anc_o[j], near)
    assert diff.size <= 2, (what, diff.size)
    return lm


INIT_CASES = [(10, 5, 1000), (2, 1, 7), (64, 32, 300), (65, 20, 257), (100, 50, 1000),
              (128, 64, 513), (400, 200, 600), (512, 100, 256), (30, 0, 100), (30, 30, 100),
              (13, 6, 1)]


@pytest.mark.parametrize("L,N,Nc", INIT_CASES)
def test_init_bit_exact(L, N, Nc):
    print(f"init L={L} N={N} Nc={Nc}", flush=True)
    p, o = make(L, N, 0.1, Nc, 0.5, seed=77 + L)
    S = pd.Sampler(p)
    words, K = S.get_population()
    occ, K0 = o.init()
    assert np.array_equal(words, pack(occ))
    assert np.array_equal(K, K0)


STEP_CASES = [
    (10, 5, 0.4, MOD, 0.1, 1000), (10, 5, -0.4, DIR, 0.1, 1000), (10, 5, 0.0, MOD, 3.0, 300),
    (100, 50, 0.002, MOD, 0.5, 1000), (100, 50, -0.001, DIR, 0.5, 700),
    (65, 30, -0.1, MOD, 1.0, 777), (64, 63, 0.2, MOD, 1.0, 256), (128, 1, 0.3, DIR, 2.0, 300),
    (400, 200, 1.25e-4, MOD, 1.0, 300), (512, 256, 0.0, DIR, 0.3, 256),
    (2, 1, 0.3, MOD, 2.0, 64), (3, 1, -0.2, MOD, 1.5, 65), (20, 0, 0.5, MOD, 1.0, 50),
    (20, 20, 0.5, DIR, 1.0, 50), (13, 6, 0.7, MOD, 5.0, 1),
    # 4297 tiles: more than the prefix kernel keeps in registers (16 per thread)
    (10, 5, 0.4, MOD, 0.1, 1_100_000),
]


@pytest.mark.parametrize("L,N,s,mode,dt,Nc", STEP_CASES)
def test_one_cycle_bit_exact(L, N, s, mode, dt, Nc):
    print(f"step L={L} N={N} s={s} mode={mode} dt={dt} Nc={Nc}", flush=True)
    p, o = make(L, N, s, Nc, dt, M=4, seed=1234, mode=mode, instance=5)
    S = pd.Sampler(p)
    occ = inputs.random_population(L, N, Nc, seed=L * 1000 + Nc)
    K = inputs.random_counts(Nc, seed=Nc)
    S.set_population(pack(occ), K)
    S.step()
    w_gpu, K_gpu = S.get_population()
    Kb_g, A_g, ell_g = S.step_outputs()

    occ_o, K_o = occ.copy(), K.copy()
    Kb_o, A_o, ell_o = o.step(1, occ_o, K_o)
    assert np.array_equal(Kb_g, Kb_o)
    assert np.array_equal(w_gpu, pack(occ_o))
    assert np.array_equal(K_gpu, K_o)
    assert np.allclose(A_g, A_o, rtol=1e-12, atol=1e-300)
    assert np.allclose(ell_g, ell_o, rtol=1e-12, atol=1e-300)

    S.resample()
    anc = S.ancestors()
    assert np.all(np.diff(anc) >= 0) and anc.min() >= 0 and anc.max() < Nc
    lm = check_selection(anc, ell_g, o.eq_offset(1), "cycle 1")
    w2, K2 = S.get_population()
    assert np.array_equal(w2, w_gpu[:, anc]) and np.array_equal(K2, K_gpu[anc])
    e = S.estimates()
    assert e["cycles"] == 1 and e["hops"] == int(Kb_o.sum())
    # the oracle sums the Nc weights one after the other: relative error of the
    # total below (Nc - 1) u, which dominates at a million clones
    assert e["psi"] * dt == pytest.approx(lm, rel=1e-12, abs=1e-15 + Nc * 2.0 ** -53)


@pytest.mark.parametrize("L,N,s,mode,Nc", [(10, 5, 0.4, MOD, 1000), (10, 5, -0.3, DIR, 600),
                                           (100, 50, 0.003, MOD, 1500), (200, 100, -0.0005, MOD, 513)])
def test_lockstep_cycles(L, N, s, mode, Nc):
    """Many cycles through the fused gather: every interval's state, K and
    ancestor map equal the oracle's."""
    print(f"lockstep L={L} s={s} mode={mode} Nc={Nc}", flush=True)
    dt = 0.1 if L == 10 else 0.5
    M = 25
    p, o = make(L, N, s, Nc, dt, M=M, seed=99, mode=mode)
    S = pd.Sampler(p)
    occ, K = o.init()
    for beta in range(1, M + 1):
        S.step()
        Kb_o, A_o, ell_o = o.step(beta, occ, K)
        w_gpu, K_gpu = S.get_population()
        assert np.array_equal(w_gpu, pack(occ)), beta
        assert np.array_equal(K_gpu, K), beta
        S.resample()
        anc = S.ancestors()
        check_selection(anc, ell_o, o.eq_offset(beta), "interval %d" % beta)
        occ, K = np.ascontiguousarray(occ[anc]), K[anc]   # identical unless a certified near-tie
    assert S.estimates()["cycles"] == M


@pytest.mark.parametrize("Nc", [20_000, 300_000])
def test_concentrated_weights_selection(Nc):
    """Strongly concentrated weights (direct form, s = -4, dt = 2: ln Ups = 4 K^beta
    spreads over tens of units) put most new slots on one or a few clones, whose
    long offspring ranges the whole wave writes.  The ancestor map equals the
    oracle's selection on the same weights, and the population follows it."""
    L, N, s, dt = 10, 5, -4.0, 2.0
    print(f"concentrated weights Nc={Nc}", flush=True)
    p, o = make(L, N, s, Nc, dt, M=3, seed=17, mode=DIR)
    S = pd.Sampler(p)
    biggest = 0
    for beta in (1, 2):
        S.step()
        w_gpu, K_gpu = S.get_population()
        _, _, ell = S.step_outputs()
        S.resample()
        anc = S.ancestors()
        assert np.all(np.diff(anc) >= 0) and anc.min() >= 0 and anc.max() < Nc
        check_selection(anc, ell, o.eq_offset(beta), "interval %d" % beta)
        biggest = max(biggest, int(np.bincount(anc, minlength=Nc).max()))
        w2, K2 = S.get_population()
        assert np.array_equal(w2, w_gpu[:, anc]) and np.array_equal(K2, K_gpu[anc])
    assert biggest > Nc // 10, biggest     # the long-range path is exercised


@pytest.mark.parametrize("s,mode", [(-0.4, MOD), (0.4, MOD), (0.2, DIR), (-0.2, DIR)])
def test_whole_run_psi(s, mode):
    w = inputs.SMALL
    M = int(round(w["t_obs"] / w["dt"]))
    print(f"whole run s={s} mode={mode}", flush=True)
    p, o = make(w["L"], w["N"], s, w["Nc"], w["dt"], M=M, seed=w["seed0"], mode=mode)
    S = pd.Sampler(p)
    S.run(M)
    e = S.estimates()
    r = o.run()
    assert e["cycles"] == M
    assert e["hops"] == r["hops"]
    assert e["psi"] == pytest.approx(r["psi"], rel=1e-9)
    assert e["k_hat"] == pytest.approx(r["k_hat"], rel=1e-12)


@pytest.mark.parametrize("mode", [MOD, DIR])
def test_zero_bias_exact_identity(mode):
    p, _ = make(10, 5, 0.0, 1000, 0.1, M=200, seed=3, mode=mode)
    S = pd.Sampler(p)
    S.run(199)
    S.step()
    S.resample()
    assert np.array_equal(S.ancestors(), np.arange(1000, dtype=np.int32))
    e = S.estimates()
    assert e["psi"] == 0.0 and e["cycles"] == 200


def test_graph_run_equals_stepwise_and_checkpoint():
    L, N, Nc, M = 100, 50, 2000, 40
    p, _ = make(L, N, 0.0015, Nc, 0.5, M=M, seed=5)
    A = pd.Sampler(p)
    A.run(M)                       # graph replays
    B = pd.Sampler(p)
    for _ in range(M):             # single launches
        B.step()
        B.resample()
    ea, eb = A.estimates(), B.estimates()
    assert ea == eb
    wa, Ka = A.get_population()
    wb, Kb = B.get_population()
    assert np.array_equal(wa, wb) and np.array_equal(Ka, Kb)
    # checkpoint half way, restore into a fresh context, continue
    C = pd.Sampler(p)
    C.run(M // 2)
    blob = C.save()
    D = pd.Sampler(p)
    D.load(blob)
    D.run(M - M // 2)
    assert D.estimates() == ea
    wd, Kd = D.get_population()
    assert np.array_equal(wd, wa) and np.array_equal(Kd, Ka)


IID = pd.PD_SEL_IID


@pytest.mark.parametrize("L,N,s,mode,Nc", [(10, 5, 0.4, MOD, 1000), (100, 50, 0.003, DIR, 1500),
                                           (65, 30, -0.1, MOD, 257)])
def test_iid_cycles_bit_exact(L, N, s, mode, Nc):
    """[iid] selection: every new slot's ancestor equals the oracle's for the
    same points (near-ties certified), through several cycles."""
    print(f"iid L={L} s={s} Nc={Nc}", flush=True)
    dt, M = 0.5, 6
    p, o = make(L, N, s, Nc, dt, M=M, seed=31, mode=mode, sel=IID)
    S = pd.Sampler(p)
    occ, K = o.init()
    for beta in range(1, M + 1):
        S.step()
        Kb_o, A_o, ell_o = o.step(beta, occ, K)
        w_gpu, K_gpu = S.get_population()
        assert np.array_equal(w_gpu, pack(occ)) and np.array_equal(K_gpu, K), beta
        S.resample()
        anc = S.ancestors()
        pts = o.iid_points(beta)
        anc_o, _ = oracle.select(ell_o, points=pts)
        diff = np.nonzero(anc != anc_o)[0]
        if diff.size:
            w = np.exp(ell_o - ell_o.max())
            y = np.cumsum(w) * Nc / w.sum()
            for j in diff:
                assert np.min(np.abs(y - pts[j])) < 1e-9 * max(1.0, pts[j]), (beta, j)
        assert diff.size <= 2
        occ, K = np.ascontiguousarray(occ[anc]), K[anc]


def test_iid_whole_run_and_variance_against_eq():
    """[iid] whole runs match the oracle; and over seeds the spread of k-hat
    is larger with [iid] than with [eq] (Sec. 4.3)."""
    w = inputs.SMALL
    M = int(round(w["t_obs"] / w["dt"]))
    s = 0.2
    p, o = make(w["L"], w["N"], s, w["Nc"], w["dt"], M=M, seed=5, sel=IID)
    S = pd.Sampler(p)
    S.run(M)
    r = o.run()
    e = S.estimates()
    assert e["hops"] == r["hops"] and e["psi"] == pytest.approx(r["psi"], rel=1e-9)
    R = 32
    spread = {}
    for sel in (pd.PD_SEL_EQ, IID):
        params = [pd.make_params(w["L"], w["N"], s, w["Nc"], w["t_obs"], w["dt"], seed=900 + i,
                                 selection=sel, instance=i) for i in range(R)]
        B = pd.Sampler(params)
        B.run(M)
        spread[sel] = np.std([B.estimates(i)["k_hat"] for i in range(R)], ddof=1)
    assert spread[pd.PD_SEL_EQ] < spread[IID], spread


GUIDED = pd.PD_W_GUIDED


def _guide_tensor(table):
    return torch.from_numpy(table.view(np.int32).copy()).cuda()


@pytest.mark.parametrize("L,N,s,Nc,table_seed", [(10, 5, 0.3, 1000, 1), (100, 50, 0.002, 1500, 2),
                                                 (30, 14, -0.05, 300, 3), (400, 200, 1e-4, 257, 4),
                                                 (6, 3, 0.5, 64, 5), (25, 12, 0.1, 300, 6),
                                                 (26, 13, 0.1, 300, 7), (65, 32, 0.01, 777, 8),
                                                 (512, 256, 1e-4, 130, 9), (12, 12, 0.2, 70, 10)])
def test_guided_cycles_bit_exact(L, N, s, Nc, table_seed):
    """Guided dynamics: states, hop counts and carried K bit-exact with the
    oracle for the same guide table, weights to 1e-12, over several cycles.
    L = 25 and 26 sit either side of the switch from recomputing the summed
    guide rate after a hop to updating it over the 14 changed neighbourhoods;
    L = 65 crosses a word, 512 is the largest ring, and a full ring has no
    allowed bond."""
    from guide_tables import random_table
    print(f"guided L={L} s={s} Nc={Nc}", flush=True)
    _guided_cycles(L, N, s, Nc, random_table(table_seed), dt=0.5, M=5)


def test_guided_wide_table_bit_exact():
    """A guide whose entries reach 2^31 - 1 (the largest allowed): the summed
    rate change of a hop then needs more than 32 bits, the other branch of the
    step kernel's update."""
    from guide_tables import random_table
    print("guided wide table", flush=True)
    table = random_table(12, lo=1 << 30, hi=(1 << 31) - 1)
    _guided_cycles(30, 14, 0.05, 200, table, dt=0.004, M=4)
    _guided_cycles(100, 50, 0.0, 64, table, dt=0.001, M=3)


def _guided_cycles(L, N, s, Nc, table, dt, M):
    p = pd.make_params(L, N, s, Nc, M * dt, dt, seed=17, weight_mode=GUIDED)
    o = oracle.Oracle(L, N, s, Nc, dt, M=M, seed=17, mode=GUIDED, guide=table)
    S = pd.Sampler(p)
    S.set_guide(_guide_tensor(table))
    occ, K = o.init()
    for beta in range(1, M + 1):
        S.step()
        Kb_o, A_o, ell_o = o.step(beta, occ, K)
        w_gpu, K_gpu = S.get_population()
        Kb_g, A_g, ell_g = S.step_outputs()
        assert np.array_equal(Kb_g, Kb_o), beta
        assert np.array_equal(w_gpu, pack(occ)) and np.array_equal(K_gpu, K), beta
        assert np.allclose(A_g, A_o, rtol=1e-12) and np.allclose(ell_g, ell_o, rtol=1e-11,
                                                                 atol=1e-12), beta
        S.resample()
        anc = S.ancestors()
        check_selection(anc, ell_o, o.eq_offset(beta), "guided interval %d" % beta)
        occ, K = np.ascontiguousarray(occ[anc]), K[anc]


def test_full_size_iid_direct_sampled():
    """Direct weights (e^{-s K}) and [iid] selection at Nc = 1e6: 2000 sampled
    clones stepped by the oracle, bit-exact; every new slot's point (the
    oracle's [iid] points) lies in the interval of the clone the GPU chose,
    with the intervals from a long-double cumulative sum of the GPU's weights
    and a tolerance of 1e-6 spacings (the GPU's two-level FP64 scan is good to
    ~2e-7 here, the oracle's sequential one only to ~1e-4)."""
    L, N, lam, Nc, dt = 100, 50, 20.0, 1_000_000, 0.5
    s = inputs.s_of_lambda(lam, L)
    print(f"full size iid direct L={L} Nc={Nc}", flush=True)
    p, o = make(L, N, s, Nc, dt, M=10, seed=2025, mode=DIR, sel=IID)
    S = pd.Sampler(p)
    S.run(3)
    words, K = S.get_population()
    rng = np.random.default_rng(1)
    slots = np.sort(rng.choice(Nc, 2000, replace=False))
    occ_s = unpack(words[:, slots], L)
    K_s = K[slots].copy()
    S.step()
    w_gpu, K_gpu = S.get_population()
    Kb_g, A_g, ell_g = S.step_outputs()
    Kb_o, A_o, ell_o = o.step_slots(4, slots, occ_s, K_s)
    assert np.array_equal(Kb_g[slots], Kb_o)
    assert np.array_equal(w_gpu[:, slots], pack(occ_s))
    assert np.array_equal(K_gpu[slots], K_s)
    assert np.allclose(ell_g[slots], ell_o, rtol=1e-12, atol=1e-300)
    S.resample()
    anc = S.ancestors().astype(np.int64)
    assert anc.min() >= 0 and anc.max() < Nc
    pts = o.iid_points(4)
    w = np.exp((ell_g - ell_g.max()).astype(np.longdouble))
    y = np.cumsum(w)
    y = y * Nc / y[-1]
    lo = np.where(anc > 0, y[np.maximum(anc - 1, 0)], 0.0)
    hi = np.where(anc < Nc - 1, y[anc], np.inf)
    tol = 1e-6
    assert np.all(lo - tol <= pts) and np.all(pts < hi + tol)


def test_twenty_million_clones_sampled():
    """Nc = 2e7 (78125 tiles: 31-bit slot arithmetic, the prefix kernel's path
    that re-reads its tiles, interval ends up to 2e7 spacings): 2000 sampled
    clones stepped by the oracle; the selection by its defining properties
    (a non-decreasing map, every clone copied floor or ceil of Nc w_k / sum w
    times), since the oracle's own sequential sum of 2e7 weights is only good
    to ~0.04 spacings here; psi against the exactly rounded sum of the GPU's
    weights."""
    import math
    L, N, s, Nc, dt = 10, 5, 0.3, 20_000_000, 0.1
    print(f"large population L={L} Nc={Nc}", flush=True)
    p, o = make(L, N, s, Nc, dt, M=4, seed=77)
    S = pd.Sampler(p)
    S.run(2)
    words, K = S.get_population()
    rng = np.random.default_rng(9)
    slots = np.sort(rng.choice(Nc, 2000, replace=False))
    occ_s = unpack(words[:, slots], L)
    K_s = K[slots].copy()
    psi2 = S.estimates()["psi"] * 2 * dt
    S.step()
    w_gpu, K_gpu = S.get_population()
    Kb_g, A_g, ell_g = S.step_outputs()
    Kb_o, A_o, ell_o = o.step_slots(3, slots, occ_s, K_s)
    assert np.array_equal(Kb_g[slots], Kb_o)
    assert np.array_equal(w_gpu[:, slots], pack(occ_s))
    assert np.array_equal(K_gpu[slots], K_s)
    assert np.allclose(ell_g[slots], ell_o, rtol=1e-12, atol=1e-300)
    S.resample()
    anc = S.ancestors()
    assert np.all(np.diff(anc) >= 0) and anc[0] >= 0 and anc[-1] < Nc
    counts = np.bincount(anc, minlength=Nc)
    wgt = np.exp(ell_g - ell_g.max())
    mean = Nc * wgt / wgt.sum()
    assert np.all(counts >= np.floor(mean - 1e-6)) and np.all(counts <= np.ceil(mean + 1e-6))
    exact = ell_g.max() + math.log(math.fsum(wgt) / Nc)
    lb3 = S.estimates()["psi"] * 3 * dt - psi2
    assert lb3 == pytest.approx(exact, rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("L,N,s,dt", [(100, 50, 0.002, 0.5), (400, 200, 1e-4, 1.0)])
def test_guided_full_size_sampled(L, N, s, dt):
    """A guided launch large enough to be split in two (3907 tiles), with 2- and
    7-word states: the third cycle runs with an event budget from the second,
    so clones are handed on to the second launch; 2000 sampled clones stepped
    by the oracle, bit-exact, and the selection (which reads the third launch's
    tile aggregates) checked against the oracle's on the GPU's log-weights."""
    from guide_tables import random_table
    Nc = 1_000_000
    print(f"guided full size L={L} Nc={Nc}", flush=True)
    table = random_table(6)
    p = pd.make_params(L, N, s, Nc, 10 * dt, dt, seed=41, weight_mode=GUIDED)
    o = oracle.Oracle(L, N, s, Nc, dt, M=10, seed=41, mode=GUIDED, guide=table)
    S = pd.Sampler(p)
    S.set_guide(_guide_tensor(table))
    S.run(2)
    words, K = S.get_population()
    rng = np.random.default_rng(5)
    slots = np.sort(rng.choice(Nc, 2000, replace=False))
    occ_s = unpack(words[:, slots], L)
    K_s = K[slots].copy()
    S.step()
    w_gpu, K_gpu = S.get_population()
    Kb_g, A_g, ell_g = S.step_outputs()
    Kb_o, A_o, ell_o = o.step_slots(3, slots, occ_s, K_s)
    # the budget is 1.1 x the mean events + 2: a quarter of the clones or so
    # exceed it and finish in the second launch
    assert np.mean(Kb_g + 1 > 1.1 * (Kb_g.mean() + 1) + 2) > 0.05
    assert np.array_equal(Kb_g[slots], Kb_o)
    assert np.array_equal(w_gpu[:, slots], pack(occ_s))
    assert np.array_equal(K_gpu[slots], K_s)
    assert np.allclose(A_g[slots], A_o, rtol=1e-12)
    assert np.allclose(ell_g[slots], ell_o, rtol=1e-11, atol=1e-12)
    S.resample()
    check_selection(S.ancestors(), ell_g, o.eq_offset(3), "guided full size")


def test_bench_guided_launch_sampled():
    """The guided leg of bench.py's guided-rate workload as it is timed: 32
    guided instances x Nc=1e5 at L=100, lambda=15 in one context (the stage in
    two launches, escape rates carried between intervals), 8 single cycles and
    16 graph-replayed ones; then one cycle checked on 1000 sampled clones of
    three instances against the oracle and those instances' whole selections."""
    from guide_tables import random_table
    L, N, lam, dt, Nc = 100, 50, 15.0, 0.5, 100_000
    s = inputs.s_of_lambda(lam, L)
    table = random_table(12)
    print("bench guided: 32 instances x Nc=%d" % Nc, flush=True)
    params = [pd.make_params(L, N, s, Nc, 60 * dt, dt, seed=2000 + i, instance=i,
                             weight_mode=GUIDED) for i in range(32)]
    S = pd.Sampler(params)
    S.set_guide(_guide_tensor(table))
    S.set_tuning(4, 13, 16, 1)
    S.run(0)
    S.run(8)
    S.run(16)
    beta = 25
    assert S.estimates(0)["cycles"] == beta - 1
    rng = np.random.default_rng(6)
    picks = [0, 17, 31]
    before = {}
    for i in picks:
        words, K = S.get_population(i)
        slots = np.sort(rng.choice(Nc, 1000, replace=False))
        before[i] = (slots, unpack(words[:, slots], L), K[slots].copy())
    S.step()
    ells = {}
    for i in picks:
        slots, occ_s, K_s = before[i]
        o = oracle.Oracle(L, N, s, Nc, dt, M=60, seed=2000 + i, instance=i, mode=GUIDED,
                          guide=table)
        Kb_o, A_o, ell_o = o.step_slots(beta, slots, occ_s, K_s)
        w_g, K_g = S.get_population(i)
        Kb_g, A_g, ell_g = S.step_outputs(i)
        assert np.array_equal(Kb_g[slots], Kb_o), i
        assert np.array_equal(w_g[:, slots], pack(occ_s)), i
        assert np.array_equal(K_g[slots], K_s), i
        assert np.allclose(A_g[slots], A_o, rtol=1e-12), i
        assert np.allclose(ell_g[slots], ell_o, rtol=1e-11, atol=1e-12), i
        ells[i] = (ell_g, o.eq_offset(beta))
    S.resample()
    for i in picks:
        check_selection(S.ancestors(i), ells[i][0], ells[i][1], "bench guided %d" % i)


def test_guided_whole_run_and_guide_validation():
    from guide_tables import constant_table, random_table
    w = inputs.SMALL
    M = 200
    table = random_table(9)
    p = pd.make_params(w["L"], w["N"], 0.3, w["Nc"], M * w["dt"], w["dt"], seed=3,
                       weight_mode=GUIDED)
    S = pd.Sampler(p)
    with pytest.raises(pd.PdError) as e:
        S.run(1)
    assert e.value.status == pd.PD_ESTATE
    bad = table.copy()
    bad[0] = 5   # a non-hop neighbourhood must hold 0
    with pytest.raises(pd.PdError) as e:
        S.set_guide(_guide_tensor(bad))
    assert e.value.status == pd.PD_EINVAL
    shifted = torch.zeros(8193, dtype=torch.int32, device="cuda")
    shifted[1:] = _guide_tensor(table)
    with pytest.raises(pd.PdError) as e:   # 4 bytes past a 16-byte boundary
        S.set_guide(shifted[1:])
    assert e.value.status == pd.PD_EINVAL
    S.set_guide(_guide_tensor(table))
    S.run(M)
    r = oracle.Oracle(w["L"], w["N"], 0.3, w["Nc"], w["dt"], M=M, seed=3, mode=GUIDED,
                      guide=table).run()
    e = S.estimates()
    assert e["hops"] == r["hops"] and e["psi"] == pytest.approx(r["psi"], rel=1e-9)
    # constant table at s = 0: exactly the modified dynamics' identity weights
    p0 = pd.make_params(w["L"], w["N"], 0.0, 500, 20 * w["dt"], w["dt"], weight_mode=GUIDED)
    S0 = pd.Sampler(p0)
    S0.set_guide(_guide_tensor(constant_table()))
    S0.run(20)
    assert S0.estimates()["psi"] == 0.0


def test_origin_tracking_composes_ancestor_maps():
    """Carried origins equal the composition of the cloning stages' ancestor
    maps, and descendant counts sum to Nc."""
    L, N, Nc, M = 100, 50, 3000, 12
    p = pd.make_params(L, N, 0.002, Nc, 40 * 0.5, 0.5, seed=4, track_origin=1)
    S = pd.Sampler(p)
    S.run(5)
    S.reset_origin()
    assert np.array_equal(S.origin(), np.arange(Nc, dtype=np.int32))
    comp = np.arange(Nc)
    for _ in range(M):
        S.step()
        S.resample()
        comp = comp[S.ancestors()]
    assert np.array_equal(S.origin(), comp)
    assert np.bincount(S.origin(), minlength=Nc).sum() == Nc


def test_checkpoint_and_autotune_keep_origins():
    """Carried origins survive a checkpoint round trip, and the autotuner (which
    runs trial cycles and restores the context) leaves them as an uninterrupted
    run has them."""
    p = pd.make_params(60, 30, 0.01, 2000, 10.0, 0.5, seed=93, track_origin=1)
    A = pd.Sampler(p)
    A.run(3)
    A.reset_origin()
    A.run(5)
    blob = A.save()
    A.run(4)
    want = A.origin()
    A.load(blob)
    A.run(4)
    assert np.array_equal(A.origin(), want)
    B = pd.Sampler(p)
    B.run(3)
    B.reset_origin()
    B.run(5)
    B.autotune(2)
    B.run(4)
    assert np.array_equal(B.origin(), want)
    assert B.estimates() == A.estimates()


def test_load_rejects_a_corrupt_checkpoint():
    """pd_load checks a checkpoint whole before uploading any of it: an origin
    outside [0, Nc), a bit beyond site L, a missing particle or a wrong magic
    is rejected with the context unchanged, and a nonzero guided hand-on count
    in the image is not taken over."""
    L, Nc = 60, 2000
    p = pd.make_params(L, 30, 0.01, Nc, 10.0, 0.5, seed=95, track_origin=1)
    A = pd.Sampler(p)
    A.run(3)
    A.reset_origin()
    A.run(2)
    blob = A.save()
    A.run(4)
    want = (A.get_population(), A.origin(), A.estimates())
    ctl = blob.nbytes - 24 - 8 * Nc * 2 - (4 * Nc + 7) // 8 * 8   # InstCtl image
    states = 24 + ctl                                             # [W=1][Nc] words, then K
    origins = states + 16 * Nc
    B = pd.Sampler(p)
    B.run(3)
    B.reset_origin()
    B.run(2)

    def corrupt(edit):
        bad = blob.copy()
        edit(bad)
        with pytest.raises(pd.PdError) as e:
            B.load(bad)
        assert e.value.status == pd.PD_EINVAL

    def set_origin(b):
        b[origins + 4 * 7:origins + 4 * 8] = np.array([Nc], np.int32).view(np.uint8)
    corrupt(set_origin)

    def set_bit_beyond_L(b):
        w = b[states + 8 * 11:states + 8 * 12].view(np.uint64)
        w[0] |= np.uint64(1) << np.uint64(L)
    corrupt(set_bit_beyond_L)

    def drop_particle(b):
        w = b[states + 8 * 13:states + 8 * 14].view(np.uint64)
        w[0] &= w[0] - np.uint64(1)
    corrupt(drop_particle)

    def wrong_magic(b):
        b[0] ^= 1
    corrupt(wrong_magic)

    B.run(4)   # every load was refused: B runs on as A did
    assert np.array_equal(B.get_population()[0], want[0][0])
    assert np.array_equal(B.origin(), want[1]) and B.estimates() == want[2]

    hand_on = blob.copy()
    hand_on[24 + 8:24 + 12] = np.array([12345], np.uint32).view(np.uint8)
    B.load(hand_on)
    B.run(4)
    assert np.array_equal(B.get_population()[0], want[0][0])
    assert np.array_equal(B.origin(), want[1]) and B.estimates() == want[2]


def test_compacting_variant_carries_origins():
    """Variant 4 (compaction between rounds) carries origin ids exactly as
    variant 0 does."""
    out = []
    for variant in (0, 4):
        p = pd.make_params(100, 50, 0.01, 3000, 5.0, 0.5, seed=91, track_origin=1)
        S = pd.Sampler(p)
        S.set_tuning(variant, 8, 16)
        S.run(2)
        S.reset_origin()
        S.run(8)
        out.append((S.origin(), S.get_population(), S.estimates()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1][0], out[1][1][0]) and out[0][2] == out[1][2]


def test_launch_variants_bit_identical():
    """Neither kernel variant nor refill threshold nor graph length nor scan
    tiling changes any result: every random number is keyed by clone slot, and
    every tile is scanned the same way."""
    specs = [(10, 5, 0.3, 1000, 0.1, MOD), (100, 50, 0.002, 3000, 0.5, MOD),
             (400, 200, 1e-4, 700, 1.0, MOD), (65, 32, -0.05, 257, 0.5, DIR),
             (512, 256, 0.0, 300, 0.2, MOD), (30, 0, 0.1, 100, 0.5, MOD),
             (200, 100, 5e-4, 2000, 2.0, DIR)]
    M = 10
    params = [pd.make_params(L, N, s, Nc, M * dt, dt, seed=70 + i, instance=i, weight_mode=wm)
              for i, (L, N, s, Nc, dt, wm) in enumerate(specs)]
    ref = None
    for variant, refill, graph, tpb in [(0, 8, 16, 1), (1, 1, 16, 1), (1, 8, 0, 2), (1, 32, 4, 1),
                                        (1, 64, 2, 4), (4, 8, 16, 8), (4, 8, 0, 1), (2, 8, 2, 1),
                                        (3, 16, 16, 2), (5, 13, 16, 1), (5, 8, 0, 2)]:
        S = pd.Sampler(params)
        S.set_tuning(variant, refill, graph, tpb)
        S.run(M)
        out = [(S.estimates(i), S.get_population(i)) for i in range(len(params))]
        if ref is None:
            ref = out
            continue
        for (ea, (wa, Ka)), (eb, (wb, Kb)) in zip(ref, out):
            assert ea == eb, (variant, refill)
            assert np.array_equal(wa, wb) and np.array_equal(Ka, Kb), (variant, refill)


def test_autotune_leaves_the_run_unchanged():
    p, _ = make(100, 50, 0.002, 5000, 0.5, M=30, seed=8)
    A = pd.Sampler(p)
    A.run(10)
    best = A.autotune(2)
    assert best["step_variant"] in (0, 1, 2, 3, 4)
    A.run(20)
    B = pd.Sampler(p)
    B.run(30)
    assert A.estimates() == B.estimates()
    wa, Ka = A.get_population()
    wb, Kb = B.get_population()
    assert np.array_equal(wa, wb) and np.array_equal(Ka, Kb)


def test_batch_equals_separate():
    specs = [(10, 5, 0.3, 1000, 0.1), (100, 50, 0.002, 3000, 0.5), (400, 200, 1e-4, 700, 1.0),
             (65, 32, -0.05, 257, 0.5)]
    M = 12
    params = [pd.make_params(L, N, s, Nc, M * dt, dt, seed=40 + i, instance=i)
              for i, (L, N, s, Nc, dt) in enumerate(specs)]
    B = pd.Sampler(params)
    B.run(M)
    for i, q in enumerate(params):
        S = pd.Sampler(q)
        S.run(M)
        assert S.estimates() == B.estimates(i)
        ws, Ks = S.get_population()
        wb, Kb = B.get_population(i)
        assert np.array_equal(ws, wb) and np.array_equal(Ks, Kb)


@pytest.mark.parametrize("variant", [4, 5])
def test_mixed_forms_in_one_context_equal_separate(variant):
    """One context holding instances of every weight form and both selections
    (modified, direct, guided; [eq] and [iid]), of uneven L and Nc, run through
    graph-replayed cycles with origins tracked: each instance equals, bit for
    bit, the same instance alone in a context of its own (with the plain
    instances in one launch per word count, or all in one persistent launch)."""
    from guide_tables import random_table
    table = _guide_tensor(random_table(11))
    EQ = pd.PD_SEL_EQ
    specs = [(40, 20, 0.05, 1500, 0.5, MOD, EQ), (100, 50, 0.002, 2600, 0.5, GUIDED, EQ),
             (30, 14, 0.1, 777, 0.3, DIR, IID), (20, 9, 0.2, 300, 0.4, GUIDED, IID),
             (512, 256, 1e-4, 130, 1.0, MOD, IID)]
    M = 9
    params = [pd.make_params(L, N, s, Nc, M * dt, dt, seed=80 + i, instance=i, weight_mode=mode,
                             selection=sel, track_origin=1)
              for i, (L, N, s, Nc, dt, mode, sel) in enumerate(specs)]
    B = pd.Sampler(params)
    B.set_guide(table)
    B.set_tuning(variant, 13, 16, 1)
    B.run(3)
    for i in range(len(params)):
        B.reset_origin(i)
    B.run(M - 3)
    for i, q in enumerate(params):
        S = pd.Sampler(q)
        if q.weight_mode == GUIDED:
            S.set_guide(table)
        S.run(3)
        S.reset_origin()
        S.run(M - 3)
        assert S.estimates() == B.estimates(i), i
        ws, Ks = S.get_population()
        wb, Kb = B.get_population(i)
        assert np.array_equal(ws, wb) and np.array_equal(Ks, Kb), i
        assert np.array_equal(S.origin(), B.origin(i)), i
        S.close()


@pytest.mark.parametrize("guided", [False, True])
def test_split_launch_equals_unsplit(guided):
    """Four instances of 938 tiles each, in one context (a step launch of 3752
    tiles; the guided stage is then split in two, the clones past the event
    budget finishing in a second launch), also restored from a mid-run
    checkpoint, and each alone (one launch).  Every result, the carried origins
    included, is the same bit for bit."""
    from guide_tables import random_table
    specs = [(10, 5, 0.3, 0.1), (30, 14, -0.05, 0.5), (64, 30, 0.01, 0.3), (20, 9, 0.2, 0.4)]
    Nc, M = 240_000, 4
    mode = GUIDED if guided else MOD
    params = [pd.make_params(L, N, s, Nc, M * dt, dt, seed=60 + i, instance=i, weight_mode=mode,
                             track_origin=1)
              for i, (L, N, s, dt) in enumerate(specs)]
    table = _guide_tensor(random_table(8)) if guided else None
    print(f"split vs unsplit guided={guided}", flush=True)

    def sampler(q):
        S = pd.Sampler(q)
        if guided:
            S.set_guide(table)
        for i in range(S.n):
            S.reset_origin(i)
        return S

    B = sampler(params)
    B.run(2)
    blob = B.save()      # mid-run checkpoint: the event budget is part of it
    B.run(M - 2)
    R = sampler(params)
    R.load(blob)
    R.run(M - 2)
    for i, q in enumerate(params):
        S = sampler(q)
        S.run(M)
        for X in (B, R):
            assert S.estimates() == X.estimates(i), i
            ws, Ks = S.get_population()
            wb, Kb = X.get_population(i)
            assert np.array_equal(ws, wb) and np.array_equal(Ks, Kb), i
            assert np.array_equal(S.origin(), X.origin(i)), i


def test_small_workload_matches_exact_diagonalisation():
    """All 9 biases x 16 seeds of the L=10 workload as one batch; the mean of
    psi-hat over seeds is within 3 sigma of (1/t_obs) ln Z(s, t_obs)."""
    w = inputs.SMALL
    M = int(round(w["t_obs"] / w["dt"]))
    R = 16
    params = []
    for si, s in enumerate(w["s_values"]):
        for r in range(R):
            params.append(pd.make_params(w["L"], w["N"], s, w["Nc"], w["t_obs"], w["dt"],
                                         seed=w["seed0"] + r, instance=si))
    B = pd.Sampler(params)
    B.run(M)
    for si, s in enumerate(w["s_values"]):
        psis = np.array([B.estimates(si * R + r)["psi"] for r in range(R)])
        target = ed.finite_time_scgf(w["L"], w["N"], s, w["t_obs"])
        sig = psis.std(ddof=1) / np.sqrt(R)
        assert abs(psis.mean() - target) < 3 * sig + 2e-4, (s, psis.mean(), target, sig)
        if s == 0.0:
            assert np.all(psis == 0.0)


def test_edge_fillings_and_single_particle():
    for N in (0, 12):
        p, _ = make(12, N, 0.5, 300, 0.5, M=20, seed=1)
        S = pd.Sampler(p)
        S.run(20)
        e = S.estimates()
        assert e["psi"] == 0.0 and e["hops"] == 0 and e["k_hat"] == 0.0
    s = 0.3
    p, _ = make(10, 1, s, 500, 0.1, M=100, seed=2)
    S = pd.Sampler(p)
    S.run(100)
    assert S.estimates()["psi"] == pytest.approx(2 * (np.exp(-s) - 1), abs=1e-12)


def test_call_order_and_validation():
    p, _ = make(10, 5, 0.1, 100, 0.1, M=10)
    S = pd.Sampler(p)
    with pytest.raises(pd.PdError) as e:
        S.resample()
    assert e.value.status == pd.PD_ESTATE
    S.step()
    with pytest.raises(pd.PdError) as e:
        S.step()
    assert e.value.status == pd.PD_ESTATE
    with pytest.raises(pd.PdError) as e:
        S.ancestors()
    assert e.value.status == pd.PD_ESTATE
    S.resample()
    bad = pack(inputs.random_population(10, 4, 100, 0))
    with pytest.raises(pd.PdError) as e:
        S.set_population(bad, np.zeros(100, np.uint64))
    assert e.value.status == pd.PD_EINVAL


def test_bench_sweep_launch_sampled():
    """The headline workload in the launch configuration bench.py times: the
    L=100 transition sweep (32 lambdas x Nc=1e5 in one context), the
    autotuner's choice with graphs of 10 cycles, 5 warm-up cycles and 20
    graph-replayed ones.  The next cycle is checked on 1000 sampled clones of
    three instances against the oracle (states, hops, log-weights), and the
    whole selection of those instances against the oracle's on the GPU's
    log-weights."""
    w = inputs.SWEEP
    L, N, dt, Nc = w["L"], w["N"], w["dt"], 100_000
    lams = w["lambdas"]
    print("bench sweep: %d instances x Nc=%d" % (len(lams), Nc), flush=True)
    params = [pd.make_params(L, N, inputs.s_of_lambda(lam, L), Nc, 60 * dt, dt,
                             seed=w["seed0"] + i, instance=i) for i, lam in enumerate(lams)]
    S = pd.Sampler(params)
    t = S.autotune(8)
    S.set_tuning(t["step_variant"], t["refill"], 10, t["scan_tiles"])
    S.run(0)
    S.run(5)
    S.run(20)
    beta = 26
    assert S.estimates(0)["cycles"] == beta - 1
    rng = np.random.default_rng(5)
    picks = [0, 13, 31]
    before = {}
    for i in picks:
        words, K = S.get_population(i)
        slots = np.sort(rng.choice(Nc, 1000, replace=False))
        before[i] = (slots, unpack(words[:, slots], L), K[slots].copy())
    S.step()
    ells = {}
    for i in picks:
        slots, occ_s, K_s = before[i]
        o = oracle.Oracle(L, N, inputs.s_of_lambda(lams[i], L), Nc, dt, M=60,
                          seed=w["seed0"] + i, instance=i)
        Kb_o, A_o, ell_o = o.step_slots(beta, slots, occ_s, K_s)
        w_g, K_g = S.get_population(i)
        Kb_g, A_g, ell_g = S.step_outputs(i)
        assert np.array_equal(Kb_g[slots], Kb_o), i
        assert np.array_equal(w_g[:, slots], pack(occ_s)), i
        assert np.array_equal(K_g[slots], K_s), i
        assert np.allclose(ell_g[slots], ell_o, rtol=1e-12, atol=1e-300), i
        ells[i] = (ell_g, o.eq_offset(beta))
    S.resample()
    for i in picks:
        check_selection(S.ancestors(i), ells[i][0], ells[i][1], "bench sweep %d" % i)


@pytest.mark.parametrize("L,N,lam,Nc,dt", [(100, 50, 20.0, 100_000, 0.5),
                                           (100, 50, 20.0, 1_000_000, 0.5),
                                           (400, 200, 20.0, 1_000_000, 1.0)])
def test_full_size_sampled(L, N, lam, Nc, dt):
    """At the full workload sizes: one cycle from a GPU-evolved population,
    2000 sampled clones stepped by the oracle; the whole selection checked
    against the oracle's on the GPU's log-weights."""
    print(f"full size L={L} Nc={Nc}", flush=True)
    s = inputs.s_of_lambda(lam, L)
    p, o = make(L, N, s, Nc, dt, M=10, seed=2024)
    S = pd.Sampler(p)
    S.run(3)
    words, K = S.get_population()
    rng = np.random.default_rng(0)
    slots = np.sort(rng.choice(Nc, 2000, replace=False))
    occ_s = unpack(words[:, slots], L)
    K_s = K[slots].copy()
    assert np.all(occ_s.sum(axis=1) == N)
    S.step()
    w_gpu, K_gpu = S.get_population()
    Kb_g, A_g, ell_g = S.step_outputs()
    Kb_o, A_o, ell_o = o.step_slots(4, slots, occ_s, K_s)
    assert np.array_equal(Kb_g[slots], Kb_o)
    assert np.array_equal(w_gpu[:, slots], pack(occ_s))
    assert np.array_equal(K_gpu[slots], K_s)
    assert np.allclose(ell_g[slots], ell_o, rtol=1e-12, atol=1e-300)
    S.resample()
    anc = S.ancestors()
    check_selection(anc, ell_g, o.eq_offset(4), "full size")
    counts = np.bincount(anc, minlength=Nc)
    wgt = np.exp(ell_g - ell_g.max())
    mean = Nc * wgt / wgt.sum()
    assert np.all(counts >= np.floor(mean - 1e-6)) and np.all(counts <= np.ceil(mean + 1e-6))
