"""What the trained guide gains over the method without it.

The guide is trained on the GPU from the plain algorithm's own populations
and ancestries (descendant counts after a lag, Sec. 2.4) and applied with the
exact compensating weights of Sec. 2.2, so psi-hat keeps its target; what
changes is the spread and the finite-Nc bias of the estimates.

  * L = 14 (exact diagonalisation over C(14, 7) = 3432 configurations): the
    learned f(C) tracks ln v(C) of the tilted generator, and at Nc = 100 the
    guided estimator's RMS error against the exact finite-time target
    (1/t) ln Z(s, t) is well below the plain one.
  * L = 50, lambda = 50 (the phase-separated state point of the paper's
    Nc-convergence study, Sec. 5.2, Delta t = 10, t_obs = 1e4): at Nc = 1e3
    the guided estimates of psi and of the activity k carry far less finite-Nc
    bias than plain ones, measured against plain runs at Nc = 1e5.

These are statistical statements about seeded runs; the margins are a factor
of about two below what the runs show.
"""
import numpy as np
import pytest
import torch

from layout import pack
from oracle import ed
from paper_1711_05095_amd import guide, inputs, pd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pd.lib()


def batch(L, N, s, Nc, t_obs, dt, reps, mode, eg=None, seed=77, burn_in=0):
    ps = [pd.make_params(L, N, s, Nc, t_obs, dt, seed=seed, weight_mode=mode, instance=i + 1,
                         burn_in=burn_in) for i in range(reps)]
    sm = pd.Sampler(ps)
    if eg is not None:
        sm.set_guide(eg)
    sm.run(int(round(t_obs / dt)))
    est = [sm.estimates(i) for i in range(reps)]
    sm.close()
    return est


def test_guide_learns_ln_v_and_reduces_error_small_ring():
    L, N, s = 14, 7, 0.2
    r = guide.train_guide(L, N, s, Nc=20000, dt=0.5, lag_cycles=20, snapshots=10,
                          burn_cycles=100, epochs=10, batch=8192, lr=3e-3, decay=1.0, gmax=1.0,
                          seed=1)
    assert r["history"]["val"][-1] < 0.8 * r["history"]["val"][0]
    basis = ed.basis(L, N)
    occ = np.array([[(c >> i) & 1 for i in range(L)] for c in basis], np.uint8)
    f = r["trainer"].f(torch.from_numpy(pack(occ).view(np.int64)).cuda()).cpu().numpy()
    _, v = ed.dominant(L, N, s)
    w = v / v.sum()
    lv = np.log(v)
    fm, lm = (w * f).sum(), (w * lv).sum()
    corr = (w * (f - fm) * (lv - lm)).sum() / np.sqrt((w * (f - fm) ** 2).sum()
                                                      * (w * (lv - lm) ** 2).sum())
    assert corr > 0.95, corr

    t_obs, reps = 200.0, 32
    target = ed.finite_time_scgf(L, N, s, t_obs)
    plain = np.array([e["psi"] for e in batch(L, N, s, 100, t_obs, 0.5, reps, pd.PD_W_MODIFIED)])
    guided = np.array([e["psi"] for e in batch(L, N, s, 100, t_obs, 0.5, reps, pd.PD_W_GUIDED,
                                               r["eg"])])
    rms_p = np.sqrt(np.mean((plain - target) ** 2))
    rms_g = np.sqrt(np.mean((guided - target) ** 2))
    assert rms_g < 0.75 * rms_p, (rms_g, rms_p)


def test_guide_reduces_finite_population_bias_phase_separated():
    L, N, lam, dt, t_obs = 50, 25, 50.0, 10.0, 1.0e4
    s = inputs.s_of_lambda(lam, L)
    r = guide.train_guide(L, N, s, Nc=100000, dt=dt, lag_cycles=5, snapshots=10,
                          burn_cycles=100, epochs=10, batch=8192, lr=1e-3, decay=0.8, gmax=1.0,
                          distill="conditional", min_count=4, seed=3)
    ref = batch(L, N, s, 100000, t_obs, dt, 2, pd.PD_W_MODIFIED, seed=21, burn_in=100)
    psi_ref = np.mean([e["psi_burn"] for e in ref])
    k_ref = np.mean([e["k_hat"] for e in ref])
    plain = batch(L, N, s, 1000, t_obs, dt, 8, pd.PD_W_MODIFIED, seed=21, burn_in=100)
    guided = batch(L, N, s, 1000, t_obs, dt, 8, pd.PD_W_GUIDED, r["eg"], seed=21, burn_in=100)
    bias = lambda est, key, ref_v: abs(np.mean([e[key] for e in est]) - ref_v)
    assert bias(guided, "psi_burn", psi_ref) < 0.5 * bias(plain, "psi_burn", psi_ref)
    assert bias(guided, "k_hat", k_ref) < 0.6 * bias(plain, "k_hat", k_ref)
