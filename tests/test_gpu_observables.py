"""Observables over the population through the C ABI (pd_density_mode,
pd_mean, pd_histogram) against the plain definitions in oracle/observables.py,
and two physical checks of the density mode (eq. fourdens): its exact mean
over the uniform distribution at s = 0, and the phase separation of Sec. 3.3
at lambda = 50 > lambda_c = 2 pi^2."""
import numpy as np
import pytest
import torch

from layout import unpack
from oracle import observables as ob
from paper_1711_05095_amd import inputs, pd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pd.lib()


@pytest.mark.parametrize("L,N,s,Nc,n", [(13, 6, 0.2, 700, 1), (100, 50, 0.002, 3000, 1),
                                        (100, 50, 0.002, 3000, -3), (400, 200, 1e-4, 1025, 2)])
def test_density_mode_and_means_match_oracle(L, N, s, Nc, n):
    p = pd.make_params(L, N, s, Nc, 20.0, 0.5, seed=5, track_origin=1)
    S = pd.Sampler(p)
    S.run(3)
    S.reset_origin()
    rho0 = S.density_mode(n)
    words, _ = S.get_population()
    want0 = ob.density_mode(unpack(words, L), n)
    assert np.allclose(rho0.cpu().numpy(), want0, rtol=1e-12, atol=1e-13)
    assert S.mean(rho0) == pytest.approx(ob.population_mean(want0), rel=1e-12)
    S.run(7)
    origin = S.origin()
    assert S.mean(rho0, ancestral=True) == pytest.approx(ob.ancestral_mean(want0, origin),
                                                         rel=1e-12)
    rho1 = S.density_mode(n)
    words, _ = S.get_population()
    assert np.allclose(rho1.cpu().numpy(), ob.density_mode(unpack(words, L), n), rtol=1e-12,
                       atol=1e-13)


def test_mean_needs_origins_and_rejects_mid_cycle():
    p = pd.make_params(20, 10, 0.1, 100, 5.0, 0.5, seed=1)
    S = pd.Sampler(p)
    v = torch.zeros(100, dtype=torch.float64, device="cuda")
    with pytest.raises(pd.PdError) as e:
        S.mean(v, ancestral=True)
    assert e.value.status == pd.PD_ESTATE
    S.step()
    with pytest.raises(pd.PdError) as e:
        S.mean(v)
    assert e.value.status == pd.PD_ESTATE
    S.resample()
    assert S.mean(v) == 0.0


def test_density_mode_physics():
    L, N, Nc = 50, 25, 100_000
    # s = 0: the population stays uniform over C(L, N), where the mean is exact
    S = pd.Sampler(pd.make_params(L, N, 0.0, Nc, 50.0, 0.5, seed=3))
    S.run(20)
    r = S.density_mode(1)
    exact = N * (L - N) / (L * (L - 1))
    se = r.std().item() / np.sqrt(Nc)
    assert abs(S.mean(r) - exact) <= 5 * se
    # lambda = 50: the biased population phase-separates (Sec. 3.3, Fig. dpqGraph)
    S = pd.Sampler(pd.make_params(L, N, inputs.s_of_lambda(50.0, L), Nc, 3000.0, 10.0, seed=4))
    S.run(300)
    assert S.mean(S.density_mode(1)) > 4 * exact


@pytest.mark.parametrize("L,N,s,Nc", [(100, 50, 0.002, 3000), (20, 10, 0.3, 600_000)])
def test_histogram_matches_oracle(L, N, s, Nc):
    """pd_histogram against the oracle, count for count: the activity K^beta of
    the last interval over the current clones (p_end) and the same quantity
    recorded at an origin reset, over the ancestors of the clones some cycles
    later (p_ave); the density mode in fine bins; and values that are NaN,
    infinite or outside the range.  Nc = 6e5 runs the kernel's grid-stride
    loop (2048 blocks)."""
    p = pd.make_params(L, N, s, Nc, 20.0, 0.5, seed=8, track_origin=1)
    S = pd.Sampler(p)
    S.run(3)
    S.step()
    Kb, _, _ = S.step_outputs()
    S.resample()
    kb_now = Kb[S.ancestors()].astype(np.float64)    # K^beta of each current clone
    kb = torch.from_numpy(kb_now).cuda()
    S.reset_origin()
    top = float(kb_now.max()) + 2
    for lo, width, nb in [(-0.5, 1.0, int(top) + 1), (0.0, 1.0, int(top)), (2.0, 3.0, 7),
                          (0.0, 1.0, 1)]:
        assert np.array_equal(S.histogram(kb, lo, width, nb), ob.histogram(kb_now, lo, width, nb))
    S.run(6)
    origin = S.origin()
    assert np.array_equal(S.histogram(kb, -0.5, 1.0, int(top) + 1, ancestral=True),
                          ob.histogram(kb_now, -0.5, 1.0, int(top) + 1, origin=origin))
    rho = S.density_mode(1)
    r = rho.cpu().numpy()
    assert np.array_equal(S.histogram(rho, 0.0, 0.05, 4096), ob.histogram(r, 0.0, 0.05, 4096))
    odd = r.copy()
    odd[::7] = np.nan
    odd[3::11] = np.inf
    odd[5::13] = -1.0
    t = torch.from_numpy(odd).cuda()
    assert np.array_equal(S.histogram(t, 0.0, 0.25, 40), ob.histogram(odd, 0.0, 0.25, 40))
    assert S.histogram(t, 1e6, 1.0, 10).sum() == 0


def test_histogram_validation():
    p = pd.make_params(20, 10, 0.1, 100, 5.0, 0.5, seed=1)
    S = pd.Sampler(p)
    v = torch.zeros(100, dtype=torch.float64, device="cuda")
    for lo, width, nb in [(0.0, 1.0, 0), (0.0, 1.0, 4097), (0.0, 0.0, 10), (0.0, -1.0, 10),
                          (float("nan"), 1.0, 10), (0.0, float("inf"), 10)]:
        with pytest.raises(pd.PdError) as e:
            S.histogram(v, lo, width, nb)
        assert e.value.status == pd.PD_EINVAL, (lo, width, nb)
    with pytest.raises(pd.PdError) as e:
        S.histogram(v, 0.0, 1.0, 10, ancestral=True)
    assert e.value.status == pd.PD_ESTATE
    S.step()
    with pytest.raises(pd.PdError) as e:
        S.histogram(v, 0.0, 1.0, 10)
    assert e.value.status == pd.PD_ESTATE
    S.resample()
    assert S.histogram(v, -0.5, 1.0, 3).tolist() == [100, 0, 0]


def test_descendant_counts_equal_origin_histogram():
    """pd_descendant_counts counts, per slot of the last origin reset, the
    current clones that descend from it: the histogram of the carried origins
    (Sec. 2.4), for [eq] and [iid] selection, through a graph-replayed run."""
    for sel in (pd.PD_SEL_EQ, pd.PD_SEL_IID):
        Nc = 70_000
        p = pd.make_params(40, 20, 0.05, Nc, 30 * 0.5, 0.5, seed=3, selection=sel, track_origin=1)
        S = pd.Sampler(p)
        S.run(5)
        S.reset_origin()
        S.run(25)
        counts = S.descendant_counts().cpu().numpy().view(np.uint32)
        want = np.bincount(S.origin(), minlength=Nc)
        assert np.array_equal(counts, want)
        assert counts.sum() == Nc and (counts == 0).any() and counts.max() > 1
    q = pd.make_params(40, 20, 0.05, 100, 1.0, 0.5, seed=3)
    with pytest.raises(pd.PdError):
        pd.Sampler(q).descendant_counts()       # origins not tracked
