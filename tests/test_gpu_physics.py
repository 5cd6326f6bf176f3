"""The paper's published activity at its own state points (Sec. 5, Tables 1
and 2), reproduced on the GPU: periodic SSEP, N = L/2, Delta t = 10,
t_obs = 1e4, uniform initial configurations, R = 10 independent replicas (as
in the paper's runs), with [eq] and with [iid] selection (the two columns of
each table).  The replica mean of k-hat (eq. khat, divided by Nc as the text
requires) must sit within the paper's 2 per cent accuracy target of the value
its fits predict for the same (L, lambda, Nc, t_obs, selection); the fitted
constants are stored in tests/golden/paper_activity_fits.json with their
source.  Nc is chosen where the paper's own fits say the finite-Nc correction
is below a few tenths of a per cent.  The replicas also give the per-run
spread (the paper's sigma, Sec. 4.2), reported and checked to be small
against the tolerance, so a pass is not luck.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_1711_05095_amd import inputs, pd

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_activity_fits.json")))
R = 10
SEL = {"eq": pd.PD_SEL_EQ, "iid": pd.PD_SEL_IID}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pd.lib()


def k_hat(L, lam, Nc, sel, seed):
    """k-hat of R independent replicas (one batch)."""
    dt, t_obs = 10.0, 1.0e4
    ps = [pd.make_params(L, L // 2, inputs.s_of_lambda(lam, L), Nc, t_obs, dt, seed=seed,
                         instance=r + 1, selection=SEL[sel]) for r in range(R)]
    S = pd.Sampler(ps)
    S.run(int(round(t_obs / dt)))
    k = np.array([S.estimates(i)["k_hat"] for i in range(R)])
    S.close()
    return k


def check(k, want, what):
    sigma = k.std(ddof=1)
    print("%s: k-hat %.5f +- %.5f (sigma %.5f over %d replicas), paper %.5f, diff %+.2f%%"
          % (what, k.mean(), sigma / np.sqrt(len(k)), sigma, len(k), want,
             100 * (k.mean() / want - 1)), flush=True)
    assert abs(k.mean() - want) <= 0.02 * want
    assert sigma / np.sqrt(len(k)) < 0.005 * want


@pytest.mark.parametrize("sel", ["eq", "iid"])
@pytest.mark.parametrize("L,Nc", [(20, 100_000), (50, 100_000), (80, 1_000_000)])
def test_activity_lambda28_matches_table1(L, Nc, sel):
    f = GOLD["lambda28_tobs_fit" + ("" if sel == "eq" else "_iid")][str(L)]
    want = f["k_inf"] * (1 + f["A"] / 1.0e4)
    k = k_hat(L, 28.0, Nc, sel, seed=600 + L)
    check(k, want, "L=%d lambda=28 [%s]" % (L, sel))


@pytest.mark.parametrize("sel", ["eq", "iid"])
def test_activity_lambda50_matches_table2(sel):
    """L = 50 at Nc = 1e6.  L = 80 is left out: there the paper's own fit moves
    by 2.0-2.4 per cent when its Nc = 1e6 point is included (Table 2), so it
    fixes no value to 2 per cent."""
    L, Nc = 50, 1_000_000
    f = GOLD["lambda50_nc_fit" + ("" if sel == "eq" else "_iid")][str(L)]
    want = f["k_inf"] * (1 + f["A"] / Nc)
    k = k_hat(L, 50.0, Nc, sel, seed=700 + L)
    check(k, want, "L=%d lambda=50 [%s]" % (L, sel))
