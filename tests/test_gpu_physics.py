"""The paper's published activity at its own state points (Sec. 5, Tables 1
and 2), reproduced on the GPU: periodic SSEP, N = L/2, [eq] selection,
Delta t = 10, t_obs = 1e4, uniform initial configurations.  k-hat (eq. khat,
divided by Nc as the text requires) must sit within the paper's 2 per cent
accuracy target of the value its fits predict for the same (L, lambda, Nc,
t_obs); the fitted constants are stored in tests/golden/paper_activity_fits.json
with their source.  Nc is chosen where the paper's own fits say the finite-Nc
correction is below a few tenths of a per cent.
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


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pd.lib()


def k_hat(L, lam, Nc, reps, seed):
    dt, t_obs = 10.0, 1.0e4
    ps = [pd.make_params(L, L // 2, inputs.s_of_lambda(lam, L), Nc, t_obs, dt, seed=seed,
                         instance=r + 1) for r in range(reps)]
    S = pd.Sampler(ps)
    S.run(int(round(t_obs / dt)))
    k = np.array([S.estimates(i)["k_hat"] for i in range(reps)])
    S.close()
    return k


@pytest.mark.parametrize("L,Nc,reps", [(20, 100_000, 2), (50, 100_000, 2), (80, 1_000_000, 1)])
def test_activity_lambda28_matches_table1(L, Nc, reps):
    f = GOLD["lambda28_tobs_fit"][str(L)]
    want = f["k_inf"] * (1 + f["A"] / 1.0e4)
    k = k_hat(L, 28.0, Nc, reps, seed=600 + L)
    print("L=%d lambda=28: k-hat %.5f, paper %.5f" % (L, k.mean(), want), flush=True)
    assert abs(k.mean() - want) <= 0.02 * want


@pytest.mark.parametrize("L", [50])
def test_activity_lambda50_matches_table2(L):
    """L = 80 is left out: there the paper's own fit moves by 2.4 per cent when
    its Nc = 1e6 point is included (Table 2), so it fixes no value to 2 per
    cent."""
    f = GOLD["lambda50_nc_fit"][str(L)]
    Nc = 1_000_000
    want = f["k_inf"] * (1 + f["A"] / Nc)
    k = k_hat(L, 50.0, Nc, 1, seed=700 + L)
    print("L=%d lambda=50: k-hat %.5f, paper %.5f" % (L, k.mean(), want), flush=True)
    assert abs(k.mean() - want) <= 0.02 * want
