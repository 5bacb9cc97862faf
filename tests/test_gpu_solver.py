"""The GCP-Adam epoch driver (restore and rate decay on a failed epoch,
stop after three failures) against the same driver written on the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_20353_amd import _lib as G
from paper_2605_20353_amd import synth
from paper_2605_20353_amd.solver import OBJECTIVE_CLIENT, SolverConfig, gcp_adam

pytestmark = pytest.mark.gpu


def _case(gpu):
    dims, R = [30, 25, 20], 4
    data = synth.count_tensor(dims, 4, 900, seed=2611, dist="uniform")
    t = G.SparseTensor(dims, data.coords.to(gpu), data.vals.to(gpu))
    to = oracle.SparseTensor(dims, data.coords.numpy(), data.vals.numpy())
    A0 = 0.2 + 0.8 * synth.init_model(dims, R, 2711, dtype=torch.float64)
    return dims, R, t, to, A0


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("lr", [5e-3, 3.0])
def test_epoch_driver_matches_oracle(gpu, lr, fused):
    """lr 5e-3 lowers the objective epoch after epoch; lr 3.0 makes epochs fail,
    which restores the model and decays the rate until three failures.  The
    gradient fused, or non-fused (sampled tensor written, then its MTTKRP)."""
    dims, R, t, to, A0 = _case(gpu)
    cfg = SolverConfig(R=R, loss="poisson", p=300, q=300, obj_p=2000, obj_q=2000, iters_per_epoch=10,
                       max_epochs=6, lr=lr, decay=0.1, max_fails=3, lower=0.0, seed=77, fused=fused)
    res = gcp_adam(t, A0.to(gpu), cfg)
    A, objs, rates, fails = oracle.gcp_adam_epochs(
        to, R, A0.numpy(), "poisson", 300, 300, 2000, 2000, 10, 6, lr, 0.1, 3, 77, OBJECTIVE_CLIENT,
        oracle.AdamParams(lr, lower=0.0))
    assert res.fails == fails
    np.testing.assert_allclose(res.rates, rates, rtol=1e-15)
    np.testing.assert_allclose(res.objective, objs, rtol=1e-10)
    rel = np.linalg.norm(res.A.cpu().numpy() - A) / np.linalg.norm(A)
    assert rel <= 1e-10
    if lr < 1:
        assert res.fails == 0 and objs[-1] < objs[0]
    else:
        assert res.fails >= 1
