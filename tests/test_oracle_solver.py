"""Pins of the oracle's GCP-Adam epoch driver (CPU): the safeguard of the
paper's experiments (Sec. 5) -- an epoch that does not lower the objective on
the fixed sample set is undone and the rate is multiplied by the decay; the run
stops after max_fails such epochs -- checked through properties that hold
whatever the arithmetic: a zero rate can never lower the objective, an
exploding rate is undone bit for bit, and small steps on a smooth objective are
accepted with a strictly decreasing objective."""
import numpy as np

import oracle
from paper_2605_20353_amd import synth


def _problem(seed=3):
    dims, R = [9, 8, 7], 3
    data = synth.count_tensor(dims, R, 120, seed=seed)
    t = oracle.SparseTensor(dims, data.coords.numpy(), data.vals.numpy())
    A0 = synth.init_model(dims, R, seed + 1).numpy()
    return t, dims, R, A0


def _run(t, R, A0, lr, decay=0.1, max_epochs=6, iters=5):
    return oracle.gcp_adam_epochs(t, R, A0, "poisson", 40, 40, 200, 200, iters, max_epochs, lr, decay, 3,
                                  seed=11, obj_client=1 << 62, ap=oracle.AdamParams(lower=0.0))


def test_zero_rate_is_undone_three_times_then_stops():
    t, dims, R, A0 = _problem()
    A, objs, rates, fails = _run(t, R, A0, lr=0.0)
    assert fails == 3 and rates == [0.0, 0.0, 0.0]
    assert len(objs) == 1                          # only the initial objective
    np.testing.assert_array_equal(A, A0.reshape(-1))


def test_exploding_rate_is_undone_exactly_and_decayed():
    t, dims, R, A0 = _problem(seed=5)
    A, objs, rates, fails = _run(t, R, A0, lr=50.0, decay=0.5, max_epochs=2)
    # both epochs move the factors far from the data: undone, rate halved
    assert rates == [50.0, 25.0] and fails == 2 and len(objs) == 1
    np.testing.assert_array_equal(A, A0.reshape(-1))


def test_small_steps_are_accepted_and_lower_the_objective():
    t, dims, R, A0 = _problem(seed=7)
    A, objs, rates, fails = _run(t, R, A0, lr=1e-3, max_epochs=3)
    assert fails == 0 and rates == [1e-3] * 3 and len(objs) == 4
    assert all(b < a for a, b in zip(objs, objs[1:]))
    assert np.abs(A - A0.reshape(-1)).max() > 0
