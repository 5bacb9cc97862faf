"""The oracle's timing-only OpenMP step (thread-private gradients, summed)
draws the same samples and takes the same Adam step as the serial step,
up to the order of the gradient's additions."""
import numpy as np

import oracle
from paper_2605_20353_amd import synth


def test_parallel_step_equals_serial_step():
    dims, R = [40, 30, 20], 6
    data = synth.count_tensor(dims, 3, 1500, seed=2641)
    t = oracle.SparseTensor(dims, data.coords.numpy(), data.vals.numpy())
    A0 = 0.1 + np.random.default_rng(1).uniform(size=sum(dims) * R)
    ap = oracle.AdamParams(lr=1e-2, lower=0.0)
    A1, B1, C1 = A0.copy(), np.zeros_like(A0), np.zeros_like(A0)
    A2, B2, C2 = A0.copy(), np.zeros_like(A0), np.zeros_like(A0)
    ps = oracle.ParallelStepper(t, R, 700, 900, threads=4)
    for k in range(3):
        G1, _ = oracle.sgd_step(t, R, A1, B1, C1, k + 1, "poisson", 700, 900, 20353, k, ap)
        G2 = ps.step(A2, B2, C2, k + 1, "poisson", 20353, k, ap)
        sc, _, _ = oracle.sample_stratified(t, 700, 900, 20353, k)
        np.testing.assert_array_equal(ps.coords, sc)
        np.testing.assert_allclose(G2, G1, rtol=1e-12, atol=1e-12 * np.abs(G1).max())
    np.testing.assert_allclose(A2, A1, rtol=1e-11, atol=1e-12)
    assert 1 <= ps.threads_used <= 4
