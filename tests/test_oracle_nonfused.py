"""Pins of the oracle's two non-fused steps (Sec. 3.1.2): the sampled
tensor's derivative values and the sampled MTTKRP of a given sampled tensor.

  * mttkrp equals an independent numpy scatter (np.add.at of gathered row
    products), and on a list of every cell of a small dense tensor the
    textbook MTTKRP X_(k) (Khatri-Rao of the other factors) by einsum;
  * sample_derivatives equals w times a central finite difference in m of
    the oracle's loss f (itself pinned to scipy's log-likelihoods), with the
    semi-stratified difference for the first n_semi samples;
  * together they give the oracle's fused sampled gradient.
"""
import numpy as np
import pytest

import oracle


def _case(seed, dims=(6, 5, 4), R=3, n=400):
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.2, 1.0, sum(dims) * R)
    coords = np.stack([rng.integers(0, I, n) for I in dims], axis=1).astype(np.int64)
    return list(dims), R, A, coords, rng


def test_mttkrp_equals_numpy_scatter():
    dims, R, A, coords, rng = _case(1)
    y = rng.normal(size=coords.shape[0])
    G = oracle.mttkrp(dims, R, A, coords, y).reshape(-1, R)
    off = np.concatenate([[0], np.cumsum(dims)])
    rows = [A.reshape(-1, R)[off[k] + coords[:, k]] for k in range(len(dims))]
    ref = np.zeros_like(G)
    for k in range(len(dims)):
        prod = y[:, None] * np.prod([rows[j] for j in range(len(dims)) if j != k], axis=0)
        np.add.at(ref, off[k] + coords[:, k], prod)
    np.testing.assert_allclose(G, ref, rtol=1e-13, atol=1e-13)


def test_mttkrp_over_every_cell_is_the_textbook_mttkrp():
    dims, R = [4, 3, 5], 2
    rng = np.random.default_rng(2)
    facs = [rng.normal(size=(I, R)) for I in dims]
    A = np.concatenate(facs).reshape(-1)
    X = rng.normal(size=dims)
    coords = np.array(list(np.ndindex(*dims)), dtype=np.int64)
    G = oracle.mttkrp(dims, R, A, coords, X.reshape(-1)).reshape(-1, R)
    ref = [np.einsum("ijk,jr,kr->ir", X, facs[1], facs[2]),
           np.einsum("ijk,ir,kr->jr", X, facs[0], facs[2]),
           np.einsum("ijk,ir,jr->kr", X, facs[0], facs[1])]
    np.testing.assert_allclose(G, np.concatenate(ref), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("loss", ["gaussian", "poisson", "bernoulli_logit"])
def test_sample_derivatives_are_w_times_df(loss):
    dims, R, A, coords, rng = _case(3, n=60)
    n = coords.shape[0]
    x = rng.integers(0, 2 if loss == "bernoulli_logit" else 4, n).astype(np.float64)
    w = rng.uniform(1, 50, n)
    n_semi = 20
    y = oracle.sample_derivatives(dims, R, A, coords, x, w, loss, n_semi=n_semi)
    for s in range(n):
        m = oracle.model_value(dims, R, A, coords[s])
        h = 1e-6 * max(1.0, abs(m))
        fd = (oracle.f(loss, x[s], m + h) - oracle.f(loss, x[s], m - h)) / (2 * h)
        if s < n_semi:
            fd -= (oracle.f(loss, 0.0, m + h) - oracle.f(loss, 0.0, m - h)) / (2 * h)
        assert abs(y[s] - w[s] * fd) <= 1e-6 * w[s] * max(1.0, abs(fd)), (s, y[s], w[s] * fd)


def test_nonfused_steps_give_the_fused_gradient():
    dims, R, A, coords, rng = _case(4)
    x = rng.poisson(1.5, coords.shape[0]).astype(np.float64)
    w = np.full(coords.shape[0], 7.5)
    Gf, _ = oracle.loss_grad(dims, R, A, coords, x, w, "poisson", n_semi=100)
    y = oracle.sample_derivatives(dims, R, A, coords, x, w, "poisson", n_semi=100)
    np.testing.assert_allclose(oracle.mttkrp(dims, R, A, coords, y), Gf, rtol=1e-12, atol=1e-12)
