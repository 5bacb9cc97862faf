"""Pins for the oracle's losses, model values, sampled gradient and Adam.

Each check ties the C oracle to something other than itself: scipy's
log-densities (loss definitions), a numpy einsum MTTKRP and a pure-Python cell
loop (eq. gcp-gradient), central finite differences, the Gaussian identity
G_k = MTTKRP(M - X), zero gradient at an exactly fitted model, unbiasedness of
the stratified estimator, torch.autograd on the sampled objective, and
torch.optim.Adam (Alg. adam-update with epsilon = 0).
"""
import math

import numpy as np
import pytest
import torch
from scipy import special, stats

import oracle
from oracle import brute

LOSS_NAMES = ["gaussian", "poisson", "bernoulli_logit"]


def _factors(dims, R, seed, kind="uniform"):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return [rng.uniform(0.2, 1.0, (n, R)) for n in dims]
    return [rng.normal(0.0, 0.7, (n, R)) for n in dims]


def _data(loss, dims, seed):
    rng = np.random.default_rng(seed + 100)
    if loss == "gaussian":
        return rng.normal(0, 1, dims)
    if loss == "poisson":
        return rng.poisson(1.5, dims).astype(np.float64)
    return rng.integers(0, 2, dims).astype(np.float64)


def _all_cells(dims):
    return np.array(list(np.ndindex(*dims)), dtype=np.int64)


def _stack(factors):
    return np.concatenate(factors, axis=0).reshape(-1)


# ----------------------------------------------------------------- losses --

@pytest.mark.parametrize("x,m", [(0.0, 0.3), (2.0, 1.7), (5.0, 0.01), (1.0, 40.0)])
def test_poisson_loss_is_negative_log_likelihood(x, m):
    mu = m + 1e-10
    nll = -stats.poisson.logpmf(x, mu) - special.gammaln(x + 1)   # drop the x-only term
    assert oracle.f("poisson", x, m) == pytest.approx(nll - 1e-10, rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("x,m", [(0.0, 0.3), (-1.2, 2.5), (3.0, -4.0)])
def test_gaussian_loss_is_negative_log_likelihood(x, m):
    nll = -stats.norm.logpdf(x, loc=m, scale=1.0) - 0.5 * math.log(2 * math.pi)
    assert oracle.f("gaussian", x, m) == pytest.approx(nll, rel=1e-13, abs=1e-14)


@pytest.mark.parametrize("x", [0.0, 1.0])
@pytest.mark.parametrize("m", [-30.0, -2.0, 0.0, 0.7, 25.0, 700.0])
def test_bernoulli_logit_loss_is_negative_log_likelihood(x, m):
    # -log P(x | p = sigmoid(m)), evaluated stably by scipy's log_expit
    nll = -(x * special.log_expit(m) + (1 - x) * special.log_expit(-m))
    assert oracle.f("bernoulli_logit", x, m) == pytest.approx(nll, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("loss", LOSS_NAMES)
def test_loss_derivative_matches_central_difference(loss):
    rng = np.random.default_rng(1)
    for _ in range(30):
        m = rng.uniform(0.2, 3.0)
        x = float(rng.integers(0, 2)) if loss == "bernoulli_logit" else rng.uniform(0, 3)
        h = 1e-6
        fd = (oracle.f(loss, x, m + h) - oracle.f(loss, x, m - h)) / (2 * h)
        assert oracle.df(loss, x, m) == pytest.approx(fd, rel=1e-7, abs=1e-8)


@pytest.mark.parametrize("loss", LOSS_NAMES)
def test_dense_loss_copies_agree(loss):
    rng = np.random.default_rng(2)
    M = rng.uniform(0.1, 3.0, 50)
    X = _data(loss, (50,), 3)
    for i in range(50):
        assert brute.f_dense(loss, X[i], M[i]) == pytest.approx(oracle.f(loss, X[i], M[i]), rel=1e-13)
        assert brute.df_dense(loss, X[i], M[i]) == pytest.approx(oracle.df(loss, X[i], M[i]),
                                                                   rel=1e-12, abs=1e-14)


def test_bernoulli_extremes_are_finite():
    assert oracle.df("bernoulli_logit", 1.0, -800.0) == -1.0
    assert oracle.df("bernoulli_logit", 0.0, 800.0) == 1.0
    assert oracle.f("bernoulli_logit", 0.0, 800.0) == pytest.approx(800.0)


# ------------------------------------------------------------ model value --

def test_model_value_rank_one_is_product():
    dims = (4, 3, 5)
    facs = _factors(dims, 1, 0)
    A = _stack(facs)
    for idx in [(0, 0, 0), (3, 2, 4), (1, 2, 0)]:
        want = facs[0][idx[0], 0] * facs[1][idx[1], 0] * facs[2][idx[2], 0]
        assert oracle.model_value(dims, 1, A, idx) == pytest.approx(want, rel=1e-15)


@pytest.mark.parametrize("dims", [(4, 3, 5), (3, 4, 2, 3)])
@pytest.mark.parametrize("R", [1, 2, 3])
def test_model_value_matches_einsum(dims, R):
    facs = _factors(dims, R, 4, kind="normal")
    full = brute.full_model(facs)
    A = _stack(facs)
    for idx in np.ndindex(*dims):
        assert oracle.model_value(dims, R, A, idx) == pytest.approx(full[idx], rel=1e-13, abs=1e-14)


# -------------------------------------------------------- gradient (full) --

@pytest.mark.parametrize("dims", [(4, 3, 5), (3, 4, 2, 3)])
@pytest.mark.parametrize("R", [1, 2, 3])
@pytest.mark.parametrize("loss", LOSS_NAMES)
def test_all_cells_gradient_equals_einsum_mttkrp(dims, R, loss):
    """P1: a sample list enumerating every cell once with weight 1 gives the
    full gradient of eq. gcp-gradient and the full objective of eq. gcp-model."""
    facs = _factors(dims, R, 5)
    X = _data(loss, dims, 6)
    cells = _all_cells(dims)
    x = X.reshape(-1)
    G, F = oracle.loss_grad(dims, R, _stack(facs), cells, x, np.ones(len(cells)), loss)
    ref = np.concatenate(brute.full_gradient(loss, X, facs), axis=0).reshape(-1)
    np.testing.assert_allclose(G, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert F == pytest.approx(brute.full_objective(loss, X, facs), rel=1e-12)


def test_einsum_mttkrp_matches_cell_loop():
    """The einsum route against a pure-Python loop over cells (3 modes)."""
    dims, R = (3, 2, 4), 2
    facs = _factors(dims, R, 7, kind="normal")
    Y = np.random.default_rng(8).normal(size=dims)
    for k in range(3):
        ref = np.zeros((dims[k], R))
        for idx in np.ndindex(*dims):
            for r in range(R):
                prod = Y[idx]
                for n in range(3):
                    if n != k:
                        prod *= facs[n][idx[n], r]
                ref[idx[k], r] += prod
        np.testing.assert_allclose(brute.mttkrp(Y, facs, k), ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("loss", LOSS_NAMES)
def test_full_gradient_matches_finite_differences(loss):
    """P2: the full gradient is the derivative of the full objective."""
    dims, R = (3, 4, 2), 2
    facs = _factors(dims, R, 9)
    X = _data(loss, dims, 10)
    cells = _all_cells(dims)
    G, _ = oracle.loss_grad(dims, R, _stack(facs), cells, X.reshape(-1), np.ones(len(cells)), loss)
    fd = np.concatenate(brute.fd_gradient(loss, X, facs), axis=0).reshape(-1)
    err = np.linalg.norm(G - fd) / np.linalg.norm(fd)
    assert err < 1e-7


def test_gaussian_gradient_is_mttkrp_of_residual():
    """P3: for the Gaussian loss dF/dA_k = MTTKRP(M - X) with the dense residual."""
    dims, R = (4, 3, 2, 3), 3
    facs = _factors(dims, R, 11, kind="normal")
    X = np.random.default_rng(12).normal(size=dims)
    cells = _all_cells(dims)
    G, _ = oracle.loss_grad(dims, R, _stack(facs), cells, X.reshape(-1), np.ones(len(cells)),
                            "gaussian")
    resid = brute.full_model(facs) - X
    ref = np.concatenate([brute.mttkrp(resid, facs, k) for k in range(4)], axis=0).reshape(-1)
    np.testing.assert_allclose(G, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("loss", LOSS_NAMES)
def test_zero_gradient_at_exact_fit(loss):
    """P4: with X = link(M) every cell has df/dm = 0, so the full gradient and
    every uniformly sampled gradient vanish."""
    dims, R = (4, 3, 5), 2
    facs = _factors(dims, R, 13)
    Mfull = brute.full_model(facs)
    if loss == "bernoulli_logit":
        X = special.expit(Mfull)
    else:
        X = Mfull.copy()
    cells = _all_cells(dims)
    A = _stack(facs)
    G, _ = oracle.loss_grad(dims, R, A, cells, X.reshape(-1), np.ones(len(cells)), loss)
    scale = np.abs(A).max() ** 2 * len(cells)
    assert np.abs(G).max() <= 1e-9 * scale
    sc, sx, sw = oracle.sample_uniform(dims, X, 200, seed=3)
    Gs, _ = oracle.loss_grad(dims, R, A, sc, sx, sw, loss)
    assert np.abs(Gs).max() <= 1e-9 * scale * 60 / 200 * 10


# ---------------------------------------------------- sampled estimators --

def _sparse_case(seed=14, dims=(4, 3, 5), nnz=12, R=2):
    rng = np.random.default_rng(seed)
    lin = rng.choice(int(np.prod(dims)), nnz, replace=False)
    coords = np.stack(np.unravel_index(lin, dims), axis=1).astype(np.int64)
    vals = rng.integers(1, 6, nnz).astype(np.float64)
    X = np.zeros(dims)
    X[tuple(coords.T)] = vals
    facs = _factors(dims, R, seed + 1)
    return oracle.SparseTensor(dims, coords, vals), X, facs


def _estimator_moments(t, facs, R, loss, p, q, K, semi=False):
    A = _stack(facs)
    acc = np.zeros(int(t.dims.sum()) * R)
    acc2 = np.zeros_like(acc)
    for seed in range(K):
        sc, sx, sw = oracle.sample_stratified(t, p, q, seed=seed, semi=semi)
        G, _ = oracle.loss_grad(t.dims, R, A, sc, sx, sw, loss, n_semi=p if semi else 0)
        acc += G
        acc2 += G * G
    mean = acc / K
    se = np.sqrt(np.maximum(acc2 / K - mean ** 2, 0) / K)
    return mean, se


@pytest.mark.parametrize("loss", ["poisson", "gaussian"])
def test_stratified_estimator_is_unbiased(loss):
    """P6: E[G~] = G for stratified sampling with weights N/p and (M-N)/q."""
    t, X, facs = _sparse_case()
    R = 2
    full = np.concatenate(brute.full_gradient(loss, X, facs), axis=0).reshape(-1)
    mean, se = _estimator_moments(t, facs, R, loss, p=6, q=6, K=4096)
    z = np.abs(mean - full) / np.maximum(se, 1e-12)
    assert z.max() < 4.5, z.max()


def test_semi_stratified_bias_is_order_density():
    """Semi-stratified sampling with the zero weight left at (M-N)/q has mean
    G - (N/M) MTTKRP(df/dm(0, M)) (the zero samples also land on nonzeros)."""
    loss = "poisson"
    t, X, facs = _sparse_case(seed=21)
    R = 2
    Mfull = brute.full_model(facs)
    full = np.concatenate(brute.full_gradient(loss, X, facs), axis=0).reshape(-1)
    Y0 = brute.df_dense(loss, np.zeros_like(Mfull), Mfull)
    bias = -(t.nnz / t.cells) * np.concatenate(
        [brute.mttkrp(Y0, facs, k) for k in range(3)], axis=0).reshape(-1)
    mean, se = _estimator_moments(t, facs, R, loss, p=6, q=6, K=4096, semi=True)
    z = np.abs(mean - (full + bias)) / np.maximum(se, 1e-12)
    assert z.max() < 4.5, z.max()
    # and the bias is really there: the unbiased hypothesis is rejected
    z0 = np.abs(mean - full) / np.maximum(se, 1e-12)
    assert z0.max() > 8.0


@pytest.mark.parametrize("loss", LOSS_NAMES)
def test_sampled_gradient_is_autograd_of_sampled_objective(loss):
    """P7: G~ is the gradient of F~ = sum_s w_s f(x_s, m_s) with the samples
    fixed (torch.autograd in float64, an independent route)."""
    t, X, facs = _sparse_case(seed=31, dims=(5, 4, 6), nnz=30, R=3)
    if loss == "bernoulli_logit":
        vals = np.ones(t.nnz)
        t = oracle.SparseTensor(t.dims, t.coords, vals)
    R = 3
    A = _stack(facs)
    sc, sx, sw = oracle.sample_stratified(t, 20, 25, seed=4)
    G, F = oracle.loss_grad(t.dims, R, A, sc, sx, sw, loss)

    At = torch.tensor(A.reshape(-1, R), dtype=torch.float64, requires_grad=True)
    off = np.concatenate([[0], np.cumsum(t.dims)])
    rows = [torch.tensor(sc[:, k] + off[k]) for k in range(t.d)]
    prod = At[rows[0]]
    for k in range(1, t.d):
        prod = prod * At[rows[k]]
    m = prod.sum(dim=1)
    x = torch.tensor(sx)
    w = torch.tensor(sw)
    if loss == "gaussian":
        fv = 0.5 * (m - x) ** 2
    elif loss == "poisson":
        fv = m - x * torch.log(m + 1e-10)
    else:
        fv = torch.nn.functional.softplus(m) - x * m
    Ft = (w * fv).sum()
    Ft.backward()
    np.testing.assert_allclose(G, At.grad.numpy().reshape(-1), rtol=1e-11, atol=1e-11)
    assert F == pytest.approx(Ft.item(), rel=1e-12)


def test_duplicate_samples_sum_as_separate_entries():
    dims, R = (3, 3, 3), 2
    facs = _factors(dims, R, 40)
    A = _stack(facs)
    one = np.array([[1, 2, 0]], dtype=np.int64)
    G1, F1 = oracle.loss_grad(dims, R, A, one, [2.0], [1.5], "poisson")
    G3, F3 = oracle.loss_grad(dims, R, A, np.repeat(one, 3, axis=0), [2.0] * 3, [1.5] * 3, "poisson")
    np.testing.assert_allclose(G3, 3 * G1, rtol=1e-15)
    assert F3 == pytest.approx(3 * F1, rel=1e-15)


# ------------------------------------------------------------------- Adam --

def test_adam_equals_torch_adam_with_eps_zero():
    """P9: with epsilon = 0 and no lower bound Alg. adam-update is torch's Adam."""
    rng = np.random.default_rng(50)
    n = 40
    A = rng.normal(size=n)
    B = np.zeros(n)
    Cm = np.zeros(n)
    p = torch.tensor(A.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.8, 0.95), eps=0.0)
    for t in range(1, 8):
        G = rng.normal(size=n)
        oracle.adam(A, G, B, Cm, t, lr=1e-2, beta1=0.8, beta2=0.95, eps=0.0)
        p.grad = torch.tensor(G)
        opt.step()
        np.testing.assert_allclose(A, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_first_step_is_sign_step():
    rng = np.random.default_rng(51)
    A = rng.normal(size=30)
    A0 = A.copy()
    G = rng.normal(size=30)
    oracle.adam(A, G, np.zeros(30), np.zeros(30), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(A, A0 - 0.01 * np.sign(G), rtol=1e-15, atol=1e-16)


def test_adam_epsilon_sits_inside_the_root():
    # first step: G / sqrt(G^2 + eps); for G = sqrt(3 eps) the step is lr sqrt(3)/2
    eps = 1e-4
    A = np.zeros(1)
    oracle.adam(A, [math.sqrt(3 * eps)], np.zeros(1), np.zeros(1), 1, lr=1.0, eps=eps)
    assert A[0] == pytest.approx(-math.sqrt(3) / 2, rel=1e-13)


def test_adam_lower_bound_clamps():
    A = np.array([0.001, 0.5, -0.2])
    G = np.array([1.0, 1.0, -1.0])
    oracle.adam(A, G, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0, lower=0.0)
    np.testing.assert_allclose(A, [0.0, 0.49, 0.0], atol=1e-16)
