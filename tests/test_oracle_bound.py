"""Pins for the oracle's per-element rounding-error bound of a sampled
gradient (ora_loss_grad_bound / oracle.grad_error_bound).

The bound is what the GPU parity tests hold every gradient element to, so it
is tied here to things other than itself:
  * its counts and magnitude sums equal an independent numpy computation;
  * a binary32 emulation of the device arithmetic (model value summed over
    the rank in a random order, the loss derivative in float32, the weight
    rounded to float32, leave-one-out products in a random mode order, and
    the contributions added in a random order, as atomics would) stays
    inside it, for every loss, semi-stratified samples and samples planted
    where the derivative cancels;
  * it is not vacuous (far below the gradient's own size), and its term for
    the error of y is needed: without it the planted cancellations break it.
"""
import numpy as np
import pytest

import oracle

F32 = np.float32


def _case(loss, seed, dims=(6, 5, 4), R=8, n=600, semi=0, cancel=0):
    rng = np.random.default_rng(seed)
    if loss == "poisson":
        A = rng.uniform(0.2, 1.0, (sum(dims), R))
    else:
        A = rng.normal(0.0, 0.8, (sum(dims), R))
    A = A.astype(F32).astype(np.float64).reshape(-1)
    coords = np.stack([rng.integers(0, I, n) for I in dims], axis=1).astype(np.int64)
    if loss == "poisson":
        x = rng.poisson(2.0, n).astype(np.float64)
    elif loss == "gaussian":
        x = rng.normal(0, 1, n)
    else:
        x = rng.integers(0, 2, n).astype(np.float64)
    # planted cancellation: x equal (in binary32) to the sample's model value
    # for Poisson and Gaussian, so that f'(x, m) is at the rounding level
    for s in range(cancel):
        m = oracle.model_value(dims, R, A, coords[s])
        x[s] = float(F32(m))
    x = x.astype(F32).astype(np.float64)
    w = np.full(n, 1234.567)
    return list(dims), R, A, coords, x, w


def _df32(loss, x, m):
    if loss == "gaussian":
        return m - x
    if loss == "poisson":
        return F32(1) - x / (m + F32(1e-10))
    out = np.empty_like(m)
    pos = m >= 0
    out[pos] = F32(1) / (F32(1) + np.exp(-m[pos]))
    e = np.exp(m[~pos])
    out[~pos] = e / (F32(1) + e)
    return out - x


def _emulate_f32(dims, R, A, coords, x, w, loss, n_semi, rng):
    """The sampled gradient in binary32 with random operation orders."""
    d = len(dims)
    off = np.concatenate([[0], np.cumsum(dims)])
    A32 = A.astype(F32).reshape(-1, R)
    rows = [A32[off[k] + coords[:, k]] for k in range(d)]        # [n, R] per mode
    n = coords.shape[0]
    order = rng.permutation(d)
    prod = rows[order[0]].copy()
    for k in order[1:]:
        prod = prod * rows[k]
    m = np.zeros(n, dtype=F32)
    for r in rng.permutation(R):
        m = m + prod[:, r]
    x32, w32 = x.astype(F32), w.astype(F32)
    y = w32 * _df32(loss, x32, m)
    if n_semi:
        y0 = w32[:n_semi] * _df32(loss, np.zeros(n_semi, dtype=F32), m[:n_semi])
        y[:n_semi] = y[:n_semi] - y0
    G = np.zeros((off[-1], R), dtype=F32)
    for k in range(d):
        others = [j for j in rng.permutation(d) if j != k]
        c = y[:, None].copy()
        for j in others:
            c = c * rows[j]
        perm = rng.permutation(n)
        np.add.at(G, off[k] + coords[perm, k], c[perm])
    return G.reshape(-1).astype(np.float64)


def test_counts_and_magnitude_sums_match_numpy():
    dims, R, A, coords, x, w = _case("poisson", 1)
    abssum, yerr, count = oracle.loss_grad_bound_parts(dims, R, A, coords, x, w, "poisson", oracle.U_F32)
    off = np.concatenate([[0], np.cumsum(dims)])
    want = np.concatenate([np.bincount(coords[:, k], minlength=dims[k]) for k in range(3)])
    np.testing.assert_array_equal(count, want)
    A2 = np.abs(A.reshape(-1, R))
    m = np.array([oracle.model_value(dims, R, A, c) for c in coords])
    y = np.abs(w * (1.0 - x / (m + 1e-10)))
    ref = np.zeros((off[-1], R))
    rows = [A2[off[k] + coords[:, k]] for k in range(3)]
    for k in range(3):
        q = np.prod([rows[j] for j in range(3) if j != k], axis=0)
        np.add.at(ref, off[k] + coords[:, k], y[:, None] * q)
    np.testing.assert_allclose(abssum.reshape(-1, R), ref, rtol=1e-12, atol=0)
    assert (yerr > 0).all() == (count.repeat(R) > 0).all()
    assert np.all(yerr[count.repeat(R) == 0] == 0)


@pytest.mark.parametrize("loss", ["poisson", "gaussian", "bernoulli_logit"])
@pytest.mark.parametrize("semi", [0, 200])
def test_binary32_emulation_stays_inside_the_bound(loss, semi):
    cancel = 150 if loss != "bernoulli_logit" else 0
    dims, R, A, coords, x, w = _case(loss, 2 + semi, semi=semi, cancel=cancel)
    G64, _ = oracle.loss_grad(dims, R, A, coords, x, w, loss, n_semi=semi)
    bound = oracle.grad_error_bound(dims, R, A, coords, x, w, loss, oracle.U_F32, n_semi=semi)
    bound += oracle.grad_error_bound(dims, R, A, coords, x, w, loss, oracle.U_F64, n_semi=semi)
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(12):
        G32 = _emulate_f32(dims, R, A, coords, x, w, loss, semi, rng)
        err = np.abs(G32 - G64)
        assert np.all(err <= 2 * bound), np.max(err / np.maximum(bound, 1e-300))
        worst = max(worst, float(np.max(err / np.maximum(bound, 1e-300))))
    # the bound is reached within a few orders of magnitude, not vacuous
    assert worst > 1e-3
    nz = np.abs(G64) > 0
    assert np.median(bound[nz] / np.abs(G64[nz])) < 1e-4


def test_the_y_error_term_is_needed_where_the_derivative_cancels():
    """Poisson samples with x equal to their model value: f' is at the
    rounding level, so the error of y dwarfs |y| and the magnitude term alone
    cannot cover what binary32 arithmetic produces."""
    dims, R, A, coords, x, w = _case("poisson", 3, n=300, cancel=300)
    G64, _ = oracle.loss_grad(dims, R, A, coords, x, w, "poisson")
    abssum, yerr, count = oracle.loss_grad_bound_parts(dims, R, A, coords, x, w, "poisson", oracle.U_F32)
    depth = np.repeat(np.maximum(count - 1, 0), R)
    gam = lambda n: n * oracle.U_F32 / (1 - n * oracle.U_F32)
    magnitude_only = (gam(3) + gam(depth)) * abssum
    full = oracle.grad_error_bound(dims, R, A, coords, x, w, "poisson", oracle.U_F32)
    rng = np.random.default_rng(11)
    G32 = _emulate_f32(dims, R, A, coords, x, w, "poisson", 0, rng)
    err = np.abs(G32 - G64)
    assert np.any(err > 2 * magnitude_only)
    assert np.all(err <= 2 * full)


def test_a_planted_error_is_caught():
    """One gradient element moved by one part in 10^4 of its size is outside
    the bound (what the GPU tests rely on to see a wrong element)."""
    dims, R, A, coords, x, w = _case("gaussian", 4)
    G64, _ = oracle.loss_grad(dims, R, A, coords, x, w, "gaussian")
    bound = oracle.grad_error_bound(dims, R, A, coords, x, w, "gaussian", oracle.U_F32)
    i = int(np.argmax(np.abs(G64)))
    bad = G64.copy()
    bad[i] *= 1.0001
    assert np.abs(bad - G64)[i] > 2 * bound[i]


def test_poisson_bound_is_infinite_where_rounding_can_flip_the_model_value():
    """m + 1e-10 within the model value's own rounding error of zero (terms
    of opposite sign cancel): no finite bound holds for 1/(m + eps)."""
    dims, R = [2, 2, 2], 2
    A = np.array([1.0, -1.0, 1.0, 1.0] + [1.0] * 8)
    coords = np.array([[0, 0, 0]], dtype=np.int64)
    b = oracle.grad_error_bound(dims, R, A, coords, np.array([1.0]), np.array([1.0]), "poisson", oracle.U_F32)
    assert np.isinf(b[0])
