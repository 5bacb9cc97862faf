"""Dense brute force for tiny tensors (numpy only).

TEST INFRASTRUCTURE ONLY, like the rest of this package.  Used to pin the C
oracle on tensors small enough to visit every cell:

  * ``full_model``      -- eq. cp: the dense Kruskal tensor, by einsum;
  * ``full_objective``  -- eq. gcp-model: F = sum over all cells of f(x, m);
  * ``mttkrp``          -- the mode-k MTTKRP Y_(k) (Khatri-Rao of the other
                           factors), by one numpy einsum per mode;
  * ``full_gradient``   -- eq. gcp-gradient with y = df/dm over all cells;
  * ``fd_gradient``     -- central finite differences of full_objective.

The loss formulas are written out again here in vectorised numpy; the tests
pin both copies against scipy's log-densities and against each other.
"""
from __future__ import annotations

import numpy as np

_LETTERS = "abcdefgh"


def split_factors(A: np.ndarray, dims, R: int):
    """Views of the contiguous model array, one [I_k, R] matrix per mode."""
    A = np.asarray(A).reshape(-1, R)
    out, off = [], 0
    for n in dims:
        out.append(A[off:off + n])
        off += n
    return out


def full_model(factors) -> np.ndarray:
    d = len(factors)
    spec = ",".join(_LETTERS[k] + "r" for k in range(d)) + "->" + _LETTERS[:d]
    return np.einsum(spec, *factors)


def f_dense(loss: str, X: np.ndarray, M: np.ndarray) -> np.ndarray:
    if loss == "gaussian":
        return 0.5 * (M - X) ** 2
    if loss == "poisson":
        return M - X * np.log(M + 1e-10)
    if loss == "bernoulli_logit":
        return np.logaddexp(0.0, M) - X * M
    raise ValueError(loss)


def df_dense(loss: str, X: np.ndarray, M: np.ndarray) -> np.ndarray:
    if loss == "gaussian":
        return M - X
    if loss == "poisson":
        return 1.0 - X / (M + 1e-10)
    if loss == "bernoulli_logit":
        return 0.5 * (1.0 + np.tanh(0.5 * M)) - X
    raise ValueError(loss)


def full_objective(loss: str, X: np.ndarray, factors) -> float:
    return float(f_dense(loss, X, full_model(factors)).sum())


def mttkrp(Y: np.ndarray, factors, k: int) -> np.ndarray:
    """G[i, r] = sum over cells with i_k = i of Y * prod_{n != k} A_n[i_n, r]."""
    d = len(factors)
    others = [n for n in range(d) if n != k]
    spec = (_LETTERS[:d] + "," + ",".join(_LETTERS[n] + "r" for n in others)
            + "->" + _LETTERS[k] + "r")
    return np.einsum(spec, Y, *[factors[n] for n in others])


def full_gradient(loss: str, X: np.ndarray, factors):
    Y = df_dense(loss, X, full_model(factors))
    return [mttkrp(Y, factors, k) for k in range(len(factors))]


def fd_gradient(loss: str, X: np.ndarray, factors, rel_h: float = 1e-6):
    """Central differences of the full objective, one entry at a time."""
    grads = []
    for k, Ak in enumerate(factors):
        g = np.zeros_like(Ak)
        for i in range(Ak.shape[0]):
            for r in range(Ak.shape[1]):
                h = rel_h * max(1.0, abs(Ak[i, r]))
                fs = [np.array(a, copy=True) for a in factors]
                fs[k][i, r] = Ak[i, r] + h
                fp = full_objective(loss, X, fs)
                fs[k][i, r] = Ak[i, r] - h
                fm = full_objective(loss, X, fs)
                g[i, r] = (fp - fm) / (2 * h)
        grads.append(g)
    return grads
