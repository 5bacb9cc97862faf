"""Seeded synthetic inputs: sparse count / binary tensors, dense Gaussian
tensors, initial Kruskal models and GCP-FedAdam client blocks.

This module draws INPUTS only.  It holds none of the method's arithmetic (no
sampling of the gradient, no model values, no losses, no MTTKRP, no Adam), so
the HIP path and the oracle can both be fed from it.

Recipe (count tensors): a low-rank nonnegative CP model with column weights
lambda_r is normalised so each factor column sums to one; events are drawn in
fixed-size batches as r ~ Cat(lambda / sum lambda), then i_k ~ Cat(column r of
factor k) by inverse CDF (searchsorted); events are counted per cell until the
number of distinct cells reaches the target; the first ``nnz`` distinct cells
in draw order are kept, with their event counts as values.  This is the usual
"events from a normalised Kruskal tensor" construction for synthetic count
data.  Binary tensors keep the same cells with value 1.

All draws use a torch.Generator seeded from the caller's seed on the device the
caller names.  A given (seed, device type) pair is reproducible; CPU and GPU
streams differ, which is fine because every consumer is fed the same arrays.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(int(seed))
    return g


def factor_matrices(dims, R: int, seed: int, dist: str = "gamma", device="cpu",
                    dtype=torch.float64):
    """Random factor matrices [I_k, R]: 'gamma' = Gamma(1, 1) (exponential),
    'uniform' = U(0, 1), 'normal' = N(0, 1)."""
    g = _gen(seed, device)
    out = []
    for n in dims:
        if dist == "gamma":
            a = torch.empty(int(n), R, dtype=dtype, device=device).exponential_(1.0, generator=g)
        elif dist == "uniform":
            a = torch.rand(int(n), R, dtype=dtype, device=device, generator=g)
        elif dist == "normal":
            a = torch.randn(int(n), R, dtype=dtype, device=device, generator=g)
        else:
            raise ValueError(dist)
        out.append(a)
    return out


def strides(dims):
    s = [1] * len(dims)
    for k in range(len(dims) - 2, -1, -1):
        s[k] = s[k + 1] * int(dims[k + 1])
    return s


def events_to_tensor(dims, factors, lam, nnz: int, seed: int, device="cpu",
                     batch: int | None = None, max_batches: int = 10000):
    """Count tensor with exactly ``nnz`` distinct nonzeros drawn as events from
    the normalised CP model (factors [I_k, R], weights lam [R]).
    Returns (coords int64 [nnz, d], counts float64 [nnz]) as torch tensors on
    ``device``, coords in first-draw order."""
    d = len(dims)
    R = int(lam.numel())
    total = 1
    for n in dims:
        total *= int(n)
    if nnz > total:
        raise ValueError("nnz exceeds the number of cells")
    g = _gen(seed + 1, device)
    lam = lam.to(device=device, dtype=torch.float64)
    probs = lam / lam.sum()
    # one flattened, strictly increasing CDF per mode: column r occupies
    # (r, r+1] so a single searchsorted serves every component
    flat_cdf = []
    for k in range(d):
        col = factors[k].to(device=device, dtype=torch.float64)
        col = col / col.sum(dim=0, keepdim=True)
        cdf = torch.cumsum(col.t(), dim=1)              # [R, I_k]
        cdf[:, -1] = 1.0
        cdf = cdf + torch.arange(R, device=device, dtype=torch.float64)[:, None]
        flat_cdf.append(cdf.reshape(-1).contiguous())
    st = strides(dims)
    # Above 2^63 cells the int64 linear key wraps; the wrapped bit pattern is
    # still one-to-one with the cell (the count is below 2^64), so duplicates
    # are still found on it, and the coordinates are kept per event instead of
    # being divided back out of the key.
    wide = total >= (1 << 63)
    if batch is None:
        batch = max(1 << 12, min(max(1 << 25, nnz // 8), nnz // 4 + 1))
    keys, ev_coords = [], []
    n_events = 0
    for _ in range(max_batches):
        r = torch.multinomial(probs, batch, replacement=True, generator=g)
        key = torch.zeros(batch, dtype=torch.int64, device=device)
        if wide:
            cs = torch.empty(batch, d, dtype=torch.int32, device=device)
        for k in range(d):
            u = torch.rand(batch, dtype=torch.float64, device=device, generator=g)
            pos = torch.searchsorted(flat_cdf[k], r.to(torch.float64) + u)
            i = pos - r * int(dims[k])
            i = i.clamp_(0, int(dims[k]) - 1)
            if wide:
                cs[:, k] = i.to(torch.int32)
                key += i * (st[k] if st[k] < (1 << 63) else st[k] - (1 << 64))   # modulo 2^64
            else:
                key += i * st[k]
        keys.append(key)
        if wide:
            ev_coords.append(cs)
        n_events += batch
        distinct = torch.unique(torch.cat(keys)).numel()
        if distinct >= nnz:
            break
    else:
        raise RuntimeError("event sampling did not reach the nonzero target")
    allk = torch.cat(keys)
    del keys
    uniq, inv, counts = torch.unique(allk, sorted=True, return_inverse=True, return_counts=True)
    pos = torch.arange(allk.numel(), device=device)
    first = torch.full((uniq.numel(),), allk.numel(), dtype=torch.int64, device=device)
    first.scatter_reduce_(0, inv, pos, reduce="amin")
    order = torch.argsort(first)[:nnz]
    vals = counts[order].to(torch.float64)
    if wide:
        coords = torch.cat(ev_coords)[first[order]].to(torch.int64)
        return coords, vals
    keep = uniq[order]
    coords = torch.empty(nnz, d, dtype=torch.int64, device=device)
    rem = keep.clone()
    for k in range(d):
        coords[:, k] = torch.div(rem, st[k], rounding_mode="floor")
        rem -= coords[:, k] * st[k]
    return coords, vals


@dataclass
class SparseData:
    dims: list
    coords: torch.Tensor      # int64 [nnz, d]
    vals: torch.Tensor        # float64 [nnz]
    true_factors: list = field(default_factory=list)

    @property
    def nnz(self) -> int:
        return int(self.coords.shape[0])


def count_tensor(dims, R: int, nnz: int, seed: int, dist: str = "gamma", lam=None,
                 device="cpu", binary: bool = False) -> SparseData:
    """Sparse count (or binary) tensor from a rank-R nonnegative CP model."""
    facs = factor_matrices(dims, R, seed, dist=dist, device=device)
    if lam is None:
        lam = torch.ones(R, dtype=torch.float64)
    lam = torch.as_tensor(lam, dtype=torch.float64)
    coords, vals = events_to_tensor(dims, facs, lam, nnz, seed, device=device)
    if binary:
        vals = torch.ones_like(vals)
    return SparseData(list(int(n) for n in dims), coords, vals, facs)


def dense_gaussian(dims, R: int, seed: int, noise: float = 0.1, device="cpu",
                   dtype=torch.float32):
    """Dense tensor full(A) + noise * N(0,1) with A_k ~ N(0,1) [I_k, R],
    returned flat in row-major order."""
    facs = factor_matrices(dims, R, seed, dist="normal", device=device, dtype=dtype)
    g = _gen(seed + 7, device)
    d = len(dims)
    # Khatri-Rao of the leading and trailing halves of the modes, then one
    # 2-D product: X = KR(first) @ KR(rest)^T, reshaped row-major
    h = d // 2

    def kr(mats):
        out = mats[0]
        for m in mats[1:]:
            out = (out[:, None, :] * m[None, :, :]).reshape(-1, out.shape[1])
        return out

    left = kr(facs[:h]).contiguous()
    right = kr(facs[h:]).contiguous()
    X = torch.matmul(left, right.t().contiguous()).reshape(-1)
    X += noise * torch.randn(X.numel(), dtype=dtype, device=device, generator=g)
    return X, facs


def init_model(dims, R: int, seed: int, dist: str = "uniform", scale: float = 1.0,
               device="cpu", dtype=torch.float64) -> torch.Tensor:
    """Initial Kruskal model as ONE contiguous [sum_k I_k, R] array (mode 0's
    rows first).  dist 'uniform' = scale * U(0,1); 'normal' = scale * N(0,1)."""
    g = _gen(seed, device)
    rows = int(sum(int(n) for n in dims))
    if dist == "uniform":
        A = torch.rand(rows, R, dtype=dtype, device=device, generator=g)
    elif dist == "normal":
        A = torch.randn(rows, R, dtype=dtype, device=device, generator=g)
    else:
        raise ValueError(dist)
    return (A * scale).contiguous()


def normal_init_scale(R: int, d: int) -> float:
    """N(0,1) * R^(-1/(2d)) keeps model entries O(1) at any rank and order."""
    return float(R) ** (-1.0 / (2.0 * d))


@dataclass
class FedBlock:
    client: int
    grid_pos: tuple            # block coordinates in the process-grid sense
    row_base: list             # first global row of the block in each mode
    data: SparseData           # block-local coordinates


def fed_blocks(global_dims, grid, R: int, nnz_min: float, nnz_max: float, seed: int,
               device="cpu", dist: str = "gamma") -> list:
    """Client blocks of a d-way block grid over a global count tensor.

    Client c's nonzero count is round(nnz_min * (nnz_max/nnz_min)^(pi(c)/(K-1)))
    for a seeded permutation pi of 0..K-1 (log-uniform over the clients).  Each
    block is drawn by event sampling from the global rank-R gamma model
    restricted to the block's rows (its column weights are the restricted
    column masses)."""
    d = len(global_dims)
    K = int(np.prod(grid))
    rng = np.random.default_rng(seed)
    perm = rng.permutation(K)
    gfac = factor_matrices(global_dims, R, seed, dist=dist, device=device)
    bsz = [int(global_dims[k]) // int(grid[k]) for k in range(d)]
    blocks = []
    for c in range(K):
        pos = np.unravel_index(c, grid)
        base = [int(pos[k]) * bsz[k] for k in range(d)]
        ldims = [bsz[k] if pos[k] < grid[k] - 1 else int(global_dims[k]) - base[k]
                 for k in range(d)]
        facs = [gfac[k][base[k]:base[k] + ldims[k]] for k in range(d)]
        lam = torch.ones(R, dtype=torch.float64, device=device)
        for k in range(d):
            lam = lam * facs[k].sum(dim=0)
        frac = perm[c] / max(1, K - 1)
        nnz = int(round(nnz_min * (nnz_max / nnz_min) ** frac))
        coords, vals = events_to_tensor(ldims, facs, lam, nnz, seed + 1000 * (c + 1),
                                        device=device)
        blocks.append(FedBlock(c, tuple(int(p) for p in pos), base,
                               SparseData(ldims, coords, vals, facs)))
    return blocks


def cells(dims) -> int:
    return int(math.prod(int(n) for n in dims))
