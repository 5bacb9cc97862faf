"""GPU parity: the HIP path against the FP64 CPU oracle, through the C ABI.

Samples must match bit for bit.  Gradients are compared with the oracle fed
the same factors (float32 factors upcast to float64) element by element --
every element within the rounding-error bound of the GPU's arithmetic for any
summation order (parity_util) -- and per mode as ||G_gpu - G_oracle||_F /
||G_oracle||_F: <= 1e-12 for the float64 build and <= 1e-5 for float32.
Sampled objectives: same relative bounds.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_20353_amd import _lib as G
from paper_2605_20353_amd import synth
from parity_util import assert_grad_close

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
LOSSES = ["poisson", "gaussian", "bernoulli_logit"]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------------ cases --

CASES = {
    # name: dims, nnz, R
    "cfg1_50x40x30": ([50, 40, 30], 3000, 5),
    "4way": ([12, 10, 8, 6], 400, 8),
    "5way": ([6, 5, 4, 3, 7], 150, 3),
    "1way": ([300], 40, 4),
    "r32": ([64, 48, 40], 2000, 32),
    "r64_4way": ([30, 20, 16, 8], 900, 64),
    "8way": ([3, 4, 2, 5, 3, 2, 4, 3], 500, 4),          # the most modes a tensor may have
    "r1_unit_mode": ([40, 1, 30], 300, 1),              # rank 1, and a mode of one index (no key bits)
    "5way_r33": ([6, 5, 4, 3, 7], 200, 33),             # general order, odd rank: 64 lanes of one column
    "2way": ([50, 40], 600, 6),                         # matrix: general-order kernels, 30% dense
}


def make_case(name, dtype, gpu, binary=False, seed=2606):
    dims, nnz, R = CASES[name]
    data = synth.count_tensor(dims, 3, nnz, seed=seed, binary=binary)
    coords = data.coords
    vals = data.vals
    t_gpu = G.SparseTensor(dims, coords.to(gpu), vals.to(dtype).to(gpu))
    # the oracle sees exactly the values the GPU holds
    t_ora = oracle.SparseTensor(dims, coords.numpy(), vals.to(dtype).double().numpy())
    return t_gpu, t_ora, dims, R


def model(dims, R, dtype, gpu, seed=7, dist="uniform", lo=0.2):
    A = synth.init_model(dims, R, seed, dist=dist, dtype=torch.float64)
    if dist == "uniform":
        A = lo + (1 - lo) * A
    return A.to(dtype).to(gpu).contiguous()


class Ref:
    """The oracle's gradient and objective of one sample set, and the
    per-element check of a GPU gradient against them."""

    def __init__(self, dims, R, A, coords, x, w, loss, n_semi=0):
        self.dims, self.R, self.loss, self.n_semi = list(dims), R, loss, n_semi
        self.A64 = A.double().cpu().numpy().reshape(-1)
        self.coords, self.x, self.w = coords, x, w
        self.G, self.F = oracle.loss_grad(self.dims, R, self.A64, coords, x, w, loss, n_semi=n_semi)

    def check(self, Gg, dtype, what="", scale=1.0, bound_scale=None):
        """Gg ~ scale * G element by element; bound_scale widens the bound
        (several results added together)."""
        bs = abs(scale) if bound_scale is None else bound_scale
        return assert_grad_close(Gg.double().cpu().numpy(), scale * np.asarray(self.G), self.dims, self.R, self.A64,
                                 self.coords, self.x, self.w, self.loss, dtype, n_semi=self.n_semi, what=str(what),
                                 scale=bs)

    def check_loss(self, Lg, dtype, factor=1.0):
        assert abs(Lg.item() - factor * self.F) <= TOL[dtype] * abs(factor * self.F), (Lg.item(), self.F)


def oracle_ref(t_ora, dims, R, A, loss, sp: G.SampleParams) -> Ref:
    semi = sp.kind == "semi_stratified"
    sc, sx, sw = oracle.sample_stratified(t_ora, sp.p, sp.q, sp.seed, sp.step, sp.client,
                                          sp.max_attempts, semi=semi)
    return Ref(dims, R, A, sc, sx, sw, loss, n_semi=sp.p if semi else 0)


# --------------------------------------------------------------- sampling --

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("pq", [(1000, 1000), (37, 91), (0, 64), (65, 0)])
def test_samples_bit_exact(gpu, dtype, name, pq):
    t_gpu, t_ora, dims, R = make_case(name, dtype, gpu)
    p, q = pq
    sp = G.SampleParams("stratified", p, q, seed=20353, step=11, client=3)
    say(f"sample {name} {dtype} p={p} q={q}")
    c, x, w = G.gcp_sample(t_gpu, sp)
    t_gpu.status()
    oc, ox, ow = oracle.sample_stratified(t_ora, p, q, 20353, 11, 3)
    np.testing.assert_array_equal(c.cpu().numpy(), oc)
    np.testing.assert_array_equal(x.cpu().numpy(), ox.astype(x.cpu().numpy().dtype))
    np.testing.assert_array_equal(w.cpu().numpy(), ow.astype(w.cpu().numpy().dtype))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_samples_bit_exact_mostly_full_tensor(gpu, dtype):
    """7 of every 8 cells are nonzeros: most zero-sample attempts land on a
    stored nonzero, so the membership probe (slot pairs, scanning on past a
    pair) and the redraw loop run for nearly every zero sample.  Draws and
    the sampled gradient on them equal the oracle's."""
    dims = [20, 20, 20]
    rng = np.random.default_rng(2611)
    cells = rng.permutation(8000)[:7000]
    coords = np.stack(np.unravel_index(cells, dims), axis=1).astype(np.int64)
    vals = rng.integers(1, 6, size=7000).astype(np.float64)
    t_gpu = G.SparseTensor(dims, torch.from_numpy(coords).to(gpu), torch.from_numpy(vals).to(dtype).to(gpu))
    t_ora = oracle.SparseTensor(dims, coords, vals)
    p, q = 3000, 5000
    say(f"mostly-full sample {dtype}")
    sp = G.SampleParams("stratified", p, q, seed=7, step=5, client=1, max_attempts=400)
    c, x, w = G.gcp_sample(t_gpu, sp)
    t_gpu.status()
    oc, ox, ow = oracle.sample_stratified(t_ora, p, q, 7, 5, 1, max_attempts=400)
    np.testing.assert_array_equal(c.cpu().numpy(), oc)
    np.testing.assert_array_equal(x.cpu().numpy(), ox.astype(x.cpu().numpy().dtype))
    np.testing.assert_array_equal(w.cpu().numpy(), ow.astype(w.cpu().numpy().dtype))
    assert not np.isin(np.ravel_multi_index(oc[p:].T, dims), cells).any()
    R = 8
    A = model(dims, R, dtype, gpu)
    ref = oracle_ref(t_ora, dims, R, A, "poisson", sp)
    Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson")
    t_gpu.status()
    ref.check(Gg, dtype, "mostly full")
    ref.check_loss(Lg, dtype)


def test_samples_depend_on_step_seed_client(gpu):
    t_gpu, _, _, _ = make_case("cfg1_50x40x30", torch.float64, gpu)
    base = G.gcp_sample(t_gpu, G.SampleParams("stratified", 100, 100, seed=1, step=0, client=0))[0]
    for kw in (dict(seed=2), dict(step=1), dict(client=1)):
        args = dict(seed=1, step=0, client=0)
        args.update(kw)
        other = G.gcp_sample(t_gpu, G.SampleParams("stratified", 100, 100, **args))[0]
        assert not torch.equal(base, other)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_uniform_samples_bit_exact(gpu, dtype):
    dims = [6, 5, 4, 3]
    X, _ = synth.dense_gaussian(dims, 2, seed=3, dtype=torch.float64)
    Xg = X.to(dtype).to(gpu)
    t = G.DenseTensor(dims, Xg)
    sp = G.SampleParams("uniform", 333, 0, seed=5, step=2)
    c, x, w = G.gcp_sample(t, sp)
    oc, ox, ow = oracle.sample_uniform(dims, X.to(dtype).double().numpy(), 333, 5, 2)
    np.testing.assert_array_equal(c.cpu().numpy(), oc)
    np.testing.assert_array_equal(x.double().cpu().numpy(), ox)
    np.testing.assert_array_equal(w.cpu().numpy(), ow.astype(w.cpu().numpy().dtype))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_semi_stratified_samples_bit_exact(gpu, dtype):
    t_gpu, t_ora, dims, R = make_case("4way", dtype, gpu)
    sp = G.SampleParams("semi_stratified", 200, 300, seed=9, step=4)
    c, x, w = G.gcp_sample(t_gpu, sp)
    oc, ox, ow = oracle.sample_stratified(t_ora, 200, 300, 9, 4, semi=True)
    np.testing.assert_array_equal(c.cpu().numpy(), oc)
    np.testing.assert_array_equal(w.cpu().numpy(), ow.astype(w.cpu().numpy().dtype))


# ------------------------------------------------- mixed-radix cell keys --

# coordinate bit widths summing past 63: the library keys cells by their
# row-major linear index instead of bit-packing them
RADIX_CASES = {
    "amazon_65bit": [4821207, 1774269, 1805187],     # 23 + 21 + 21 bits, M ~ 1.54e19 > 2^63
    "4way_64bit": [40000, 40000, 40000, 40000],      # 4 x 16 bits, M = 2.56e18
}


def radix_case(name, dtype, gpu, q, seed, step):
    """~20000 event-sampled nonzeros plus, planted as nonzeros, the first zero
    candidate of every other zero sample of (seed, step), so that those zero
    samples are decided by the membership test and redrawn."""
    dims = RADIX_CASES[name]
    d = len(dims)
    data = synth.count_tensor(dims, 3, 20000, seed=2613)
    planted = []
    for s in range(0, q, 2):
        o = oracle.philox4x64_10([s, step, 1, 0], [seed, 0])
        planted.append([oracle.range_map(int(o[k]), dims[k]) for k in range(d)])
    coords = np.concatenate([data.coords.numpy(), np.array(planted, dtype=np.int64)])
    vals = np.concatenate([data.vals.numpy(), np.ones(len(planted))])
    coords, first = np.unique(coords, axis=0, return_index=True)
    vals = vals[first]
    t_gpu = G.SparseTensor(dims, torch.from_numpy(coords).to(gpu), torch.from_numpy(vals).to(dtype).to(gpu))
    t_ora = oracle.SparseTensor(dims, coords, torch.from_numpy(vals).to(dtype).double().numpy())
    return t_gpu, t_ora, dims, planted


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", list(RADIX_CASES))
def test_mixed_radix_keys_match_oracle(gpu, dtype, name):
    """Bit-exact samples (stratified and semi-stratified) and gradients of the
    fused, materialised, atomic and (4-way) row-bucketed paths on tensors whose
    cells need the mixed-radix key."""
    q, seed, step, R = 2000, 13, 4, 4
    t_gpu, t_ora, dims, planted = radix_case(name, dtype, gpu, q, seed, step)
    say(f"mixed radix {name} {dtype}: {t_ora.nnz} nonzeros")
    A = model(dims, R, dtype, gpu)
    for kind in ("stratified", "semi_stratified"):
        sp = G.SampleParams(kind, 3000, q, seed=seed, step=step)
        c, x, w = G.gcp_sample(t_gpu, sp)
        t_gpu.status()
        oc, ox, ow = oracle.sample_stratified(t_ora, sp.p, q, seed, step, semi=(kind == "semi_stratified"))
        np.testing.assert_array_equal(c.cpu().numpy(), oc)
        np.testing.assert_array_equal(x.cpu().numpy(), ox.astype(x.cpu().numpy().dtype))
        np.testing.assert_array_equal(w.cpu().numpy(), ow.astype(w.cpu().numpy().dtype))
        zc = oc[sp.p:]
        if kind == "stratified":      # the planted candidates were rejected and redrawn
            assert all(list(zc[s]) != planted[s // 2] for s in range(0, q, 2))
        else:                         # semi-stratified keeps the first candidate
            assert all(list(zc[s]) == planted[s // 2] for s in range(0, q, 2))
        ref = oracle_ref(t_ora, dims, R, A, "poisson", sp)
        tiles = [G.Tile(), G.Tile(lds_modes=0, bucket_modes=0)]
        if name == "4way_64bit":
            t_gpu.reserve(sp.n, R)
            tiles.append(G.Tile(lds_modes=0, bucket_modes=15))
        for tile in tiles:
            Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", tile=tile)
            t_gpu.status()
            ref.check(Gg, dtype, (kind, tile))
            ref.check_loss(Lg, dtype)
        Gm, _ = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", samples=(c, x, w))
        ref.check(Gm, dtype, (kind, "materialised"))


# --------------------------------------------------------------- gradient --

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("loss", LOSSES)
@pytest.mark.parametrize("name", list(CASES))
def test_fused_loss_grad_matches_oracle(gpu, dtype, loss, name):
    t_gpu, t_ora, dims, R = make_case(name, dtype, gpu, binary=(loss == "bernoulli_logit"))
    dist = "normal" if loss != "poisson" else "uniform"
    A = model(dims, R, dtype, gpu, dist=dist)
    sp = G.SampleParams("stratified", 1500, 1300, seed=77, step=5)
    say(f"loss_grad {name} {loss} {dtype}")
    Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, loss)
    t_gpu.status()
    ref = oracle_ref(t_ora, dims, R, A, loss, sp)
    ref.check(Gg, dtype, (name, loss))
    ref.check_loss(Lg, dtype)


def _shapes(R, dtype):
    f32 = [(8, 1), (16, 1), (32, 1), (64, 1), (2, 4), (4, 4), (8, 4), (16, 4), (32, 4), (64, 4), (4, 2), (8, 2), (16, 2)]
    f64 = [(8, 1), (16, 1), (32, 1), (64, 1), (4, 2), (8, 2), (16, 2), (32, 2)]
    out = []
    for lanes, vec in (f32 if dtype == torch.float32 else f64):
        if R % vec == 0 and lanes * vec >= R:
            out.append((lanes, vec))
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", ["r32", "r64_4way", "cfg1_50x40x30", "8way", "r1_unit_mode"])
def test_every_tile_matches_oracle(gpu, dtype, name):
    t_gpu, t_ora, dims, R = make_case(name, dtype, gpu)
    A = model(dims, R, dtype, gpu)
    sp = G.SampleParams("stratified", 777, 555, seed=3, step=1)
    ref = oracle_ref(t_ora, dims, R, A, "poisson", sp)
    for lanes, vec in _shapes(R, dtype):
        for block in (64, 256, 1024):
            for lds in (0, (1 << len(dims)) - 1):
                tile = G.Tile(lanes=lanes, vec=vec, block=block, lds_modes=lds)
                Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", tile=tile)
                ref.check(Gg, dtype, (lanes, vec, block, lds))
                ref.check_loss(Lg, dtype)
    # a small grid forces many chunks per wave (grid-stride path)
    Gg, _ = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", tile=G.Tile(grid=1, block=64))
    ref.check(Gg, dtype, "grid 1")


BUCKET_TILES = [
    dict(),                                                          # automatic
    dict(bucket_modes=7, lds_modes=0, bucket_lds_bytes=8192, bucket_block_samples=512, bucket_splits=3),
    dict(bucket_modes=5, lds_modes=0, bucket_block_samples=1024, bucket_splits=1, bucket_block=64),
    dict(bucket_modes=7, lds_modes=0, bucket_block_samples=512, bucket_splits=7, bucket_block=192),
    dict(bucket_modes=7, lds_modes=2, bucket_block_samples=4096, bucket_block=1024),
    dict(bucket_modes=7, lds_modes=0, bucket_block_samples=8192, bucket_lds_bytes=65536),
    dict(block=1024, bucket_modes=-1, bucket_block_samples=4096, bucket_splits=16, bucket_block=1024),
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", ["r32", "r64_4way"])
def test_bucketed_scatter_every_lane_shape(gpu, dtype, name):
    """The owner pass adds 1, 2 or 4 columns per lane (float column pairs by
    one 64-bit compare-and-swap): every lane shape, bucketed alone and with
    the LDS-private strategy on one mode, against the oracle, with 256- and
    1024-thread owner workgroups and one or two splits per row block."""
    t_gpu, t_ora, dims, R = make_case(name, dtype, gpu)
    pq = (20000, 9001)
    t_gpu.reserve(sum(pq), R)
    A = model(dims, R, dtype, gpu)
    sp = G.SampleParams("stratified", pq[0], pq[1], seed=37, step=4)
    ref = oracle_ref(t_ora, dims, R, A, "poisson", sp)
    every = (1 << len(dims)) - 1
    for lanes, vec in _shapes(R, dtype):
        for lds, bblock, splits in ((0, 256, 2), (1, 256, 2), (0, 1024, 1), (1, 1024, 2)):
            tl = dict(lanes=lanes, vec=vec, bucket_modes=every & ~lds, lds_modes=lds, bucket_block_samples=1024,
                      bucket_splits=splits, bucket_block=bblock)
            say(f"bucketed shape {name} {dtype} {tl}")
            Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", tile=G.Tile(**tl))
            t_gpu.status()
            ref.check(Gg, dtype, tl)
            ref.check_loss(Lg, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("loss", LOSSES)
@pytest.mark.parametrize("pq", [(70000, 50001), (3000, 2000)])
def test_bucketed_scatter_matches_oracle(gpu, dtype, loss, pq):
    """Row-bucketed (sort-by-row) scatter, alone and mixed with the LDS and
    atomic strategies, ragged sample counts, every loss, against the oracle."""
    t_gpu, t_ora, dims, R = make_case("r32", dtype, gpu, binary=(loss == "bernoulli_logit"))
    t_gpu.reserve(sum(pq), R)
    A = model(dims, R, dtype, gpu, dist="uniform" if loss == "poisson" else "normal")
    sp = G.SampleParams("stratified", pq[0], pq[1], seed=31, step=2)
    ref = oracle_ref(t_ora, dims, R, A, loss, sp)
    for tl in BUCKET_TILES:
        say(f"bucketed {dtype} {loss} {pq} {tl}")
        Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, loss, tile=G.Tile(**tl))
        t_gpu.status()
        ref.check(Gg, dtype, tl)
        ref.check_loss(Lg, dtype)
    # a scale and accumulation go through the bucketed path too: two halves
    # added, each within half the bound, plus the rounding of their sum
    scale = torch.tensor([0.5], dtype=dtype, device=gpu)
    Gs, _ = G.gcp_loss_grad(t_gpu, sp, A, R, loss, scale=scale, tile=G.Tile(bucket_modes=7, lds_modes=0))
    Gs, _ = G.gcp_loss_grad(t_gpu, sp, A, R, loss, G=Gs, accumulate=True, scale=scale,
                            tile=G.Tile(bucket_modes=7, lds_modes=0))
    ref.check(Gs, dtype, "scaled and accumulated", bound_scale=2.0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", ["1way", "2way", "5way", "8way", "5way_r33"])
def test_bucketed_scatter_general_order(gpu, dtype, name):
    """The general-order owner pass (the modes other than the owned one in
    compile-time slots, unused slots multiplying as ones): orders 1, 2, 5 and
    8, and an odd rank, every mode row-bucketed or mixed with LDS-private
    modes, several sorted blocks with ragged ends, against the oracle."""
    t_gpu, t_ora, dims, R = make_case(name, dtype, gpu)
    d = len(dims)
    full = (1 << d) - 1
    sp = G.SampleParams("stratified", 1300, 901, seed=37, step=3)
    t_gpu.reserve(sp.n, R)
    A = model(dims, R, dtype, gpu)
    ref = oracle_ref(t_ora, dims, R, A, "poisson", sp)
    tiles = [dict(bucket_modes=full, lds_modes=0, bucket_block_samples=512),
             dict(bucket_modes=full, lds_modes=0, bucket_block_samples=1024, bucket_splits=3, bucket_block=64)]
    if d > 1:
        tiles.append(dict(bucket_modes=full & ~1, lds_modes=1, bucket_block_samples=512))
    for tl in tiles:
        say(f"bucketed general order {name} {dtype} {tl}")
        Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", tile=G.Tile(**tl))
        t_gpu.status()
        ref.check(Gg, dtype, tl)
        ref.check_loss(Lg, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_bucketed_scatter_4way_r64(gpu, dtype):
    t_gpu, t_ora, dims, R = make_case("r64_4way", dtype, gpu)
    t_gpu.reserve(40000, R)
    A = model(dims, R, dtype, gpu)
    sp = G.SampleParams("stratified", 20000, 19999, seed=5, step=9)
    ref = oracle_ref(t_ora, dims, R, A, "poisson", sp)
    for tl in (dict(bucket_modes=15, lds_modes=0), dict(bucket_modes=15, lds_modes=0, bucket_lds_bytes=8192)):
        Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", tile=G.Tile(**tl))
        ref.check(Gg, dtype, tl)


def test_bucketed_scatter_needs_workspace(gpu):
    t_gpu, _, dims, R = make_case("r32", torch.float32, gpu)
    A = model(dims, R, torch.float32, gpu)
    sp = G.SampleParams("stratified", 1000, 1000, seed=1)
    with pytest.raises(G.GCPError):
        G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", tile=G.Tile(bucket_modes=1))
    t_gpu.reserve(1000, R)
    with pytest.raises(G.GCPError):     # reserved for fewer samples than requested
        G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", tile=G.Tile(bucket_modes=1))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_materialised_equals_fused(gpu, dtype):
    t_gpu, t_ora, dims, R = make_case("4way", dtype, gpu)
    A = model(dims, R, dtype, gpu)
    sp = G.SampleParams("stratified", 900, 700, seed=12, step=2)
    smp = G.gcp_sample(t_gpu, sp)
    Gm, Lm = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", samples=smp)
    Gf, Lf = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson")
    ref = oracle_ref(t_ora, dims, R, A, "poisson", sp)
    for name, (Gx, Lx) in (("materialised", (Gm, Lm)), ("fused", (Gf, Lf))):
        ref.check(Gx, dtype, name)
        ref.check_loss(Lx, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("loss", LOSSES)
def test_semi_stratified_grad_matches_oracle(gpu, dtype, loss):
    t_gpu, t_ora, dims, R = make_case("r32", dtype, gpu, binary=(loss == "bernoulli_logit"))
    A = model(dims, R, dtype, gpu, dist="normal" if loss != "poisson" else "uniform")
    sp = G.SampleParams("semi_stratified", 1000, 1200, seed=8, step=3)
    Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, loss)
    ref = oracle_ref(t_ora, dims, R, A, loss, sp)
    ref.check(Gg, dtype, ("semi-stratified", loss))
    ref.check_loss(Lg, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_uniform_dense_grad_matches_oracle(gpu, dtype):
    dims, R = [20, 16, 12, 6], 16
    X, _ = synth.dense_gaussian(dims, 4, seed=3, dtype=torch.float64)
    t = G.DenseTensor(dims, X.to(dtype).to(gpu))
    A = model(dims, R, dtype, gpu, dist="normal")
    sp = G.SampleParams("uniform", 5000, 0, seed=4, step=0)
    oc, ox, ow = oracle.sample_uniform(dims, X.to(dtype).double().numpy(), 5000, 4, 0)
    ref = Ref(dims, R, A, oc, ox, ow, "gaussian")
    for lds in (-1, 0, 15):
        Gg, Lg = G.gcp_loss_grad(t, sp, A, R, "gaussian", tile=G.Tile(lds_modes=lds))
        ref.check(Gg, dtype, ("uniform", lds))
        ref.check_loss(Lg, dtype)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_flags_scale_accumulate_loss_only(gpu, dtype):
    t_gpu, t_ora, dims, R = make_case("cfg1_50x40x30", dtype, gpu)
    A = model(dims, R, dtype, gpu)
    sp = G.SampleParams("stratified", 500, 500, seed=1, step=0)
    ref = oracle_ref(t_ora, dims, R, A, "poisson", sp)
    scale = torch.tensor([-2.5], dtype=dtype, device=gpu)
    Gs, Ls = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", scale=scale)
    ref.check(Gs, dtype, "scaled", scale=-2.5)
    ref.check_loss(Ls, dtype)                                      # objective not scaled
    Ga, La = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", G=Gs.clone(), loss_out=Ls.clone(), accumulate=True)
    # -2.5 G (bound 2.5 b) plus G (bound b), plus the rounding of their sum
    ref.check(Ga, dtype, "accumulated", scale=-1.5, bound_scale=4.5)
    ref.check_loss(La, dtype, factor=2.0)
    _, Lo = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", loss_only=True)
    ref.check_loss(Lo, dtype)


# ------------------------------------------------------------------- Adam --

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1, 7, 1000, 4099])
def test_adam_matches_oracle(gpu, dtype, n):
    rng = np.random.default_rng(n)
    A0 = rng.normal(size=n)
    Gr = rng.normal(size=n)
    B0 = rng.normal(size=n) * 0.1
    C0 = rng.uniform(0, 1, n)
    dev = lambda a: torch.tensor(a, dtype=dtype, device=gpu)
    A, Gt, B, Cm = dev(A0), dev(Gr), dev(B0), dev(C0)
    G.gcp_adam_step(A, Gt, B, Cm, 3, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-8, lower=-0.5, zero_grad=True)
    Ao, Bo, Co = (v.to(dtype).double().cpu().numpy() for v in (dev(A0), dev(B0), dev(C0)))
    oracle.adam(Ao, dev(Gr).double().cpu().numpy(), Bo, Co, 3, 1e-2, 0.9, 0.99, 1e-8, -0.5)
    tol = 1e-14 if dtype == torch.float64 else 1e-6
    np.testing.assert_allclose(A.double().cpu().numpy(), Ao, rtol=tol, atol=tol)
    np.testing.assert_allclose(B.double().cpu().numpy(), Bo, rtol=tol, atol=tol)
    np.testing.assert_allclose(Cm.double().cpu().numpy(), Co, rtol=tol, atol=tol)
    assert torch.count_nonzero(Gt).item() == 0


def test_config1_fp64_trajectory_20_steps(gpu):
    """50x40x30 Poisson, rank 5, 1000 + 1000 samples, 20 Adam steps, lr 1e-3:
    the FP64 GPU trajectory equals the oracle's within 1e-10 relative."""
    t_gpu, t_ora, dims, R = make_case("cfg1_50x40x30", torch.float64, gpu)
    A = model(dims, R, torch.float64, gpu, seed=2605, lo=0.0)
    Bg, Cg, Gg = torch.zeros_like(A), torch.zeros_like(A), torch.zeros_like(A)
    Ao = A.cpu().numpy().copy()
    Bo, Co = np.zeros_like(Ao), np.zeros_like(Ao)
    ap = oracle.AdamParams(lr=1e-3, lower=0.0)
    for step in range(20):
        sp = G.SampleParams("stratified", 1000, 1000, seed=20353, step=step)
        G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", G=Gg, want_loss=False)
        G.gcp_adam_step(A, Gg, Bg, Cg, step + 1, lr=1e-3, lower=0.0)
        oracle.sgd_step(t_ora, R, Ao, Bo, Co, step + 1, "poisson", 1000, 1000, 20353, step, ap)
    t_gpu.status()
    err = np.linalg.norm(A.cpu().numpy() - Ao) / np.linalg.norm(Ao)
    assert err <= 1e-10, err


# ----------------------------------------------------------------- errors --

def test_rejection_exhaustion_is_reported(gpu):
    dims = [4, 3, 2]
    allc = torch.tensor(list(np.ndindex(*dims)), dtype=torch.int64)
    t = G.SparseTensor(dims, allc[1:].to(gpu), torch.ones(23, dtype=torch.float64, device=gpu))
    G.gcp_sample(t, G.SampleParams("stratified", 0, 64, seed=1, max_attempts=1))
    with pytest.raises(G.GCPError) as e:
        t.status()
    assert e.value.code == G.GCP_ERR_SAMPLING
    t.status()                                   # the word was cleared
    c, _, _ = G.gcp_sample(t, G.SampleParams("stratified", 0, 16, seed=1, max_attempts=2000))
    t.status()
    assert (c.cpu() == allc[0]).all()


def test_bad_data_is_rejected(gpu):
    dims = [4, 4]
    with pytest.raises(G.GCPError) as e:
        G.SparseTensor(dims, torch.tensor([[0, 1], [2, 3], [0, 1]], device=gpu),
                       torch.ones(3, dtype=torch.float64, device=gpu))
    assert e.value.code == G.GCP_ERR_DATA
    with pytest.raises(G.GCPError) as e:
        G.SparseTensor(dims, torch.tensor([[0, 4]], device=gpu), torch.ones(1, dtype=torch.float64, device=gpu))
    assert e.value.code == G.GCP_ERR_DATA
    t = G.SparseTensor(dims, torch.tensor([[0, 1]], device=gpu), torch.ones(1, dtype=torch.float64, device=gpu))
    A = torch.ones(8 * 2, dtype=torch.float64, device=gpu)
    bad = (torch.tensor([[0, 9]], device=gpu), torch.ones(1, dtype=torch.float64, device=gpu),
           torch.ones(1, dtype=torch.float64, device=gpu))
    G.gcp_loss_grad(t, G.SampleParams("stratified", 1, 0), A, 2, "poisson", samples=bad)
    with pytest.raises(G.GCPError) as e:
        t.status()
    assert e.value.code == G.GCP_ERR_DATA


def test_argument_errors(gpu):
    t_gpu, _, dims, R = make_case("cfg1_50x40x30", torch.float32, gpu)
    A = model(dims, R, torch.float32, gpu)
    with pytest.raises(G.GCPError):      # no zeros to sample in a full tensor
        full = torch.tensor(list(np.ndindex(2, 2)), device=gpu)
        tf = G.SparseTensor([2, 2], full, torch.ones(4, device=gpu))
        G.gcp_sample(tf, G.SampleParams("stratified", 1, 1))
    with pytest.raises(G.GCPError):      # uniform sampling needs a dense tensor
        G.gcp_sample(t_gpu, G.SampleParams("uniform", 10, 0))
    with pytest.raises(G.GCPError):      # vec does not divide R = 5
        G.gcp_loss_grad(t_gpu, G.SampleParams("stratified", 10, 10), A, R, "poisson", tile=G.Tile(vec=4))
    with pytest.raises(G.GCPError):      # too few lanes
        G.gcp_loss_grad(t_gpu, G.SampleParams("stratified", 10, 10), A, R, "poisson", tile=G.Tile(lanes=2, vec=1))
    with pytest.raises(G.GCPError):      # R outside [1, 256]
        G.gcp_loss_grad(t_gpu, G.SampleParams("stratified", 10, 10), torch.zeros(0, device=gpu), 0, "poisson")
    assert G.lib().gcp_loss_grad(t_gpu.handle, None, None, None, 0, 1, 0, None, None, None, None,
                                 None) == G.GCP_ERR_ARG


def test_empty_sample_set(gpu):
    t_gpu, _, dims, R = make_case("cfg1_50x40x30", torch.float32, gpu)
    A = model(dims, R, torch.float32, gpu)
    Gg, Lg = G.gcp_loss_grad(t_gpu, G.SampleParams("stratified", 0, 0), A, R, "poisson",
                             G=torch.full_like(A, 3.0))
    assert torch.count_nonzero(Gg).item() == 0 and Lg.item() == 0.0
