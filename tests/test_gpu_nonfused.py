"""The non-fused sampled gradient (Sec. 3.1.2) on the GPU, through the C ABI:
gcp_sample_y writes the sampled tensor (coordinates bit-exact against the
oracle's draws, values y = w f'(x, m) against the oracle's), gcp_mttkrp
reads a sampled tensor and gathers the factor rows again (element by element
against the oracle's MTTKRP within the rounding bound), and the two together
give the oracle's sampled gradient, for every loss, sampling scheme and
scatter strategy."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_20353_amd import _lib as G
from paper_2605_20353_amd import synth
from parity_util import SAFETY, assert_grad_close, frob_rel_errs

pytestmark = pytest.mark.gpu

LOSSES = ["poisson", "gaussian", "bernoulli_logit"]
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(gpu, dtype, dims, nnz, R, binary, seed=2651):
    data = synth.count_tensor(dims, 3, nnz, seed=seed, binary=binary)
    t = G.SparseTensor(dims, data.coords.to(gpu), data.vals.to(dtype).to(gpu))
    to = oracle.SparseTensor(dims, data.coords.numpy(), data.vals.to(dtype).double().numpy())
    return t, to


def _model(dims, R, dtype, gpu, loss, seed=5):
    if loss == "poisson":
        A = 0.2 + 0.8 * synth.init_model(dims, R, seed, dtype=torch.float64)
    else:
        A = 0.5 * synth.init_model(dims, R, seed, dist="normal", dtype=torch.float64)
    return A.to(dtype).to(gpu).contiguous()


def _gamma(n, u):
    n = np.asarray(n, dtype=np.float64)
    return n * u / (1 - n * u)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("loss", LOSSES)
@pytest.mark.parametrize("kind", ["stratified", "semi_stratified"])
def test_sample_y_matches_oracle(gpu, dtype, loss, kind):
    dims, R = [60, 50, 40], 16
    t, to = _case(gpu, dtype, dims, 3000, R, binary=(loss == "bernoulli_logit"))
    A = _model(dims, R, dtype, gpu, loss)
    sp = G.SampleParams(kind, 1777, 1301, seed=41, step=3)
    Lg = torch.zeros(1, dtype=torch.float64, device=gpu)
    c, y, _ = G.gcp_sample_y(t, sp, A, R, loss, loss_out=Lg)
    t.status()
    semi = kind == "semi_stratified"
    oc, ox, ow = oracle.sample_stratified(to, sp.p, sp.q, sp.seed, sp.step, semi=semi)
    np.testing.assert_array_equal(c.cpu().numpy(), oc)
    A64 = A.double().cpu().numpy().reshape(-1)
    yo = oracle.sample_derivatives(dims, R, A64, oc, ox, ow, loss, n_semi=sp.p if semi else 0)
    Go, Fo = oracle.loss_grad(dims, R, A64, oc, ox, ow, loss, n_semi=sp.p if semi else 0)
    if dtype == torch.float64:
        err = np.abs(y.cpu().numpy() - yo)
        assert np.all(err <= 1e-12 * (np.abs(yo) + np.abs(ow))), err.max()
    # the stored values feed the gradient: their MTTKRP (in FP64 on the host)
    # is the oracle's gradient within the rounding bound of y
    Gy = oracle.mttkrp(dims, R, A64, oc, y.double().cpu().numpy())
    assert_grad_close(Gy, Go, dims, R, A64, oc, ox, ow, loss, dtype, n_semi=sp.p if semi else 0,
                      what=f"y of {loss} {kind}")
    assert abs(Lg.item() - Fo) <= TOL[dtype] * abs(Fo)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("tile", ["atomic", "lds", "bucketed", "auto"])
def test_mttkrp_matches_oracle(gpu, dtype, tile):
    dims, R = [300, 200, 100], 32
    t, _ = _case(gpu, dtype, dims, 5000, R, binary=False)
    rng = np.random.default_rng(7)
    n = 70001
    coords = np.stack([rng.integers(0, I, n) for I in dims], axis=1).astype(np.int64)
    y = rng.normal(size=n).astype(np.float32).astype(np.float64)        # exact in either format
    A = _model(dims, R, dtype, gpu, "gaussian")
    t.reserve(n, R)
    tiles = {"atomic": G.Tile(lds_modes=0, bucket_modes=0), "lds": G.Tile(lds_modes=4, bucket_modes=0),
             "bucketed": G.Tile(lds_modes=0, bucket_modes=7, bucket_block_samples=1024),
             "auto": G.Tile()}
    Gg = G.gcp_mttkrp(t, torch.from_numpy(coords).to(gpu), torch.from_numpy(y).to(dtype).to(gpu), A, R,
                      tile=tiles[tile])
    t.status()
    A64 = A.double().cpu().numpy().reshape(-1)
    Go = oracle.mttkrp(dims, R, A64, coords, y)
    # rounding bound of the MTTKRP of exact values: d - 1 products per
    # contribution, count - 1 additions per element in any order
    u = oracle.U_F32 if dtype == torch.float32 else oracle.U_F64
    absG = oracle.mttkrp(dims, R, np.abs(A64), coords, np.abs(y))
    off = np.concatenate([[0], np.cumsum(dims)])
    count = np.concatenate([np.bincount(coords[:, k], minlength=dims[k]) for k in range(3)])
    bound = SAFETY * (_gamma(3, u) + _gamma(np.repeat(np.maximum(count - 1, 0), R), u)) * absG * (1 + 2**-53 / u)
    err = np.abs(Gg.double().cpu().numpy().reshape(-1) - Go)
    assert np.all(err <= bound + 1e-300), (err / np.maximum(bound, 1e-300)).max()
    assert max(frob_rel_errs(Gg.double().cpu().numpy(), Go, dims, R)) <= TOL[dtype]
    # accumulate and scale
    scale = torch.tensor([-0.5], dtype=dtype, device=gpu)
    G.gcp_mttkrp(t, torch.from_numpy(coords).to(gpu), torch.from_numpy(y).to(dtype).to(gpu), A, R, G=Gg,
                 accumulate=True, scale=scale, tile=tiles[tile])
    assert max(frob_rel_errs(Gg.double().cpu().numpy(), 0.5 * Go, dims, R)) <= 4 * TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("loss", LOSSES)
def test_nonfused_gradient_matches_oracle_and_fused(gpu, dtype, loss):
    """gcp_sample_y then gcp_mttkrp (rows gathered twice) against the oracle's
    gradient, and against the fused call on the same samples."""
    dims, R = [120, 90, 70], 32
    t, to = _case(gpu, dtype, dims, 20000, R, binary=(loss == "bernoulli_logit"))
    A = _model(dims, R, dtype, gpu, loss)
    sp = G.SampleParams("stratified", 40000, 30001, seed=43, step=1)
    t.reserve(sp.n, R)
    c, y, _ = G.gcp_sample_y(t, sp, A, R, loss)
    Gn = G.gcp_mttkrp(t, c, y, A, R)
    Gf, _ = G.gcp_loss_grad(t, sp, A, R, loss)
    t.status()
    oc, ox, ow = oracle.sample_stratified(to, sp.p, sp.q, sp.seed, sp.step)
    A64 = A.double().cpu().numpy().reshape(-1)
    Go, _ = oracle.loss_grad(dims, R, A64, oc, ox, ow, loss)
    for name, Gx in (("non-fused", Gn), ("fused", Gf)):
        assert_grad_close(Gx.cpu().numpy(), Go, dims, R, A64, oc, ox, ow, loss, dtype, what=f"{name} {loss}")


def test_nonfused_argument_errors(gpu):
    dims, R = [20, 10, 5], 4
    t, _ = _case(gpu, torch.float32, dims, 100, R, binary=False)
    A = _model(dims, R, torch.float32, gpu, "poisson")
    sp = G.SampleParams("stratified", 10, 10, seed=1)
    assert G.lib().gcp_sample_y(t.handle, G.C.byref(sp.c()), G._ptr(A), R, 1, None, None, None, None,
                                None) == G.GCP_ERR_ARG
    bad = torch.tensor([[0, 0, 7]], device=gpu)       # coordinate 7 outside mode 2 (5 rows)
    G.gcp_mttkrp(t, bad, torch.ones(1, device=gpu), A, R)
    with pytest.raises(G.GCPError) as e:
        t.status()
    assert e.value.code == G.GCP_ERR_DATA
