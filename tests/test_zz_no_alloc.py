"""gcp_loss_grad_noalloc (the entry point for callers that cannot allocate)
against gcp_loss_grad with a reserved workspace, through the C ABI.

Both run the row-bucketed scatter (requested explicitly, so a call that did
not bucket would have failed) on the same samples; each gradient is held to
the oracle element by element (the rounding-error bound for any summation
order) and per mode (1e-5 relative in float32, 1e-12 in float64), and the
two are compared with each other.  Two calls in a row, the second with a
smaller input, so the scratch region holds the first call's entries when the
second runs.  Also: the automatic choice buckets inside the scratch region,
falls back to hardware atomics when a call would need more than the region,
an explicit request that does not fit is refused on the host, and the calls
change the device's free memory by nothing.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_20353_amd import _lib as G
from paper_2605_20353_amd import synth
from parity_util import assert_grad_close, frob_rel_errs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _tensor(gpu, dtype, dims, nnz, seed, binary=False):
    data = synth.count_tensor(dims, 4, nnz, seed=seed, binary=binary)
    t = G.SparseTensor(dims, data.coords.to(gpu), data.vals.to(dtype).to(gpu))
    to = oracle.SparseTensor(dims, data.coords.numpy(), data.vals.to(dtype).double().numpy())
    return t, to


def _check_against_oracle(to, dims, R, A, sp, loss, dtype, grads, what):
    sc, sx, sw = oracle.sample_stratified(to, sp.p, sp.q, sp.seed, sp.step, sp.client)
    A64 = A.double().cpu().numpy().reshape(-1)
    Go, Fo = oracle.loss_grad(dims, R, A64, sc, sx, sw, loss)
    for name, (Gx, Lx) in grads.items():
        assert_grad_close(Gx.cpu().numpy(), Go, dims, R, A64, sc, sx, sw, loss, dtype, what=f"{what} {name}")
        rel = abs(Lx.item() - Fo) / abs(Fo)
        assert rel <= (1e-5 if dtype == torch.float32 else 1e-12), f"{what} {name}: objective rel err {rel}"


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_reserved_two_calls(gpu, dtype):
    dims, R, loss = [3000, 2500, 2000], 32, "poisson"
    t, to = _tensor(gpu, dtype, dims, 200_000, seed=2621)
    A = synth.init_model(dims, R, 2622, device=gpu, dtype=dtype).contiguous()
    t.reserve(1 << 18, R)
    tile = G.Tile(lds_modes=0, bucket_modes=7)
    # first call: several sorting workgroups and a ragged tail; second call:
    # a smaller sample set, while the scratch region still holds the first
    # call's entries and counts
    for call, (p, q) in enumerate([((1 << 16) + 333, (1 << 16) + 1001), (3000 + 17, 5000 + 5)]):
        sp = G.SampleParams("stratified", p, q, seed=20353, step=41 + call)
        say(f"noalloc {dtype} call {call}: p={p} q={q}")
        Gn = torch.empty_like(A)
        Ln = torch.zeros(1, dtype=torch.float64, device=gpu)
        G.gcp_loss_grad_noalloc(t, sp, A, R, loss, Gn, Ln, tile=tile)
        Gr, Lr = G.gcp_loss_grad(t, sp, A, R, loss, tile=tile)
        t.status()
        tol = 1e-5 if dtype == torch.float32 else 1e-12
        errs = frob_rel_errs(Gn.cpu().numpy(), Gr.cpu().numpy(), dims, R)
        assert max(errs) <= tol, f"noalloc vs reserved, call {call}: per-mode rel errors {errs}"
        _check_against_oracle(to, dims, R, A, sp, loss, dtype, {"noalloc": (Gn, Ln), "reserved": (Gr, Lr)},
                              f"{dtype} call {call}")


def test_noalloc_automatic_and_limits(gpu):
    dtype = torch.float32
    dims, R, loss = [3000, 2500, 2000], 32, "bernoulli_logit"
    t, to = _tensor(gpu, dtype, dims, 150_000, seed=2623, binary=True)
    A = (0.3 * synth.init_model(dims, R, 2624, dist="normal", device=gpu, dtype=torch.float64)).to(dtype).contiguous()
    cap = G.gcp_noalloc_scratch_bytes()
    assert cap == 128 << 20
    # automatic choice at 2^17 + 2^17 samples: bucketed inside the scratch
    sp = G.SampleParams("stratified", 1 << 17, 1 << 17, seed=20353, step=7)
    Gn = torch.empty_like(A)
    Ln = torch.zeros(1, dtype=torch.float64, device=gpu)
    say("noalloc automatic, 2^18 samples")
    G.gcp_loss_grad_noalloc(t, sp, A, R, loss, Gn, Ln)
    t.status()
    _check_against_oracle(to, dims, R, A, sp, loss, dtype, {"noalloc-auto": (Gn, Ln)}, "automatic")
    # the free device memory does not move across further calls
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for step in range(3):
        G.gcp_loss_grad_noalloc(t, G.SampleParams("stratified", 1 << 17, 1 << 17, seed=20353, step=100 + step),
                                A, R, loss, Gn, Ln)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, f"free device memory changed by {free0 - free1} bytes across noalloc calls"
    # a call that would need more than the scratch region: an explicit
    # bucketed request is refused before any launch, the automatic choice
    # takes hardware atomics and still gives the gradient
    big = G.SampleParams("stratified", 1_500_000, 1_500_000, seed=20353, step=9)
    with pytest.raises(G.GCPError) as ei:
        G.gcp_loss_grad_noalloc(t, big, A, R, loss, Gn, Ln, tile=G.Tile(bucket_modes=7, lds_modes=0))
    assert ei.value.code == G.GCP_ERR_ARG and "scratch" in str(ei.value)
    say("noalloc automatic, 3e6 samples (atomic fallback)")
    G.gcp_loss_grad_noalloc(t, big, A, R, loss, Gn, Ln)
    Ga, La = G.gcp_loss_grad(t, big, A, R, loss, tile=G.Tile(bucket_modes=0))
    t.status()
    errs = frob_rel_errs(Gn.cpu().numpy(), Ga.cpu().numpy(), dims, R)
    assert max(errs) <= 1e-5, f"atomic fallback vs atomic call: per-mode rel errors {errs}"
    assert abs(Ln.item() - La.item()) <= 1e-5 * abs(La.item())
