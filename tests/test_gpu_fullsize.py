"""Parity at the full benchmark sizes, in the launch configurations bench.py
times.

10000 x 8000 x 6000 Poisson tensor with 5e7 nonzeros, rank 32, 2^20 + 2^20
stratified samples: every one of the 2^21 samples is checked bit for bit
against the oracle's own draw (its sorted-tuple binary search against the
GPU's hash table), and the whole gradient of the fused kernel -- atomic,
row-bucketed (the automatic choice, and the exact launch shape the benchmark
times, read from the traffic summary it pairs its timing with) and
bit-reproducible -- against the oracle's gradient on its own samples, element
by element within the float32 rounding bound.

GCP-FedAdam, 64 clients on a 4 x 4 x 4 grid over 20000 x 20000 x 2000 with
1e5..5e6 nonzeros per client: one batched (graph-replayed) round, with the
automatic (row-bucketed at this size) and with the atomic scatter, and one
per-client round with each call's automatic scatter, equal one round of
per-client launches with hardware atomics (U, every M_c and every B_c).
"""
import json
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2605_20353_amd import _lib as G
from paper_2605_20353_amd import synth
from paper_2605_20353_amd.fedadam import FedAdam, FedConfig, FedTile, Plain
from parity_util import assert_grad_close

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_config2_full_size_samples_and_gradient(gpu):
    dims, R, nnz, P, Q = [10000, 8000, 6000], 32, 50_000_000, 1 << 20, 1 << 20
    t0 = time.time()
    data = synth.count_tensor(dims, R, nnz, seed=2607, device=gpu)
    t = G.SparseTensor(dims, data.coords, data.vals.to(torch.float32))
    t.reserve(P + Q, R)
    A = synth.init_model(dims, R, 2707, device=gpu, dtype=torch.float32)
    sp = G.SampleParams("stratified", P, Q, seed=20353, step=3)
    c, x, w = G.gcp_sample(t, sp)
    Ga, La = G.gcp_loss_grad(t, sp, A, R, "poisson", tile=G.Tile(bucket_modes=0, lds_modes=0))
    Gb, Lb = G.gcp_loss_grad(t, sp, A, R, "poisson")                     # automatic: row-bucketed
    # the benchmark's launch shape: the tile of its traffic summary
    with open(os.path.join(os.path.dirname(__file__), "..", "profiles", "loss_grad_cfg2_traffic.json")) as f:
        bench_tile = G.Tile(**json.load(f)["tile"])
    Gt, Lt = G.gcp_loss_grad(t, sp, A, R, "poisson", tile=bench_tile)
    Gd, Ld = G.gcp_loss_grad(t, sp, A, R, "poisson", deterministic=True)
    Gd2, Ld2 = G.gcp_loss_grad(t, sp, A, R, "poisson", deterministic=True)
    t.status()
    assert torch.equal(Gd, Gd2) and torch.equal(Ld, Ld2), "deterministic runs differ"
    say(f"config 2: GPU side done in {time.time() - t0:.1f} s; building the oracle's sorted index")
    coords = data.coords.cpu().numpy()
    vals = data.vals.to(torch.float32).double().cpu().numpy()
    del data
    to = oracle.SparseTensor(dims, coords, vals)
    say(f"config 2: oracle index built at {time.time() - t0:.1f} s")
    oc, ox, ow = oracle.sample_stratified(to, P, Q, 20353, 3)
    np.testing.assert_array_equal(c.cpu().numpy(), oc)
    np.testing.assert_array_equal(x.cpu().numpy(), ox.astype(np.float32))
    np.testing.assert_array_equal(w.cpu().numpy(), ow.astype(np.float32))
    Go, Fo = oracle.loss_grad(dims, R, A.double().cpu().numpy(), oc, ox, ow, "poisson")
    say(f"config 2: oracle gradient at {time.time() - t0:.1f} s")
    Go = Go.reshape(-1, R)
    A64 = A.double().cpu().numpy().reshape(-1)
    for name, (Gx, Lx) in (("atomic", (Ga, La)), ("bucketed", (Gb, Lb)), (f"benchmark tile {bench_tile}", (Gt, Lt)),
                           ("deterministic", (Gd, Ld))):
        # every element within the rounding bound of float32 arithmetic in
        # any summation order, and per mode within 1e-5 relative
        frob, worst = assert_grad_close(Gx.cpu().numpy(), Go, dims, R, A64, oc, ox, ow, "poisson", torch.float32,
                                        what=f"config 2 {name}")
        say(f"config 2 {name}: per-mode rel err {frob:.2e}, worst element at {worst:.2f} of its bound")
        assert abs(Lx.item() - Fo) <= 1e-5 * abs(Fo)


def test_config5_full_size_batched_equals_plain(gpu):
    gd, grid, R = [20000, 20000, 2000], (4, 4, 4), 32
    blocks = synth.fed_blocks(gd, grid, R, 1e5, 5e6, seed=2610, device=gpu)
    total = sum(b.data.nnz for b in blocks)
    assert 7e7 < total < 9.5e7
    clients = [(G.SparseTensor(b.data.dims, b.data.coords, b.data.vals.to(torch.float32)), b.row_base)
               for b in blocks]
    del blocks
    U0 = synth.init_model(gd, R, 2710, device=gpu, dtype=torch.float32)
    cfg = FedConfig(R=R, tau=10, loss="poisson", p=1 << 16, q=1 << 16, seed=20353, lr=1e-3, meta_lr=1e-3,
                    lower=0.0)
    state = {}
    modes = (("plain", lambda: Plain(clients, gd, U0, cfg, scatter="atomic")),
             ("plain_auto", lambda: Plain(clients, gd, U0, cfg, scatter="auto")),
             ("graph", lambda: FedAdam(clients, gd, U0, cfg, batched=True, use_graph=True)),
             ("graph_atomic", lambda: FedAdam(clients, gd, U0, cfg, batched=True, use_graph=True,
                                              tile=FedTile(bucket_modes=0))))
    forms = {"plain": "per_client", "plain_auto": "per_client", "graph": "row_bucketed",
             "graph_atomic": "persistent"}
    for name, make in modes:
        fed = make()
        assert fed.info()["form"] == forms[name], (name, fed.info())
        fed.round(0)
        fed.status()
        # U, and the clients' models and first moments (B_c is not invariant
        # to the gradients' scale)
        state[name] = (fed.U.double().cpu().numpy(),
                       [(c.M.double().cpu().numpy(), c.B.double().cpu().numpy()) for c in fed.clients])
        say(f"config 5: {name} round done")
        fed.close()
    U_ref, cl_ref = state["plain"]
    for name in ("plain_auto", "graph", "graph_atomic"):
        U, cls = state[name]
        rel = np.linalg.norm(U - U_ref) / np.linalg.norm(U_ref)
        assert rel <= 1e-5, (name, "U", rel)
        for c, ((M, B), (Mr, Br)) in enumerate(zip(cls, cl_ref)):
            assert np.linalg.norm(M - Mr) / np.linalg.norm(Mr) <= 1e-5, (name, "M", c)
            assert np.linalg.norm(B - Br) / np.linalg.norm(Br) <= 1e-5, (name, "B", c)
    assert np.abs(state["graph"][0] - U0.double().cpu().numpy().reshape(-1)).max() > 0     # the round moved U
