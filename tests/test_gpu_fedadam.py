"""GCP-FedAdam rounds on the GPU (batched persistent launch, with and without
HIP-graph replay, and per-client launches) against the oracle's FedAdam round
(Alg. gcp-fed-iter) and against each other."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_20353_amd import _lib as G
from paper_2605_20353_amd import synth
from paper_2605_20353_amd.autotune import tune_fedadam
from paper_2605_20353_amd.fedadam import FedAdam, FedConfig, FedTile

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _blocks(gdims, grid, R, nmin, nmax, seed):
    return synth.fed_blocks(gdims, grid, R, nmin, nmax, seed=seed)


def _gpu_clients(blocks, dtype, gpu):
    out = []
    for bl in blocks:
        t = G.SparseTensor(bl.data.dims, bl.data.coords.to(gpu), bl.data.vals.to(dtype).to(gpu))
        out.append((t, bl.row_base))
    return out


def _oracle_clients(blocks, R, dtype):
    out = []
    for bl in blocks:
        t = oracle.SparseTensor(bl.data.dims, bl.data.coords.numpy(), bl.data.vals.to(dtype).double().numpy())
        n = sum(bl.data.dims) * R
        out.append(oracle.FedClient(t, np.array(bl.row_base), np.zeros(n), np.zeros(n), np.zeros(n)))
    return out


def _run_oracle(blocks, gdims, R, U0, cfg, rounds, dtype):
    ocl = _oracle_clients(blocks, R, dtype)
    U = U0.double().cpu().numpy().reshape(-1).copy()
    Bs, Cs = np.zeros_like(U), np.zeros_like(U)
    ap_c = oracle.AdamParams(cfg.lr, cfg.beta1, cfg.beta2, cfg.eps, cfg.lower)
    ap_s = oracle.AdamParams(cfg.meta_lr, cfg.beta1, cfg.beta2, cfg.eps, cfg.lower)
    st = 0
    for r in range(rounds):
        st = oracle.fedadam_round(ocl, gdims, R, U, Bs, Cs, st, r, cfg.tau, cfg.loss, cfg.p, cfg.q, cfg.seed,
                                  ap_c, ap_s)
    return U, ocl


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


SMALL = dict(gdims=[40, 36, 20], grid=(2, 2, 2), R=3, nmin=30, nmax=150)


# batched variants of the gradient scatter: atomics (default for few samples),
# every mode row-bucketed, and an LDS-private mode next to bucketed ones
SCATTER = {"atomic": FedTile(), "bucketed": FedTile(lds_modes=0, bucket_modes=7),
           "lds_and_bucketed": FedTile(lds_modes=4, bucket_modes=3)}


@pytest.mark.parametrize("mode", ["batched_graph", "batched", "plain", "batched_graph_bucketed", "batched_bucketed",
                                  "batched_graph_lds_and_bucketed"])
def test_fp64_rounds_match_oracle(gpu, mode):
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], SMALL["nmax"], seed=2609)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2709, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=3, loss="poisson", p=64, q=64, seed=20353, lr=1e-2, meta_lr=1e-2, lower=0.0)
    scatter = "lds_and_bucketed" if mode.endswith("lds_and_bucketed") else (
        "bucketed" if mode.endswith("bucketed") else "atomic")
    say(f"fedadam fp64 {mode}")
    fed = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg,
                  batched=mode != "plain", use_graph=mode.startswith("batched_graph"), tile=SCATTER[scatter])
    for r in range(2):
        fed.round(r)
    fed.status()
    Uo, ocl = _run_oracle(blocks, gdims, R, U0, cfg, 2, torch.float64)
    assert _rel(fed.U.cpu().numpy(), Uo) <= 1e-10
    for cl, oc in zip(fed.clients, ocl):
        assert _rel(cl.M.cpu().numpy(), oc.M) <= 1e-10
        assert _rel(cl.B.cpu().numpy(), oc.B) <= 1e-10
        assert torch.count_nonzero(cl.G).item() == 0


def test_fp64_workgroups_per_client_sweep(gpu):
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], 400, seed=2610)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2710, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=300, q=200, seed=5, lr=1e-2, meta_lr=1e-2, lower=0.0)
    Uo, _ = _run_oracle(blocks, gdims, R, U0, cfg, 1, torch.float64)
    for tile in (FedTile(1, 64), FedTile(3, 128), FedTile(16, 256), FedTile(2, 1024)):
        fed = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg, tile=tile)
        fed.round(0)
        fed.status()
        assert _rel(fed.U.cpu().numpy(), Uo) <= 1e-10, tile
        fed.close()


@pytest.mark.parametrize("tile", [FedTile(1, 64, lds_modes=0, bucket_modes=7, bucket_block_samples=512),
                                  FedTile(3, 128, lds_modes=0, bucket_modes=7, bucket_block_samples=512),
                                  FedTile(4, 1024, lds_modes=4, bucket_modes=3, bucket_block_samples=1024)])
def test_fp64_bucketed_blocks_and_workgroups(gpu, tile):
    """Several sorted sample blocks per client step, spread over 1..4
    workgroups per client, with ragged last blocks, against the oracle."""
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], 400, seed=2612)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2712, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=1500, q=1301, seed=7, lr=1e-2, meta_lr=1e-2, lower=0.0)
    Uo, ocl = _run_oracle(blocks, gdims, R, U0, cfg, 2, torch.float64)
    say(f"fedadam bucketed {tile}")
    fed = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg, tile=tile)
    for r in range(2):
        fed.round(r)
    fed.status()
    assert _rel(fed.U.cpu().numpy(), Uo) <= 1e-10
    for cl, oc in zip(fed.clients, ocl):
        assert _rel(cl.M.cpu().numpy(), oc.M) <= 1e-10


def test_fp64_automatic_bucketing_at_large_sample_counts(gpu):
    """At >= 2^14 samples per client step the automatic choice is the
    row-bucketed round (three launches per local step); it still matches the
    oracle."""
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], SMALL["nmax"], seed=2613)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2713, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=8192, q=8192, seed=3, lr=1e-2, meta_lr=1e-2, lower=0.0)
    Uo, ocl = _run_oracle(blocks, gdims, R, U0, cfg, 1, torch.float64)
    fed = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg, tile=FedTile(lds_modes=0))
    fed.round(0)
    fed.status()
    assert _rel(fed.U.cpu().numpy(), Uo) <= 1e-10
    for cl, oc in zip(fed.clients, ocl):
        assert _rel(cl.M.cpu().numpy(), oc.M) <= 1e-10


@pytest.mark.parametrize("shape", [(32, 1), (16, 2), (8, 4)])
def test_fp32_batched_equals_plain_and_oracle(gpu, shape):
    gdims, grid, R = [200, 160, 60], (4, 2, 2), 32
    blocks = _blocks(gdims, grid, R, 200, 2000, seed=2611)
    U0 = 0.1 + 0.9 * synth.init_model(gdims, R, 2711, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=4, loss="poisson", p=1024, q=1024, seed=11, lr=1e-3, meta_lr=1e-3, lower=0.0)
    feds = {}
    for mode in ("batched_graph", "plain", "batched_graph_bucketed"):
        tile = FedTile(lanes=shape[0], vec=shape[1], bucket_modes=7 if mode.endswith("bucketed") else 0)
        fed = FedAdam(_gpu_clients(blocks, torch.float32, gpu), gdims, U0.to(torch.float32).to(gpu), cfg,
                      batched=mode != "plain", use_graph=mode.startswith("batched_graph"), tile=tile)
        for r in range(2):
            fed.round(r)
        fed.status()
        feds[mode] = fed
    Up = feds["plain"].U.double().cpu().numpy()
    Uo, _ = _run_oracle(blocks, gdims, R, U0.to(torch.float32), cfg, 2, torch.float32)
    for mode in ("batched_graph", "batched_graph_bucketed"):
        Ub = feds[mode].U.double().cpu().numpy()
        assert _rel(Ub, Up) <= 1e-5, mode
        assert _rel(Ub, Uo) <= 1e-5, mode


@pytest.mark.parametrize("scatter", ["atomic", "bucketed"])
def test_graph_replays_stay_exact(gpu, scatter):
    """Several graph replays (the persistent launch, or the row-bucketed
    round's three launches per local step) with eager work and
    synchronisations in between each equal the eager batched rounds."""
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], SMALL["nmax"], seed=2612)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2712, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=64, q=64, seed=9, lr=1e-2, meta_lr=1e-2, lower=0.0)
    tile = SCATTER[scatter]
    fg = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg, use_graph=True, tile=tile)
    fe = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg, use_graph=False, tile=tile)
    for r in range(4):
        fg.round(r)
        fe.round(r)
        junk = torch.randn(1000, device=gpu).sum().item()     # eager work between replays
        torch.cuda.synchronize()
        assert junk == junk
        assert _rel(fg.U.cpu().numpy(), fe.U.cpu().numpy()) <= 1e-12, r


def test_autotuner_keeps_state_and_picks_a_shape(gpu, tmp_path, monkeypatch):
    monkeypatch.setenv("GCP_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], SMALL["nmax"], seed=2613)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2713, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=64, q=64, seed=3, lr=1e-2, meta_lr=1e-2, lower=0.0)
    fed = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg)
    before = fed.U.clone()
    tile = tune_fedadam(fed, candidates=[FedTile(1, 256), FedTile(4, 256), FedTile(2, 512)])
    assert torch.equal(fed.U, before)
    assert (tmp_path / "tune.json").exists()
    fed.round(0)
    fed.status()
    Uo, _ = _run_oracle(blocks, gdims, R, U0, cfg, 1, torch.float64)
    assert _rel(fed.U.cpu().numpy(), Uo) <= 1e-10
    assert isinstance(tile, FedTile)


@pytest.mark.parametrize("scatter", ["atomic", "bucketed"])
def test_fp64_four_way_rounds_match_oracle(gpu, scatter):
    """4-way client blocks: the general-order kernels of both batched forms."""
    gdims, R = [20, 18, 12, 8], 3
    blocks = _blocks(gdims, (2, 2, 1, 2), R, 30, 120, seed=2615)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2715, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=200, q=150, seed=6, lr=1e-2, meta_lr=1e-2, lower=0.0)
    tile = FedTile() if scatter == "atomic" else FedTile(lds_modes=0, bucket_modes=15, bucket_block_samples=512)
    fed = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg, tile=tile)
    for r in range(2):
        fed.round(r)
    fed.status()
    Uo, ocl = _run_oracle(blocks, gdims, R, U0, cfg, 2, torch.float64)
    assert _rel(fed.U.cpu().numpy(), Uo) <= 1e-10
    for cl, oc in zip(fed.clients, ocl):
        assert _rel(cl.M.cpu().numpy(), oc.M) <= 1e-10


def test_batched_and_plain_classes_equal_the_flags(gpu):
    from paper_2605_20353_amd.fedadam import Batched, Plain
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], SMALL["nmax"], seed=2614)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2714, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=64, q=64, seed=4, lr=1e-2, meta_lr=1e-2, lower=0.0)
    a = Batched(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg)
    b = Plain(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg)
    assert a.batched and a.use_graph and not b.batched
    a.round(0)
    b.round(0)
    a.status()
    b.status()
    assert _rel(a.U.cpu().numpy(), b.U.cpu().numpy()) <= 1e-12


def test_create_errors(gpu):
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], SMALL["nmax"], seed=2614)
    U0 = synth.init_model(gdims, R, 1, dtype=torch.float64).to(gpu)
    cfg = FedConfig(R=R, tau=1, p=8, q=8)
    cl = _gpu_clients(blocks, torch.float64, gpu)
    bad = [(t, [b[0] + 30, b[1], b[2]]) for t, b in cl]          # blocks outside the global dims
    with pytest.raises(G.GCPError) as e:
        FedAdam(bad, gdims, U0, cfg)
    assert e.value.code == G.GCP_ERR_ARG
    with pytest.raises(G.GCPError) as e:                         # more workgroups than the GPU holds
        FedAdam(cl, gdims, U0, cfg, tile=FedTile(workgroups_per_client=100000))
    assert e.value.code == G.GCP_ERR_UNSUPPORTED
