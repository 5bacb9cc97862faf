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


FP32_TOL = 1e-5


def _assert_state_matches(fed, Uo, ocl, tol, what):
    """U and every client's M_c, B_c, C_c against the oracle's round state.
    B_c (the first moment, (1 - beta1) times a sum of sampled gradients) is
    not invariant to the gradients' scale, so it catches magnitude errors
    that Adam's sign-like early steps hide in U and M_c."""
    assert _rel(fed.U.double().cpu().numpy(), Uo) <= tol, f"{what}: U"
    for c, (cl, oc) in enumerate(zip(fed.clients, ocl)):
        assert _rel(cl.M.double().cpu().numpy(), oc.M) <= tol, f"{what}: M_{c}"
        assert _rel(cl.B.double().cpu().numpy(), oc.B) <= tol, f"{what}: B_{c}"
        assert _rel(cl.C.double().cpu().numpy(), oc.C) <= tol, f"{what}: C_{c}"
        assert torch.count_nonzero(cl.G).item() == 0, f"{what}: G_{c} not left zeroed"


@pytest.mark.parametrize("shape", [(32, 1), (16, 2), (8, 4)])
def test_fp32_batched_equals_plain_and_oracle(gpu, shape):
    gdims, grid, R = [200, 160, 60], (4, 2, 2), 32
    blocks = _blocks(gdims, grid, R, 200, 2000, seed=2611)
    U0 = 0.1 + 0.9 * synth.init_model(gdims, R, 2711, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=4, loss="poisson", p=1024, q=1024, seed=11, lr=1e-3, meta_lr=1e-3, lower=0.0)
    feds = {}
    # the client blocks' modes all fit the LDS budget, so the bucketed mode
    # turns LDS-private accumulation off to really row-bucket every mode
    tiles = {"batched_graph": FedTile(lanes=shape[0], vec=shape[1], bucket_modes=0),
             "plain": FedTile(lanes=shape[0], vec=shape[1], bucket_modes=0),
             "batched_graph_bucketed": FedTile(lanes=shape[0], vec=shape[1], lds_modes=0, bucket_modes=7)}
    forms = {"batched_graph": "persistent", "plain": "per_client", "batched_graph_bucketed": "row_bucketed"}
    for mode, tile in tiles.items():
        fed = FedAdam(_gpu_clients(blocks, torch.float32, gpu), gdims, U0.to(torch.float32).to(gpu), cfg,
                      batched=mode != "plain", use_graph=mode.startswith("batched_graph"), tile=tile)
        info = fed.info()
        assert info["form"] == forms[mode], (mode, info)
        if mode.endswith("bucketed"):
            assert info["bucket_modes"] == 7 and info["lds_modes"] == 0, info
        for r in range(2):
            fed.round(r)
        fed.status()
        feds[mode] = fed
    Uo, ocl = _run_oracle(blocks, gdims, R, U0.to(torch.float32), cfg, 2, torch.float32)
    for mode, fed in feds.items():
        _assert_state_matches(fed, Uo, ocl, FP32_TOL, f"{mode} {shape}")
    for mode in ("batched_graph", "batched_graph_bucketed"):
        for cb, cp in zip(feds[mode].clients, feds["plain"].clients):
            assert _rel(cb.B.double().cpu().numpy(), cp.B.double().cpu().numpy()) <= FP32_TOL, mode


# client blocks 1200 x 1000 x 200 at rank 32 in float32: modes 0 and 1 exceed
# the 64 KiB LDS budget of a batched client (150 and 125 KiB), mode 2 fits
BIG = dict(gdims=[2400, 2000, 400], grid=(2, 2, 2), R=32, nmin=3000, nmax=20000)


@pytest.mark.parametrize("lds", ["auto", "none"])
def test_fp32_row_bucketed_round_matches_oracle(gpu, lds):
    """The FP32 row-bucketed batched round -- k_fed_sample / k_fed_owner with
    eight lanes of four columns, the form config-5 rounds take -- against the
    oracle's FedAdam rounds: 2^13 + 2^13 samples per client step (the
    automatic choice row-buckets from 2^14), three local steps, two rounds.
    With the automatic LDS choice mode 2 stays LDS-private next to the two
    bucketed modes; without it every mode is bucketed."""
    gdims, grid, R = BIG["gdims"], BIG["grid"], BIG["R"]
    blocks = _blocks(gdims, grid, R, BIG["nmin"], BIG["nmax"], seed=2631)
    U0 = 0.1 + 0.9 * synth.init_model(gdims, R, 2731, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=3, loss="poisson", p=1 << 13, q=1 << 13, seed=13, lr=1e-3, meta_lr=1e-3, lower=0.0)
    tile = FedTile() if lds == "auto" else FedTile(lds_modes=0)
    say(f"fedadam fp32 row-bucketed, lds {lds}")
    fed = FedAdam(_gpu_clients(blocks, torch.float32, gpu), gdims, U0.to(torch.float32).to(gpu), cfg, tile=tile)
    info = fed.info()
    assert info["form"] == "row_bucketed", info
    assert (info["lanes"], info["vec"]) == (8, 4), info
    assert info["bucket_modes"] == (3 if lds == "auto" else 7) and info["lds_modes"] == (4 if lds == "auto" else 0), info
    for r in range(2):
        fed.round(r)
    fed.status()
    Uo, ocl = _run_oracle(blocks, gdims, R, U0.to(torch.float32), cfg, 2, torch.float32)
    _assert_state_matches(fed, Uo, ocl, FP32_TOL, f"row-bucketed lds={lds}")


def test_fp32_per_client_automatic_scatter_matches_oracle(gpu):
    """Per-client rounds with each gcp_loss_grad call's automatic scatter
    (row-bucketed at 2^16 samples, on the client workspaces the Plain class
    reserves) against the oracle."""
    from paper_2605_20353_amd.fedadam import Plain
    gdims, grid, R = BIG["gdims"], BIG["grid"], BIG["R"]
    blocks = _blocks(gdims, grid, R, BIG["nmin"], BIG["nmax"], seed=2632)
    U0 = 0.1 + 0.9 * synth.init_model(gdims, R, 2732, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=1 << 15, q=1 << 15, seed=17, lr=1e-3, meta_lr=1e-3, lower=0.0)
    fed = Plain(_gpu_clients(blocks, torch.float32, gpu), gdims, U0.to(torch.float32).to(gpu), cfg, scatter="auto")
    info = fed.info()
    assert info["form"] == "per_client" and info["bucket_modes"] == -1, info
    assert all(cl.tensor.reserved_samples >= cfg.p + cfg.q for cl in fed.clients)
    fed.round(0)
    fed.status()
    Uo, ocl = _run_oracle(blocks, gdims, R, U0.to(torch.float32), cfg, 1, torch.float32)
    _assert_state_matches(fed, Uo, ocl, FP32_TOL, "per-client automatic scatter")


def test_barrier_timeout_fails_the_round_cleanly(gpu):
    """A persistent round whose group barriers may wait no time at all: the
    first early arrival gives up (workgroups without samples reach the
    barrier after the gradient long before those with samples), every
    workgroup leaves the launch, the server step is skipped, U is unchanged,
    the next round is refused on the host, and the status reports and clears
    the failure."""
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], SMALL["nmax"], seed=2633)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2733, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=3, loss="poisson", p=64, q=64, seed=3, lr=1e-2, meta_lr=1e-2, lower=0.0,
                    barrier_timeout_s=1e-9)
    fed = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg, use_graph=False,
                  tile=FedTile(workgroups_per_client=4, block=64, bucket_modes=0))
    assert fed.info()["form"] == "persistent"
    U_before = fed.U.clone()
    fed.round(0)
    torch.cuda.synchronize()
    assert torch.equal(fed.U, U_before)
    with pytest.raises(G.GCPError) as e:
        fed.round(1)
    assert e.value.code == G.GCP_ERR_HIP
    with pytest.raises(G.GCPError) as e:
        fed.status()
    assert e.value.code == G.GCP_ERR_HIP
    fed.status()                                    # cleared


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


@pytest.mark.parametrize("scatter", ["atomic", "bucketed"])
def test_fp32_four_way_rounds_match_oracle(gpu, scatter):
    """4-way client blocks in FP32 (the general-order kernels of both batched
    forms at rank 16) against the oracle's rounds: U, every M_c, B_c, C_c."""
    gdims, R = [40, 36, 24, 16], 16
    blocks = _blocks(gdims, (2, 2, 1, 2), R, 200, 900, seed=2616)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2716, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=600, q=500, seed=8, lr=1e-3, meta_lr=1e-3, lower=0.0)
    tile = (FedTile(workgroups_per_client=3) if scatter == "atomic" else
            FedTile(lds_modes=0, bucket_modes=15, bucket_block_samples=512))
    say(f"fedadam fp32 4-way {scatter}")
    fed = FedAdam(_gpu_clients(blocks, torch.float32, gpu), gdims, U0.to(torch.float32).to(gpu), cfg, tile=tile)
    assert fed.info()["form"] == ("persistent" if scatter == "atomic" else "row_bucketed")
    for r in range(2):
        fed.round(r)
    fed.status()
    Uo, ocl = _run_oracle(blocks, gdims, R, U0.to(torch.float32), cfg, 2, torch.float32)
    _assert_state_matches(fed, Uo, ocl, FP32_TOL, f"4-way {scatter}")


@pytest.mark.parametrize("gdims,grid", [([60, 48], (2, 2)), ([12, 10, 8, 8, 6], (2, 1, 2, 1, 2))],
                         ids=["2-way", "5-way"])
@pytest.mark.parametrize("scatter", ["atomic", "bucketed", "lds_and_bucketed"])
def test_fp32_two_and_five_way_rounds_match_oracle(gpu, gdims, grid, scatter):
    """Orders 2 and 5 through the general-order kernels of both batched forms
    in FP32; the 5-way blocks draw their fifth coordinate from the second
    Philox block of each counter."""
    R = 8
    d = len(gdims)
    blocks = _blocks(gdims, grid, R, 60, 300, seed=2618 + d)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2718 + d, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=300, q=200, seed=9, lr=1e-3, meta_lr=1e-3, lower=0.0)
    full = (1 << d) - 1
    tile = {"atomic": FedTile(workgroups_per_client=3),
            "bucketed": FedTile(lds_modes=0, bucket_modes=full, bucket_block_samples=512),
            "lds_and_bucketed": FedTile(lds_modes=1, bucket_modes=full & ~1, bucket_block_samples=512)}[scatter]
    say(f"fedadam fp32 {d}-way {scatter}")
    fed = FedAdam(_gpu_clients(blocks, torch.float32, gpu), gdims, U0.to(torch.float32).to(gpu), cfg, tile=tile)
    assert fed.info()["form"] == ("persistent" if scatter == "atomic" else "row_bucketed")
    for r in range(2):
        fed.round(r)
    fed.status()
    Uo, ocl = _run_oracle(blocks, gdims, R, U0.to(torch.float32), cfg, 2, torch.float32)
    _assert_state_matches(fed, Uo, ocl, FP32_TOL, f"{d}-way {scatter}")


def test_fp32_mixed_radix_client_blocks_match_oracle(gpu):
    """Client blocks shaped like the Amazon tensor (4821207 x 1774269 x
    1805187: 23 + 21 + 21 coordinate bits, so each block's cells take the
    mixed-radix key) through both batched forms against the oracle's rounds
    (one oracle run for both: its Adam over 3.4e7 client parameters per step
    is the slow part)."""
    gdims, R = [2 * 4821207, 1774269, 1805187], 4
    blocks = _blocks(gdims, (2, 1, 1), R, 300, 600, seed=2619)
    assert all(b.data.dims == [4821207, 1774269, 1805187] for b in blocks)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2719, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=700, q=500, seed=10, lr=1e-3, meta_lr=1e-3, lower=0.0)
    say("fedadam fp32 mixed-radix blocks: oracle")
    Uo, ocl = _run_oracle(blocks, gdims, R, U0.to(torch.float32), cfg, 2, torch.float32)
    for scatter, tile in (("atomic", FedTile()),
                          ("bucketed", FedTile(lds_modes=0, bucket_modes=7, bucket_block_samples=512))):
        say(f"fedadam fp32 mixed-radix blocks {scatter}")
        fed = FedAdam(_gpu_clients(blocks, torch.float32, gpu), gdims, U0.to(torch.float32).to(gpu), cfg, tile=tile)
        assert fed.info()["form"] == ("persistent" if scatter == "atomic" else "row_bucketed")
        for r in range(2):
            fed.round(r)
        fed.status()
        _assert_state_matches(fed, Uo, ocl, FP32_TOL, f"mixed radix {scatter}")
        fed.close()
        del fed
        torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,R", [(torch.float64, 48), (torch.float64, 100), (torch.float64, 200),
                                     (torch.float32, 96), (torch.float32, 256)])
@pytest.mark.parametrize("scatter", ["atomic", "bucketed"])
def test_wide_rank_rounds_match_oracle(gpu, dtype, R, scatter):
    """Ranks past 32 (FP64) and 64 (FP32): 64 lanes of 1, 2 or 4 columns in
    both batched forms against the oracle's rounds."""
    gdims = SMALL["gdims"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], SMALL["nmax"], seed=2617)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2717, dtype=torch.float64)
    cfg = FedConfig(R=R, tau=2, loss="poisson", p=64, q=64, seed=20353, lr=1e-2, meta_lr=1e-2, lower=0.0)
    tile = FedTile() if scatter == "atomic" else FedTile(lds_modes=0, bucket_modes=7, bucket_block_samples=512)
    say(f"fedadam wide rank R={R} {dtype} {scatter}")
    fed = FedAdam(_gpu_clients(blocks, dtype, gpu), gdims, U0.to(dtype).to(gpu), cfg, tile=tile)
    info = fed.info()
    assert info["lanes"] == 64 and info["lanes"] * info["vec"] >= R, info
    for r in range(2):
        fed.round(r)
    fed.status()
    Uo, ocl = _run_oracle(blocks, gdims, R, U0.to(dtype), cfg, 2, dtype)
    _assert_state_matches(fed, Uo, ocl, 1e-10 if dtype == torch.float64 else FP32_TOL, f"R={R} {scatter}")


def test_automatic_workgroups_per_client(gpu):
    """The persistent launch's automatic workgroups per client: one for a
    local step of two 64-sample chunks; for 128 chunks at 256 threads (four
    wavefronts) enough for four chunks per wavefront, 8, which the GPU holds
    for 8 clients -- and that round matches the oracle."""
    gdims, R = SMALL["gdims"], SMALL["R"]
    blocks = _blocks(gdims, SMALL["grid"], R, SMALL["nmin"], SMALL["nmax"], seed=2620)
    U0 = 0.2 + 0.8 * synth.init_model(gdims, R, 2720, dtype=torch.float64)
    for pq, want in ((64, 1), (4096, 8)):
        cfg = FedConfig(R=R, tau=2, loss="poisson", p=pq, q=pq, seed=12, lr=1e-2, meta_lr=1e-2, lower=0.0)
        fed = FedAdam(_gpu_clients(blocks, torch.float64, gpu), gdims, U0.to(gpu), cfg, tile=FedTile(bucket_modes=0))
        info = fed.info()
        assert info["form"] == "persistent" and info["block"] == 256, info
        assert info["workgroups_per_client"] == want, (pq, info)
        if pq == 4096:
            fed.round(0)
            fed.status()
            Uo, ocl = _run_oracle(blocks, gdims, R, U0, cfg, 1, torch.float64)
            assert _rel(fed.U.cpu().numpy(), Uo) <= 1e-10
            for cl, oc in zip(fed.clients, ocl):
                assert _rel(cl.B.cpu().numpy(), oc.B) <= 1e-10
        fed.close()


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
