"""Benchmark: GCP-SGD/Adam sampled-gradient steps on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (the configuration the headline metric is quoted on): a 3-way sparse
Poisson count tensor 10000 x 8000 x 6000 with 5e7 nonzeros drawn from a
rank-32 gamma(1,1) CP model, rank-32 FP32 Kruskal model, 2^20 nonzero +
2^20 zero stratified samples per step.  One step = the fused sampled
loss/gradient kernel (sampling, model values, Poisson derivative, sampled
MTTKRP) + the Adam kernel (lower bound 0).  Inputs are generated on the GPU
and resident in HBM before the timed region.

Prints ONE JSON line.  `value` = samples (p + q) per second over the timed
steps (whole step, wall clock between two device synchronisations).
`roofline` prices the sampled-gradient kernel: algorithmic bytes per launch
(1180 B per nonzero sample, 1160 B per zero sample: int64 coordinates and
value or one 8-byte probe, d gathered factor rows, d read-modify-written
gradient rows) over its mean duration from HIP events on the launch stream,
against the 8 TB/s HBM3E peak.  `cpu_baseline` times the FP64 CPU oracle on
the host over a bounded number of full steps of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_2605_20353_amd import _lib as G  # noqa: E402
from paper_2605_20353_amd import autotune, synth  # noqa: E402
from paper_2605_20353_amd.autograd import gcp_loss  # noqa: E402
from paper_2605_20353_amd.fedadam import FedAdam, FedConfig, FedTile, Plain  # noqa: E402

HBM_PEAK_GBS = 8000.0
DIMS = [10000, 8000, 6000]
NNZ = 50_000_000
RANK = 32
P = Q = 1 << 20
DATA_SEED = 2607
SAMPLE_SEED = 20353
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "loss_grad_cfg2_traffic.json")
KERNEL_SOURCES = ["paper_2605_20353_amd/csrc/loss_grad.hip", "paper_2605_20353_amd/csrc/lg_kernels.hpp",
                  "paper_2605_20353_amd/csrc/lg_core.hpp", "paper_2605_20353_amd/csrc/sampling.hpp",
                  "paper_2605_20353_amd/csrc/gcp_internal.hpp"]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(d: int, R: int, p: int, q: int, w: int = 4) -> int:
    per_nz = d * 8 + w + d * R * w + 2 * d * R * w
    per_z = 8 + d * R * w + 2 * d * R * w
    return p * per_nz + q * per_z


def traffic_record():
    """The committed rocprofv3 counter summary of the sampled-gradient call
    (DRAM bytes per launch and the tile it was taken at), if it was taken on
    the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec


CEILINGS_FILE = os.path.join(ROOT, "profiles", "ceilings.json")


def binding_ceiling(kernel_ms: float):
    """The sampled-gradient call's lower bound from the measured hardware
    ceilings (profiles/ceilings.json, written by --ceilings), if present."""
    try:
        with open(CEILINGS_FILE) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    lb = c.get("config2_call_lower_bound_ms")
    if not lb:
        return None
    return {"name": c.get("binding"), "lower_bound_ms": lb, "frac": round(lb / kernel_ms, 4),
            "source": "profiles/ceilings.json (bench.py --ceilings)"}


TILE_FIELDS = ("lanes", "vec", "block", "grid", "lds_modes", "bucket_modes", "bucket_lds_bytes",
               "bucket_block_samples", "bucket_splits", "bucket_block")


def parse_tile(spec: str) -> G.Tile:
    if spec == "default":
        return G.Tile()
    kw = {}
    for part in spec.split(","):
        k, _, v = part.partition("=")
        if k.strip() not in TILE_FIELDS:
            raise SystemExit(f"--tile: unknown field {k!r}; fields are {', '.join(TILE_FIELDS)}")
        kw[k.strip()] = int(v)
    return G.Tile(**kw)


def tile_dict(tile: G.Tile) -> dict:
    return {f: getattr(tile, f) for f in TILE_FIELDS}


def build_workload(dev):
    log(f"generating {DIMS} with {NNZ} nonzeros (rank-{RANK} gamma model) on {dev}")
    t0 = time.time()
    data = synth.count_tensor(DIMS, RANK, NNZ, seed=DATA_SEED, dist="gamma", device=dev)
    log(f"  generated in {time.time() - t0:.1f} s")
    t = G.SparseTensor(DIMS, data.coords, data.vals.to(torch.float32))
    t.reserve(P + Q, RANK)
    torch.cuda.synchronize()
    log(f"  tensor handle: {t.device_bytes() / 2**30:.2f} GiB of records, membership table and workspace")
    A = synth.init_model(DIMS, RANK, DATA_SEED + 100, dist="uniform", device=dev, dtype=torch.float32)
    return data, t, A


def run_gpu(t, A, steps: int, warmup: int, tile):
    Gr = torch.zeros_like(A)
    B = torch.zeros_like(A)
    Cm = torch.zeros_like(A)
    n_params = A.numel()

    def step(k):
        sp = G.SampleParams("stratified", P, Q, seed=SAMPLE_SEED, step=k)
        G.gcp_loss_grad(t, sp, A, RANK, "poisson", G=Gr, accumulate=True, want_loss=False, tile=tile)
        return sp

    for k in range(warmup):
        step(k)
        G.gcp_adam_step(A, Gr, B, Cm, k + 1, lr=1e-3, lower=0.0, zero_grad=True)
    torch.cuda.synchronize()
    t.status()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        step(warmup + k)
        ev[k][1].record()
        G.gcp_adam_step(A, Gr, B, Cm, warmup + k + 1, lr=1e-3, lower=0.0, zero_grad=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    t.status()
    kms = [a.elapsed_time(b) for a, b in ev]
    # objective estimate at the final model (outside the timed region)
    sp = G.SampleParams("stratified", P, Q, seed=SAMPLE_SEED, step=warmup + steps)
    _, L = G.gcp_loss_grad(t, sp, A, RANK, "poisson", loss_only=True)
    torch.cuda.synchronize()
    return (t1 - t0), kms, float(L.item()), n_params


def _time_ms(fn, reps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def _median_ms(fn, reps: int, warmup: int) -> float:
    """Median over reps of one call each, wall clock between device synchronisations."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - t0))
    return float(np.median(ts))


# GCP-FedAdam workloads: global dims, client block grid, nonzeros per client
# (log-uniform between the two), generator seed
FED_WORKLOADS = {
    "3way": ([20000, 20000, 2000], (4, 4, 4), 1e5, 5e6, 2610),
    "4way": ([4000, 4000, 400, 100], (2, 2, 2, 2), 1e5, 1e6, 2610),
}


def run_fedadam(dev, rounds: int, tune: bool = True, workload: str = "3way"):
    """GCP-FedAdam, by default 64 clients on a 4x4x4 block grid over
    20000x20000x2000, 1e5..5e6 nonzeros per client (log-uniform); "4way" is
    16 clients on a 2x2x2x2 grid over 4000x4000x400x100 with 1e5..1e6 (the
    general-order kernels).  Rank 32 FP32, tau = 10 local steps of
    2^16 + 2^16 samples, then the server step.  Median ms per round of four
    forms on the same state:
      plain_atomic  per-client launches (a gcp_loss_grad and a gcp_adam_step
                    per client and local step), hardware-atomic scatter;
      plain_auto    per-client launches, each call's automatic scatter
                    (row-bucketed at 2^17 samples, on reserved workspaces);
      persistent    one persistent launch for every client and local step
                    (group barriers, atomic and LDS-private scatter), graph
                    replay, the autotuner's best persistent shape;
      bucketed      three launches over all clients per local step (sample
                    and sort, row-block owners, Adam), graph replay, the
                    autotuner's best row-bucketed shape.
    The speedup is the best batched form against the best per-client form,
    so the choice of scatter is not counted as a gain of batching."""
    gd, grid, nnz_min, nnz_max, gseed = FED_WORKLOADS[workload]
    R = 32
    K = int(np.prod(grid))
    log(f"fedadam: generating {K} client blocks")
    blocks = synth.fed_blocks(gd, grid, R, nnz_min, nnz_max, seed=gseed, device=dev)
    nnz = sum(b.data.nnz for b in blocks)
    clients = [(G.SparseTensor(b.data.dims, b.data.coords, b.data.vals.to(torch.float32)), b.row_base)
               for b in blocks]
    del blocks
    U0 = synth.init_model(gd, R, 2710, device=dev, dtype=torch.float32)
    cfg = FedConfig(R=R, tau=10, loss="poisson", p=1 << 16, q=1 << 16, seed=SAMPLE_SEED, lr=1e-3, meta_lr=1e-3,
                    lower=0.0)
    out = {"workload": f"GCP-FedAdam, {K} clients ({'x'.join(map(str, grid))} grid over "
                       f"{'x'.join(map(str, gd))}), {nnz} nonzeros, rank 32 FP32, tau 10 x (2^16 + 2^16) samples "
                       "per client",
           "nnz": nnz, "forms": {}}

    def measure(name, fed):
        ms = _median_ms(lambda: fed.round(0), rounds, 1)
        fed.status()
        info = fed.info()
        out["forms"][name] = {"ms_per_round": ms, "launches_per_round": info["launches_per_round"],
                              "shape": {k: info[k] for k in ("form", "workgroups_per_client", "block", "lanes",
                                                             "vec", "lds_modes", "bucket_modes")}}
        log(f"fedadam: {name} {ms:.2f} ms per round ({info['form']}, {info['launches_per_round']} launches)")
        fed.close()

    measure("plain_atomic", Plain(clients, gd, U0, cfg, scatter="atomic"))
    measure("plain_auto", Plain(clients, gd, U0, cfg, scatter="auto"))
    for name, cands in (("persistent", "persistent"), ("bucketed", "bucketed")):
        fed = FedAdam(clients, gd, U0, cfg, batched=True, use_graph=True,
                      tile=FedTile(bucket_modes=0) if name == "persistent" else FedTile())
        if tune:
            pool = [c for c in autotune.fed_candidates(R, torch.float32, len(clients), nmodes=len(gd))
                    if (c.bucket_modes == 0) == (cands == "persistent")]
            autotune.tune_fedadam(fed, candidates=pool, rounds=1, warmup=1, use_cache=False)
        measure(name, fed)
    f = out["forms"]
    best_plain = min(("plain_atomic", "plain_auto"), key=lambda k: f[k]["ms_per_round"])
    best_batched = min(("persistent", "bucketed"), key=lambda k: f[k]["ms_per_round"])
    out["best_plain"], out["best_batched"] = best_plain, best_batched
    out["plain_ms_per_round"] = f[best_plain]["ms_per_round"]
    out["batched_ms_per_round"] = f[best_batched]["ms_per_round"]
    out["speedup"] = out["plain_ms_per_round"] / out["batched_ms_per_round"]
    out["speedup_same_scatter"] = {
        "atomic (persistent vs plain_atomic)": f["plain_atomic"]["ms_per_round"] / f["persistent"]["ms_per_round"],
        "row-bucketed (bucketed vs plain_auto)": f["plain_auto"]["ms_per_round"] / f["bucketed"]["ms_per_round"]}
    out["samples_per_round"] = K * 10 * (cfg.p + cfg.q)
    out["batched_samples_per_s"] = out["samples_per_round"] / (out["batched_ms_per_round"] * 1e-3)
    log(f"fedadam: best per-client {best_plain} {out['plain_ms_per_round']:.2f} ms, best batched {best_batched} "
        f"{out['batched_ms_per_round']:.2f} ms per round -> {out['speedup']:.2f}x")
    return out


def run_autograd(dev, which: str, reps: int):
    """Forward + backward of the sampled objective as a torch.autograd
    Function (backward recomputes the samples and model values)."""
    if which == "dense_gaussian":
        dims, R, loss, s = [200, 200, 200, 50], 16, "gaussian", 1 << 22
        X, _ = synth.dense_gaussian(dims, 16, seed=2608, device=dev, dtype=torch.float32)
        t = G.DenseTensor(dims, X)
        sp = G.SampleParams("uniform", s, 0, seed=SAMPLE_SEED, step=0)
        desc = "dense Gaussian 200x200x200x50 FP32, rank 16, 2^22 uniform samples"
    else:
        dims, R, loss, s = [5000, 5000, 500, 100], 64, "bernoulli_logit", 1 << 23
        data = synth.count_tensor(dims, 64, 100_000_000, seed=2609, device=dev, binary=True)
        t = G.SparseTensor(dims, data.coords, data.vals.to(torch.float32))
        t.reserve(s, R)
        del data
        sp = G.SampleParams("stratified", s // 2, s // 2, seed=SAMPLE_SEED, step=0)
        desc = "binary 5000x5000x500x100 with 1e8 ones, Bernoulli-logit, rank 64 FP32, 2^22 + 2^22 samples"
    A = (synth.init_model(dims, R, 2708, dist="normal", device=dev, dtype=torch.float32)
         * synth.normal_init_scale(R, len(dims))).requires_grad_(True)

    def fb():
        A.grad = None
        gcp_loss(A, t, R, loss, sp).backward()

    ms = _median_ms(fb, reps, 3)
    log(f"autograd {which}: {ms:.3f} ms per forward+backward (median of {reps})")
    return {"workload": desc, "ms_per_forward_backward": ms, "samples_per_s": s / (ms * 1e-3)}


def host_threads() -> int:
    """Threads the host share allows: OMP_NUM_THREADS when set, else the CPU
    count."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    return n if n > 0 else (os.cpu_count() or 1)


def run_cpu_baseline(data, A_init: np.ndarray, steps: int, par_steps: int):
    """The FP64 oracle timed on the host over full steps of the same workload:
    the serial checker (1 thread), then its timing-only OpenMP form with
    thread-private gradients (the paper's CPU MTTKRP strategy) on every
    thread the host share allows.  `value` is the all-threads figure."""
    import oracle
    log("cpu baseline: building the oracle's sorted index on the host")
    coords = data.coords.cpu().numpy()
    vals = data.vals.to(torch.float32).double().cpu().numpy()
    t_ora = oracle.SparseTensor(DIMS, coords, vals)
    ap = oracle.AdamParams(lr=1e-3, lower=0.0)

    def fresh():
        A = A_init.astype(np.float64).copy()
        return A, np.zeros_like(A), np.zeros_like(A)

    A, B, Cm = fresh()
    log(f"cpu baseline: timing {steps} full serial step(s) of {P + Q} samples")
    t0 = time.perf_counter()
    for k in range(steps):
        oracle.sgd_step(t_ora, RANK, A, B, Cm, k + 1, "poisson", P, Q, SAMPLE_SEED, k, ap)
    dt_serial = time.perf_counter() - t0
    serial = steps * (P + Q) / dt_serial
    threads = host_threads()
    ps = oracle.ParallelStepper(t_ora, RANK, P, Q, threads)
    A, B, Cm = fresh()
    ps.step(A, B, Cm, 1, "poisson", SAMPLE_SEED, 0, ap)          # first touch of the workspaces
    A, B, Cm = fresh()
    log(f"cpu baseline: timing {par_steps} full step(s) on {threads} threads")
    t0 = time.perf_counter()
    for k in range(par_steps):
        ps.step(A, B, Cm, k + 1, "poisson", SAMPLE_SEED, k, ap)
    dt_par = time.perf_counter() - t0
    par = par_steps * (P + Q) / dt_par
    return {"value": par, "unit": "samples/s", "cores": ps.threads_used, "kind": "oracle",
            "sample": f"{par_steps} full step(s) of the same workload ({P}+{Q} stratified samples, sampled "
                      f"gradient, Adam over all {A.size} parameters), FP64 C, OpenMP over samples with "
                      f"thread-private gradients on {ps.threads_used} threads, {dt_par:.1f} s; serially "
                      f"{steps} step(s) in {dt_serial:.1f} s",
            "serial": {"value": serial, "cores": 1, "steps": steps, "seconds": dt_serial},
            "parallel_speedup": par / serial}


def fused_experiment(dev, sizes, epochs: int = 2, iters: int = 100, obj_samples: int = 1_500_000):
    """Fused vs non-fused sampled gradient (Sec. 3.1.2) under the protocol of
    the paper's experiment (Sec. 5): a synthetic tensor shaped like its arXiv
    tensor (172 x 25000 x 300, 3e7 nonzeros, Poisson), semi-stratified
    sampling with as many zero as nonzero samples, swept; GCP-Adam for 2
    epochs of 100 iterations with a fixed objective set of 1.5M samples and
    the default Adam parameters.  fused = one gcp_loss_grad per iteration
    that draws the samples in the kernel and reads the factor rows once;
    non-fused = gcp_sample_y (draws, reads the rows for the model values,
    writes the sampled tensor) then gcp_mttkrp (reads the sampled tensor,
    reads the rows again), as the paper describes the unfused form.  Rank 32
    (the paper does not state the rank of this experiment).  Reported: wall
    time of the whole solve between device synchronisations, and of the
    gradient alone (sampling + MTTKRP, median of 20 after warm-up)."""
    from paper_2605_20353_amd.solver import SolverConfig, gcp_adam
    dims, R = [172, 25000, 300], 32
    log("fused experiment: generating 172x25000x300 with 3e7 nonzeros")
    data = synth.count_tensor(dims, R, 30_000_000, seed=2612, device=dev)
    t = G.SparseTensor(dims, data.coords, data.vals.to(torch.float32))
    del data
    t.reserve(2 * max(sizes), R)
    A0 = synth.init_model(dims, R, 2712, device=dev, dtype=torch.float32)
    rows = []
    for s in sizes:
        res = {"samples": 2 * s}
        for fused in (True, False):
            cfg = SolverConfig(R=R, loss="poisson", sampling="semi_stratified", p=s, q=s, obj_p=obj_samples // 2,
                               obj_q=obj_samples // 2, iters_per_epoch=iters, max_epochs=epochs, lr=1e-3,
                               lower=0.0, fused=fused)
            gcp_adam(t, A0, cfg)                       # warm-up (kernels loaded, buffers sized)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = gcp_adam(t, A0, cfg)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            sp = G.SampleParams("semi_stratified", s, s, seed=SAMPLE_SEED, step=0)
            Gr = torch.zeros_like(A0)
            if fused:
                grad = lambda: G.gcp_loss_grad(t, sp, A0, R, "poisson", G=Gr, want_loss=False)
            else:
                cb = torch.empty(2 * s, 3, dtype=torch.int64, device=dev)
                yb = torch.empty(2 * s, dtype=torch.float32, device=dev)

                def grad():
                    G.gcp_sample_y(t, sp, A0, R, "poisson", coords=cb, y=yb)
                    G.gcp_mttkrp(t, cb, yb, A0, R, G=Gr)
            key = "fused" if fused else "nonfused"
            res[f"{key}_solve_s"] = wall
            res[f"{key}_ms_per_iter"] = 1e3 * wall / (epochs * iters)
            res[f"{key}_grad_ms"] = _median_ms(grad, 20, 3)
            res[f"{key}_objective"] = out.objective[-1]
            res[f"{key}_accepted_epochs"] = sum(out.accepted)
        res["solve_ratio"] = res["nonfused_solve_s"] / res["fused_solve_s"]
        res["grad_ratio"] = res["nonfused_grad_ms"] / res["fused_grad_ms"]
        rows.append(res)
        log(f"fused experiment: {2 * s} samples: solve fused {res['fused_solve_s']:.3f} s, non-fused "
            f"{res['nonfused_solve_s']:.3f} s ({res['solve_ratio']:.2f}x); gradient {res['fused_grad_ms']:.3f} vs "
            f"{res['nonfused_grad_ms']:.3f} ms ({res['grad_ratio']:.2f}x)")
    t.status()
    return {"workload": "172x25000x300 Poisson, 3e7 nonzeros, rank 32 FP32, semi-stratified p = q, "
                        f"{epochs} epochs x {iters} iterations, {obj_samples} objective samples",
            "rows": rows}


def hbm_resident(dev, nnz: int, steps: int, warmup: int):
    """The HBM-resident-factor regime: a synthetic count tensor shaped like the
    Amazon reviews tensor (4821207 x 1774269 x 1805187; its cells need 65 key
    bits, so the mixed-radix cell key), rank 32 FP32, so the factor, gradient
    and moment arrays are 1.07 GB each -- far beyond the L2 and Infinity Cache
    -- and every factor-row gather and gradient update goes to HBM.  Same step
    as the headline benchmark: 2^20 + 2^20 stratified samples, sampled
    gradient with the library's automatic launch shape, Adam."""
    dims, R = [4821207, 1774269, 1805187], 32
    log(f"hbm-resident: generating {dims} with {nnz} nonzeros (rank-{R} gamma model)")
    t0 = time.time()
    data = synth.count_tensor(dims, R, nnz, seed=2614, dist="gamma", device=dev)
    gen_s = time.time() - t0
    torch.cuda.empty_cache()            # the generator's temporaries, before the handle's own allocations
    t = G.SparseTensor(dims, data.coords, data.vals.to(torch.float32))
    del data
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    log(f"  generated in {gen_s:.1f} s; tensor handle {t.device_bytes() / 2**30:.1f} GiB")
    A = synth.init_model(dims, R, 2714, dist="uniform", device=dev, dtype=torch.float32)
    Gr, B, Cm = torch.zeros_like(A), torch.zeros_like(A), torch.zeros_like(A)
    tile = G.Tile()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for k in range(warmup + steps):
        sp = G.SampleParams("stratified", P, Q, seed=SAMPLE_SEED, step=k)
        if k >= warmup:
            ev[k - warmup][0].record()
        G.gcp_loss_grad(t, sp, A, R, "poisson", G=Gr, accumulate=True, want_loss=False, tile=tile)
        if k >= warmup:
            ev[k - warmup][1].record()
        G.gcp_adam_step(A, Gr, B, Cm, k + 1, lr=1e-3, lower=0.0, zero_grad=True)
        if k == warmup - 1:
            torch.cuda.synchronize()
            t_start = time.perf_counter()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    t.status()
    kms = [a.elapsed_time(b) for a, b in ev]
    kmed = float(np.median(kms))
    # the same samples through the row-sorted form (GCP_DETERMINISTIC): the
    # sampled tensor written, its (row, sample) pairs sorted by row, each
    # touched gradient row summed by one wavefront and written with a plain
    # load-add-store -- against one float-atomic request per (sample, mode)
    t.reserve(P + Q, R)
    sms = []
    for k in range(5):
        sp = G.SampleParams("stratified", P, Q, seed=SAMPLE_SEED, step=k)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        G.gcp_loss_grad(t, sp, A, R, "poisson", G=Gr, accumulate=True, want_loss=False, deterministic=True)
        b.record()
        torch.cuda.synchronize()
        if k:
            sms.append(a.elapsed_time(b))
    t.status()
    alg = algorithmic_bytes(3, R, P, Q)
    return {"workload": f"Amazon-shaped count tensor {dims[0]}x{dims[1]}x{dims[2]}, {nnz} nonzeros, rank {R} "
                        f"FP32, {P}+{Q} stratified samples per step (mixed-radix cell keys)",
            "factor_bytes": A.numel() * 4, "tensor_handle_bytes": t.device_bytes(), "generation_s": gen_s,
            "steps": steps, "samples_per_s": steps * (P + Q) / wall, "ms_per_step": 1e3 * wall / steps,
            "loss_grad_ms_median": kmed, "sorted_rows_plain_stores_ms_median": float(np.median(sms)),
            "algorithmic_bytes_per_launch": alg,
            "algorithmic_gbs": alg / (kmed * 1e-3) / 1e9,
            "frac": alg / (kmed * 1e-3) / 1e9 / HBM_PEAK_GBS}


def _counter_rows(d: str):
    """Rows of the rocprofv3 --pmc CSV output under directory d."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def _median_counter(rows, counter: str, kernel_sub: str) -> float:
    vals = [float(r["Counter_Value"]) for r in rows
            if r.get("Counter_Name") == counter and kernel_sub in r.get("Kernel_Name", "")]
    if not vals:
        raise SystemExit(f"no {counter} rows for kernels matching {kernel_sub!r}")
    return float(np.median(vals)), len(vals)


def traffic_summary(dirs, tile: G.Tile) -> dict:
    """DRAM bytes per sampled-gradient call from four rocprofv3 --pmc runs,
    each counter scaled by what it reads for a copy kernel of known size;
    written to profiles/loss_grad_cfg2_traffic.json."""
    if not tile.lanes or not tile.vec:
        raise SystemExit("--traffic-summary needs the profiled tile (--tile with lanes and vec)")
    fetch, write, cfetch, cwrite = (_counter_rows(d) for d in dirs)
    out = {"kernel_source_hash": kernel_source_hash(), "tile": tile_dict(tile)}
    cf, _ = _median_counter(cfetch, "FETCH_SIZE", "k_ceil_copy")
    cw, _ = _median_counter(cwrite, "WRITE_SIZE", "k_ceil_copy")
    copy_bytes = 1 << 30
    ff, fw = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    out["copy_calibration"] = {"kernel": "k_ceil_copy", "bytes": copy_bytes, "fetch_size_kib": cf,
                               "write_size_kib": cw, "fetch_factor": ff, "write_factor": fw}
    per = {}
    total_r = total_w = 0.0
    # the exact instantiations of the benchmark's call (SRC = 0: samples drawn
    # in the kernel; the tile's lane shape)
    shape = f"3, {tile.lanes}, {tile.vec}"
    for name, match in (("k_loss_grad", f"k_loss_grad<float, {shape}, 0>"),
                        ("k_bucket_accum", f"k_bucket_accum<float, {shape}>"), ("k_adam", "k_adam<float>")):
        try:
            kf, nd = _median_counter(fetch, "FETCH_SIZE", match)
            kw, _ = _median_counter(write, "WRITE_SIZE", match)
        except SystemExit:
            continue
        per[name] = {"kernel": match, "fetch_size_kib": kf, "write_size_kib": kw, "read_bytes": kf * 1024 * ff,
                     "write_bytes": kw * 1024 * fw, "dispatches": nd}
        if name != "k_adam":
            total_r += kf * 1024 * ff
            total_w += kw * 1024 * fw
    out["per_kernel"] = per
    out["read_bytes_per_launch"] = int(total_r)
    out["write_bytes_per_launch"] = int(total_w)
    out["bytes_per_launch"] = int(total_r + total_w)
    out["what"] = ("DRAM bytes per gcp_loss_grad call of the benchmark step (k_loss_grad + k_bucket_accum), median "
                   "over dispatches, calibrated against a 1 GiB copy kernel")
    ts = ",".join(f"{k}={v}" for k, v in tile_dict(tile).items())
    out["commands"] = [
        f"rocprofv3 --pmc FETCH_SIZE --kernel-include-regex 'k_loss_grad|k_bucket_accum|k_adam' --output-format csv "
        f"-d {dirs[0]} -o cfg2 -- python3 bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-extras --tile {ts}",
        f"rocprofv3 --pmc WRITE_SIZE --kernel-include-regex 'k_loss_grad|k_bucket_accum|k_adam' --output-format csv "
        f"-d {dirs[1]} -o cfg2 -- python3 bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-extras --tile {ts}",
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {dirs[2]} -o copy -- python3 bench.py --copy-calibration",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {dirs[3]} -o copy -- python3 bench.py --copy-calibration",
        "python3 bench.py --traffic-summary " + " ".join(dirs) + f" --tile {ts}"]
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    return out


ENGINE_CLOCK_HZ = 2.4e9      # MI355X peak engine clock
CUS = 256


def ceilings(dev, reps: int = 10):
    """Measure the hardware ceilings of the sampled gradient's access patterns
    (include/gcp_ceilings.h) on this device, and from them a lower bound on
    the config-2 sampled-gradient call (2^20 + 2^20 samples, rank 32, three
    modes, row-bucketed scatter) under this model:
      sampling kernel: per sample one random record read (or probe) and three
        dependent row gathers, at the dependent-gather rate, overlapped with
        writing its 3 x 16-byte sort entries at the copy rate;
      owner pass: per entry (3 per sample) two row gathers from a streamed
        entry, at the streamed-gather rate, and R float adds into the LDS row
        block by compare-and-swap pairs, at the rate measured for the owner's
        pattern (8 lanes x 4 columns into rows drawn at random), overlapped
        with reading the entries back at the copy rate;
      the two kernels run one after the other.
    The bound is the sum over the two kernels of the slowest part of each."""
    import ctypes as C
    L = G.lib()
    st = G._stream()
    sink = torch.zeros(1 << 16, dtype=torch.int32, device=dev)

    def timed(call):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        G._check(call(), "ceiling")
        torch.cuda.synchronize()
        for a, b in ev:
            a.record()
            G._check(call(), "ceiling")
            b.record()
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    out = {"device": torch.cuda.get_device_name(0), "engine_clock_hz": ENGINE_CLOCK_HZ, "cus": CUS}
    nrec = NNZ
    rec = torch.randint(-2**31, 2**31 - 1, (nrec * 4,), dtype=torch.int32, device=dev)
    nreads = 1 << 24
    for inflight in (1, 4):
        ms = timed(lambda: L.gcp_ceiling_random_reads(C.c_void_p(rec.data_ptr()), nrec, nreads, inflight, 512,
                                                      C.c_void_p(sink.data_ptr()), st))
        out[f"random_16B_reads_{inflight}_in_flight"] = {"per_s": nreads / (ms * 1e-3), "ms": ms, "n": nreads}
    A = torch.rand(sum(DIMS) * RANK, dtype=torch.float32, device=dev)
    dims3 = (C.c_int64 * 3)(*DIMS)
    n = P + Q
    for seq, name in ((0, "dependent_record_3_row_gathers"), (1, "streamed_record_3_row_gathers")):
        best = None
        for block in (512, 1024):
            ms = timed(lambda: L.gcp_ceiling_dependent_gathers(C.c_void_p(rec.data_ptr()), nrec,
                                                               C.c_void_p(A.data_ptr()), dims3, n, seq, block,
                                                               C.c_void_p(sink.data_ptr()), st))
            if best is None or ms < best[0]:
                best = (ms, block)
        out[name] = {"samples_per_s": n / (best[0] * 1e-3), "rows_per_s": 3 * n / (best[0] * 1e-3),
                     "ms": best[0], "block": best[1], "n": n}
    iters, block = 4096, 1024
    grid = CUS * 2
    ms = timed(lambda: L.gcp_ceiling_lds_cas(iters, block, grid, C.c_void_p(sink.data_ptr()), st))
    lane_ops = grid * block * iters
    out["lds_cas64"] = {"lane_ops_per_s": lane_ops / (ms * 1e-3),
                        "wave_instr_per_clk_per_cu": lane_ops / 64 / (ms * 1e-3) / (CUS * ENGINE_CLOCK_HZ),
                        "ms": ms}
    iters_r = 2048
    for form, name in ((0, "cas64_pairs"), (1, "native_ds_add_f32"), (2, "native_ds_add_f64")):
        ms = timed(lambda: L.gcp_ceiling_lds_row_adds(form, iters_r, grid, C.c_void_p(sink.data_ptr()), st))
        out.setdefault("lds_row_adds", {})[name] = {"adds_per_s": grid * 1024 * iters_r * 4 / (ms * 1e-3),
                                                    "ms": ms}
    Gr = torch.zeros(sum(DIMS) * RANK, dtype=torch.float32, device=dev)
    nup = 1 << 22
    ms = timed(lambda: L.gcp_ceiling_global_atomics(C.c_void_p(Gr.data_ptr()), sum(DIMS), nup, 512, st))
    out["global_float_atomic_rows"] = {"requests_per_s": nup / (ms * 1e-3), "ms": ms, "n": nup}
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms = timed(lambda: L.gcp_ceiling_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, st))
    out["copy"] = {"gbs_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9, "ms": ms, "bytes": nbytes}
    del rec, src, dst

    # lower bound of the config-2 call
    d, ent_bytes = 3, 16
    copy_bps = out["copy"]["gbs_read_plus_write"] * 1e9
    t_draw = n / out["dependent_record_3_row_gathers"]["samples_per_s"]
    t_write = n * d * ent_bytes / copy_bps
    t_owner_gather = n * d * 2 / out["streamed_record_3_row_gathers"]["rows_per_s"]
    t_owner_cas = n * d * RANK / out["lds_row_adds"]["cas64_pairs"]["adds_per_s"]
    t_read = n * d * ent_bytes / copy_bps
    parts_a = {"dependent record and row gathers": t_draw, "sort-entry writes": t_write}
    parts_b = {"streamed-entry row gathers": t_owner_gather, "LDS compare-and-swap adds": t_owner_cas,
               "sort-entry reads": t_read}
    ka, kb = max(parts_a, key=parts_a.get), max(parts_b, key=parts_b.get)
    out["config2_model_ms"] = {"sampling_kernel": {k: v * 1e3 for k, v in parts_a.items()},
                               "owner_pass": {k: v * 1e3 for k, v in parts_b.items()}}
    out["config2_call_lower_bound_ms"] = (parts_a[ka] + parts_b[kb]) * 1e3
    out["binding"] = f"sampling kernel: {ka}; owner pass: {kb}"
    out["commands"] = ["python3 bench.py --ceilings"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--cpu-par-steps", type=int, default=20)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the GCP-FedAdam round and autograd measurements")
    ap.add_argument("--fed-rounds", type=int, default=5)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy five times, so that "
                         "rocprofv3's FETCH_SIZE / WRITE_SIZE can be calibrated against known bytes")
    ap.add_argument("--fused-experiment", action="store_true",
                    help="only run the fused vs non-fused sampled-gradient comparison and print its JSON")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the sampled-gradient tile instead of taking the one the committed "
                         "counter profile was taken at")
    ap.add_argument("--tile", default="",
                    help="fixed sampled-gradient tile instead of the autotuned one, as comma-separated "
                         "key=value pairs of gcp_tile fields (e.g. lanes=8,vec=4,block=256,bucket_block=1024); "
                         "'default' = the library's automatic choice")
    ap.add_argument("--hbm-resident", action="store_true",
                    help="only run the HBM-resident-factor experiment (Amazon-shaped tensor) and print its JSON")
    ap.add_argument("--hbm-nnz", type=int, default=1_700_000_000)
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write profiles/loss_grad_cfg2_traffic.json from four rocprofv3 --pmc runs (FETCH_SIZE and "
                         "WRITE_SIZE of the benchmark at --tile, then of --copy-calibration) and print it")
    ap.add_argument("--ceilings", action="store_true",
                    help="only measure the hardware ceilings of the sampled gradient's access patterns and the "
                         "lower bound they put on the benchmark call; print their JSON")
    ap.add_argument("--fedadam-only", action="store_true",
                    help="only run the GCP-FedAdam comparison (per-client vs batched round, the library's "
                         "automatic launch shape, no autotuning) and print its JSON")
    ap.add_argument("--fed-workload", choices=sorted(FED_WORKLOADS), default="3way",
                    help="GCP-FedAdam workload of --fedadam-only: 3way (64 clients over 20000x20000x2000) or 4way "
                         "(16 clients over 4000x4000x400x100, the general-order kernels)")
    args = ap.parse_args()
    if args.ceilings:
        print(json.dumps(ceilings(torch.device("cuda:0"))))
        return
    if args.fedadam_only:
        print(json.dumps(run_fedadam(torch.device("cuda:0"), args.fed_rounds, tune=False,
                                     workload=args.fed_workload)))
        return
    if args.hbm_resident:
        out = hbm_resident(torch.device("cuda:0"), args.hbm_nnz, max(1, min(args.steps, 50)), args.warmup)
        print(json.dumps(out))
        return
    if args.fused_experiment:
        out = fused_experiment(torch.device("cuda:0"), [1 << k for k in (14, 16, 18, 20, 22)])
        print(json.dumps(out))
        return
    if args.copy_calibration:
        import ctypes as C
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            G._check(G.lib().gcp_ceiling_copy(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), x.numel() * 4,
                                              G._stream()), "gcp_ceiling_copy")
        torch.cuda.synchronize()
        print(json.dumps({"copy_kernel": "k_ceil_copy", "copy_bytes_read_per_launch": x.numel() * 4,
                          "copy_bytes_written_per_launch": x.numel() * 4}))
        return
    if args.traffic_summary:
        print(json.dumps(traffic_summary(args.traffic_summary, parse_tile(args.tile) if args.tile else G.Tile()),
                         indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path; "
              "run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    data, t, A = build_workload(dev)
    A0 = A.cpu().numpy().copy()
    sp0 = G.SampleParams("stratified", P, Q, seed=SAMPLE_SEED, step=0)
    rec = traffic_record()
    if args.tile:
        tile, tile_source = parse_tile(args.tile), "fixed"
    elif args.autotune or not rec or "tile" not in rec:
        tile, tile_source = autotune.tune_loss_grad(t, sp0, A, RANK, "poisson", reps=10), "autotuned"
    else:
        # the tile the committed counter profile was taken at (itself the
        # autotuner's pick when it was profiled), so time and bytes pair up
        tile, tile_source = G.Tile(**rec["tile"]), "profiled"
    log(f"{tile_source} sampled-gradient tile: {tile}")
    log(f"timing {args.steps} steps after {args.warmup} warm-up steps")
    wall, kms, loss_est, n_params = run_gpu(t, A, args.steps, args.warmup, tile)
    ms_per_step = 1e3 * wall / args.steps
    value = args.steps * (P + Q) / wall
    kmean = float(np.mean(kms))
    alg = algorithmic_bytes(3, RANK, P, Q)
    alg_gbs = alg / (kmean * 1e-3) / 1e9
    # DRAM bytes per launch, only when the counters were taken on this kernel
    # source at this very tile
    traffic = rec.get("bytes_per_launch") if rec and rec.get("tile") == tile_dict(tile) else None
    dram_gbs = traffic / (kmean * 1e-3) / 1e9 if traffic else None
    roof = {"bound": "hbm",
            "achieved": round(dram_gbs, 1) if dram_gbs else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(dram_gbs / HBM_PEAK_GBS, 4) if dram_gbs else None,
            "traffic": traffic,
            "achieved_from": "DRAM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated against a "
                             "1 GiB copy; profiles/loss_grad_cfg2_traffic.json, same kernel source and tile) "
                             "over the mean launch duration measured here with HIP events on the launch stream",
            "kernel": "gcp_loss_grad: k_loss_grad (sampling, model values, loss derivative, scatter or "
                      "row-block sort) + k_bucket_accum (row-block owner pass) when bucketed",
            "kernel_ms_mean": round(kmean, 5), "kernel_ms_median": round(float(np.median(kms)), 5),
            "algorithmic": {
                "bytes_per_launch": alg, "rate_gbs": round(alg_gbs, 1),
                "model": "1180 B per nonzero sample (int64 coordinates and value, 3 factor rows gathered, "
                         "3 gradient rows read and written) and 1160 B per zero sample (one 8-byte probe "
                         "instead), every access charged as if there were no cache; the 3 MB factor and "
                         "gradient arrays live in the L2 and Infinity Cache here, so this rate is not an "
                         "HBM figure and may exceed the HBM peak"}}
    ceil = binding_ceiling(kmean)
    if ceil:
        roof["binding_ceiling"] = ceil
    log(f"step {ms_per_step:.4f} ms, {value:.4g} samples/s; loss_grad kernel {kmean:.4f} ms; "
        f"DRAM {dram_gbs or float('nan'):.0f} GB/s; algorithmic model {alg_gbs:.0f} GB/s")
    roof["tile"] = tile_dict(tile)
    roof["tile_source"] = tile_source
    extras = {}
    if not args.no_extras:
        # the bit-reproducible form of the same call (GCP_DETERMINISTIC)
        Gd = torch.zeros_like(A)
        extras["deterministic_call_ms"] = _median_ms(
            lambda: G.gcp_loss_grad(t, sp0, A, RANK, "poisson", G=Gd, want_loss=False, deterministic=True), 10, 2)
        log(f"deterministic call {extras['deterministic_call_ms']:.3f} ms")
        # semi-stratified sampling (zero samples kept without a membership
        # search) against stratified, same tile and timing method
        sps = G.SampleParams("semi_stratified", P, Q, seed=SAMPLE_SEED, step=0)
        for name, spx in (("stratified", sp0), ("semi_stratified", sps)):
            extras[f"{name}_call_ms"] = _median_ms(
                lambda: G.gcp_loss_grad(t, spx, A, RANK, "poisson", G=Gd, want_loss=False, tile=tile), 20, 3)
        log(f"stratified call {extras['stratified_call_ms']:.3f} ms, semi-stratified "
            f"{extras['semi_stratified_call_ms']:.3f} ms (host-synchronised timing)")
        del Gd
    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_baseline(data, A0, args.cpu_steps, args.cpu_par_steps)
        log(f"cpu baseline {cpu['value']:.4g} samples/s")
    del data, t
    torch.cuda.empty_cache()
    if not args.no_extras:
        extras["fedadam"] = run_fedadam(dev, args.fed_rounds)
        torch.cuda.empty_cache()
        extras["autograd_dense_gaussian"] = run_autograd(dev, "dense_gaussian", 20)
        torch.cuda.empty_cache()
        extras["autograd_binary_bernoulli"] = run_autograd(dev, "binary_bernoulli", 20)
    out = {
        "metric": "sampled gradient entries/sec + HBM GB/s fraction; batched vs plain speedup",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded rank-32 gamma CP event sampler, generated on the GPU)",
        "config": {"workload": "GCP-SGD/Adam step, 3-way Poisson count tensor 10000x8000x6000, "
                               "5e7 nonzeros, rank 32 FP32, 2^20 nonzero + 2^20 zero stratified "
                               "samples per step", "dims": DIMS, "nnz": NNZ, "rank": RANK,
                   "p": P, "q": Q, "loss": "poisson", "parallelism": "single GPU"},
        "loss_estimate": loss_est,
        "params": n_params,
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched_vs_plain_speedup": extras.get("fedadam", {}).get("speedup"),
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
