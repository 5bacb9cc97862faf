"""Autotuner for the launch shapes of the sampled-gradient kernel and the
batched GCP-FedAdam round.

Each candidate is timed with HIP events on the real workload (warm-up launches
first); the fastest is kept and cached per shape signature in a JSON file
(``$GCP_AUTOTUNE_CACHE`` or ``~/.cache/gcp_mi355x/autotune.json``).  Tuning a
FedAdam round snapshots the model state first and restores it after every
candidate, so tuning leaves the state as it found it.
"""
from __future__ import annotations

import json
import os
from dataclasses import asdict

import torch

from . import _lib as G
from .fedadam import FedAdam, FedTile


def cache_path() -> str:
    p = os.environ.get("GCP_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "gcp_mi355x", "autotune.json")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _time(fn, stream, reps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


# ------------------------------------------------------------ FedAdam round --

def fed_candidates(R: int, dtype, nclients: int, cus: int = 256, nmodes: int = 3):
    """Launch shapes worth trying for a batched round: the persistent launch
    with the atomic scatter over lane shapes, workgroup sizes and workgroups
    per client (0 = the library's automatic count), then the row-bucketed
    rounds (three launches per local step) over lane shapes (0 = its default)
    and workgroup sizes."""
    shapes = [(32, 1), (16, 2)] if R == 32 else [(0, 0)]
    if dtype == torch.float32 and R == 32:
        shapes.append((8, 4))
    out = []
    for block in (256, 512):
        max_w = max(1, (cus * (2048 // block)) // (2 * nclients))
        for w in sorted({0, 1, 2, 4, 8, 16, max_w}):
            if w > max_w:
                continue
            for lanes, vec in shapes:
                out.append(FedTile(workgroups_per_client=w, block=block, lanes=lanes, vec=vec, bucket_modes=0))
    all_modes = (1 << nmodes) - 1
    for block in (512, 1024):
        for lanes, vec in shapes + [(0, 0)]:
            out.append(FedTile(workgroups_per_client=0, block=block, lanes=lanes, vec=vec, bucket_modes=all_modes))
    return out


def fed_signature(fed: FedAdam) -> str:
    cfg = fed.cfg
    dims = ",".join(str(n) for n in fed.global_dims)
    return (f"fed|{torch.cuda.get_device_name(0)}|{fed.dtype}|K{len(fed.clients)}|R{cfg.R}|tau{cfg.tau}|"
            f"p{cfg.p}|q{cfg.q}|{dims}")


def tune_fedadam(fed: FedAdam, candidates=None, rounds: int = 1, warmup: int = 1, use_cache: bool = True,
                 log=None) -> FedTile:
    """Pick the fastest batched launch shape for this FedAdam workload and
    leave `fed` retiled with it (state unchanged)."""
    path = cache_path()
    key = fed_signature(fed)
    cache = _load(path) if use_cache else {}
    if key in cache:
        tile = FedTile(**cache[key]["tile"])
        fed.retile(tile)
        return tile
    cands = candidates or fed_candidates(fed.cfg.R, fed.dtype, len(fed.clients), nmodes=len(fed.global_dims))
    snap = fed.snapshot()
    results = []
    for tile in cands:
        try:
            fed.retile(tile)
            ms = _time(lambda: fed.round(0), fed.stream, rounds, warmup)
            fed.status()
        except G.GCPError as e:
            if log:
                log(f"autotune: skip {tile}: {e}")
            fed.restore(snap)
            continue
        fed.restore(snap)
        results.append((ms, tile))
        if log:
            log(f"autotune: {tile} -> {ms:.3f} ms/round")
    if not results:
        raise RuntimeError("no batched launch shape worked")
    ms, best = min(results, key=lambda r: r[0])
    fed.retile(best)
    if use_cache:
        cache[key] = {"tile": asdict(best), "ms": ms}
        _store(path, cache)
    return best


# ------------------------------------------------------- sampled gradient --

def loss_grad_candidates(R: int, dtype, reserved: bool):
    """The library's automatic choice, then the atomic scatter with one
    column per lane, then (with a reserved workspace) the row-bucketed
    scatter over a few lane shapes, workgroup sizes, samples per sorting
    workgroup, owner-pass workgroup sizes and splits."""
    out = [G.Tile()]
    out.append(G.Tile(lds_modes=0, bucket_modes=0))
    if reserved:
        wide = 4 if dtype == torch.float32 else 2
        shapes = []
        for vec in (wide, 2):
            if R % vec == 0 and (vec, R // vec) not in [(v, R // v) for v, _ in shapes]:
                lanes = 2
                while lanes * vec < R:
                    lanes *= 2
                if lanes <= 64:
                    shapes.append((vec, lanes))
        for vec, lanes in shapes:
            for block in (256, 512):
                for bblock, splits in ((1024, 0), (1024, 16), (1024, 32), (512, 0), (512, 32)):
                    out.append(G.Tile(lanes=lanes, vec=vec, block=block, lds_modes=-1, bucket_modes=-1,
                                      bucket_splits=splits, bucket_block=bblock))
            # larger sorting workgroups: fewer, longer segments per row block
            for block in (512, 1024):
                for splits in (0, 16):
                    out.append(G.Tile(lanes=lanes, vec=vec, block=block, lds_modes=-1, bucket_modes=-1,
                                      bucket_block_samples=4096, bucket_splits=splits, bucket_block=1024))
    return out


def tune_loss_grad(tensor, sp, A, R: int, loss: str, candidates=None, reps: int = 10, log=None) -> G.Tile:
    """Fastest gcp_loss_grad tile for this (tensor, samples, rank)."""
    Gr = torch.zeros_like(A)
    stream = torch.cuda.current_stream()
    cands = candidates or loss_grad_candidates(R, A.dtype, getattr(tensor, "reserved_samples", 0) >= sp.n)
    results = []
    for tile in cands:
        try:
            ms = _time(lambda: G.gcp_loss_grad(tensor, sp, A, R, loss, G=Gr, accumulate=True, want_loss=False,
                                               tile=tile), stream, reps, 2)
        except G.GCPError as e:
            if log:
                log(f"autotune: skip {tile}: {e}")
            continue
        results.append((ms, tile))
        if log:
            log(f"autotune: {tile} -> {ms:.4f} ms")
    return min(results, key=lambda r: r[0])[1]
