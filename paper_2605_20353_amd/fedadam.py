"""GCP-FedAdam (Alg. gcp-fed-iter) driver over the C ABI.

The clients' blocks, models, moments and gradient buffers and the server
model and moments are torch tensors owned here; the rounds run in the HIP
library.  Batched rounds (``batched=True``) share their launches among all
clients: either one persistent launch for every client and local step
(hardware-atomic or LDS-private scatter), or, with the row-bucketed scatter,
three launches over all clients per local step (sample and sort, row-block
owners, Adam); then one server kernel.  The round's launches are captured
once into a HIP graph and replayed.  Per-client rounds (``batched=False``,
the baseline) issue one sampled-gradient launch (two when it row-buckets)
and one Adam launch per client and local step.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import torch

from . import _lib as G


class gcp_fed_client(C.Structure):
    _fields_ = [("tensor", C.c_void_p), ("row_base", C.c_int64 * 8), ("M", C.c_void_p), ("B", C.c_void_p),
                ("C", C.c_void_p), ("G", C.c_void_p)]


class gcp_fed_desc(C.Structure):
    _fields_ = [("nclients", C.c_int32), ("R", C.c_int32), ("tau", C.c_int32), ("loss", C.c_int32),
                ("batched", C.c_int32), ("use_graph", C.c_int32), ("workgroups_per_client", C.c_int32),
                ("block", C.c_int32), ("lanes", C.c_int32), ("vec", C.c_int32), ("max_attempts", C.c_int32),
                ("lds_modes", C.c_int32), ("bucket_modes", C.c_int32), ("bucket_block_samples", C.c_int32),
                ("p", C.c_int64), ("q", C.c_int64), ("seed", C.c_uint64),
                ("global_dims", C.c_int64 * 8), ("U", C.c_void_p), ("Bs", C.c_void_p), ("Cs", C.c_void_p),
                ("lr", C.c_double), ("meta_lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("lower", C.c_double), ("clients", C.POINTER(gcp_fed_client)),
                ("barrier_timeout_s", C.c_double)]


class gcp_fed_info(C.Structure):
    _fields_ = [("form", C.c_int32), ("lds_modes", C.c_int32), ("bucket_modes", C.c_int32),
                ("workgroups_per_client", C.c_int32), ("block", C.c_int32), ("lanes", C.c_int32),
                ("vec", C.c_int32), ("bucket_block_samples", C.c_int32), ("launches_per_round", C.c_int64)]


FORMS = {0: "per_client", 1: "persistent", 2: "row_bucketed"}


def _declare():
    L = G.lib()
    if getattr(L, "_fed_declared", False):
        return L
    L.gcp_fedadam_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(gcp_fed_desc), C.c_void_p]
    L.gcp_fedadam_create.restype = C.c_int
    L.gcp_fedadam_round.argtypes = [C.c_void_p, C.c_int64, C.c_void_p]
    L.gcp_fedadam_round.restype = C.c_int
    L.gcp_fedadam_status.argtypes = [C.c_void_p, C.c_void_p]
    L.gcp_fedadam_status.restype = C.c_int
    L.gcp_fedadam_destroy.argtypes = [C.c_void_p]
    L.gcp_fedadam_destroy.restype = C.c_int
    L.gcp_fedadam_info.argtypes = [C.c_void_p, C.POINTER(gcp_fed_info)]
    L.gcp_fedadam_info.restype = C.c_int
    L._fed_declared = True
    return L


@dataclass
class FedConfig:
    R: int
    tau: int = 10
    loss: str = "poisson"
    p: int = 1 << 16
    q: int = 1 << 16
    seed: int = 20353
    lr: float = 1e-3
    meta_lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    lower: float = 0.0
    max_attempts: int = 64
    barrier_timeout_s: float = 0.0      # persistent launch's group-barrier wait bound; 0 = library default


@dataclass
class FedTile:
    """Launch shape of the batched round (0 = library default).  For
    per-client rounds only bucket_modes is used: it is passed to every
    gcp_loss_grad call (-1 = that call's automatic choice)."""
    workgroups_per_client: int = 0
    block: int = 0
    lanes: int = 0
    vec: int = 0
    lds_modes: int = -1
    bucket_modes: int = -1         # bitmask of row-bucketed modes; -1 automatic, 0 hardware atomics
    bucket_block_samples: int = 0

    def key(self):
        return (self.workgroups_per_client, self.block, self.lanes, self.vec, self.lds_modes, self.bucket_modes,
                self.bucket_block_samples)


@dataclass
class FedClient:
    tensor: G.SparseTensor
    row_base: list
    M: torch.Tensor = None
    B: torch.Tensor = None
    C: torch.Tensor = None
    G: torch.Tensor = None
    extra: dict = field(default_factory=dict)


class FedAdam:
    """GCP-FedAdam state and rounds.

    clients: list of (SparseTensor in block-local coordinates, row_base per mode).
    U0: initial server model [sum_k I_k, R] (copied).
    Per-client rounds with tile.bucket_modes != 0 reserve each client
    tensor's row-bucketing workspace (gcp_tensor_reserve) so that every
    gcp_loss_grad call may choose that scatter."""

    def __init__(self, clients, global_dims, U0: torch.Tensor, cfg: FedConfig, batched: bool = True,
                 use_graph: bool = True, tile: FedTile | None = None, stream: torch.cuda.Stream | None = None):
        _declare()
        self.cfg = cfg
        self.global_dims = [int(n) for n in global_dims]
        self.batched = bool(batched)
        self.use_graph = bool(use_graph) and self.batched
        self.tile = tile or FedTile()
        if not self.batched and tile is None:
            self.tile = FedTile(bucket_modes=0)      # the per-client baseline's default: hardware atomics
        dev = U0.device
        self.dtype = U0.dtype
        self.U = U0.detach().reshape(-1).contiguous().clone()
        self.Bs = torch.zeros_like(self.U)
        self.Cs = torch.zeros_like(self.U)
        self.clients = []
        for t, base in clients:
            n = t.model_rows * cfg.R
            z = lambda: torch.zeros(n, dtype=self.dtype, device=dev)
            self.clients.append(FedClient(t, [int(b) for b in base], z(), z(), z(), z()))
            if not self.batched and self.tile.bucket_modes != 0 and t.reserved_samples < cfg.p + cfg.q:
                t.reserve(cfg.p + cfg.q, cfg.R)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        self._h = None
        self._create()

    # ------------------------------------------------------------ handle --
    def _desc(self) -> gcp_fed_desc:
        cfg = self.cfg
        arr = (gcp_fed_client * len(self.clients))()
        for i, cl in enumerate(self.clients):
            arr[i].tensor = cl.tensor.handle.value
            for k, b in enumerate(cl.row_base):
                arr[i].row_base[k] = b
            arr[i].M, arr[i].B, arr[i].C, arr[i].G = (cl.M.data_ptr(), cl.B.data_ptr(), cl.C.data_ptr(),
                                                      cl.G.data_ptr())
        self._arr = arr
        d = gcp_fed_desc()
        d.nclients = len(self.clients)
        d.R = cfg.R
        d.tau = cfg.tau
        d.loss = G.LOSSES[cfg.loss]
        d.batched = int(self.batched)
        d.use_graph = int(self.use_graph)
        d.workgroups_per_client = self.tile.workgroups_per_client
        d.block = self.tile.block
        d.lanes = self.tile.lanes
        d.vec = self.tile.vec
        d.max_attempts = cfg.max_attempts
        d.lds_modes = self.tile.lds_modes
        d.bucket_modes = self.tile.bucket_modes
        d.bucket_block_samples = self.tile.bucket_block_samples
        d.p, d.q, d.seed = cfg.p, cfg.q, cfg.seed
        for k, n in enumerate(self.global_dims):
            d.global_dims[k] = n
        d.U, d.Bs, d.Cs = self.U.data_ptr(), self.Bs.data_ptr(), self.Cs.data_ptr()
        d.lr, d.meta_lr = cfg.lr, cfg.meta_lr
        d.beta1, d.beta2, d.eps, d.lower = cfg.beta1, cfg.beta2, cfg.eps, cfg.lower
        d.clients = C.cast(arr, C.POINTER(gcp_fed_client))
        d.barrier_timeout_s = cfg.barrier_timeout_s
        return d

    def _create(self):
        L = _declare()
        h = C.c_void_p()
        desc = self._desc()
        G._check(L.gcp_fedadam_create(C.byref(h), C.byref(desc), G._stream(self.stream)), "gcp_fedadam_create")
        self._h = h

    def retile(self, tile: FedTile) -> None:
        """Rebuild the handle with another launch shape (buffers kept)."""
        self.close_handle()
        self.tile = tile
        self._create()

    def close_handle(self):
        if self._h is not None and self._h.value:
            torch.cuda.synchronize()
            _declare().gcp_fedadam_destroy(self._h)
        self._h = None

    def close(self):
        self.close_handle()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- rounds --
    def round(self, r: int, check: bool = False) -> None:
        """Run round r on the handle's stream; the caller's current stream
        waits for it.  A barrier failure of an earlier batched round raises
        here once its status has reached the host; check=True also waits for
        this round and raises on any device error it recorded."""
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        G._check(_declare().gcp_fedadam_round(self._h, int(r), G._stream(self.stream)), "gcp_fedadam_round")
        cur.wait_stream(self.stream)
        if check:
            self.status()

    def status(self) -> None:
        G._check(_declare().gcp_fedadam_status(self._h, G._stream(self.stream)), "gcp_fedadam_status")

    def info(self) -> dict:
        """How the handle runs its rounds (gcp_fedadam_info)."""
        i = gcp_fed_info()
        G._check(_declare().gcp_fedadam_info(self._h, C.byref(i)), "gcp_fedadam_info")
        return {"form": FORMS.get(i.form, i.form), "lds_modes": i.lds_modes, "bucket_modes": i.bucket_modes,
                "workgroups_per_client": i.workgroups_per_client, "block": i.block, "lanes": i.lanes,
                "vec": i.vec, "bucket_block_samples": i.bucket_block_samples,
                "launches_per_round": i.launches_per_round}

    # -------------------------------------------------------------- state --
    def snapshot(self):
        torch.cuda.synchronize()
        s = [self.U.clone(), self.Bs.clone(), self.Cs.clone()]
        for cl in self.clients:
            s += [cl.M.clone(), cl.B.clone(), cl.C.clone(), cl.G.clone()]
        return s

    def restore(self, s) -> None:
        torch.cuda.synchronize()
        bufs = [self.U, self.Bs, self.Cs]
        for cl in self.clients:
            bufs += [cl.M, cl.B, cl.C, cl.G]
        for b, v in zip(bufs, s):
            b.copy_(v)
        torch.cuda.synchronize()


class Batched(FedAdam):
    """GCP-FedAdam with every client's local steps in shared launches (the
    persistent launch, or the row-bucketed round's three launches per local
    step), replayed from a HIP graph by default."""

    def __init__(self, clients, global_dims, U0: torch.Tensor, cfg: FedConfig, use_graph: bool = True,
                 tile: FedTile | None = None, stream: torch.cuda.Stream | None = None):
        super().__init__(clients, global_dims, U0, cfg, batched=True, use_graph=use_graph, tile=tile, stream=stream)


class Plain(FedAdam):
    """GCP-FedAdam with one sampled-gradient launch and one Adam launch per
    client and local step (the per-client reference).  scatter="atomic"
    forces hardware atomics; "auto" reserves each client's workspace and
    lets every gcp_loss_grad call choose (row-bucketed at large sample
    counts)."""

    def __init__(self, clients, global_dims, U0: torch.Tensor, cfg: FedConfig,
                 stream: torch.cuda.Stream | None = None, scatter: str = "atomic"):
        tile = FedTile(bucket_modes=0 if scatter == "atomic" else -1)
        super().__init__(clients, global_dims, U0, cfg, batched=False, use_graph=False, tile=tile, stream=stream)
