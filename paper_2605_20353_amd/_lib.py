"""ctypes binding of libgcp.so: the C ABI declared in include/gcp.h, with the
same names, plus thin handle classes.  Argument marshalling only -- every step
of the sampled gradient runs in the HIP kernels.  torch tensors serve as
device memory; the current torch stream is passed as the HIP stream.

The library is loaded from this package directory.  If it has not been built
it is built once with hipcc; if that fails, every call raises.  There is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re
import threading
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgcp.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "gcp.h")

GCP_OK = 0
GCP_ERR_ARG = -1
GCP_ERR_HIP = -2
GCP_ERR_OOM = -3
GCP_ERR_SAMPLING = -4
GCP_ERR_UNSUPPORTED = -5
GCP_ERR_DATA = -6
STATUS_NAMES = {0: "GCP_OK", -1: "GCP_ERR_ARG", -2: "GCP_ERR_HIP", -3: "GCP_ERR_OOM",
                -4: "GCP_ERR_SAMPLING", -5: "GCP_ERR_UNSUPPORTED", -6: "GCP_ERR_DATA"}

GCP_F32 = 0
GCP_F64 = 1
LOSSES = {"gaussian": 0, "poisson": 1, "bernoulli_logit": 2}
SAMPLING = {"stratified": 0, "uniform": 1, "semi_stratified": 2}

GCP_LOSS_ONLY = 1
GCP_ACCUMULATE = 2
GCP_SCALE_BY_DEV = 4
GCP_DETERMINISTIC = 8
GCP_ADAM_ZERO_GRAD = 1


class GCPError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__(f"{fn}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class gcp_sample_params(C.Structure):
    _fields_ = [("kind", C.c_int32), ("max_attempts", C.c_int32), ("p", C.c_int64), ("q", C.c_int64),
                ("seed", C.c_uint64), ("step", C.c_uint64), ("client", C.c_uint64)]


class gcp_samples(C.Structure):
    _fields_ = [("coords", C.c_void_p), ("x", C.c_void_p), ("w", C.c_void_p)]


class gcp_tile(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("vec", C.c_int32), ("block", C.c_int32), ("grid", C.c_int32),
                ("lds_modes", C.c_int32), ("bucket_modes", C.c_int32), ("bucket_lds_bytes", C.c_int32),
                ("bucket_block_samples", C.c_int32), ("bucket_splits", C.c_int32), ("bucket_block", C.c_int32)]


_lock = threading.Lock()
_lib = None


def _declare(L):
    vp, i64, u, d_ = C.c_void_p, C.c_int64, C.c_uint, C.c_double
    sig = {
        "gcp_version": ([], C.c_char_p),
        "gcp_last_error": ([], C.c_char_p),
        "gcp_tensor_create": ([C.POINTER(vp), C.c_int, C.POINTER(i64), i64, vp, vp, C.c_int, vp], C.c_int),
        "gcp_tensor_create_dense": ([C.POINTER(vp), C.c_int, C.POINTER(i64), vp, C.c_int, vp], C.c_int),
        "gcp_tensor_destroy": ([vp], C.c_int),
        "gcp_tensor_device_bytes": ([vp], i64),
        "gcp_tensor_reserve": ([vp, i64, C.c_int, vp], C.c_int),
        "gcp_device_status": ([vp, vp], C.c_int),
        "gcp_sample": ([vp, C.POINTER(gcp_sample_params), vp, vp, vp, vp], C.c_int),
        "gcp_loss_grad": ([vp, C.POINTER(gcp_sample_params), C.POINTER(gcp_samples), vp, C.c_int, C.c_int,
                           u, vp, vp, vp, C.POINTER(gcp_tile), vp], C.c_int),
        "gcp_loss_grad_noalloc": ([vp, C.POINTER(gcp_sample_params), C.POINTER(gcp_samples), vp, C.c_int,
                                   C.c_int, u, vp, vp, vp, C.POINTER(gcp_tile), vp], C.c_int),
        "gcp_noalloc_scratch_bytes": ([], i64),
        "gcp_sample_y": ([vp, C.POINTER(gcp_sample_params), vp, C.c_int, C.c_int, vp, vp, vp, C.POINTER(gcp_tile),
                          vp], C.c_int),
        "gcp_mttkrp": ([vp, i64, vp, vp, vp, C.c_int, u, vp, vp, C.POINTER(gcp_tile), vp], C.c_int),
        "gcp_ceiling_random_reads": ([vp, i64, i64, C.c_int, C.c_int, vp, vp], C.c_int),
        "gcp_ceiling_dependent_gathers": ([vp, i64, vp, C.POINTER(i64), i64, C.c_int, C.c_int, vp, vp], C.c_int),
        "gcp_ceiling_lds_cas": ([C.c_int, C.c_int, C.c_int, vp, vp], C.c_int),
        "gcp_ceiling_lds_row_adds": ([C.c_int, C.c_int, C.c_int, vp, vp], C.c_int),
        "gcp_ceiling_global_atomics": ([vp, i64, i64, C.c_int, vp], C.c_int),
        "gcp_ceiling_copy": ([vp, vp, i64, vp], C.c_int),
        "gcp_adam_step": ([vp, vp, vp, vp, i64, C.c_int, i64, d_, d_, d_, d_, d_, u, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    for name in ("gcp_fedadam_create", "gcp_fedadam_round", "gcp_fedadam_destroy", "gcp_fed_status"):
        if hasattr(L, name):
            getattr(L, name).restype = C.c_int


def lib():
    """Load libgcp.so, building it first only if it does not exist."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                from . import build as _build
                _build.build()
            L = C.CDLL(LIB_PATH)
            _declare(L)
            _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions declared in the headers under include/."""
    names = set()
    inc = os.path.dirname(HEADER)
    for h in sorted(os.listdir(inc)):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(inc, h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names.update(re.findall(r"\b(gcp_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def _check(code: int, fn: str):
    if code != GCP_OK:
        msg = lib().gcp_last_error().decode(errors="replace")
        raise GCPError(code, fn, msg)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(0)
    return C.c_void_p(t.data_ptr())


def _dt(dtype) -> int:
    if dtype == torch.float32:
        return GCP_F32
    if dtype == torch.float64:
        return GCP_F64
    raise TypeError(f"unsupported dtype {dtype}")


def _require_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("device tensors are required (tensor on %s)" % t.device)


# ----------------------------------------------------------------- tensors --

class SparseTensor:
    """Handle of a sparse COO tensor on the GPU (gcp_tensor_create)."""

    def __init__(self, dims, coords: torch.Tensor, vals: torch.Tensor, stream=None):
        _require_cuda(coords, vals)
        self.dims = [int(n) for n in dims]
        self.d = len(self.dims)
        self.dtype = vals.dtype
        coords = coords.to(torch.int64).contiguous()
        vals = vals.contiguous()
        self.nnz = int(vals.numel())
        if coords.shape != (self.nnz, self.d):
            raise ValueError(f"coords shape {tuple(coords.shape)} != ({self.nnz}, {self.d})")
        dims_c = (C.c_int64 * self.d)(*self.dims)
        h = C.c_void_p()
        _check(lib().gcp_tensor_create(C.byref(h), self.d, dims_c, self.nnz, _ptr(coords), _ptr(vals),
                                       _dt(self.dtype), _stream(stream)), "gcp_tensor_create")
        self._h = h
        self.dense = False
        self.reserved_samples = 0

    @property
    def handle(self):
        return self._h

    @property
    def cells(self) -> int:
        n = 1
        for x in self.dims:
            n *= x
        return n

    @property
    def model_rows(self) -> int:
        return sum(self.dims)

    def device_bytes(self) -> int:
        return int(lib().gcp_tensor_device_bytes(self._h))

    def reserve(self, max_samples: int, R: int, stream=None) -> None:
        """Workspace for the row-bucketed scatter (gcp_tensor_reserve)."""
        _check(lib().gcp_tensor_reserve(self._h, int(max_samples), int(R), _stream(stream)), "gcp_tensor_reserve")
        self.reserved_samples = int(max_samples)

    def status(self, stream=None) -> None:
        _check(lib().gcp_device_status(self._h, _stream(stream)), "gcp_device_status")

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().gcp_tensor_destroy(h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DenseTensor(SparseTensor):
    """Handle of a dense row-major tensor (gcp_tensor_create_dense).  Keeps a
    reference to the values, which the library borrows."""

    def __init__(self, dims, vals: torch.Tensor, stream=None):
        _require_cuda(vals)
        self.dims = [int(n) for n in dims]
        self.d = len(self.dims)
        self.dtype = vals.dtype
        self._vals = vals.contiguous()
        if self._vals.numel() != self.cells:
            raise ValueError("dense values do not match dims")
        self.nnz = self.cells
        dims_c = (C.c_int64 * self.d)(*self.dims)
        h = C.c_void_p()
        _check(lib().gcp_tensor_create_dense(C.byref(h), self.d, dims_c, _ptr(self._vals), _dt(self.dtype),
                                             _stream(stream)), "gcp_tensor_create_dense")
        self._h = h
        self.dense = True


def gcp_tensor_create(dims, coords, vals, stream=None) -> SparseTensor:
    return SparseTensor(dims, coords, vals, stream)


def gcp_tensor_create_dense(dims, vals, stream=None) -> DenseTensor:
    return DenseTensor(dims, vals, stream)


def gcp_tensor_reserve(t: SparseTensor, max_samples: int, R: int, stream=None) -> None:
    t.reserve(max_samples, R, stream)


def gcp_tensor_destroy(t: SparseTensor) -> None:
    t.close()


def gcp_device_status(t: SparseTensor, stream=None) -> None:
    t.status(stream)


# ----------------------------------------------------------------- sampling --

@dataclass
class SampleParams:
    kind: str = "stratified"
    p: int = 0
    q: int = 0
    seed: int = 0
    step: int = 0
    client: int = 0
    max_attempts: int = 64

    def c(self) -> gcp_sample_params:
        return gcp_sample_params(SAMPLING[self.kind], int(self.max_attempts), int(self.p), int(self.q),
                                 int(self.seed) & (2**64 - 1), int(self.step) & (2**64 - 1),
                                 int(self.client) & (2**64 - 1))

    @property
    def n(self) -> int:
        return int(self.p) + int(self.q)


@dataclass
class Tile:
    lanes: int = 0
    vec: int = 0
    block: int = 0
    grid: int = 0
    lds_modes: int = -1
    bucket_modes: int = -1
    bucket_lds_bytes: int = 0
    bucket_block_samples: int = 0
    bucket_splits: int = 0
    bucket_block: int = 0

    def c(self) -> gcp_tile:
        return gcp_tile(self.lanes, self.vec, self.block, self.grid, self.lds_modes, self.bucket_modes,
                        self.bucket_lds_bytes, self.bucket_block_samples, self.bucket_splits, self.bucket_block)


def gcp_sample(t: SparseTensor, sp: SampleParams, stream=None):
    """Materialised samples: (coords int64 [n, d], x [n], w [n]) on the GPU."""
    dev = torch.device("cuda", torch.cuda.current_device())
    n = sp.n
    coords = torch.empty(n, t.d, dtype=torch.int64, device=dev)
    x = torch.empty(n, dtype=t.dtype, device=dev)
    w = torch.empty(n, dtype=t.dtype, device=dev)
    spc = sp.c()
    _check(lib().gcp_sample(t.handle, C.byref(spc), _ptr(coords), _ptr(x), _ptr(w), _stream(stream)), "gcp_sample")
    return coords, x, w


def gcp_loss_grad(t: SparseTensor, sp: SampleParams, A: torch.Tensor, R: int, loss: str,
                  G: torch.Tensor | None = None, loss_out: torch.Tensor | None = None,
                  samples=None, loss_only: bool = False, accumulate: bool = False,
                  scale: torch.Tensor | None = None, tile: Tile | None = None, want_loss: bool = True,
                  stream=None, noalloc: bool = False, deterministic: bool = False):
    """Fused sampled objective and gradient.  Returns (G, loss_out) where
    loss_out is a 1-element float64 device tensor (or None).
    deterministic=True sets GCP_DETERMINISTIC (bit-identical runs; needs
    the tensor's reserved workspace).  noalloc=True
    calls gcp_loss_grad_noalloc (the library's fixed scratch region instead
    of the handle's reserved workspace); G and loss_out should then be passed
    in, or they are allocated here by torch before the call."""
    _require_cuda(A, G, loss_out, scale)
    if A.dtype != t.dtype:
        raise TypeError("model dtype must match the tensor dtype")
    if not A.is_contiguous():
        raise ValueError("A must be contiguous")
    if A.numel() != t.model_rows * R:
        raise ValueError(f"A has {A.numel()} values, expected {t.model_rows * R}")
    if G is None and not loss_only:
        G = torch.empty_like(A)
    if G is not None and (G.dtype != A.dtype or G.numel() != A.numel() or not G.is_contiguous()):
        raise ValueError("G must be a contiguous array shaped like A")
    if loss_out is None and (want_loss or loss_only):
        loss_out = torch.zeros(1, dtype=torch.float64, device=A.device)
    flags = 0
    if loss_only:
        flags |= GCP_LOSS_ONLY
    if accumulate:
        flags |= GCP_ACCUMULATE
    if scale is not None:
        if scale.dtype != A.dtype:
            raise TypeError("scale dtype must match the model dtype")
        flags |= GCP_SCALE_BY_DEV
    if deterministic:
        flags |= GCP_DETERMINISTIC
    smp_p = None
    keep = None
    if samples is not None:
        coords, x, w = samples
        _require_cuda(coords, x, w)
        keep = (coords.contiguous(), x.contiguous(), w.contiguous())
        smp = gcp_samples(keep[0].data_ptr(), keep[1].data_ptr(), keep[2].data_ptr())
        smp_p = C.byref(smp)
    spc = sp.c()
    tl = tile.c() if tile is not None else None
    fn = "gcp_loss_grad_noalloc" if noalloc else "gcp_loss_grad"
    _check(getattr(lib(), fn)(t.handle, C.byref(spc), smp_p, _ptr(A), int(R), LOSSES[loss], flags,
                              _ptr(scale), _ptr(G), _ptr(loss_out), C.byref(tl) if tl is not None else None,
                              _stream(stream)), fn)
    del keep
    return G, loss_out


def gcp_sample_y(t: SparseTensor, sp: SampleParams, A: torch.Tensor, R: int, loss: str, coords=None, y=None,
                 loss_out: torch.Tensor | None = None, tile: Tile | None = None, stream=None):
    """Non-fused sampling step: the sampled tensor (coords [n, d] int64, y [n])
    with y = w f'(x, m) of the model A.  Returns (coords, y, loss_out)."""
    _require_cuda(A, coords, y, loss_out)
    if A.dtype != t.dtype or not A.is_contiguous() or A.numel() != t.model_rows * R:
        raise ValueError("A must be a contiguous model of the tensor's dtype and shape")
    n = sp.n
    if coords is None:
        coords = torch.empty(n, t.d, dtype=torch.int64, device=A.device)
    if y is None:
        y = torch.empty(n, dtype=t.dtype, device=A.device)
    spc = sp.c()
    tl = tile.c() if tile is not None else None
    _check(lib().gcp_sample_y(t.handle, C.byref(spc), _ptr(A), int(R), LOSSES[loss], _ptr(coords), _ptr(y),
                              _ptr(loss_out), C.byref(tl) if tl is not None else None, _stream(stream)),
           "gcp_sample_y")
    return coords, y, loss_out


def gcp_mttkrp(t: SparseTensor, coords: torch.Tensor, y: torch.Tensor, A: torch.Tensor, R: int,
               G: torch.Tensor | None = None, accumulate: bool = False, scale: torch.Tensor | None = None,
               tile: Tile | None = None, stream=None) -> torch.Tensor:
    """Sampled MTTKRP of a given sampled tensor (coords [n, d], values y)."""
    _require_cuda(coords, y, A, G, scale)
    n = int(y.numel())
    coords = coords.to(torch.int64).contiguous()
    y = y.contiguous()
    if coords.shape != (n, t.d) or y.dtype != A.dtype or A.dtype != t.dtype:
        raise ValueError("coords must be [n, d] int64 and y of the model's dtype")
    if G is None:
        G = torch.empty_like(A)
    flags = GCP_ACCUMULATE if accumulate else 0
    if scale is not None:
        flags |= GCP_SCALE_BY_DEV
    tl = tile.c() if tile is not None else None
    _check(lib().gcp_mttkrp(t.handle, n, _ptr(coords), _ptr(y), _ptr(A), int(R), flags, _ptr(scale), _ptr(G),
                            C.byref(tl) if tl is not None else None, _stream(stream)), "gcp_mttkrp")
    return G


def gcp_loss_grad_noalloc(t: SparseTensor, sp: SampleParams, A: torch.Tensor, R: int, loss: str,
                          G: torch.Tensor, loss_out: torch.Tensor | None = None, **kw):
    """gcp_loss_grad_noalloc: gcp_loss_grad on the library's fixed scratch
    region, for callers that cannot allocate."""
    return gcp_loss_grad(t, sp, A, R, loss, G=G, loss_out=loss_out, noalloc=True, **kw)


def gcp_noalloc_scratch_bytes() -> int:
    return int(lib().gcp_noalloc_scratch_bytes())


def gcp_adam_step(A: torch.Tensor, G: torch.Tensor, B: torch.Tensor, Cm: torch.Tensor, t: int,
                  lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                  lower: float = float("-inf"), zero_grad: bool = False, stream=None) -> None:
    """Alg. adam-update, in place on A, B, C (and G if zero_grad)."""
    _require_cuda(A, G, B, Cm)
    n = A.numel()
    for x in (G, B, Cm):
        if x.numel() != n or x.dtype != A.dtype or not x.is_contiguous():
            raise ValueError("A, G, B, C must be contiguous arrays of one dtype and size")
    flags = GCP_ADAM_ZERO_GRAD if zero_grad else 0
    _check(lib().gcp_adam_step(_ptr(A), _ptr(G), _ptr(B), _ptr(Cm), n, _dt(A.dtype), int(t), float(lr),
                               float(beta1), float(beta2), float(eps), float(lower), flags, _stream(stream)),
           "gcp_adam_step")
