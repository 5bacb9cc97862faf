"""FP64 CPU oracle for the GCP sampled stochastic gradient.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never imports
this package and this package never imports the product library; the two share
no code.  Inputs come from the seeded generators or from the caller's own
arrays, never from the HIP path.

The arithmetic lives in ``gcp_oracle.c`` (plain serial C, double precision),
built here with gcc into ``liboracle.so``.  This module marshals numpy arrays
into it and writes the GCP-FedAdam round (Alg. gcp-fed-iter) out in numpy on
top of the C sampling, gradient and Adam routines.

Citations are to the paper's sections, equations and algorithms:
  * eq. cp / eq. gcp-model / eq. gcp-gradient (Sec. 2) -- model, objective,
    gradient (MTTKRP);
  * Sec. 3.1.1 -- stratified / semi-stratified sampling, O(log N) search;
  * Sec. 3.1.2 -- sampled MTTKRP (serial strategy here);
  * Alg. adam-update, Sec. 3.1.3 -- Adam on one contiguous vector;
  * Alg. gcp-fed-iter (Sec. 4) -- GCP-FedAdam.

Parity pins for every function are in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gcp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LOSS_GAUSSIAN = 0
LOSS_POISSON = 1
LOSS_BERNOULLI_LOGIT = 2
LOSSES = {"gaussian": LOSS_GAUSSIAN, "poisson": LOSS_POISSON,
          "bernoulli_logit": LOSS_BERNOULLI_LOGIT}

ORA_OK = 0
ORA_ERR_ARG = -1
ORA_ERR_SAMPLING = -4


def build(force: bool = False) -> str:
    """Compile gcp_oracle.c with gcc (-O2, no fast-math; OpenMP for the
    timing-only parallel step) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall",
                               "-fno-fast-math", "-fopenmp", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        i64p = C.POINTER(C.c_int64)
        f64p = C.POINTER(C.c_double)
        u64p = C.POINTER(C.c_uint64)
        L.ora_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.ora_philox4x64_10.restype = None
        L.ora_range.argtypes = [C.c_uint64, C.c_uint64]
        L.ora_range.restype = C.c_uint64
        L.ora_tensor_new.argtypes = [C.c_int, i64p, C.c_int64, i64p, f64p, C.POINTER(C.c_int)]
        L.ora_tensor_new.restype = C.c_void_p
        L.ora_tensor_free.argtypes = [C.c_void_p]
        L.ora_tensor_free.restype = None
        L.ora_find.argtypes = [C.c_void_p, i64p]
        L.ora_find.restype = C.c_int64
        L.ora_sample_stratified.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_uint64, C.c_uint64,
                                            C.c_uint64, C.c_int64, C.c_int, i64p, f64p, f64p]
        L.ora_sample_stratified.restype = C.c_int
        L.ora_sample_uniform.argtypes = [C.c_int, i64p, f64p, C.c_int64, C.c_uint64, C.c_uint64,
                                         C.c_uint64, i64p, f64p, f64p]
        L.ora_sample_uniform.restype = C.c_int
        L.ora_f.argtypes = [C.c_int, C.c_double, C.c_double]
        L.ora_f.restype = C.c_double
        L.ora_df.argtypes = [C.c_int, C.c_double, C.c_double]
        L.ora_df.restype = C.c_double
        L.ora_model_value.argtypes = [C.c_int, i64p, C.c_int, f64p, i64p]
        L.ora_model_value.restype = C.c_double
        L.ora_loss_grad.argtypes = [C.c_int, i64p, C.c_int, f64p, C.c_int64, i64p, f64p, f64p,
                                    C.c_int, C.c_int64, f64p, f64p]
        L.ora_loss_grad.restype = None
        L.ora_loss_grad_bound.argtypes = [C.c_int, i64p, C.c_int, f64p, C.c_int64, i64p, f64p, f64p,
                                          C.c_int, C.c_int64, C.c_double, f64p, f64p, i64p]
        L.ora_loss_grad_bound.restype = None
        L.ora_omp_sgd_step.argtypes = [C.c_void_p, C.c_int, f64p, f64p, f64p, C.c_int64, C.c_int, C.c_int64,
                                       C.c_int64, C.c_uint64, C.c_uint64, C.c_int64, C.c_double, C.c_double,
                                       C.c_double, C.c_double, C.c_double, C.c_int, i64p, f64p, f64p, f64p, f64p,
                                       C.POINTER(C.c_int)]
        L.ora_omp_sgd_step.restype = C.c_int
        L.ora_sample_derivatives.argtypes = [C.c_int, i64p, C.c_int, f64p, C.c_int64, i64p, f64p, f64p, C.c_int,
                                             C.c_int64, f64p]
        L.ora_sample_derivatives.restype = None
        L.ora_mttkrp.argtypes = [C.c_int, i64p, C.c_int, f64p, C.c_int64, i64p, f64p, f64p]
        L.ora_mttkrp.restype = None
        L.ora_adam.argtypes = [C.c_int64, f64p, f64p, f64p, f64p, C.c_int64, C.c_double,
                               C.c_double, C.c_double, C.c_double, C.c_double]
        L.ora_adam.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _loss_id(loss) -> int:
    return LOSSES[loss] if isinstance(loss, str) else int(loss)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


# --------------------------------------------------------------------------
# RNG: Philox4x64-10 and the exact range map.
# --------------------------------------------------------------------------

def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().ora_philox4x64_10(_p(c, C.c_uint64), _p(k, C.c_uint64), _p(out, C.c_uint64))
    return out


def range_map(u: int, n: int) -> int:
    return int(lib().ora_range(C.c_uint64(u), C.c_uint64(n)))


# --------------------------------------------------------------------------
# Tensors and sampling (Sec. 3.1.1).
# --------------------------------------------------------------------------

class SparseTensor:
    """COO tensor with the oracle's own lexicographically sorted index."""

    def __init__(self, dims, coords, vals):
        self.dims = _i64(dims)
        self.d = int(self.dims.size)
        self.coords = _i64(coords).reshape(-1, self.d)
        self.vals = _f64(vals)
        self.nnz = int(self.coords.shape[0])
        st = C.c_int(0)
        self._h = lib().ora_tensor_new(self.d, _p(self.dims, C.c_int64), self.nnz,
                                       _p(self.coords, C.c_int64), _p(self.vals, C.c_double),
                                       C.byref(st))
        if not self._h:
            raise OracleError(st.value, "ora_tensor_new (coordinate out of range or repeated)")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.ora_tensor_free(h)
            except Exception:
                pass
            self._h = None

    @property
    def cells(self) -> int:
        return int(np.prod(self.dims.astype(object)))

    def find(self, idx) -> int:
        i = _i64(idx)
        return int(lib().ora_find(self._h, _p(i, C.c_int64)))


def sample_stratified(t: SparseTensor, p: int, q: int, seed: int, step: int = 0, client: int = 0,
                      max_attempts: int = 64, semi: bool = False):
    """p nonzero samples (weight N/p) then q zero samples (weight (M-N)/q)."""
    n = p + q
    coords = np.zeros((n, t.d), dtype=np.int64)
    x = np.zeros(n)
    w = np.zeros(n)
    st = lib().ora_sample_stratified(t._h, p, q, C.c_uint64(seed), C.c_uint64(step),
                                     C.c_uint64(client), max_attempts, int(bool(semi)),
                                     _p(coords, C.c_int64), _p(x, C.c_double), _p(w, C.c_double))
    if st != ORA_OK:
        raise OracleError(st, "ora_sample_stratified")
    return coords, x, w


def sample_uniform(dims, dense, s: int, seed: int, step: int = 0, client: int = 0):
    """s cells uniform over the dense tensor, weight M/s."""
    dims = _i64(dims)
    dense = _f64(dense).reshape(-1)
    d = int(dims.size)
    coords = np.zeros((s, d), dtype=np.int64)
    x = np.zeros(s)
    w = np.zeros(s)
    st = lib().ora_sample_uniform(d, _p(dims, C.c_int64), _p(dense, C.c_double), s,
                                  C.c_uint64(seed), C.c_uint64(step), C.c_uint64(client),
                                  _p(coords, C.c_int64), _p(x, C.c_double), _p(w, C.c_double))
    if st != ORA_OK:
        raise OracleError(st, "ora_sample_uniform")
    return coords, x, w


# --------------------------------------------------------------------------
# Loss, model value, sampled gradient (eq. cp, eq. gcp-gradient).
# --------------------------------------------------------------------------

def f(loss, x: float, m: float) -> float:
    return float(lib().ora_f(_loss_id(loss), float(x), float(m)))


def df(loss, x: float, m: float) -> float:
    return float(lib().ora_df(_loss_id(loss), float(x), float(m)))


def model_value(dims, R: int, A, idx) -> float:
    dims = _i64(dims)
    A = _f64(A).reshape(-1)
    i = _i64(idx)
    return float(lib().ora_model_value(int(dims.size), _p(dims, C.c_int64), R,
                                       _p(A, C.c_double), _p(i, C.c_int64)))


def loss_grad(dims, R: int, A, coords, x, w, loss, n_semi: int = 0):
    """Return (G, F): sampled gradient (sum_k I_k x R, same layout as A) and
    the sampled objective, for the given sample list."""
    dims = _i64(dims)
    A = _f64(A).reshape(-1)
    coords = _i64(coords).reshape(-1, int(dims.size))
    x = _f64(x)
    w = _f64(w)
    n = int(coords.shape[0])
    G = np.zeros(int(dims.sum()) * R)
    F = C.c_double(0.0)
    lib().ora_loss_grad(int(dims.size), _p(dims, C.c_int64), R, _p(A, C.c_double), n,
                        _p(coords, C.c_int64), _p(x, C.c_double), _p(w, C.c_double),
                        _loss_id(loss), int(n_semi), _p(G, C.c_double), C.byref(F))
    return G, float(F.value)


def sample_derivatives(dims, R: int, A, coords, x, w, loss, n_semi: int = 0) -> np.ndarray:
    """Values of the sampled tensor of the non-fused gradient (Sec. 3.1.2):
    y_s = w_s f'(x_s, m_s), semi-stratified nonzeros w_s (f'(x_s,m_s) - f'(0,m_s))."""
    dims = _i64(dims)
    A = _f64(A).reshape(-1)
    coords = _i64(coords).reshape(-1, int(dims.size))
    x, w = _f64(x), _f64(w)
    n = int(coords.shape[0])
    y = np.zeros(n)
    lib().ora_sample_derivatives(int(dims.size), _p(dims, C.c_int64), R, _p(A, C.c_double), n,
                                 _p(coords, C.c_int64), _p(x, C.c_double), _p(w, C.c_double), _loss_id(loss),
                                 int(n_semi), _p(y, C.c_double))
    return y


def mttkrp(dims, R: int, A, coords, y) -> np.ndarray:
    """Sampled MTTKRP of a given sampled tensor: G_k[i_k, :] += y prod_{j != k} A_j[i_j, :]."""
    dims = _i64(dims)
    A = _f64(A).reshape(-1)
    coords = _i64(coords).reshape(-1, int(dims.size))
    y = _f64(y)
    G = np.zeros(int(dims.sum()) * R)
    lib().ora_mttkrp(int(dims.size), _p(dims, C.c_int64), R, _p(A, C.c_double), int(coords.shape[0]),
                     _p(coords, C.c_int64), _p(y, C.c_double), _p(G, C.c_double))
    return G


U_F32 = 2.0 ** -24      # unit roundoff of binary32
U_F64 = 2.0 ** -53      # unit roundoff of binary64


def loss_grad_bound_parts(dims, R: int, A, coords, x, w, loss, u: float, n_semi: int = 0):
    """Per-element ingredients of the rounding-error bound of a sampled
    gradient computed with unit roundoff u in any summation order (see
    ora_loss_grad_bound): (abssum, yerr) shaped like A and count per model
    row."""
    dims = _i64(dims)
    A = _f64(A).reshape(-1)
    coords = _i64(coords).reshape(-1, int(dims.size))
    x = _f64(x)
    w = _f64(w)
    n = int(coords.shape[0])
    rows = int(dims.sum())
    abssum = np.zeros(rows * R)
    yerr = np.zeros(rows * R)
    count = np.zeros(rows, dtype=np.int64)
    lib().ora_loss_grad_bound(int(dims.size), _p(dims, C.c_int64), R, _p(A, C.c_double), n,
                              _p(coords, C.c_int64), _p(x, C.c_double), _p(w, C.c_double),
                              _loss_id(loss), int(n_semi), float(u), _p(abssum, C.c_double),
                              _p(yerr, C.c_double), _p(count, C.c_int64))
    return abssum, yerr, count


def _gamma(n, u):
    n = np.asarray(n, dtype=np.float64)
    return n * u / (1.0 - n * u)


def grad_error_bound(dims, R: int, A, coords, x, w, loss, u: float, n_semi: int = 0) -> np.ndarray:
    """First-order bound, per gradient element, on |G^ - G| for a sampled
    gradient G^ computed with unit roundoff u (any order of the additions)
    against the exact gradient G of the same samples and factors:
    yerr + (gamma_d + gamma_{count-1}) abssum."""
    dims = _i64(dims)
    abssum, yerr, count = loss_grad_bound_parts(dims, R, A, coords, x, w, loss, u, n_semi)
    d = int(dims.size)
    depth = np.repeat(np.maximum(count - 1, 0), R)
    return yerr + (_gamma(d, u) + _gamma(depth, u)) * abssum


def adam(A: np.ndarray, G, B: np.ndarray, C_: np.ndarray, t: int, lr: float = 1e-3,
         beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
         lower: float = -np.inf) -> None:
    """In-place Adam update (Alg. adam-update) of the float64 arrays A, B, C_."""
    for a in (A, B, C_):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    G = _f64(G)
    lib().ora_adam(int(A.size), _p(A, C.c_double), _p(G, C.c_double), _p(B, C.c_double),
                   _p(C_, C.c_double), int(t), lr, beta1, beta2, eps, lower)


# --------------------------------------------------------------------------
# GCP-SGD/Adam steps and GCP-FedAdam (Alg. gcp-sgd-iter, Alg. gcp-fed-iter).
# --------------------------------------------------------------------------

@dataclass
class AdamParams:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    lower: float = -np.inf


def sgd_step(t: SparseTensor, R: int, A, B, C_, adam_t: int, loss, p: int, q: int, seed: int,
             step: int, ap: AdamParams, client: int = 0, max_attempts: int = 64,
             semi: bool = False):
    """One synchronous iteration on one device (Alg. gcp-sgd-iter without the
    all-reduce): sample, sampled gradient, Adam.  Returns (G, F)."""
    coords, x, w = sample_stratified(t, p, q, seed, step, client, max_attempts, semi)
    G, F = loss_grad(t.dims, R, A, coords, x, w, loss, n_semi=p if semi else 0)
    adam(A, G, B, C_, adam_t, ap.lr, ap.beta1, ap.beta2, ap.eps, ap.lower)
    return G, F


class ParallelStepper:
    """Timing-only OpenMP form of sgd_step (the paper's CPU MTTKRP with
    thread-private gradients), for the benchmark's CPU baseline: same
    samples and arithmetic, other order of the gradient's additions.  Holds
    its sample and per-thread gradient workspaces."""

    def __init__(self, t: SparseTensor, R: int, p: int, q: int, threads: int):
        self.t, self.R, self.p, self.q, self.threads = t, R, p, q, int(threads)
        n = p + q
        rows = int(t.dims.sum())
        self.coords = np.zeros((n, t.d), dtype=np.int64)
        self.x = np.zeros(n)
        self.w = np.zeros(n)
        self.G_priv = np.zeros(self.threads * rows * R)
        self.G = np.zeros(rows * R)
        self.threads_used = 0

    def step(self, A, B, C_, adam_t: int, loss, seed: int, step: int, ap: AdamParams, max_attempts: int = 64):
        used = C.c_int(0)
        st = lib().ora_omp_sgd_step(self.t._h, self.R, _p(A, C.c_double), _p(B, C.c_double), _p(C_, C.c_double),
                                    int(adam_t), _loss_id(loss), self.p, self.q, C.c_uint64(seed),
                                    C.c_uint64(step), int(max_attempts), ap.lr, ap.beta1, ap.beta2, ap.eps,
                                    ap.lower, self.threads, _p(self.coords, C.c_int64), _p(self.x, C.c_double),
                                    _p(self.w, C.c_double), _p(self.G_priv, C.c_double), _p(self.G, C.c_double),
                                    C.byref(used))
        if st != ORA_OK:
            raise OracleError(st, "ora_omp_sgd_step")
        self.threads_used = used.value
        return self.G


@dataclass
class FedClient:
    tensor: SparseTensor          # the client's block, in block-local coordinates
    row_base: np.ndarray          # per mode: first global row of the block
    M: np.ndarray                 # client (local) model, sum_k I_k^c x R
    B: np.ndarray                 # client Adam moments
    C: np.ndarray
    t: int = 0                    # client Adam update count


def fedadam_round(clients, global_dims, R: int, U: np.ndarray, Bs: np.ndarray, Cs: np.ndarray,
                  server_t: int, rnd: int, tau: int, loss, p: int, q: int, seed: int,
                  client_ap: AdamParams, server_ap: AdamParams, max_attempts: int = 64) -> int:
    """One GCP-FedAdam round (Alg. gcp-fed-iter) on float64 state, in place.

    Reading of the algorithm used here:
      1. every client copies the rows of its block from the server model U
         into its local model M_c;
      2. every client runs tau local steps (stratified samples of its block,
         sampled gradient, client Adam with its own persistent moments and
         counter), local step j of round rnd using RNG step rnd*tau + j and
         the client index as the RNG client id;
      3. D = U - M_c, averaged per row over the clients whose block covers it;
      4. server Adam on U with gradient D (lr = meta-rate), counter server_t+1.
    Returns the new server counter."""
    gd = _i64(global_dims)
    d = int(gd.size)
    goff = np.concatenate([[0], np.cumsum(gd)])
    U2 = U.reshape(-1, R)
    Dsum = np.zeros_like(U2)
    count = np.zeros(U2.shape[0])
    for c, cl in enumerate(clients):
        ldims = cl.tensor.dims
        loff = np.concatenate([[0], np.cumsum(ldims)])
        M2 = cl.M.reshape(-1, R)
        for k in range(d):
            g0 = goff[k] + cl.row_base[k]
            M2[loff[k]:loff[k + 1]] = U2[g0:g0 + ldims[k]]
        for j in range(tau):
            cl.t += 1
            sgd_step(cl.tensor, R, cl.M, cl.B, cl.C, cl.t, loss, p, q, seed, rnd * tau + j,
                     client_ap, client=c, max_attempts=max_attempts)
        for k in range(d):
            g0 = goff[k] + cl.row_base[k]
            Dsum[g0:g0 + ldims[k]] += U2[g0:g0 + ldims[k]] - M2[loff[k]:loff[k + 1]]
            count[g0:g0 + ldims[k]] += 1
    D = np.zeros_like(Dsum)
    covered = count > 0
    D[covered] = Dsum[covered] / count[covered, None]
    server_t += 1
    adam(U, D.reshape(-1), Bs, Cs, server_t, server_ap.lr, server_ap.beta1, server_ap.beta2,
         server_ap.eps, server_ap.lower)
    return server_t


def objective(t: SparseTensor, R: int, A, loss, p: int, q: int, seed: int, step: int = 0, client: int = 0,
              semi: bool = False) -> float:
    """Sampled objective F~ on the stratified sample set (seed, step, client)."""
    coords, x, w = sample_stratified(t, p, q, seed, step, client, semi=semi)
    _, F = loss_grad(t.dims, R, A, coords, x, w, loss, n_semi=p if semi else 0)
    return F


def gcp_adam_epochs(t: SparseTensor, R: int, A0, loss, p: int, q: int, obj_p: int, obj_q: int,
                    iters_per_epoch: int, max_epochs: int, lr: float, decay: float, max_fails: int,
                    seed: int, obj_client: int, ap: AdamParams):
    """GCP-Adam epochs with the restore-and-decay safeguard, written out on the
    oracle's routines: each epoch runs iters_per_epoch sampled-gradient Adam
    iterations (iteration number = RNG step, counted over all epochs, accepted
    or not); the objective is estimated on the fixed set (seed, step 0,
    obj_client); an epoch that does not lower it is undone and the rate is
    multiplied by decay; the run stops after max_fails undone epochs.
    Returns (A, objectives of accepted epochs with the initial one first,
    rates per epoch, fails)."""
    A = _f64(A0).reshape(-1).copy()
    B = np.zeros_like(A)
    Cm = np.zeros_like(A)
    f_prev = objective(t, R, A, loss, obj_p, obj_q, seed, 0, obj_client)
    objs, rates = [f_prev], []
    rate, tcount, it, fails = lr, 0, 0, 0
    for _ in range(max_epochs):
        saved = (A.copy(), B.copy(), Cm.copy(), tcount)
        for _ in range(iters_per_epoch):
            coords, x, w = sample_stratified(t, p, q, seed, it, 0)
            G, _ = loss_grad(t.dims, R, A, coords, x, w, loss)
            tcount += 1
            it += 1
            adam(A, G, B, Cm, tcount, rate, ap.beta1, ap.beta2, ap.eps, ap.lower)
        f = objective(t, R, A, loss, obj_p, obj_q, seed, 0, obj_client)
        rates.append(rate)
        if f < f_prev:
            f_prev = f
            objs.append(f)
        else:
            A[:], B[:], Cm[:] = saved[0], saved[1], saved[2]
            tcount = saved[3]
            rate *= decay
            fails += 1
            if fails >= max_fails:
                break
    return A, objs, rates, fails
