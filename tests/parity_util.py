"""Element-by-element gradient parity against the oracle.

A GPU gradient G^ is compared with the oracle's FP64 gradient G of the same
samples and factors element by element:

    |G^ - G| <= SAFETY * bound + floor

where bound is the oracle's first-order rounding-error bound for the GPU's
arithmetic (unit roundoff 2^-24 in float32, 2^-53 in float64), valid for any
order of the additions (atomics, per-workgroup partial sums, row-block
owners), plus the same bound at 2^-53 for the oracle's own FP64 rounding
(the bound is first-order in the unit roundoff, so that is the first scaled).
SAFETY = 2 covers the second-order terms the first-order bound drops; floor
(1e-37) only matters for elements whose bound is zero or underflows.
The per-mode Frobenius relative error (<= 1e-5 in float32, <= 1e-12 in
float64) is checked as well.
"""
import numpy as np
import torch

import oracle

SAFETY = 2.0
FROB_TOL = {torch.float64: 1e-12, torch.float32: 1e-5, np.float64: 1e-12, np.float32: 1e-5}


def _u(dtype):
    return oracle.U_F32 if dtype in (torch.float32, np.float32) else oracle.U_F64


def frob_rel_errs(g_gpu, g_ora, dims, R):
    g_gpu = np.asarray(g_gpu, dtype=np.float64).reshape(-1, R)
    g_ora = np.asarray(g_ora, dtype=np.float64).reshape(-1, R)
    errs, off = [], 0
    for n in dims:
        a, b = g_gpu[off:off + n], g_ora[off:off + n]
        nb = np.linalg.norm(b)
        errs.append(np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a))
        off += n
    return errs


def element_bound(dims, R, A64, coords, x, w, loss, dtype, n_semi=0):
    """Allowed |G^ - G| per element for a gradient computed in `dtype`.  The
    bound is first-order in the unit roundoff, so the oracle's own FP64
    rounding adds the same bound scaled by 2^-53 / u."""
    u = _u(dtype)
    b = oracle.grad_error_bound(dims, R, A64, coords, x, w, loss, u, n_semi=n_semi)
    return SAFETY * b * (1.0 + oracle.U_F64 / u) + 1e-37


def assert_grad_close(g_gpu, g_ora, dims, R, A64, coords, x, w, loss, dtype, n_semi=0, what="", scale=1.0):
    """Per-element bound and per-mode Frobenius check of one gradient.
    scale multiplies every y (GCP_SCALE_BY_DEV); the oracle gradient passed in
    must already include it."""
    g = np.asarray(g_gpu, dtype=np.float64).reshape(-1)
    go = np.asarray(g_ora, dtype=np.float64).reshape(-1)
    bound = element_bound(dims, R, A64, coords, x, w, loss, dtype, n_semi) * abs(scale)
    err = np.abs(g - go)
    bad = np.nonzero(~(err <= bound))[0]
    if bad.size:
        i = bad[np.argmax(err[bad] / np.maximum(bound[bad], 1e-300))]
        raise AssertionError(f"{what}: {bad.size} of {g.size} gradient elements exceed the rounding bound; "
                             f"worst element {i} (row {i // R}, column {i % R}): gpu {g[i]!r}, oracle {go[i]!r}, "
                             f"|diff| {err[i]:.3e} > bound {bound[i]:.3e}")
    errs = frob_rel_errs(g, go, dims, R)
    tol = FROB_TOL[dtype]
    assert max(errs) <= tol, f"{what}: per-mode relative errors {errs} above {tol}"
    return max(errs), float(np.max(err / np.maximum(bound, 1e-300)))
