"""The C-ABI library loads and exports every entry point of include/gcp.h,
and host-side argument checks reject bad calls before any GPU work (CPU)."""
import ctypes as C

import pytest

from paper_2605_20353_amd import _lib


def test_every_declared_symbol_is_exported():
    L = _lib.lib()
    names = _lib.header_functions()
    assert "gcp_loss_grad" in names and "gcp_sample" in names and "gcp_adam_step" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_error_string():
    L = _lib.lib()
    assert b"gfx950" in L.gcp_version()
    assert L.gcp_last_error() is not None


def test_host_argument_errors_without_gpu():
    L = _lib.lib()
    assert L.gcp_tensor_create(None, 3, None, 1, None, None, 0, None) == _lib.GCP_ERR_ARG
    h = C.c_void_p()
    dims = (C.c_int64 * 3)(4, 5, 6)
    assert L.gcp_tensor_create(C.byref(h), 0, dims, 1, None, None, 0, None) == _lib.GCP_ERR_ARG
    assert L.gcp_tensor_create(C.byref(h), 9, dims, 1, None, None, 0, None) == _lib.GCP_ERR_ARG
    assert L.gcp_tensor_create(C.byref(h), 3, dims, 0, None, None, 0, None) == _lib.GCP_ERR_ARG
    assert L.gcp_tensor_create(C.byref(h), 3, dims, 121, None, None, 0, None) == _lib.GCP_ERR_ARG
    big = (C.c_int64 * 3)(1 << 30, 1 << 30, 1 << 10)
    assert L.gcp_tensor_create(C.byref(h), 3, big, 5, None, None, 0, None) == _lib.GCP_ERR_UNSUPPORTED
    sp = _lib.gcp_sample_params(0, 64, 10, 10, 1, 0, 0)
    assert L.gcp_sample(None, C.byref(sp), None, None, None, None) == _lib.GCP_ERR_ARG
    assert L.gcp_loss_grad(None, C.byref(sp), None, None, 4, 1, 0, None, None, None, None, None) == _lib.GCP_ERR_ARG
    dummy = C.c_void_p(16)
    assert L.gcp_adam_step(dummy, dummy, dummy, dummy, -1, 0, 1, 1e-3, .9, .999, 1e-8, 0.0, 0, None) == _lib.GCP_ERR_ARG
    assert L.gcp_adam_step(dummy, dummy, dummy, dummy, 8, 0, 0, 1e-3, .9, .999, 1e-8, 0.0, 0, None) == _lib.GCP_ERR_ARG
    assert L.gcp_adam_step(dummy, dummy, dummy, dummy, 8, 0, 1, 1e-3, 1.0, .999, 1e-8, 0.0, 0, None) == _lib.GCP_ERR_ARG
    assert L.gcp_adam_step(dummy, dummy, dummy, dummy, 8, 7, 1, 1e-3, .9, .999, 1e-8, 0.0, 0, None) == _lib.GCP_ERR_ARG
    assert L.gcp_adam_step(None, dummy, dummy, dummy, 8, 0, 1, 1e-3, .9, .999, 1e-8, 0.0, 0, None) == _lib.GCP_ERR_ARG
    assert b"NULL" in L.gcp_last_error()
    # n = 0 is a no-op success
    assert L.gcp_adam_step(None, None, None, None, 0, 0, 1, 1e-3, .9, .999, 1e-8, 0.0, 0, None) == _lib.GCP_OK


def test_cell_key_limits_without_gpu():
    # a mode of 2^32 indices, a sum of dimensions of 2^32 model rows or more,
    # or 2^64 - 1 cells or more: unsupported, decided before any device work
    L = _lib.lib()
    h = C.c_void_p()
    for dims in ((1 << 32, 2, 2), (3_000_000_000, 1_500_000_000, 1), (4_000_000, 4_000_000, 4_000_000)):
        arr = (C.c_int64 * 3)(*dims)
        assert L.gcp_tensor_create(C.byref(h), 3, arr, 5, None, None, 0, None) == _lib.GCP_ERR_UNSUPPORTED, dims
    # 23 + 21 + 21 coordinate bits (more than a bit-packed key holds) but
    # under 2^64 cells: the shape is accepted and the NULL coordinates are
    # what the call rejects
    amazon = (C.c_int64 * 3)(4821207, 1774269, 1805187)
    assert L.gcp_tensor_create(C.byref(h), 3, amazon, 5, None, None, 0, None) == _lib.GCP_ERR_ARG
    assert b"coords" in L.gcp_last_error() or b"NULL" in L.gcp_last_error()


def test_struct_layouts_match_the_binding():
    import ctypes as C
    from paper_2605_20353_amd import fedadam
    L = _lib.lib()
    L.gcp_struct_size.restype = C.c_int64
    L.gcp_struct_size.argtypes = [C.c_char_p]
    for name, cls in [("gcp_sample_params", _lib.gcp_sample_params), ("gcp_samples", _lib.gcp_samples),
                      ("gcp_tile", _lib.gcp_tile), ("gcp_fed_client", fedadam.gcp_fed_client),
                      ("gcp_fed_desc", fedadam.gcp_fed_desc)]:
        assert L.gcp_struct_size(name.encode()) == C.sizeof(cls), name
    assert L.gcp_struct_size(b"nope") == -1
