"""The measurement kernels of include/gcp_ceilings.h run and do what their
rates are quoted for: the float4 copy copies, the float-atomic kernel adds
one per lane and request, the others finish with GCP_OK on small sizes; bad
arguments are rejected on the host."""
import ctypes as C
import sys

import pytest
import torch

from paper_2605_20353_amd import _lib as G

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_copy_and_atomics_do_their_work(gpu):
    L = G.lib()
    st = G._stream()
    say("ceilings: copy")
    src = torch.randint(-2**31, 2**31 - 1, (1 << 20,), dtype=torch.int32, device=gpu)
    dst = torch.zeros_like(src)
    G._check(L.gcp_ceiling_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), src.numel() * 4, st),
             "gcp_ceiling_copy")
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    say("ceilings: global atomics")
    rows, nup = 100, 10000
    Gr = torch.zeros(rows * 32, dtype=torch.float32, device=gpu)
    G._check(L.gcp_ceiling_global_atomics(C.c_void_p(Gr.data_ptr()), rows, nup, 256, st), "atomics")
    torch.cuda.synchronize()
    # every request adds 1 to each of the 32 columns of one row; each column
    # therefore holds the same count, and the counts add up to the requests
    per_row = Gr.view(rows, 32)
    assert torch.equal(per_row, per_row[:, :1].expand(rows, 32))
    assert per_row[:, 0].double().sum().item() == nup


def test_rate_kernels_run_on_small_sizes(gpu):
    L = G.lib()
    st = G._stream()
    sink = torch.zeros(1 << 14, dtype=torch.int32, device=gpu)
    rec = torch.randint(-2**31, 2**31 - 1, (1000 * 4,), dtype=torch.int32, device=gpu)
    A = torch.rand((30 + 20 + 10) * 32, dtype=torch.float32, device=gpu)
    dims3 = (C.c_int64 * 3)(30, 20, 10)
    s = C.c_void_p(sink.data_ptr())
    say("ceilings: random reads, gathers, LDS adds")
    for inflight in (1, 4):
        G._check(L.gcp_ceiling_random_reads(C.c_void_p(rec.data_ptr()), 1000, 5000, inflight, 256, s, st), "reads")
    for seq in (0, 1):
        G._check(L.gcp_ceiling_dependent_gathers(C.c_void_p(rec.data_ptr()), 1000, C.c_void_p(A.data_ptr()), dims3,
                                                 5000, seq, 256, s, st), "gathers")
    G._check(L.gcp_ceiling_lds_cas(16, 256, 8, s, st), "lds cas")
    for form in (0, 1, 2):
        G._check(L.gcp_ceiling_lds_row_adds(form, 16, 8, s, st), "lds row adds")
    torch.cuda.synchronize()
    assert L.gcp_ceiling_random_reads(C.c_void_p(rec.data_ptr()), 1000, 10, 2, 256, s, st) == G.GCP_ERR_ARG
    assert L.gcp_ceiling_lds_row_adds(3, 16, 8, s, st) == G.GCP_ERR_ARG
    assert L.gcp_ceiling_lds_cas(16, 100, 8, s, st) == G.GCP_ERR_ARG
    assert L.gcp_ceiling_copy(C.c_void_p(rec.data_ptr()), s, 10, st) == G.GCP_ERR_ARG
    bad = (C.c_int64 * 3)(30, 0, 10)
    assert L.gcp_ceiling_dependent_gathers(C.c_void_p(rec.data_ptr()), 1000, C.c_void_p(A.data_ptr()), bad, 10, 0,
                                           256, s, st) == G.GCP_ERR_ARG
