"""The widest ranks the kernels take (R up to 256: 64 lanes x 4 columns, and
ranks that are no multiple of 64) against the oracle: drawn and materialised
samples, every scatter strategy (atomic, LDS-private, row-bucketed, mixed),
the lane shapes that cover R, both dtypes."""
import sys

import pytest
import torch

import oracle
from paper_2605_20353_amd import _lib as G
from paper_2605_20353_amd import synth
from test_gpu_parity import model, oracle_ref

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _shapes(R, dtype):
    built = ([(32, 4), (64, 4), (64, 2)] if dtype == torch.float32 else [(64, 4), (64, 2)])
    return [(ln, vc) for ln, vc in built if ln * vc >= R and R % vc == 0]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("R", [96, 200, 256])
def test_wide_ranks_match_oracle(gpu, dtype, R):
    dims = [40, 30, 20]
    data = synth.count_tensor(dims, 3, 2000, seed=2607)
    t_gpu = G.SparseTensor(dims, data.coords.to(gpu), data.vals.to(dtype).to(gpu))
    t_ora = oracle.SparseTensor(dims, data.coords.numpy(), data.vals.to(dtype).double().numpy())
    sp = G.SampleParams("stratified", 3000 + 7, 2000 + 3, seed=41, step=5)
    t_gpu.reserve(sp.n, R)
    A = model(dims, R, dtype, gpu)
    ref = oracle_ref(t_ora, dims, R, A, "poisson", sp)
    tiles = [dict(),                                                        # automatic
             dict(lds_modes=0, bucket_modes=0),                             # atomic
             dict(lds_modes=1, bucket_modes=0),                             # mode 0 in LDS, the rest atomic
             dict(lds_modes=0, bucket_modes=7, bucket_block_samples=1024, bucket_splits=2),
             dict(lds_modes=4, bucket_modes=3, bucket_block_samples=512, bucket_block=256)]
    tiles += [dict(lanes=ln, vec=vc, lds_modes=0, bucket_modes=bm) for ln, vc in _shapes(R, dtype) for bm in (0, 7)]
    for tl in tiles:
        say(f"wide rank R={R} {dtype} {tl}")
        Gg, Lg = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", tile=G.Tile(**tl))
        t_gpu.status()
        ref.check(Gg, dtype, (R, tl))
        ref.check_loss(Lg, dtype)
    smp = G.gcp_sample(t_gpu, sp)
    Gm, Lm = G.gcp_loss_grad(t_gpu, sp, A, R, "poisson", samples=smp)
    t_gpu.status()
    ref.check(Gm, dtype, (R, "materialised"))
    ref.check_loss(Lm, dtype)
