"""The seeded generators produce what they promise (CPU)."""
import numpy as np
import torch

from paper_2605_20353_amd import synth


def test_count_tensor_exact_nnz_distinct_and_deterministic():
    a = synth.count_tensor([30, 20, 10], 4, 500, seed=3)
    b = synth.count_tensor([30, 20, 10], 4, 500, seed=3)
    assert a.nnz == 500
    assert torch.equal(a.coords, b.coords) and torch.equal(a.vals, b.vals)
    lin = np.ravel_multi_index(a.coords.numpy().T, (30, 20, 10))
    assert len(np.unique(lin)) == 500
    assert (a.coords.min(0).values >= 0).all()
    assert (a.coords.max(0).values < torch.tensor([30, 20, 10])).all()
    assert (a.vals >= 1).all() and torch.equal(a.vals, a.vals.round())


def test_binary_and_blocks():
    b = synth.count_tensor([10, 10, 10, 4], 3, 200, seed=1, binary=True)
    assert torch.equal(b.vals, torch.ones(200, dtype=torch.float64))
    blocks = synth.fed_blocks([8, 8, 4], (2, 2, 1), 3, 20, 60, seed=2)
    assert len(blocks) == 4
    n = sorted(bl.data.nnz for bl in blocks)
    assert n[0] == 20 and n[-1] == 60
    for bl in blocks:
        assert bl.data.dims == [4, 4, 4]


def test_dense_gaussian_shape():
    X, facs = synth.dense_gaussian([4, 3, 5, 2], 2, seed=0, noise=0.0, dtype=torch.float64)
    full = torch.einsum("ar,br,cr,dr->abcd", *facs).reshape(-1)
    assert torch.allclose(X, full)
