"""Pins for the oracle's RNG and sampling (Sec. 3.1.1), on the CPU.

The oracle's Philox4x64-10 is pinned to the published known-answer vectors
and to numpy's independent Philox implementation; the range map to its exact
bucket boundaries; stratified sampling to brute-force membership and to
uniformity over the nonzeros and over the zeros of tiny tensors.
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")
U64 = (1 << 64) - 1


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    out = oracle.philox4x64_10(ctr, key)
    assert [int(v) for v in out] == expect


def test_philox_matches_numpy():
    # numpy's Philox is Philox4x64-10; it advances the 256-bit counter by one
    # before producing each block of four words.
    rng = np.random.default_rng(123)
    for _ in range(200):
        ctr = rng.integers(0, 2**63, 4, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 4, dtype=np.uint64)
        key = rng.integers(0, 2**63, 2, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 2, dtype=np.uint64)
        if int(ctr[0]) == 0:
            continue
        prev = ctr.copy()
        prev[0] = np.uint64(int(ctr[0]) - 1)
        ref = np.random.Philox(key=key, counter=prev).random_raw(4)
        assert [int(v) for v in oracle.philox4x64_10(ctr, key)] == [int(v) for v in ref]


@pytest.mark.parametrize("n", [1, 2, 3, 7, 50, 10000, 6000, 5 * 10**7, (1 << 40) + 12345, U64])
def test_range_map_bucket_boundaries(n):
    # floor(u n / 2^64) = j exactly on [ceil(j 2^64 / n), ceil((j+1) 2^64 / n))
    for j in [0, 1, n // 3, n // 2, n - 2, n - 1]:
        if j < 0 or j >= n:
            continue
        lo = -((-j << 64) // n)            # ceil(j * 2^64 / n)
        assert oracle.range_map(lo, n) == j
        if lo > 0:
            assert oracle.range_map(lo - 1, n) == j - 1
    assert oracle.range_map(0, n) == 0
    assert oracle.range_map(U64, n) == n - 1


def test_range_map_uniform_chi_square():
    n = 37
    counts = np.zeros(n)
    for s in range(20000):
        u = int(oracle.philox4x64_10([s, 5, 0, 0], [99, 0])[0])
        counts[oracle.range_map(u, n)] += 1
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, n - 1) > 1e-4


def _tiny_tensor(seed=0, dims=(5, 4, 3), nnz=17):
    rng = np.random.default_rng(seed)
    M = int(np.prod(dims))
    lin = rng.choice(M, nnz, replace=False)
    coords = np.stack(np.unravel_index(lin, dims), axis=1).astype(np.int64)
    vals = rng.integers(1, 9, nnz).astype(np.float64)
    return oracle.SparseTensor(dims, coords, vals), coords, vals


def test_find_brute_force():
    t, coords, vals = _tiny_tensor()
    present = {tuple(c): j for j, c in enumerate(coords.tolist())}
    for idx in np.ndindex(*t.dims):
        j = t.find(idx)
        if idx in present:
            assert j == present[idx]
        else:
            assert j == -1


def test_tensor_rejects_duplicates_and_out_of_range():
    with pytest.raises(oracle.OracleError):
        oracle.SparseTensor([3, 3], [[0, 1], [2, 2], [0, 1]], [1.0, 2.0, 3.0])
    with pytest.raises(oracle.OracleError):
        oracle.SparseTensor([3, 3], [[0, 3]], [1.0])


def test_stratified_samples_valid_and_weighted():
    t, coords, vals = _tiny_tensor()
    present = {tuple(c): v for c, v in zip(coords.tolist(), vals)}
    p, q = 40, 60
    sc, sx, sw = oracle.sample_stratified(t, p, q, seed=7, step=3)
    M = int(np.prod(t.dims))
    N = t.nnz
    for s in range(p):
        assert tuple(sc[s]) in present and sx[s] == present[tuple(sc[s])]
        assert sw[s] == N / p
    for s in range(p, p + q):
        assert tuple(sc[s]) not in present and sx[s] == 0.0
        assert sw[s] == (M - N) / q
        assert all(0 <= sc[s, k] < t.dims[k] for k in range(t.d))


def test_stratified_is_deterministic_and_step_dependent():
    t, _, _ = _tiny_tensor()
    a = oracle.sample_stratified(t, 10, 10, seed=1, step=0)
    b = oracle.sample_stratified(t, 10, 10, seed=1, step=0)
    c = oracle.sample_stratified(t, 10, 10, seed=1, step=1)
    assert np.array_equal(a[0], b[0])
    assert not np.array_equal(a[0], c[0])


def test_nonzero_draw_uniform_over_nonzeros():
    t, coords, _ = _tiny_tensor(seed=3)
    index = {tuple(c): j for j, c in enumerate(coords.tolist())}
    counts = np.zeros(t.nnz)
    for step in range(60):
        sc, _, _ = oracle.sample_stratified(t, 200, 0, seed=11, step=step)
        for c in sc.tolist():
            counts[index[tuple(c)]] += 1
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, t.nnz - 1) > 1e-4


def test_zero_draw_uniform_over_zeros():
    # rejection sampling gives the uniform distribution over the zero cells
    t, coords, _ = _tiny_tensor(seed=4, dims=(4, 3, 2), nnz=10)
    zeros = [idx for idx in np.ndindex(*t.dims) if t.find(idx) < 0]
    index = {z: i for i, z in enumerate(zeros)}
    counts = np.zeros(len(zeros))
    for step in range(100):
        sc, _, _ = oracle.sample_stratified(t, 0, 200, seed=5, step=step)
        for c in sc.tolist():
            counts[index[tuple(c)]] += 1
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, len(zeros) - 1) > 1e-4


def test_rejection_exhaustion_reports_sampling_error():
    # 23 of 24 cells are nonzero: with one attempt allowed some zero draw fails
    dims = (4, 3, 2)
    allc = np.array(list(np.ndindex(*dims)), dtype=np.int64)
    t = oracle.SparseTensor(dims, allc[1:], np.ones(len(allc) - 1))
    with pytest.raises(oracle.OracleError) as e:
        oracle.sample_stratified(t, 0, 64, seed=1, max_attempts=1)
    assert e.value.code == oracle.ORA_ERR_SAMPLING
    # with enough attempts the only zero cell is found every time
    sc, _, _ = oracle.sample_stratified(t, 0, 16, seed=1, max_attempts=2000)
    assert (sc == allc[0]).all()


def test_no_zero_cells_is_an_argument_error():
    dims = (2, 2)
    allc = np.array(list(np.ndindex(*dims)), dtype=np.int64)
    t = oracle.SparseTensor(dims, allc, np.ones(4))
    with pytest.raises(oracle.OracleError) as e:
        oracle.sample_stratified(t, 1, 1, seed=1)
    assert e.value.code == oracle.ORA_ERR_ARG


def test_zero_candidates_follow_counter_layout():
    # attempt a of zero sample s draws i_k = floor(out_k * I_k / 2^64) from
    # Philox(ctr = (s, step, 1 | a << 8, 0), key = (seed, client)); an empty
    # tensor accepts attempt 0
    dims = (7, 5, 3, 2, 9)            # d = 5 uses a second block for mode 4
    t = oracle.SparseTensor(dims, np.zeros((0, 5), dtype=np.int64), np.zeros(0))
    sc, _, sw = oracle.sample_stratified(t, 0, 4, seed=42, step=9, client=3)
    for s in range(4):
        o0 = oracle.philox4x64_10([s, 9, 1, 0], [42, 3])
        o1 = oracle.philox4x64_10([s, 9, 1, 1], [42, 3])
        want = [oracle.range_map(int(o0[k]), dims[k]) for k in range(4)]
        want.append(oracle.range_map(int(o1[0]), dims[4]))
        assert sc[s].tolist() == want
    assert (sw == np.prod(dims) / 4).all()


def test_zero_weight_exact_beyond_int64_cell_counts():
    # Amazon-shaped dimensions: M = 4821207 * 1774269 * 1805187 ~ 1.54e19 cells,
    # above 2^63.  The zero weight (M - N) / q comes from the exact count
    # (Python integers here), the zeros are drawn by the range map per mode and
    # never hit a stored nonzero.
    dims = (4821207, 1774269, 1805187)
    M = dims[0] * dims[1] * dims[2]
    assert (1 << 63) < M < (1 << 64)
    rng = np.random.default_rng(5)
    coords = np.unique(np.stack([rng.integers(0, n, 300) for n in dims], axis=1), axis=0)
    t = oracle.SparseTensor(dims, coords, np.ones(len(coords)))
    assert t.cells == M
    sc, sx, sw = oracle.sample_stratified(t, 8, 64, seed=3, step=1)
    assert (sw[8:] == float(M - len(coords)) / 64).all()
    assert (sw[:8] == len(coords) / 8).all()
    present = set(map(tuple, coords.tolist()))
    for s in range(8, 72):
        assert tuple(sc[s]) not in present and sx[s] == 0.0
        o = oracle.philox4x64_10([s - 8, 1, 1, 0], [3, 0])
        assert sc[s].tolist() == [oracle.range_map(int(o[k]), dims[k]) for k in range(3)]


def test_uniform_sampling_reads_dense_values():
    dims = (3, 4, 5)
    dense = np.arange(60, dtype=np.float64) * 0.5
    sc, sx, sw = oracle.sample_uniform(dims, dense, 50, seed=2, step=1)
    for s in range(50):
        assert sx[s] == dense[np.ravel_multi_index(tuple(sc[s]), dims)]
    assert (sw == 60 / 50).all()


def test_semi_stratified_skips_search():
    t, coords, _ = _tiny_tensor(seed=9, dims=(3, 3, 2), nnz=9)
    present = {tuple(c) for c in coords.tolist()}
    sc, sx, sw = oracle.sample_stratified(t, 0, 400, seed=3, semi=True)
    hits = sum(tuple(c) in present for c in sc.tolist())
    assert hits > 0                       # nonzero cells are kept as "zeros"
    assert (sx == 0).all()
