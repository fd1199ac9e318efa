"""Pins for the oracle's grid/FOV and index sampler (CPU only)."""
import math
import os

import numpy as np
import pytest

from oracle import grid, sampler

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("N", [1, 2, 7, 8, 16, 33, 128])
def test_fov_count_integer_form(N):
    # c(i)^2 + c(j)^2 <= 1  <=>  (2i+1-N)^2 + (2j+1-N)^2 <= N^2 (exact integers)
    brute = sum(1 for i in range(N) for j in range(N)
                if (2 * i + 1 - N) ** 2 + (2 * j + 1 - N) ** 2 <= N * N)
    assert grid.fov_indices(2, N).size == brute
    assert grid.fov_indices(3, N).size == brute * N


def test_fov_counts_of_workloads():
    # C1 and C2 grids and the 3D slices computed by the integer form
    for N in (128, 512, 256, 501):
        brute = sum(1 for i in range(N) for j in range(N)
                    if (2 * i + 1 - N) ** 2 + (2 * j + 1 - N) ** 2 <= N * N)
        assert grid.fov_mask(2, N).sum() == brute


def test_coords_roundtrip():
    N = 9
    idx = grid.fov_indices(3, N)
    X = grid.coords(3, N, idx)
    ijk = np.rint((X + 1) * N / 2 - 0.5).astype(int)
    assert np.array_equal(ijk[:, 0] + N * ijk[:, 1] + N * N * ijk[:, 2], idx)
    assert np.all(X[:, 0] ** 2 + X[:, 1] ** 2 <= 1)


def test_mix64_matches_published_splitmix64_outputs():
    lines = [l.strip() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
             if l.strip() and not l.startswith("#")]
    for i, hexv in enumerate(lines, start=1):
        z = (i * sampler.GOLDEN) & sampler.M64
        assert sampler.mix64(z) == int(hexv, 16)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 100, 1000, 4099])
def test_permutation_is_bijection(n):
    out = [sampler.permute(j, n, seed=12345, step=7) for j in range(n)]
    assert sorted(out) == list(range(n))


def test_half_bits_domain():
    for n in range(1, 3000):
        hb = sampler.half_bits(n)
        assert (1 << (2 * hb)) >= n
        assert (1 << (2 * hb)) < 4 * max(n, 4) + 1


def test_sample_sorted_distinct_and_keyed():
    n, k = 5000, 300
    a = sampler.sample_ranks(n, k, seed=1, step=0)
    b = sampler.sample_ranks(n, k, seed=1, step=1)
    c = sampler.sample_ranks(n, k, seed=2, step=0)
    assert a.size == k and np.all(np.diff(a) > 0) and a.min() >= 0 and a.max() < n
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(a, sampler.sample_ranks(n, k, seed=1, step=0))
    # k = n gives every rank
    assert np.array_equal(sampler.sample_ranks(50, 50, 3, 4), np.arange(50))


def test_inclusion_frequency_uniform():
    # P(i in I) = k/n for every i: chi-square over 400 draws
    n, k, draws = 40, 10, 400
    cnt = np.zeros(n)
    for s in range(draws):
        cnt[sampler.sample_ranks(n, k, seed=99, step=s)] += 1
    p = k / n
    expected = draws * p
    var = draws * p * (1 - p)
    chi2 = float(((cnt - expected) ** 2 / var).sum())
    # 39 degrees of freedom (sum is fixed); 99.9% quantile ~ 72.1
    assert chi2 < 72.1
    # pairwise: P(i, j both in I) = k(k-1)/(n(n-1)) on average
    assert abs(cnt.sum() - draws * k) == 0


def test_vectorised_sampler_equals_scalar_spec():
    for n, k in [(1, 1), (7, 7), (5000, 300), (70001, 1000)]:
        assert np.array_equal(sampler.sample_ranks_np(n, k, 31, 2),
                              sampler.sample_ranks(n, k, 31, 2))
