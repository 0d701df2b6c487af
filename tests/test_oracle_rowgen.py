"""Pins of the oracle's seeded minibatch generator (Sec. IV: every iteration draws its rows
uniformly at random) and agreement of the library's host generator with it, bit for bit.

The generator is SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) with iteration k taking outputs
k 2^32 + 1, ... of the sequence seeded with `seed`, and a partial Fisher-Yates shuffle that maps
draw u at step j to position j + floor(hi32(u) (n - j) / 2^32).  Pins: the published first
outputs of SplitMix64 from seed 0, a worked example of the shuffle computed by hand from them,
and properties of a uniform draw without replacement."""
import numpy as np
import pytest

import oracle

# First three outputs of SplitMix64 from seed 0, as published with the algorithm's reference code.
SPLITMIX64_SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_splitmix64_published_outputs():
    g = oracle.splitmix64(0)
    assert [next(g) for _ in range(3)] == SPLITMIX64_SEED0


def test_shuffle_worked_example():
    """seed 0, iteration 0, M = 10, B = 3, by hand from the three outputs above:
    hi32 0xE220A839 = 3793791033: j = 0, r = floor(3793791033 * 10 / 2^32) = 8, row 8;
    hi32 0x6E789E6A = 1853398634: j = 1, r = 1 + floor(1853398634 * 9 / 2^32) = 1 + 3 = 4, row 4;
    hi32 0x06C45D18 = 113532184:  j = 2, r = 2 + floor(113532184 * 8 / 2^32) = 2 + 0 = 2, row 2."""
    assert oracle.rows_generate(0, 0, 1, 10, 3).tolist() == [[8, 4, 2]]


@pytest.mark.parametrize("M,B", [(1, 1), (5, 5), (97, 13), (4096, 256)])
def test_rows_distinct_and_in_range(M, B):
    t = oracle.rows_generate(12345, 3, 6, M, B)
    assert t.shape == (6, B)
    for row in t:
        assert len(set(row.tolist())) == B
        assert row.min() >= 0 and row.max() < M
    if B == M:
        for row in t:
            assert sorted(row.tolist()) == list(range(M))


def test_prefix_and_start_iter():
    """A smaller minibatch is the prefix of a larger one drawn with the same stream, and a table
    split over calls at start_iter equals one call (each iteration has its own stream)."""
    a = oracle.rows_generate(7, 0, 5, 300, 40)
    b = oracle.rows_generate(7, 0, 5, 300, 25)
    assert np.array_equal(a[:, :25], b)
    c = np.vstack([oracle.rows_generate(7, 0, 2, 300, 40), oracle.rows_generate(7, 2, 3, 300, 40)])
    assert np.array_equal(a, c)
    assert not np.array_equal(a[0], a[1])
    assert not np.array_equal(oracle.rows_generate(8, 0, 1, 300, 40), a[:1])


def test_rows_uniform():
    """7000 draws of 3 of 7 rows: every row is drawn about 3000 times, and the first row of the
    minibatch is uniform over the 7 (chi-square with 6 degrees of freedom below 35, p < 1e-5)."""
    t = oracle.rows_generate(2024, 0, 7000, 7, 3)
    counts = np.bincount(t.ravel(), minlength=7)
    chi = np.sum((counts - 3000.0) ** 2 / 3000.0)
    first = np.bincount(t[:, 0], minlength=7)
    chi_first = np.sum((first - 1000.0) ** 2 / 1000.0)
    assert chi < 35 and chi_first < 35, (counts, first)


def test_subsets_follow_the_stream():
    """Frequencies are the stream's first nf draws (so they equal a row draw of size nf over F);
    transmitters and receivers are distinct subsets of their arrays."""
    f, t, r = oracle.subsets_generate(99, 4, 3, 64, 32, 24, 16, 8, 12)
    assert np.array_equal(f, oracle.rows_generate(99, 4, 3, 64, 16))
    for a, n in ((f, 64), (t, 32), (r, 24)):
        for row in a:
            assert len(set(row.tolist())) == row.size and row.min() >= 0 and row.max() < n


@pytest.fixture(scope="module")
def bd():
    from paper_2509_00774_amd import binding
    binding.load_library()
    return binding


@pytest.mark.parametrize("seed,start,iters,M,B", [
    (0, 0, 1, 10, 3), (12345, 3, 6, 97, 13), (2 ** 64 - 1, 1000, 2, 4096, 4096), (31337, 7, 2, 230400, 16384)])
def test_library_generator_matches_oracle(bd, seed, start, iters, M, B):
    """The library's host generator (used by spgm_solve_ex when no rows are given) gives the
    oracle's rows bit for bit, including the largest workload's M and B."""
    assert np.array_equal(bd.rows_generate(seed, start, iters, M, B), oracle.rows_generate(seed, start, iters, M, B))


def test_library_subsets_match_oracle(bd):
    got = bd.subsets_generate(5, 2, 4, 64, 32, 32, 16, 16, 16)
    ref = oracle.subsets_generate(5, 2, 4, 64, 32, 32, 16, 16, 16)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_library_generator_rejects_bad_sizes(bd):
    with pytest.raises(bd.SpgmError):
        bd.rows_generate(0, 0, 1, 10, 11)
    with pytest.raises(bd.SpgmError):
        bd.subsets_generate(0, 0, 1, 8, 8, 8, 9, 1, 1)
