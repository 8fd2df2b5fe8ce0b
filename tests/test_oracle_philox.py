"""Pin: the oracle's Philox4x64-10 is bit-exact against numpy.random.Philox.

numpy's generator increments its 256-bit counter before producing a block,
so numpy started at counter c - 1 yields block(c)."""
import numpy as np

import oracle
import workloads


def _numpy_block(ctr, key):
    c = (int(ctr[0]) | (int(ctr[1]) << 64) | (int(ctr[2]) << 128) | (int(ctr[3]) << 192)) - 1
    c &= (1 << 256) - 1
    words = np.array([(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return g.random_raw(4)


def test_philox_matches_numpy_random_counters():
    rng = np.random.default_rng(123)
    for _ in range(300):
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 4).astype(np.uint64)
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64) * np.uint64(2)
        assert np.array_equal(oracle.philox4x64(ctr, key), _numpy_block(ctr, key))


def test_philox_edge_counters():
    M = (1 << 64) - 1
    for ctr in [(0, 0, 0, 0), (M, 0, 0, 0), (0, M, 0, 0), (M, M, M, M), (5, 7, 1, 4), (1, 0, 0, 2)]:
        for key in [(0, 0), (1, 0), (1, 999), (M, M)]:
            assert np.array_equal(oracle.philox4x64(ctr, key), _numpy_block(ctr, key)), (ctr, key)


def test_input_generator_block_matches_oracle():
    for e in (0, 1, 77):
        for i in (0, 3):
            assert np.array_equal(workloads.philox_block(1, e, i, 0, 0, 2), oracle.philox4x64((i, 0, 0, 2), (1, e)))


def test_unit_mapping_open_interval():
    # ((w >> 12) + 0.5) * 2^-52 lies strictly inside (0, 1) for the extreme words
    assert workloads.unit(0) > 0.0
    assert workloads.unit((1 << 64) - 1) < 1.0
