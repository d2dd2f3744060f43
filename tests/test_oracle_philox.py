"""Pins for the oracle's Philox4x64-10 generator.

The generator is checked against numpy.random.Philox, an independent
implementation of the same published algorithm (Salmon et al., SC'11).
numpy increments its 256-bit counter before each block, so the block for
counter c is the first output of a generator started at c - 1.
"""
import numpy as np

from oracle import philox


def _numpy_block(ctr, key):
    cint = sum(int(v) << (64 * i) for i, v in enumerate(ctr))
    bg = np.random.Philox(counter=(cint - 1) % (1 << 256), key=int(key[0]) | (int(key[1]) << 64))
    return [int(x) for x in bg.random_raw(4)]


def test_scalar_and_vector_match_numpy_philox():
    rng = np.random.default_rng(12345)
    for _ in range(300):
        ctr = [int(v) for v in rng.integers(0, 2 ** 63, size=4, dtype=np.uint64) * 2 + rng.integers(0, 2, size=4)]
        key = [int(v) for v in rng.integers(0, 2 ** 63, size=2, dtype=np.uint64) * 2 + rng.integers(0, 2, size=2)]
        ref = _numpy_block(ctr, key)
        assert list(philox.philox4x64_scalar(ctr, key)) == ref
        vec = philox.philox4x64(*[np.uint64(c) for c in ctr], np.uint64(key[0]), np.uint64(key[1]))
        assert [int(v) for v in vec] == ref


def test_method_stream_layout_matches_numpy():
    # u for (seed, chain, grid, sweep, slice, stream) = top 53 bits of word 0
    # of the block at counter (slice, sweep, 0, stream), key (seed+chain, grid).
    for seed, chain, grid, sweep, sl, stream in [(0, 0, 0, 0, 0, 0), (7, 3, 2, 1234, 399, 0),
                                                 (2 ** 40, 255, 6, 2 ** 33 + 5, 17, 1)]:
        x0 = _numpy_block([sl, sweep, 0, stream], [seed + chain, grid])[0]
        ref = (x0 >> 11) * 2.0 ** -53
        got = philox.uniform(seed, chain, grid, sweep, sl, stream)
        assert float(got) == ref


def test_uniform_range_and_chi2():
    u = philox.uniform(0, np.arange(64)[:, None], 0, 5, np.arange(4096)[None, :], 0).ravel()
    assert u.min() >= 0.0 and u.max() < 1.0
    counts, _ = np.histogram(u, bins=64, range=(0.0, 1.0))
    exp = u.size / 64
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    # 63 degrees of freedom: mean 63, sd ~11.2; 5 sd bound
    assert chi2 < 63 + 5 * 11.3


def test_streams_are_distinct():
    a = philox.uniform(0, 0, 0, 0, np.arange(100), 0)
    b = philox.uniform(0, 0, 0, 0, np.arange(100), 1)
    c = philox.uniform(0, 1, 0, 0, np.arange(100), 0)
    d = philox.uniform(0, 0, 1, 0, np.arange(100), 0)
    for x, y in [(a, b), (a, c), (a, d), (b, c)]:
        assert not np.any(x == y)


def test_initial_field_is_balanced():
    s = np.concatenate([philox.initial_field(0, c, 0, 400) for c in range(50)])
    assert set(np.unique(s)) == {-1, 1}
    assert abs(float(np.mean(s))) < 5.0 / np.sqrt(s.size)
