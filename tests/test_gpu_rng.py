"""The device generator bit for bit against the oracle's Philox4x64-10.

The oracle's generator is pinned to numpy.random.Philox (an independent
implementation of the same published algorithm) on the CPU; here the uniforms
the sweep kernels draw, written out by hfqmc_uniforms, must equal it exactly:
about 1.7e7 draws over both streams, large seeds and sweep counters beyond
2^32, chains and grids of a batched launch.
"""
import numpy as np
import pytest

from oracle import philox

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("seed,chain,grid,sweep0,n_sweeps,L,stream", [
    (0, 0, 0, 0, 2200, 400, 0),               # the headline chain 0: 8.8e5 draws
    (1 << 32, 255, 7, 0, 1, 4096, 1),         # initial field of a long grid
    (12345, 31, 3, (1 << 33) + 17, 4, 2000, 0),
    (2 ** 63 + 5, 17, 1, 0, 3584, 4096, 0),  # 1.5e7 draws; key word 0 wraps past 2^64
])
def test_device_uniforms_equal_the_oracle(ctx, seed, chain, grid, sweep0, n_sweeps, L, stream):
    import paper_0801_1222_amd as P
    got = P.hfqmc_uniforms(ctx, seed, chain, grid, sweep0, n_sweeps, L, stream)
    sw = np.arange(sweep0, sweep0 + n_sweeps, dtype=np.uint64)[:, None]
    sl = np.arange(L, dtype=np.uint64)[None, :]
    ref = philox.uniform(seed, chain, grid, sw, sl, stream)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref), int(np.count_nonzero(got != ref))
    # a few values also against the scalar reference on Python integers
    for s_, l_ in [(0, 0), (n_sweeps - 1, L - 1), (n_sweeps // 2, L // 3)]:
        x0 = philox.philox4x64_scalar([l_, sweep0 + s_, 0, stream],
                                      [(seed + chain) % (1 << 64), grid])[0]
        assert got[s_, l_] == (x0 >> 11) * 2.0 ** -53


def test_uniform_arguments_are_checked(ctx):
    import paper_0801_1222_amd as P
    for a in [(0, -1, 0, 0, 1, 4, 0), (0, 0, 0, 0, 0, 4, 0), (0, 0, 0, 0, 1, 4, 2),
              (0, 0, 0, 0, 1 << 20, 1 << 9, 0)]:
        with pytest.raises(P.HFQMCError) as e:
            P.hfqmc_uniforms(ctx, *a)
        assert e.value.code == -1
