"""The allocation-free entry point against hfqmc_solve_dev (through the C ABI).

hfqmc_solve_dev_noalloc runs the same kernels with every buffer in the
library's static per-device array, so its outputs must equal those of
hfqmc_solve_dev bit for bit.  Two calls in a row, the second smaller than the
first (the array keeps the first call's contents), then the limits.
"""
import numpy as np
import pytest

from oracle import bath as OB

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _run(P, ctx, fn, g0, L, U, beta, seed, **kw):
    import torch
    g0_d = torch.tensor(g0, dtype=torch.float64, device="cuda")
    g = torch.full((L + 1,), np.nan, dtype=torch.float64, device="cuda")
    e = torch.full((L + 1,), np.nan, dtype=torch.float64, device="cuda")
    d = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st = fn(ctx, g0_d.data_ptr(), L, U, beta, beta / L, seed, g.data_ptr(), e.data_ptr(),
            d.data_ptr(), **kw)
    torch.cuda.synchronize()
    return g.cpu().numpy(), e.cpu().numpy(), d.cpu().numpy(), st


CASES = [
    # beta, U, L, seed, options: a large call, then a smaller one
    (40.0, 4.5, 400, 3, dict(n_chains=40, warmup=2, sweeps=4, mode="mixed", delay_k=64)),
    (13.0, 4.8, 130, 5, dict(n_chains=24, warmup=2, sweeps=8, mode="rank1")),
]


def test_noalloc_equals_solve_dev_two_calls(ctx):
    import paper_0801_1222_amd as P
    for beta, U, L, seed, kw in CASES:
        g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
        a = _run(P, ctx, P.hfqmc_solve_dev_noalloc, g0, L, U, beta, seed, **kw)
        b = _run(P, ctx, P.hfqmc_solve_dev, g0, L, U, beta, seed, **kw)
        for x, y in zip(a[:3], b[:3]):
            assert np.all(np.isfinite(x))
            assert np.array_equal(x, y), np.abs(x - y).max()
        sa, sb = a[3], b[3]
        for key in ("n_proposed", "n_accepted", "n_recomputes", "n_flushes", "n_bad_ratio",
                    "max_drift", "max_drift_gtau", "delay_k", "recompute_every", "lu_panel"):
            assert sa[key] == sb[key], key
        assert sa["graph"] == 0 and sa["autotuned"] == 0
        assert 1 <= sa["n_workgroups"] <= kw["n_chains"]


def test_noalloc_repeat_after_a_larger_call_is_unchanged(ctx):
    # the array keeps the last call's contents: a repeat of the small call after the
    # large one returns the same values
    import paper_0801_1222_amd as P
    beta, U, L, seed, kw = CASES[1]
    g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    first = _run(P, ctx, P.hfqmc_solve_dev_noalloc, g0, L, U, beta, seed, **kw)
    bb, UU, LL, ss, kk = CASES[0]
    g0b = OB.bath_to_tau(OB.semicircle_iw(bb, 1.0, 20000), 1.0, bb, LL)
    _run(P, ctx, P.hfqmc_solve_dev_noalloc, g0b, LL, UU, bb, ss, **kk)
    again = _run(P, ctx, P.hfqmc_solve_dev_noalloc, g0, L, U, beta, seed, **kw)
    for x, y in zip(first[:3], again[:3]):
        assert np.array_equal(x, y)


def test_noalloc_limits(ctx):
    import paper_0801_1222_amd as P
    beta, U = 100.0, 4.5
    L = 1000
    g0 = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    with pytest.raises(P.HFQMCError) as e:      # beyond the buffer
        _run(P, ctx, P.hfqmc_solve_dev_noalloc, g0, L, U, beta, 0, n_chains=2, mode="rank1")
    assert e.value.code == -1 and "exceeds" in str(e.value)
    L = 40
    g0 = OB.bath_to_tau(OB.semicircle_iw(4.0, 1.0, 20000), 1.0, 4.0, L)
    with pytest.raises(P.HFQMCError) as e:      # the autotuner would allocate
        _run(P, ctx, P.hfqmc_solve_dev_noalloc, g0, L, U, 4.0, 0, n_chains=2, mode="mixed")
    assert e.value.code == -1 and "delay_k" in str(e.value)
