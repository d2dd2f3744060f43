"""Run-to-run determinism: two identical calls give bit-identical results.

Every reduction in the path has a fixed order (per-chain accumulators in
device memory, the chain reduction one grid per workgroup in chain order, no
floating-point atomics), so the workgroup that happens to take a unit from the
queue, and the launch's timing, cannot change a bit of the output.  Checked
for each update form and the batched, split launch.
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


def _bath(beta, L):
    return OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 8000), 1.0, beta, L)


@pytest.mark.parametrize("kw", [dict(mode="rank1"), dict(mode="delayed", delay_k=32),
                                dict(mode="mixed", delay_k=64), dict(mode="mixed", delay_k=64, ph=True),
                                dict(mode="mixed", delay_k=64, g_fp32=True)])
def test_identical_calls_are_bit_identical(ctx, kw):
    import paper_0801_1222_amd as P
    beta, U, L = 20.0, 4.5, 200
    g0 = _bath(beta, L)
    runs = [P.hfqmc_solve(ctx, g0, U, beta, beta / L, 11, n_chains=48, warmup=5, sweeps=20, **kw)
            for _ in range(2)]
    a, b = runs
    assert np.array_equal(a["g"], b["g"]) and np.array_equal(a["g_err"], b["g_err"])
    assert a["D"] == b["D"] and a["D_err"] == b["D_err"]
    assert a["stats"]["n_accepted"] == b["stats"]["n_accepted"]
    assert a["stats"]["max_drift"] == b["stats"]["max_drift"]


def test_split_batched_launch_is_bit_identical(ctx):
    import paper_0801_1222_amd as P
    beta, U = 16.0, 4.0
    Ls = [32, 64, 160]
    g0s = [_bath(beta, L) for L in Ls]
    runs = [P.hfqmc_solve_grids(ctx, Ls, g0s, U, beta, 3, n_chains=8, warmup=10, sweeps=64,
                                mode="mixed", delay_k=32, balance=True) for _ in range(2)]
    for i in range(len(Ls)):
        assert np.array_equal(runs[0]["g"][i], runs[1]["g"][i])
        assert runs[0]["D"][i] == runs[1]["D"][i]
    assert max(st["chain_split"] for st in runs[0]["stats"]) > 1
