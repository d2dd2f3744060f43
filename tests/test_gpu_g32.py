"""GPU parity of the mixed path with G stored in FP32 between recomputes
(HFQMC_FLAG_G_FP32), through the C ABI.

Bars as for the mixed path with FP64-stored G: under replay of the FP64
oracle's flips, G(tau) and D within 1e-5 (the storage rounding, ~6e-8
relative per flush and recompute, is far below the FP32 flush products' own
error), the drift reported and bounded; without replay, the atomic limit's
closed form within the statistical errors.
"""
import numpy as np
import pytest

from oracle import bath as OB
from oracle import hfqmc as OH

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _bath(beta, L, t=1.0):
    return OB.bath_to_tau(OB.semicircle_iw(beta, t, 20000), t * t, beta, L)


def _codes(ref, L):
    return [sw * L + l for sw, l in ref["flips"]]


@pytest.mark.parametrize("L,k,ph", [(130, 16, False), (400, 64, False), (400, 64, True),
                                    (251, 32, True)])
def test_g32_replay_within_1e5(ctx, L, k, ph):
    import paper_0801_1222_amd as P
    beta, U, seed, sweeps = L * 0.1, 4.5, 0, 3
    g0 = _bath(beta, L)
    refs = [OH.run_chain(g0, U, beta, seed, chain=c, warmup=0, sweeps=sweeps, n_rec=4 * k)
            for c in (0, 1)]
    kw = dict(n_chains=2, warmup=0, sweeps=sweeps, mode="mixed", delay_k=k,
              replay=[_codes(r, L) for r in refs], flip_cap=20000, want_chain=True, ph=ph)
    out = P.hfqmc_solve(ctx, g0, U, beta, 0.1, seed, g_fp32=True, **kw)
    f64 = P.hfqmc_solve(ctx, g0, U, beta, 0.1, seed, **kw)
    for c in (0, 1):
        assert list(out["flips"][c]) == _codes(refs[c], L)
        n = out["chain_n"][c][0]
        got = out["chain_g"][c][0] / n
        exp = refs[c]["bins_g"][0] / refs[c]["bins_n"][0]
        assert np.abs(got - exp).max() < 1e-5
        assert abs(out["chain_d"][c][0] / n - refs[c]["bins_d"][0] / refs[c]["bins_n"][0]) < 1e-5
        # against the same replay with FP64-stored G: the storage rounding only
        assert np.abs(got - f64["chain_g"][c][0] / n).max() < 1e-6
    st = out["stats"]
    assert st["n_recomputes"] == refs[0]["n_recomputes"] + refs[1]["n_recomputes"]
    assert 1e-12 < st["max_drift"] < 1e-3
    assert st["n_bad_ratio"] == 0 and st["n_singular"] == 0


def test_g32_final_green_close_to_exact(ctx):
    # after the last flush the stored G differs from the exact G of the final
    # field by the mixed path's drift since the last recompute, plus rounding
    import paper_0801_1222_amd as P
    beta, U, L, k, seed = 20.0, 4.5, 200, 32, 3
    g0 = _bath(beta, L)
    ref = OH.run_chain(g0, U, beta, seed, chain=0, warmup=0, sweeps=2, n_rec=4 * k)
    out = P.hfqmc_solve(ctx, g0, U, beta, 0.1, seed, n_chains=1, warmup=0, sweeps=2, n_bins=1,
                        mode="mixed", delay_k=k, replay=[_codes(ref, L)], flip_cap=20000,
                        want_green=True, g_fp32=True)
    Gu, Gd = OH.green_from_field(OH.g0_matrix(g0), ref["field"], OH.hs_lambda(U, 0.1))
    d = max(np.abs(out["green"][0, 0] - Gu).max(), np.abs(out["green"][0, 1] - Gd).max())
    assert d < 1e-3
    # values are FP32 numbers
    g = out["green"][0, 0]
    assert np.array_equal(g, g.astype(np.float32).astype(np.float64))


def test_g32_free_running_atomic_limit(ctx):
    import paper_0801_1222_amd as P
    beta, U, L = 4.0, 4.0, 40
    out = P.hfqmc_solve(ctx, np.full(L, 0.5), U, beta, beta / L, 9, n_chains=32, warmup=20,
                        sweeps=300, mode="mixed", delay_k=16, g_fp32=True)
    tau = np.arange(L + 1) * beta / L
    z = np.abs(out["g"] - OH.atomic_limit_g(U, beta, tau))[1:L] / out["g_err"][1:L]
    assert z.max() < 4.5
    assert abs(out["D"] - OH.atomic_limit_d(U, beta)) < 4.0 * out["D_err"]


def test_g32_autotuned_and_rejected_outside_mixed(ctx):
    import paper_0801_1222_amd as P
    beta, U, L = 20.0, 4.5, 200
    g0 = _bath(beta, L)
    out = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 1, n_chains=8, warmup=1, sweeps=3, mode="mixed",
                        delay_k=0, g_fp32=True)
    st = out["stats"]
    assert st["autotuned"] == 1 and st["delay_k"] in (16, 32, 64)
    assert abs(out["g"][0] - 0.5) < 1e-5 and np.abs(out["g"] - out["g"][::-1]).max() < 1e-3
    for mode in ("rank1", "delayed"):
        with pytest.raises(P.HFQMCError):
            P.hfqmc_solve(ctx, g0, U, beta, 0.1, 1, n_chains=2, sweeps=2, mode=mode, g_fp32=True)
