"""GPU parity of the delayed rank-k paths (FP64 flush and FP32-MFMA flush).

FP64 delayed updates are an exact reformulation of successive rank-1 updates,
so they must reproduce the oracle's flip sequence and its G(tau)
accumulators to 1e-10.  The mixed-precision flush is checked under replay of
the oracle's flips: G(tau) within 1e-5, drift reported.
"""
import numpy as np
import pytest

from oracle import bath as OB
from oracle import hfqmc as OH

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _bath(beta, L, t=1.0):
    return OB.bath_to_tau(OB.semicircle_iw(beta, t, 20000), t * t, beta, L)


def _codes(ref, L):
    return [sw * L + l for sw, l in ref["flips"]]


@pytest.mark.parametrize("beta,U,L,k,n_rec,chains,sweeps", [
    (10.0, 4.0, 20, 4, 100, 3, 60),      # window = whole sweep
    (7.0, 5.0, 37, 7, 23, 2, 20),        # odd L, recompute not a multiple of k
    (13.0, 4.8, 130, 32, 128, 2, 6),     # several windows per sweep, ragged last window
    (20.0, 4.8, 160, 64, 256, 2, 4),     # k = window size
])
def test_delayed_fp64_matches_oracle(ctx, beta, U, L, k, n_rec, chains, sweeps):
    import paper_0801_1222_amd as P
    g0 = _bath(beta, L)
    seed = 4
    out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, n_chains=chains, warmup=1,
                        sweeps=sweeps, mode="delayed", delay_k=k, recompute_every=n_rec,
                        flip_cap=50000, want_chain=True)
    for c in range(chains):
        ref = OH.run_chain(g0, U, beta, seed, chain=c, warmup=1, sweeps=sweeps, n_rec=n_rec)
        assert list(out["flips"][c]) == _codes(ref, L)
        got = out["chain_g"][c][0] / out["chain_n"][c][0]
        exp = ref["bins_g"][0] / ref["bins_n"][0]
        assert np.abs(got - exp).max() < 1e-10
        assert abs(out["chain_d"][c][0] / out["chain_n"][c][0]
                   - ref["bins_d"][0] / ref["bins_n"][0]) < 1e-10
    st = out["stats"]
    assert st["n_bad_ratio"] == 0 and st["n_singular"] == 0
    assert st["max_drift"] < 1e-10
    assert st["delay_k"] == k


@pytest.mark.parametrize("L,k", [(130, 16), (400, 32), (400, 64)])
def test_mixed_replay_within_1e5(ctx, L, k):
    import paper_0801_1222_amd as P
    beta, U, seed, sweeps = L * 0.1, 4.5, 0, 3
    g0 = _bath(beta, L)
    chains = [0, 1]
    refs = [OH.run_chain(g0, U, beta, seed, chain=c, warmup=0, sweeps=sweeps, n_rec=4 * k)
            for c in chains]
    out = P.hfqmc_solve(ctx, g0, U, beta, 0.1, seed, n_chains=2, warmup=0, sweeps=sweeps,
                        mode="mixed", delay_k=k, replay=[_codes(r, L) for r in refs],
                        flip_cap=20000, want_chain=True)
    for c in chains:
        assert list(out["flips"][c]) == _codes(refs[c], L)
        got = out["chain_g"][c][0] / out["chain_n"][c][0]
        exp = refs[c]["bins_g"][0] / refs[c]["bins_n"][0]
        assert np.abs(got - exp).max() < 1e-5
    drift = out["stats"]["max_drift"]
    assert 1e-12 < drift < 1e-3


def test_mixed_free_running_statistics(ctx):
    """Mixed path without replay on the atomic limit: closed form within errors."""
    import paper_0801_1222_amd as P
    beta, U, L = 4.0, 4.0, 40
    out = P.hfqmc_solve(ctx, np.full(L, 0.5), U, beta, beta / L, 9, n_chains=32, warmup=20,
                        sweeps=300, mode="mixed", delay_k=16)
    tau = np.arange(L + 1) * beta / L
    z = np.abs(out["g"] - OH.atomic_limit_g(U, beta, tau))[1:L] / out["g_err"][1:L]
    assert z.max() < 4.5
    assert abs(out["D"] - OH.atomic_limit_d(U, beta)) < 4.0 * out["D_err"]


def test_delayed_c2_shape_sampled_chains(ctx):
    """beta=40, U=4.5, L=400, 256 chains, k=32, recompute every 4k: chains 0 and 200
    against the oracle (FP64 flush: identical flips)."""
    import paper_0801_1222_amd as P
    beta, U, L, k = 40.0, 4.5, 400, 32
    g0 = _bath(beta, L)
    out = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 0, n_chains=256, warmup=1, sweeps=2,
                        mode="delayed", delay_k=k, flip_cap=4096, want_chain=True)
    for c in (0, 200):
        ref = OH.run_chain(g0, U, beta, 0, chain=c, warmup=1, sweeps=2, n_rec=4 * k)
        assert list(out["flips"][c]) == _codes(ref, L)
        got = out["chain_g"][c][0] / out["chain_n"][c][0]
        assert np.abs(got - ref["bins_g"][0] / ref["bins_n"][0]).max() < 1e-10


def test_drift_limit_raises_and_sampled_drift_is_reported(ctx):
    # the FP32 flush leaves a drift far above 1e-12: the limit turns it into
    # HFQMC_EDRIFT; a generous limit passes and the sampled drift is reported
    import paper_0801_1222_amd as P
    beta, U, L = 20.0, 4.5, 200
    g0 = _bath(beta, L)
    kw = dict(n_chains=4, warmup=1, sweeps=4, mode="mixed", delay_k=32)
    with pytest.raises(P.HFQMCError) as e:
        P.hfqmc_solve(ctx, g0, U, beta, 0.1, 3, drift_limit=1e-12, **kw)
    assert e.value.code == -5
    out = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 3, drift_limit=1.0, **kw)
    st = out["stats"]
    assert st["n_recomputes"] > 4 and 1e-12 < st["max_drift"] < 1.0
    # FP64 delayed: the same chains whether or not the drift is sampled at a
    # recompute (the recompute replaces G): identical to the oracle flip for flip
    ref = OH.run_chain(g0, U, beta, 3, chain=0, warmup=1, sweeps=12, n_rec=128)
    f64 = P.hfqmc_solve(ctx, g0, U, beta, 0.1, 3, n_chains=1, warmup=1, sweeps=12, n_bins=1,
                        mode="delayed", delay_k=32, flip_cap=20000, want_chain=True)
    assert ref["n_recomputes"] > 8
    assert list(f64["flips"][0]) == _codes(ref, L)
    assert np.abs(f64["chain_g"][0][0] / f64["chain_n"][0][0]
                  - ref["bins_g"][0] / ref["bins_n"][0]).max() < 1e-10
