"""GPU parity of the particle-hole symmetric single-matrix path (only G_up
stored, G_dn = 1 - G_up^T) against the two-matrix CPU oracle, through the C ABI.

The identity G_dn = 1 - G_up^T holds for every field when the bath is
particle-hole symmetric (G0 = 1 - G0^T) and V_dn = -V_up; the oracle keeps both
matrices and updates them separately, so agreement here tests the identity as
well as the single-matrix kernels.  Bars as for the two-matrix path: identical
flips and 1e-10 in FP64, 1e-5 under replay in the mixed path.
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


@pytest.mark.parametrize("mode,k,L,beta", [("rank1", 0, 40, 10.0), ("rank1", 0, 37, 8.0),
                                           ("delayed", 16, 130, 13.0), ("delayed", 64, 200, 20.0)])
def test_single_matrix_matches_two_matrix_oracle(ctx, mode, k, L, beta):
    import paper_0801_1222_amd as P
    U, seed, warmup, sweeps = 4.5, 3, 2, 6
    g0 = _bath(beta, L)
    n_rec = 100 if mode == "rank1" else 4 * k
    out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, n_chains=3, warmup=warmup,
                        sweeps=sweeps, mode=mode, delay_k=k, flip_cap=40000, want_chain=True,
                        ph=True)
    assert out["stats"]["n_recomputes"] > 0
    for c in range(3):
        ref = OH.run_chain(g0, U, beta, seed, chain=c, warmup=warmup, sweeps=sweeps, n_rec=n_rec)
        assert list(out["flips"][c]) == _codes(ref, L), "chain %d flips differ" % c
        n = out["chain_n"][c][0]
        got = out["chain_g"][c][0] / n
        exp = ref["bins_g"][0] / ref["bins_n"][0]
        assert np.abs(got - exp).max() < 1e-10
        assert abs(out["chain_d"][c][0] / n - ref["bins_d"][0] / ref["bins_n"][0]) < 1e-10


def test_single_matrix_mixed_replay_within_1e5(ctx):
    import paper_0801_1222_amd as P
    L, k = 400, 64
    beta, U, seed, sweeps = 40.0, 4.5, 0, 3
    g0 = _bath(beta, L)
    refs = [OH.run_chain(g0, U, beta, seed, chain=c, warmup=0, sweeps=sweeps, n_rec=4 * k)
            for c in (0, 1)]
    out = P.hfqmc_solve(ctx, g0, U, beta, 0.1, seed, n_chains=2, warmup=0, sweeps=sweeps,
                        mode="mixed", delay_k=k, replay=[_codes(r, L) for r in refs],
                        flip_cap=20000, want_chain=True, ph=True)
    for c in (0, 1):
        assert list(out["flips"][c]) == _codes(refs[c], L)
        got = out["chain_g"][c][0] / out["chain_n"][c][0]
        exp = refs[c]["bins_g"][0] / refs[c]["bins_n"][0]
        assert np.abs(got - exp).max() < 1e-5
    assert 1e-12 < out["stats"]["max_drift"] < 1e-3


def test_single_matrix_equals_two_matrix_gpu(ctx):
    # FP64 delayed at the production size: both storage forms take the same chain
    import paper_0801_1222_amd as P
    L, beta, U, seed = 400, 40.0, 4.5, 11
    g0 = _bath(beta, L)
    kw = dict(n_chains=4, warmup=1, sweeps=3, mode="delayed", delay_k=64, flip_cap=20000,
              want_chain=True)
    two = P.hfqmc_solve(ctx, g0, U, beta, 0.1, seed, **kw)
    one = P.hfqmc_solve(ctx, g0, U, beta, 0.1, seed, ph=True, **kw)
    for c in range(4):
        assert np.array_equal(one["flips"][c], two["flips"][c])
        assert np.abs(one["chain_g"][c] - two["chain_g"][c]).max() < 1e-10 * one["chain_n"][c][0]
    assert abs(one["D"] - two["D"]) < 1e-10
    assert one["stats"]["n_recomputes"] == two["stats"]["n_recomputes"]
    # one Dyson solve per recompute instead of two (the spins' systems have equal size)
    assert 2 * one["stats"]["n_reduced_rows"] == two["stats"]["n_reduced_rows"]


@pytest.mark.parametrize("mode,k", [("rank1", 0), ("delayed", 32)])
def test_single_matrix_final_green_is_exact(ctx, mode, k):
    import paper_0801_1222_amd as P
    beta, U, L, seed = 10.0, 4.0, 50, 5
    g0 = _bath(beta, L)
    n_rec = 37 if mode == "rank1" else 4 * k
    out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, n_chains=2, warmup=2, sweeps=3,
                        mode=mode, delay_k=k, recompute_every=n_rec, flip_cap=20000,
                        want_green=True, ph=True)
    lam = OH.hs_lambda(U, beta / L)
    G0 = OH.g0_matrix(g0)
    for c in range(2):
        ref = OH.run_chain(g0, U, beta, seed, chain=c, warmup=2, sweeps=3, n_rec=n_rec)
        Gu, Gd = OH.green_from_field(G0, ref["field"], lam)
        assert np.abs(out["green"][c, 0] - Gu).max() < 1e-10
        assert np.abs(out["green"][c, 1] - Gd).max() < 1e-10


def test_single_matrix_device_entry_and_graph(ctx):
    import torch
    import paper_0801_1222_amd as P
    beta, U, L, seed = 20.0, 4.5, 200, 2
    g0 = _bath(beta, L)
    kw = dict(n_chains=6, warmup=1, sweeps=3, mode="mixed", delay_k=0, ph=True)
    # device entry first: its autotuner reads the bath from device memory
    g0d = torch.tensor(g0, device="cuda", dtype=torch.float64)
    gd = torch.zeros(L + 1, device="cuda", dtype=torch.float64)
    dd = torch.zeros(2, device="cuda", dtype=torch.float64)
    torch.cuda.synchronize()
    st = P.hfqmc_solve_dev(ctx, g0d.data_ptr(), L, U, beta, beta / L, seed, gd.data_ptr(), None,
                           dd.data_ptr(), **kw)
    torch.cuda.synchronize()
    assert st["graph"] == 1 and st["autotuned"] == 1 and st["seconds_autotune"] > 0
    host = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, **kw)
    assert host["stats"]["seconds_autotune"] == 0.0
    assert host["stats"]["delay_k"] == st["delay_k"]
    assert np.array_equal(gd.cpu().numpy(), host["g"])
    assert dd.cpu().numpy()[0] == host["D"]


def test_single_matrix_rejects_asymmetric_bath(ctx):
    import paper_0801_1222_amd as P
    beta, U, L = 10.0, 4.0, 20
    g0 = _bath(beta, L, t=1.0)
    g0[3] += 1e-6                                # G0(tau) != G0(beta - tau)
    with pytest.raises(P.HFQMCError):
        P.hfqmc_solve(ctx, g0, U, beta, beta / L, 0, n_chains=2, sweeps=2, ph=True)
    g1 = _bath(beta, L)
    g1[0] = 0.49                                 # G0(0+) != 1/2
    with pytest.raises(P.HFQMCError):
        P.hfqmc_solve(ctx, g1, U, beta, beta / L, 0, n_chains=2, sweeps=2, ph=True)
