"""GPU parity of the solver with spin-dependent baths (hfqmc_solve_spin),
through the C ABI: the method with a magnetic field or in magnetic phases,
both Green matrices with baths of their own.

* FP64 paths (rank-1, delayed): the oracle's flip sequence and its
  spin-resolved accumulators to 1e-10; mixed path under replay within 1e-5.
* U = 0: each spin's G(tau) is its own bath (exact).
* One bath given for both spins: the same chain as hfqmc_solve.
* The Hubbard atom in a Zeeman field (Trotter-exact for every L): Monte Carlo
  against the closed form per spin within the statistical errors.
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


def _baths(beta, L, eps_dn=-0.4):
    tau = np.arange(L) * beta / L
    up = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    return up, OH.atomic_level_bath(eps_dn, beta, tau)


def _codes(ref, L):
    return [sw * L + l for sw, l in ref["flips"]]


@pytest.mark.parametrize("mode,k,L,beta,U", [("rank1", 0, 32, 8.0, 4.0), ("rank1", 0, 37, 6.0, 5.0),
                                             ("delayed", 16, 130, 13.0, 4.5),
                                             ("delayed", 32, 200, 20.0, 4.5)])
def test_spin_baths_match_oracle(ctx, mode, k, L, beta, U):
    import paper_0801_1222_amd as P
    bu, bd = _baths(beta, L)
    seed, warmup, sweeps = 6, 2, 6
    n_rec = 37 if mode == "rank1" else 4 * k
    out = P.hfqmc_solve_spin(ctx, bu, bd, U, beta, beta / L, seed, n_chains=3, warmup=warmup,
                             sweeps=sweeps, mode=mode, delay_k=k, recompute_every=n_rec,
                             flip_cap=40000, want_chain=True)
    assert out["stats"]["n_recomputes"] > 0
    assert out["chain_g"].shape == (3, 1, 2, L + 1)
    for c in range(3):
        ref = OH.run_chain((bu, bd), U, beta, seed, chain=c, warmup=warmup, sweeps=sweeps,
                           n_rec=n_rec)
        assert list(out["flips"][c]) == _codes(ref, L), "chain %d flips differ" % c
        n = out["chain_n"][c][0]
        got = out["chain_g"][c][0] / n
        exp = ref["bins_gs"][0] / ref["bins_n"][0]
        assert np.abs(got - exp).max() < 1e-10
        assert abs(out["chain_d"][c][0] / n - ref["bins_d"][0] / ref["bins_n"][0]) < 1e-10


def test_spin_baths_mixed_replay_within_1e5(ctx):
    import paper_0801_1222_amd as P
    L, k, beta, U, seed = 200, 32, 20.0, 4.5, 1
    bu, bd = _baths(beta, L, eps_dn=0.3)
    refs = [OH.run_chain((bu, bd), U, beta, seed, chain=c, warmup=0, sweeps=3, n_rec=4 * k)
            for c in (0, 1)]
    out = P.hfqmc_solve_spin(ctx, bu, bd, U, beta, beta / L, seed, n_chains=2, warmup=0, sweeps=3,
                             mode="mixed", delay_k=k, replay=[_codes(r, L) for r in refs],
                             flip_cap=20000, want_chain=True)
    for c in (0, 1):
        assert list(out["flips"][c]) == _codes(refs[c], L)
        got = out["chain_g"][c][0] / out["chain_n"][c][0]
        assert np.abs(got - refs[c]["bins_gs"][0] / refs[c]["bins_n"][0]).max() < 1e-5
    # the elementwise drift before a recompute is reported, not bounded by the
    # method; the bar is on G(tau) above (the atomic-level bath of spin down
    # has entries near 1, the FP32 flush products a few 1e-3 of error there)
    assert 1e-12 < out["stats"]["max_drift"] < 1e-2


@pytest.mark.parametrize("mode,k", [("rank1", 0), ("delayed", 16), ("mixed", 16)])
def test_spin_baths_u0_return_each_bath(ctx, mode, k):
    import paper_0801_1222_amd as P
    beta, L = 10.0, 50
    bu, bd = _baths(beta, L)
    out = P.hfqmc_solve_spin(ctx, bu, bd, 0.0, beta, beta / L, 3, n_chains=2, warmup=1, sweeps=3,
                             mode=mode, delay_k=k)
    assert np.abs(out["g_up"][:L] - bu).max() < 1e-12
    assert np.abs(out["g_dn"][:L] - bd).max() < 1e-12
    assert abs(out["g_up"][L] - (1.0 - bu[0])) < 1e-12 and abs(out["g_dn"][L] - (1.0 - bd[0])) < 1e-12


@pytest.mark.parametrize("mode,k", [("rank1", 0), ("delayed", 16)])
def test_one_bath_for_both_spins_equals_plain_solve(ctx, mode, k):
    import paper_0801_1222_amd as P
    beta, U, L = 12.0, 4.0, 60
    g0, _ = _baths(beta, L)
    kw = dict(n_chains=4, warmup=1, sweeps=5, mode=mode, delay_k=k, flip_cap=20000)
    a = P.hfqmc_solve(ctx, g0, U, beta, beta / L, 8, **kw)
    b = P.hfqmc_solve_spin(ctx, g0, g0, U, beta, beta / L, 8, **kw)
    for c in range(4):
        assert np.array_equal(a["flips"][c], b["flips"][c])
    assert np.abs(0.5 * (b["g_up"] + b["g_dn"]) - a["g"]).max() < 1e-12
    assert abs(a["D"] - b["D"]) < 1e-12


@pytest.mark.parametrize("mode", ["rank1", "delayed", "mixed"])
def test_atom_in_a_field_matches_closed_form(ctx, mode):
    import paper_0801_1222_amd as P
    beta, U, L, eu, ed = 4.0, 4.0, 16, -0.5, 0.3
    tau = np.arange(L) * beta / L
    out = P.hfqmc_solve_spin(ctx, OH.atomic_level_bath(eu, beta, tau), OH.atomic_level_bath(ed, beta, tau),
                             U, beta, beta / L, 21, n_chains=64, warmup=20, sweeps=400, mode=mode,
                             delay_k=16 if mode != "rank1" else 0)
    ex_u, ex_d = OH.atomic_field_g(eu, ed, U, beta, np.arange(L + 1) * beta / L)
    for got, err, ex in ((out["g_up"], out["err_up"], ex_u), (out["g_dn"], out["err_dn"], ex_d)):
        z = np.abs(got - ex)[1:L] / err[1:L]
        assert z.max() < 4.5, z.max()
        assert abs(got[0] + got[L] - 1.0) < 1e-12
    # the field polarises the atom: n_up > n_dn
    assert out["g_up"][L] - out["g_dn"][L] > 4 * np.hypot(out["err_up"][L], out["err_dn"][L])
    assert abs(out["D"] - OH.atomic_field_d(eu, ed, U, beta)) < 4.5 * out["D_err"]


def test_spin_baths_reject_single_matrix_and_fp32_storage(ctx):
    import paper_0801_1222_amd as P
    beta, L = 10.0, 20
    bu, bd = _baths(beta, L)
    with pytest.raises(P.HFQMCError):
        P._native.check(P._native.lib.hfqmc_solve_spin(ctx.handle, None, None, L, 4.0, beta, beta / L,
                                                      0, None, None, None, None, None), "null")
    import paper_0801_1222_amd.api as A
    for extra in (dict(ph=True), dict(g_fp32=True, mode="mixed")):
        o = A._opts(2, extra.get("mode", "rank1"), 0, 2, 0, 0, 0, 0.0,
                    A._flags(ph=extra.get("ph", False), g_fp32=extra.get("g_fp32", False)))
        g = np.zeros(2 * (L + 1))
        rc = P._native.lib.hfqmc_solve_spin(ctx.handle, P._native.ptr(np.ascontiguousarray(bu)),
                                           P._native.ptr(np.ascontiguousarray(bd)), L, 4.0, beta,
                                           beta / L, 0, A.C.byref(o), P._native.ptr(g), None, None,
                                           None)
        assert rc == -1


def test_spin_single_chain_bins_and_final_green(ctx):
    # one chain: 20 bins of the spin-resolved estimator, then the final G of
    # each spin against the exact Dyson solution with that spin's bath
    import paper_0801_1222_amd as P
    from oracle import philox
    beta, U, L, seed = 6.0, 4.0, 24, 4
    bu, bd = _baths(beta, L, eps_dn=0.35)
    out = P.hfqmc_solve_spin(ctx, bu, bd, U, beta, beta / L, seed, n_chains=1, warmup=3, sweeps=40,
                             mode="delayed", delay_k=8, flip_cap=20000, want_chain=True,
                             want_green=True)
    ref = OH.run_chain((bu, bd), U, beta, seed, chain=0, warmup=3, sweeps=40, n_rec=32, n_bins=20)
    assert out["chain_g"].shape == (1, 20, 2, L + 1)
    assert list(out["flips"][0]) == _codes(ref, L)
    for b in range(20):
        n = out["chain_n"][0][b]
        assert n == ref["bins_n"][b] == 2
        assert np.abs(out["chain_g"][0][b] / n - ref["bins_gs"][b] / n).max() < 1e-10
    # binned mean and error of each spin
    samples = ref["bins_gs"] / ref["bins_n"][:, None, None]
    assert np.abs(out["g_up"] - samples[:, 0].mean(axis=0)).max() < 1e-10
    assert np.abs(out["err_dn"] - samples[:, 1].std(axis=0, ddof=1) / np.sqrt(20)).max() < 1e-10
    field = philox.initial_field(seed, 0, 0, L).astype(np.int64)
    for code in out["flips"][0]:
        field[code % L] *= -1
    Gu, Gd = OH.green_from_field((OH.g0_matrix(bu), OH.g0_matrix(bd)), field, OH.hs_lambda(U, beta / L))
    assert np.abs(out["green"][0, 0] - Gu).max() < 1e-10
    assert np.abs(out["green"][0, 1] - Gd).max() < 1e-10
