"""GPU tests of the launch machinery: captured-graph replays against eager
launches, the k / panel-width autotuner, the device-pointer entry point, and
the heat-bath acceptance rule against the oracle (through the C ABI).
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


def _eager_work():
    # unrelated device work and a synchronisation between graph replays
    import torch
    x = torch.arange(1 << 20, device="cuda", dtype=torch.float64)
    y = (x * 0.5 + 1.0).sum().item()
    torch.cuda.synchronize()
    assert y > 0


def _same(a, b):
    assert np.array_equal(a["g"], b["g"])
    assert np.array_equal(a["g_err"], b["g_err"])
    assert a["D"] == b["D"] and a["D_err"] == b["D_err"]
    assert np.array_equal(a["flip_count"], b["flip_count"])
    for x, y in zip(a["flips"], b["flips"]):
        assert np.array_equal(x, y)
    for k in ("n_accepted", "n_proposed", "n_recomputes", "n_flushes"):
        assert a["stats"][k] == b["stats"][k]


@pytest.mark.parametrize("mode,k", [("rank1", 0), ("mixed", 16), ("delayed", 32)])
def test_graph_replays_equal_eager(ctx, mode, k):
    import paper_0801_1222_amd as P
    beta, U, L, seed = 8.0, 4.5, 64, 5
    g0 = _bath(beta, L)
    kw = dict(n_chains=6, warmup=1, sweeps=4, mode=mode, delay_k=k, flip_cap=4000)
    ref = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, eager=True, **kw)
    assert ref["stats"]["graph"] == 0
    for rep in range(3):
        out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, **kw)
        assert out["stats"]["graph"] == 1
        _same(out, ref)
        _eager_work()
    # the sweep kernel's own events (event-record nodes of the graph, or eager records)
    for st in (ref["stats"], out["stats"]):
        assert 0.0 < st["seconds_sweep_kernel"] <= st["seconds_kernel"]


def test_graph_replay_with_new_bath(ctx):
    # same shapes, different bath values: the cached graph is replayed on the new input
    import paper_0801_1222_amd as P
    beta, L, seed = 8.0, 48, 2
    kw = dict(n_chains=4, warmup=1, sweeps=3, mode="mixed", delay_k=32, flip_cap=4000)
    for U, t in ((4.0, 1.0), (4.0, 0.8), (4.0, 1.2)):
        g0 = _bath(beta, L, t)
        a = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, **kw)
        _eager_work()
        b = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, eager=True, **kw)
        _same(a, b)


def test_autotune_choice_is_cached_and_deterministic(ctx):
    import paper_0801_1222_amd as P
    beta, U, L, seed = 20.0, 4.5, 200, 3
    g0 = _bath(beta, L)
    kw = dict(n_chains=16, warmup=1, sweeps=2, mode="mixed", delay_k=0, flip_cap=2000)
    a = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, **kw)
    sa = a["stats"]
    assert sa["autotuned"] == 1
    assert sa["delay_k"] in (16, 32, 64)
    assert sa["recompute_every"] == 4 * sa["delay_k"]
    assert sa["lu_panel"] in (16, 32)
    b = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, **kw)
    sb = b["stats"]
    assert sb["seconds_autotune"] == 0.0
    assert (sb["delay_k"], sb["lu_panel"]) == (sa["delay_k"], sa["lu_panel"])
    _same(a, b)


def test_device_pointer_entry_matches_host_entry(ctx):
    import torch
    import paper_0801_1222_amd as P
    beta, U, L, seed = 10.0, 4.0, 40, 9
    g0 = _bath(beta, L)
    host = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, n_chains=5, warmup=2, sweeps=6,
                         mode="delayed", delay_k=16)
    g0d = torch.tensor(g0, device="cuda", dtype=torch.float64)
    gd = torch.zeros(L + 1, device="cuda", dtype=torch.float64)
    ed = torch.zeros(L + 1, device="cuda", dtype=torch.float64)
    dd = torch.zeros(2, device="cuda", dtype=torch.float64)
    torch.cuda.synchronize()
    st = P.hfqmc_solve_dev(ctx, g0d.data_ptr(), L, U, beta, beta / L, seed, gd.data_ptr(),
                           ed.data_ptr(), dd.data_ptr(), n_chains=5, warmup=2, sweeps=6,
                           mode="delayed", delay_k=16)
    torch.cuda.synchronize()
    assert np.array_equal(gd.cpu().numpy(), host["g"])
    assert np.array_equal(ed.cpu().numpy(), host["g_err"])
    assert dd.cpu().numpy()[0] == host["D"]
    assert st["n_accepted"] == host["stats"]["n_accepted"]


@pytest.mark.parametrize("mode,k", [("rank1", 0), ("delayed", 8)])
def test_heat_bath_matches_oracle(ctx, mode, k):
    import paper_0801_1222_amd as P
    beta, U, L, seed = 10.0, 4.0, 20, 4
    g0 = _bath(beta, L)
    out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, n_chains=3, warmup=5, sweeps=60,
                        mode=mode, delay_k=k, flip_cap=20000, want_chain=True, heat_bath=True)
    for c in range(3):
        ref = OH.run_chain(g0, U, beta, seed, chain=c, warmup=5, sweeps=60,
                           n_rec=100 if mode == "rank1" else 4 * k, heat_bath=True)
        assert list(out["flips"][c]) == [sw * L + l for sw, l in ref["flips"]]
        n = out["chain_n"][c][0]
        got = out["chain_g"][c][0] / n
        exp = ref["bins_g"][0] / ref["bins_n"][0]
        assert np.abs(got - exp).max() < 1e-10


@pytest.mark.parametrize("mode,k,L", [("rank1", 0, 60), ("delayed", 16, 130), ("mixed", 32, 400)])
def test_reduced_recompute_equals_direct(ctx, mode, k, L):
    # the block elimination against the uniform-field references and the full
    # L x L LU give the same chain: identical flips, accumulators within 1e-10
    import paper_0801_1222_amd as P
    beta, U, seed = L / 10.0, 4.5, 8
    g0 = _bath(beta, L)
    kw = dict(n_chains=3, warmup=1, sweeps=4, mode=mode, delay_k=k, flip_cap=20000,
              want_chain=True)
    red = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, **kw)
    dirc = P.hfqmc_solve(ctx, g0, U, beta, beta / L, seed, direct=True, **kw)
    assert red["stats"]["recompute_reduced"] == 1 and dirc["stats"]["recompute_reduced"] == 0
    assert 0 < red["stats"]["n_reduced_rows"] <= (L // 2) * 2 * (red["stats"]["n_recomputes"] + 3)
    for c in range(3):
        assert np.array_equal(red["flips"][c], dirc["flips"][c])
        assert np.abs(red["chain_g"][c] - dirc["chain_g"][c]).max() < 1e-10 * red["chain_n"][c][0]
    assert red["stats"]["max_drift"] < (1e-3 if mode == "mixed" else 1e-10)


def test_measured_peaks_are_plausible(ctx):
    # the probes measure what the device achieves: positive and not above
    # the datasheet figures (8 TB/s, 78.6 / 157.3 / 78.6 TFLOP/s)
    import paper_0801_1222_amd as P
    pk = P.hfqmc_measure_peaks(ctx)
    assert 500.0 < pk["hbm_copy_gbs"] < 8000.0 * 1.05
    assert 500.0 < pk["hbm_read_gbs"] < 8000.0 * 1.05
    assert 5.0 < pk["fp64_mfma_tflops"] < 78.6 * 1.05
    assert 5.0 < pk["fp32_mfma_tflops"] < 157.3 * 1.05
    assert 2.0 < pk["fp64_fma_tflops"] < 78.6 * 1.05
