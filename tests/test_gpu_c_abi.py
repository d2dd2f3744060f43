"""The device entry points called from plain C (no Python or PyTorch in the
process): tests/c_abi/solve.c, compiled with gcc against include/hfqmc.h and
linked to the library, must print the same numbers as the Python binding's
calls with the same arguments (same seeds: identical results)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ctx():
    import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
    import paper_0801_1222_amd as P
    c = P.Context(0)
    yield c
    c.close()


def test_c_caller_matches_the_python_binding(ctx, tmp_path):
    import paper_0801_1222_amd as P
    from paper_0801_1222_amd import _native as N
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "solve")
    libdir = os.path.dirname(N.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-O1", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi", "solve.c"), "-L", libdir, "-lhfqmc",
                    "-Wl,-rpath," + libdir, "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    lines = [l.split() for l in res.stdout.splitlines()]
    beta, U, L, t = 10.0, 4.0, 20, 1.0
    bath = P.bethe_semicircle_bath(beta, t, 4096)
    g0 = P.bath_to_tau(bath, t * t, beta, L)
    for mode, name, k in ((0, "rank1", 0), (2, "mixed", 16)):
        out = P.hfqmc_solve(ctx, g0, U, beta, beta / L, 3, n_chains=4, warmup=20, sweeps=200,
                            mode=name, delay_k=k)
        dl = [x for x in lines if x[:3] == ["solve", str(mode), "D"]][0]
        assert float(dl[3]) == out["D"] and float(dl[4]) == out["D_err"]
        gc = np.array([float(x[4]) for x in lines if x[:3] == ["solve", str(mode), "g"]])
        assert np.array_equal(gc, out["g"])
    m = P.multigrid_solve(ctx, bath, t * t, U, beta, [0.5, 0.4, 0.25], 5, n_fine=41, n_chains=4,
                          warmup=20, sweeps=200, mode="rank1")
    dl = [x for x in lines if x[:2] == ["multigrid", "D"]][0]
    assert float(dl[2]) == m["D"] and float(dl[3]) == m["D_err"]
    gc = np.array([float(x[3]) for x in lines if x[:2] == ["multigrid", "g"]])
    assert np.array_equal(gc, m["g"])
