"""CPU checks of the native library: it loads, exports every declared symbol,
and its host-only routines agree with the oracle."""
import os
import re

import numpy as np
import pytest

from oracle import bath as OB
from oracle import multigrid as OMG

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hfqmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char\s*\*|const char\s*\*)\s*\*?\s*(\w+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_0801_1222_amd import _native as N
    names = _declared()
    assert "hfqmc_solve" in names and "multigrid_solve" in names and "dmft_bethe_step" in names
    for n in names:
        assert hasattr(N.lib, n), n
    assert sorted(N.EXPORTED) == names


def test_context_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_0801_1222_amd as P
    with pytest.raises(P.HFQMCError) as e:
        P.Context(0)
    assert e.value.code == -3


def test_semicircle_and_bath_transform_match_oracle():
    import paper_0801_1222_amd as P
    for beta, L in [(10.0, 20), (40.0, 400), (20.0, 57)]:
        b = P.bethe_semicircle_bath(beta, 1.0, 8000)
        bo = OB.semicircle_iw(beta, 1.0, 8000)
        assert np.abs(b - bo).max() < 1e-15
        g = P.bath_to_tau(b, 1.0, beta, L)
        go = OB.bath_to_tau(bo, 1.0, beta, L)
        assert np.abs(g - go).max() < 1e-12


def test_atomic_seed_matches_oracle():
    import paper_0801_1222_amd as P
    for beta, U in [(45.0, 5.0), (10.0, 0.0), (100.0, 4.8)]:
        b = P.bethe_atomic_bath(beta, 1.0, U, 6000)
        assert np.abs(b - OB.atomic_seed_iw(beta, 1.0, U, 6000)).max() < 1e-15


def test_bethe_step_matches_oracle_and_fixed_point():
    import paper_0801_1222_amd as P
    beta, t = 10.0, 1.0
    b = OB.semicircle_iw(beta, t, 3000)
    tf = OMG.fine_grid(beta, 200)
    gf = OB.iw_to_tau(b, 1.0, beta, tf)
    # U = 0: fixed point
    assert np.abs(P.dmft_bethe_step(gf, b, 1.0, 0.0, beta, t) - b).max() < 1e-12
    # U > 0 with a perturbed G: same result as the oracle's spline transform
    gp = gf + 0.01 * np.sin(np.pi * tf / beta) ** 2
    new = P.dmft_bethe_step(gp, b, 1.0, 3.0, beta, t)
    ref = OMG.dmft_bethe_step(gp, tf, b, 1.0, 3.0, beta, t)
    assert np.abs(new - ref).max() < 1e-11


def test_host_argument_errors():
    import paper_0801_1222_amd as P
    with pytest.raises(P.HFQMCError):
        P.bath_to_tau(np.zeros(4, dtype=complex), 1.0, 10.0, 20)   # n_iw < 16
    with pytest.raises(P.HFQMCError):
        P.dmft_bethe_step(np.zeros(3), np.zeros(100, dtype=complex), 1.0, 0.0, 10.0, 1.0)
    with pytest.raises(P.HFQMCError):
        P.bethe_atomic_bath(10.0, 1.0, -1.0, 100)                  # U < 0


def test_general_filling_host_routines_match_oracle():
    # away from half filling: the lattice bath at mu, the transform with the 1/(i w)^2
    # moment and the closure at mu (reference model at the density G(beta-))
    import paper_0801_1222_amd as P
    beta, t, U = 10.0, 1.0, 2.5
    for mu in (0.6, -0.9):
        b = P.bethe_lattice_bath(beta, t, mu, 4000)
        bo = OB.bethe_lattice_iw(beta, t, mu, 4000)
        assert np.abs(b - bo).max() < 1e-14
        g = P.bath_to_tau_m2(b, -mu, mu * mu + t * t, beta, 57)
        assert np.abs(g - OB.bath_to_tau(bo, mu * mu + t * t, beta, 57, m2=-mu)).max() < 1e-12
        tau = OMG.fine_grid(beta, 101)
        # an interacting-looking G: the reference model at n plus a smooth bump
        gf = OMG.reference_tau_n(bo, -mu, mu * mu + t * t, U, beta, tau, 0.55) \
            + 1e-3 * np.sin(np.pi * tau / beta)
        new = P.dmft_bethe_step_mu(gf, b, -mu, mu * mu + t * t, U, beta, t, mu)
        ref = OMG.dmft_bethe_step_n(gf, tau, bo, -mu, mu * mu + t * t, U, beta, t, mu)
        assert np.abs(new - ref).max() < 1e-11


def test_plain_c_caller_of_the_host_entry_points(tmp_path):
    """The C ABI from C: tests/c_abi/host_calls.c compiled with gcc against
    include/hfqmc.h and linked to the library, its output equal to the Python
    binding's (and the oracle's transform)."""
    import shutil
    import subprocess
    import paper_0801_1222_amd as P
    from paper_0801_1222_amd import _native as N
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "host_calls")
    libdir = os.path.dirname(N.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-O1", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi", "host_calls.c"), "-L", libdir, "-lhfqmc",
                    "-Wl,-rpath," + libdir, "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    g = [float(l.split()[2]) for l in out if l.startswith("g ")]
    f = [int(l.split()[2]) for l in out if l.startswith("f ")]
    bath = P.bethe_semicircle_bath(10.0, 1.0, 4096)
    assert np.array_equal(np.array(g), P.bath_to_tau(bath, 1.0, 10.0, 20))
    ref = OB.bath_to_tau(OB.semicircle_iw(10.0, 1.0, 4096), 1.0, 10.0, 20)
    assert np.abs(np.array(g) - ref).max() < 1e-12
    plan = P.hfqmc_plan_balance([250, 286, 333, 400, 500, 667, 1000, 2000], 32, 100, 1000, 1, 256)
    assert f == plan["factor"]
    assert any(l.startswith("error ") and "n_grids" in l for l in out)
