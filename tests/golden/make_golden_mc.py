"""Writes the oracle's Monte Carlo estimates used as statistical pins by the GPU tests.

Calls only the oracle (FP64 rank-1 chains, exact recompute every 100 accepted
flips), with seeds disjoint from the GPU tests' (chain keys start at 2^40), so
a GPU run at the same parameters is an independent sample of the same
fixed-dtau expectation and must agree within the combined error bars:

  oracle_mc_b40_u45_L400   the headline shape: half-filled Bethe-lattice
                           impurity (t = 1, W = 4t, the semi-elliptic DOS of the
                           Benchmark results section), beta = 40, U = 4.5,
                           dtau = 0.1 (L = 400), 64 chains x (200 + 800) sweeps;
                           G(tau_k), k = 0..L, its error and D
  oracle_mc_b20_u48_mg7    a multigrid step (section "Multigrid HF-QMC method",
                           steps (i) and (ii)) on seven grids, beta = 20,
                           U = 4.8, dtau in {0.4, 1/3, 2/7, 0.25, 0.2, 1/6,
                           0.125} (L = 50 .. 160), 64 chains per grid x
                           (200 + 2000) sweeps: the extrapolated G on the
                           200-point fine grid and D, each grid's G(tau_k) and D

The chains are independent, so they run in a process pool (one BLAS thread
each); the pool only maps the oracle's own chain function.  About an hour on
six cores:

  python tests/golden/make_golden_mc.py [n_procs]
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bath as B  # noqa: E402
from oracle import hfqmc as H  # noqa: E402
from oracle import multigrid as MG  # noqa: E402

SEED = 1 << 40
N_IW = 20000


def _init_worker():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _write(path, header, rows):
    with open(path, "w") as f:
        for h in header:
            f.write("# " + h + "\n")
        for r in rows:
            f.write(r + "\n")
    print("wrote", path, flush=True)


def headline(pool):
    beta, U, L, t, nch, warm, sw = 40.0, 4.5, 400, 1.0, 64, 200, 800
    g_tau = B.bath_to_tau(B.semicircle_iw(beta, t, N_IW), t * t, beta, L)
    t0 = time.time()
    r = H.solve(g_tau, U, beta, SEED, n_chains=nch, warmup=warm, sweeps=sw, n_rec=100,
                mapper=pool.map)
    acc = sum(c["n_accepted"] for c in r["chains"]) / sum(c["n_proposed"] for c in r["chains"])
    rows = ["D %.17g %.17g" % (r["D"], r["D_err"])]
    rows += ["G %d %.17g %.17g" % (k, r["g"][k], r["g_err"][k]) for k in range(L + 1)]
    _write(os.path.join(HERE, "oracle_mc_b40_u45_L400.txt"),
           ["oracle Monte Carlo (FP64 rank-1, recompute every 100 accepted flips), written by",
            "make_golden_mc.py (oracle only); half-filled Bethe lattice t=%g (W=4t)" % t,
            "beta=%r U=%r L=%d n_iw=%d seed=%d chains=%d warmup=%d sweeps=%d" % (
                beta, U, L, N_IW, SEED, nch, warm, sw),
            "acceptance %.4f; columns: D mean err / G k mean err (tau_k = k beta/L, k = L is beta-)"
            % acc, "%.0f s" % (time.time() - t0)],
           rows)


def multigrid(pool):
    beta, U, t, nch, warm, sw, n_fine = 20.0, 4.8, 1.0, 64, 200, 2000, 200
    dtaus = [0.4, 1 / 3, 2 / 7, 0.25, 0.2, 1 / 6, 0.125]
    bath = B.semicircle_iw(beta, t, N_IW)
    t0 = time.time()
    r = MG.multigrid_solve(bath, t * t, U, beta, dtaus, SEED, nch, warm, sw, n_rec=100,
                           n_fine=n_fine, mapper=pool.map)
    rows = ["D %.17g %.17g" % (r["D"], r["D_err"])]
    rows += ["F %d %.17g %.17g" % (j, r["g"][j], r["g_err"][j]) for j in range(n_fine)]
    for i, (L, gr) in enumerate(zip(r["Ls"], r["grids"])):
        rows.append("GD %d %d %.17g %.17g" % (i, L, gr["D"], gr["D_err"]))
        rows += ["GG %d %d %.17g %.17g" % (i, k, gr["g"][k], gr["g_err"][k]) for k in range(L + 1)]
    _write(os.path.join(HERE, "oracle_mc_b20_u48_mg7.txt"),
           ["oracle multigrid solve (FP64 rank-1 chains, recompute every 100), written by",
            "make_golden_mc.py (oracle only); half-filled Bethe lattice t=%g (W=4t)" % t,
            "beta=%r U=%r Ls=%s n_iw=%d seed=%d chains per grid=%d warmup=%d sweeps=%d n_fine=%d"
            % (beta, U, r["Ls"], N_IW, SEED, nch, warm, sw, n_fine),
            "columns: D (extrapolated) mean err / F j g err (tau_j = j beta/(n_fine-1)) /",
            "GD grid L D err / GG grid k g err (tau_k = k beta/L)", "%.0f s" % (time.time() - t0)],
           rows)


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 2)
    with mp.get_context("fork").Pool(procs, initializer=_init_worker) as pool:
        headline(pool)
        multigrid(pool)


if __name__ == "__main__":
    main()
