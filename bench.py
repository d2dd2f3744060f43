"""Throughput of the Hirsch-Fye QMC hot path on one MI355X.

Workload (the headline configuration): half-filled single-band Hubbard
impurity, Bethe-lattice semicircular DOS (t = 1), beta = 40, U = 4.5,
dtau = 0.1 (L = 400), 256 independent chains (seeds 0..255), 200 warm-up +
2000 measured sweeps per chain.  One step = one full solve of that workload
(all chains, all sweeps, chain init, recomputes, measurement and reduction).

Prints ONE JSON line: metric sweeps/s over all chains for the production
path, the plain FP64 rank-1 path timed beside it, the roofline of the
persistent sweep kernel and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

WORKLOAD = dict(beta=40.0, U=4.5, dtau=0.1, L=400, n_chains=256, warmup=200, sweeps=2000,
                t=1.0, seed=0)


def algorithmic_work(L, st, n_chains, measured_sweeps, mode, k):
    """Algorithmic HBM bytes and FP64 flops of one solve (Measurement)."""
    L2 = float(L) * L
    n_acc = st["n_accepted"]
    n_rec = st["n_recomputes"] + 2 * n_chains  # plus the initial G of each chain (both spins counted below)
    meas = float(n_chains) * measured_sweeps
    if mode == "rank1":
        upd_bytes = 32.0 * L2 * n_acc
    else:
        # one read+write of both G per flush of up to k pending flips
        upd_bytes = 32.0 * L2 * n_acc / k
    bytes_ = upd_bytes + 16.0 * L2 * meas + 24.0 * L2 * n_rec
    flops = 4.0 * L2 * n_acc + n_rec * (8.0 / 3.0) * L2 * L
    return bytes_, flops


def cpu_baseline(sample_chains, warmup, sweeps, procs):
    """Oracle (as it stands) on the host cores over a bounded sample of the workload."""
    import multiprocessing as mp
    w = WORKLOAD
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        pool.map(_oracle_chain, [(c, warmup, sweeps) for c in range(sample_chains)])
    dt = time.perf_counter() - t0
    return dict(value=sample_chains * (warmup + sweeps) / dt, unit="sweeps/s", cores=procs,
                kind="oracle",
                sample="%d chains x (%d+%d) sweeps of the beta=40 U=4.5 L=400 workload, "
                       "one chain per process, %d processes, %.1f s" % (sample_chains, warmup,
                                                                           sweeps, procs, dt))


def _oracle_chain(args):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    c, warmup, sweeps = args
    from oracle import bath as OB
    from oracle import hfqmc as OH
    w = WORKLOAD
    g0 = OB.bath_to_tau(OB.semicircle_iw(w["beta"], w["t"], 20000), w["t"] ** 2, w["beta"], w["L"])
    OH.run_chain(g0, w["U"], w["beta"], w["seed"], chain=c, warmup=warmup, sweeps=sweeps, n_rec=100)
    return c


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="rank1", choices=["rank1", "delayed", "mixed"])
    ap.add_argument("--delay-k", type=int, default=0)
    ap.add_argument("--chain-sweeps", type=int, default=None,
                    help="measured sweeps per chain (default: the workload's 2000)")
    ap.add_argument("--chain-warmup", type=int, default=None)
    ap.add_argument("--rank1-sweeps", type=int, default=40,
                    help="measured sweeps of the plain FP64 comparison solve (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-chains", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported "
              "(independent chains shard across GPUs, see DESIGN.md)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_0801_1222_amd as P

    w = dict(WORKLOAD)
    if args.chain_sweeps is not None:
        w["sweeps"] = args.chain_sweeps
    if args.chain_warmup is not None:
        w["warmup"] = args.chain_warmup
    L = w["L"]
    bath = P.bethe_semicircle_bath(w["beta"], w["t"], 20000)
    g0 = P.bath_to_tau(bath, w["t"] ** 2, w["beta"], L)
    ctx = P.Context(0)
    stream = torch.cuda.current_stream()
    ctx.set_stream(stream)

    def solve(mode, warmup, sweeps):
        return P.hfqmc_solve(ctx, g0, w["U"], w["beta"], w["dtau"], w["seed"],
                             n_chains=w["n_chains"], warmup=warmup, sweeps=sweeps, mode=mode,
                             delay_k=args.delay_k)

    for _ in range(args.warmup):
        solve(args.mode, w["warmup"], w["sweeps"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for _ in range(args.steps):
        outs.append(solve(args.mode, w["warmup"], w["sweeps"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    chain_sweeps = w["n_chains"] * (w["warmup"] + w["sweeps"])
    value = chain_sweeps * args.steps / elapsed
    kern = [o["stats"]["seconds_kernel"] for o in outs]
    st = outs[-1]["stats"]
    k_used = st["delay_k"]
    by, fl = algorithmic_work(L, st, w["n_chains"], w["sweeps"], args.mode, max(k_used, 1))
    t_k = float(np.mean(kern))
    achieved = by / t_k / 1e9
    g = outs[-1]["g"]
    checks = dict(
        ph_symmetry_max=float(np.abs(g[1:L] - g[1:L][::-1]).max()),
        g0_minus_half=float(abs(g[0] - 0.5)),
        max_drift=float(st["max_drift"]),
        acc_rate=float(st["acc_rate"]),
        bad_ratios=int(st["n_bad_ratio"]),
        docc=float(outs[-1]["D"]),
        docc_err=float(outs[-1]["D_err"]),
    )
    rank1 = None
    if args.rank1_sweeps > 0 and args.mode != "rank1":
        r = solve("rank1", 0, args.rank1_sweeps)
        rank1 = dict(sweeps_per_s=w["n_chains"] * args.rank1_sweeps / r["stats"]["seconds_kernel"],
                     chain_sweeps=w["n_chains"] * args.rank1_sweeps,
                     kernel_s=r["stats"]["seconds_kernel"])
    cpu = None
    if not args.no_cpu_baseline:
        procs = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        procs = max(1, min(procs, 16))
        n_ch = args.cpu_chains or procs
        cpu = cpu_baseline(n_ch, 0, 2, procs)
    line = {
        "metric": "HF-QMC sweeps/s (all chains, L=400)",
        "value": value,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.mode != "mixed" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "half-filled Bethe-lattice impurity beta=40 U=4.5 dtau=0.1 L=400, "
                               "256 chains x (%d+%d) sweeps" % (w["warmup"], w["sweeps"]),
                   "mode": args.mode, "delay_k": k_used, "recompute_every": st["recompute_every"],
                   "n_chains": w["n_chains"], "L": L, "parallelism": "chains"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_sweeps", "kernel_ms": t_k * 1e3,
                     "fp64_tflops": fl / t_k / 1e12},
        "rank1_fp64": rank1,
        "cpu_baseline": cpu,
        "checks": checks,
        "phases_chain_s": {k: st[k] for k in ("chain_s_sweep", "chain_s_flush",
                                              "chain_s_recompute", "chain_s_measure",
                                              "chain_s_lu_build", "chain_s_lu_panel",
                                              "chain_s_lu_strip", "chain_s_lu_back")},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
