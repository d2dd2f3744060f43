"""Throughput of the Hirsch-Fye QMC hot path on one MI355X.

Workload (the headline configuration): half-filled single-band Hubbard
impurity, Bethe-lattice semicircular DOS (t = 1), beta = 40, U = 4.5,
dtau = 0.1 (L = 400), 256 independent chains (seeds 0..255), 200 warm-up +
2000 measured sweeps per chain.  One step = one full solve of that workload
(all chains, all sweeps: chain init, Metropolis sweeps, delayed updates,
Dyson recomputes, measurement and chain reduction) in one persistent launch.

Prints ONE JSON line on stdout with the production path's sweeps/s over all
chains, the plain FP64 rank-1 path timed beside it on the same chains, the
roofline of the persistent sweep kernel (k_sweeps) from HIP events, and the
CPU oracle timed on a bounded sample of the workload.  Progress goes to stderr.

  python bench.py                      # mixed precision, autotuned k (default)
  python bench.py --mode delayed       # delayed rank-k, FP64 flush
  python bench.py --delay-k 64         # fixed k instead of the autotuner
  python bench.py --calib-copy         # copy kernel used to scale PMC counters

Other workloads (one JSON line per DMFT iteration, then a summary line):

  python bench.py --workload c5 --iterations 3 --state c5.json
      the eight-grid multigrid DMFT cycle near the Mott transition: beta = 100,
      U = 4.8, dtau 0.4 .. 0.05 (L = 250 .. 2000), 32 chains per grid, mixed
      path with autotuned k, single-matrix form, 4001-point fine grid; the bath,
      iteration count and history are kept in --state, so a run of many
      iterations can be split over several calls (each call continues the
      random streams where the last one stopped)
  python bench.py --workload range-scan
      the grid-range bias of the multigrid fixed point (the study of Fig. 4):
      U = 4, beta = 45, the DMFT cycle converged separately on three dtau
      ranges of five grids each; D of the last iterations per range
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
KERNEL_SRC = os.path.join(ROOT, "paper_0801_1222_amd", "csrc", "hfqmc_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweeps_traffic.json")

WORKLOAD = dict(beta=40.0, U=4.5, dtau=0.1, L=400, n_chains=256, warmup=200, sweeps=2000,
                t=1.0, seed=0)

_T0 = time.perf_counter()


def progress(msg):
    print("[bench %7.1fs] %s" % (time.perf_counter() - _T0, msg), file=sys.stderr, flush=True)


def algorithmic_work(L, st, n_chains, measured_sweeps, mode, spins=2, dense=False):
    """Algorithmic HBM bytes and FP64/FP32 flops of one solve.

    Per unit (both spins, L x L FP64 Green matrices; with spins=1, the
    particle-hole symmetric single-matrix form, every figure halves):
      rank-1 accepted flip     32 L^2 bytes (read + write G), 4 L^2 FP64 flops
      delayed flush of rank m  32 L^2 bytes; its flips cost 4 L^2 flops each
                               (FP32 in the mixed path, FP64 otherwise)
      Dyson recompute          24 L^2 bytes (read G0 twice, write G); the FP64 flops
                               the recompute executes (executed_recompute_flops: the
                               reduced system's LU, solves and product), or with
                               dense=True those of the full solve, 2 (8/3) L^3
      measurement              16 L^2 bytes
    The accepted-flip, flush and recompute counts come from the kernel's stats.
    """
    L2 = float(L) * L
    n_acc = st["n_accepted"]
    n_rec = st["n_recomputes"] + n_chains            # plus the initial recompute of each chain
    n_flush = st.get("n_flushes", 0)
    meas = float(n_chains) * measured_sweeps
    if mode == "rank1":
        upd_bytes = 32.0 * L2 * n_acc
        f64, f32 = 4.0 * L2 * n_acc, 0.0
    else:
        upd_bytes = 32.0 * L2 * n_flush
        f64, f32 = (0.0, 4.0 * L2 * n_acc) if mode == "mixed" else (4.0 * L2 * n_acc, 0.0)
    bytes_ = upd_bytes + 16.0 * L2 * meas + 24.0 * L2 * n_rec
    h = spins / 2.0
    if dense:
        f64 += n_rec * 2.0 * (8.0 / 3.0) * L2 * L
    else:
        # (already per spin form: executed_recompute_flops counts the solves it is given)
        f64 += executed_recompute_flops(L, st, n_chains, spins) / h
    return bytes_ * h, f64 * h, f32 * h


def executed_recompute_flops(L, st, n_chains, spins=2):
    """FP64 flops the recompute actually executes.

    Reduced form (the default): per spin solve with |S| = s rows, an LU of the
    s x s system (2/3 s^3), its forward and back substitution on L right-hand
    sides (2 s^2 L) and the GEMM for the other L - s rows (2 (L - s) s L);
    |S| is the mean over all solves (stats n_reduced_rows).  Full form:
    (8/3) L^3 per spin.
    """
    n_solves = spins * (st["n_recomputes"] + n_chains)
    if not st.get("recompute_reduced"):
        return n_solves * (8.0 / 3.0) * float(L) ** 3
    s = st["n_reduced_rows"] / max(n_solves, 1.0)
    return n_solves * ((2.0 / 3.0) * s ** 3 + 2.0 * s * s * L + 2.0 * (L - s) * s * L)


def composite_bound_s(L, st, n_chains, measured_sweeps, mode, spins=2):
    """Sum over phases of max(bytes / HBM peak, flops / matrix-core peak) (phases not
    overlapped); the recompute's flops are those it executes."""
    L2 = float(L) * L
    n_acc = st["n_accepted"]
    n_rec = st["n_recomputes"] + n_chains
    n_flush = st.get("n_flushes", 0)
    bw, f64p, f32p = HBM_PEAK_GBS * 1e9, FP64_PEAK_TFLOPS * 1e12, FP32_PEAK_TFLOPS * 1e12
    if mode == "rank1":
        upd = max(32.0 * L2 * n_acc / bw, 4.0 * L2 * n_acc / f64p)
    else:
        upd = max(32.0 * L2 * n_flush / bw, 4.0 * L2 * n_acc / (f32p if mode == "mixed" else f64p))
    rec_f = executed_recompute_flops(L, st, n_chains, spins) * 2.0 / spins
    rec = max(24.0 * L2 * n_rec / bw, rec_f / f64p)
    meas = 16.0 * L2 * n_chains * measured_sweeps / bw
    return (upd + rec + meas) * spins / 2.0


def roofline(L, st, n_chains, measured_sweeps, mode, t_kernel, spins=2):
    """Roofline entry of the sweep kernel: the resource whose lower-bound time is largest.

    Flops are those the kernel executes (the reduced recompute's, not the full
    solve's); the full-solve figure is kept under "dense_recompute"."""
    by, f64, f32 = algorithmic_work(L, st, n_chains, measured_sweeps, mode, spins)
    t_hbm = by / (HBM_PEAK_GBS * 1e9)
    t_mfma = f64 / (FP64_PEAK_TFLOPS * 1e12) + f32 / (FP32_PEAK_TFLOPS * 1e12)
    hbm = {"bound": "hbm", "achieved": by / t_kernel / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    # matrix-core work expressed at the FP64 rate (FP32 flops count half)
    f64e = f64 + f32 * FP64_PEAK_TFLOPS / FP32_PEAK_TFLOPS
    mf = {"bound": "mfma", "achieved": f64e / t_kernel / 1e12, "peak": FP64_PEAK_TFLOPS,
          "unit": "TFLOP/s"}
    mf["frac"] = mf["achieved"] / mf["peak"]
    main, other = (hbm, mf) if t_hbm >= t_mfma else (mf, hbm)
    main = dict(main)
    main["secondary"] = other
    main["lower_bound_s"] = {"hbm": t_hbm, "mfma_fp64_equiv": t_mfma}
    main["algorithmic"] = {"bytes": by, "fp64_flops": f64, "fp32_flops": f32}
    main["composite_frac"] = composite_bound_s(L, st, n_chains, measured_sweeps, mode,
                                               spins) / t_kernel
    # the same work with the recompute priced as the full (8/3) L^3 solve per spin
    _, f64d, _ = algorithmic_work(L, st, n_chains, measured_sweeps, mode, spins, dense=True)
    f64de = f64d + f32 * FP64_PEAK_TFLOPS / FP32_PEAK_TFLOPS
    main["dense_recompute"] = {
        "fp64_flops": f64d,
        "fp64_equiv_tflops": f64de / t_kernel / 1e12,
        "frac": f64de / t_kernel / 1e12 / FP64_PEAK_TFLOPS,
        "mean_reduced_rows": st["n_reduced_rows"]
        / max(spins * (st["n_recomputes"] + n_chains), 1.0),
        "note": "algorithmic flops of the full L x L solve the reduced recompute replaces; "
                "not executed"}
    return main


def add_measured_peaks(entry, peaks):
    """Fraction of the achievable peak the library's probe kernels measured."""
    if not peaks:
        return
    m = (max(peaks["hbm_copy_gbs"], peaks["hbm_read_gbs"]) if entry["bound"] == "hbm"
         else peaks["fp64_mfma_tflops"])
    entry["measured_peak"] = m
    entry["frac_of_measured_peak"] = entry["achieved"] / m if m > 0 else None


def batched_grids(P, ctx, name, beta, U, dtaus, n_chains, warmup, sweeps, mode, t=1.0):
    """One persistent launch over several grids; per-grid work and the whole-launch rate.

    Each grid's chain-seconds come from the kernel's own phase clocks; its
    L=400-equivalent chain-sweeps scale by (L/400)^3, the rank-1 cost law.
    """
    Ls = [int(round(beta / d)) for d in dtaus]
    bath = P.bethe_semicircle_bath(beta, t, 20000)
    g0s = [P.bath_to_tau(bath, t * t, beta, L) for L in Ls]
    kw = dict(n_chains=n_chains, warmup=warmup, sweeps=sweeps, mode=mode)
    P.hfqmc_solve_grids(ctx, Ls, g0s, U, beta, 0, **kw)           # autotune, capture
    out = P.hfqmc_solve_grids(ctx, Ls, g0s, U, beta, 0, **kw)
    st = out["stats"]
    tk = st[0]["seconds_kernel"]
    per = []
    eq = 0.0
    flips = 0
    for L, s_ in zip(Ls, st):
        cs = n_chains * (warmup + sweeps)
        busy = sum(s_[k] for k in ("chain_s_sweep", "chain_s_flush", "chain_s_recompute",
                                   "chain_s_measure"))
        per.append(dict(L=L, chain_sweeps=cs, accepted=s_["n_accepted"],
                        acc_rate=s_["acc_rate"], chain_seconds=busy,
                        chain_sweeps_per_chain_s=cs / busy if busy > 0 else None,
                        recomputes=s_["n_recomputes"], delay_k=s_["delay_k"]))
        eq += cs * (L / 400.0) ** 3
        flips += s_["n_accepted"]
    return dict(workload="%s: beta=%g U=%g L=%s, %d chains per grid x (%d+%d) sweeps, mode %s"
                % (name, beta, U, Ls, n_chains, warmup, sweeps, mode),
                kernel_s=tk, chain_sweeps_per_s=sum(p_["chain_sweeps"] for p_ in per) / tk,
                l400_equiv_sweeps_per_s=eq / tk, accepted_flips_per_s=flips / tk, grids=per,
                workgroups=st[0]["n_workgroups"])


def single_chain_l20(P, ctx):
    """The smallest workload: one chain, beta=10 U=4 dtau=0.5 (L=20), seed 0,
    1000+20000 sweeps, FP64 rank-1, recompute every 100, 20 bins; beside it the
    oracle on the same chain for 100+2000 sweeps on one host core."""
    from threadpoolctl import threadpool_limits

    from oracle import bath as OB
    from oracle import hfqmc as OH
    beta, U, L = 10.0, 4.0, 20
    g0 = P.bath_to_tau(P.bethe_semicircle_bath(beta, 1.0, 20000), 1.0, beta, L)
    r = P.hfqmc_solve(ctx, g0, U, beta, beta / L, 0, n_chains=1, warmup=1000, sweeps=20000,
                      mode="rank1")
    st = r["stats"]
    g0o = OB.bath_to_tau(OB.semicircle_iw(beta, 1.0, 20000), 1.0, beta, L)
    t0 = time.perf_counter()
    with threadpool_limits(1):
        OH.run_chain(g0o, U, beta, 0, warmup=100, sweeps=2000, n_bins=20)
    dt = time.perf_counter() - t0
    return dict(workload="one chain, beta=10 U=4 dtau=0.5 (L=20), 1000+20000 sweeps, rank-1",
                sweeps_per_s=21000 / st["seconds_kernel"], kernel_s=st["seconds_kernel"],
                acc_rate=st["acc_rate"], D=float(r["D"]), D_err=float(r["D_err"]),
                g_beta_half=float(r["g"][L // 2]), g_beta_half_err=float(r["g_err"][L // 2]),
                oracle_sweeps_per_s=2100 / dt,
                note="latency-bound: one workgroup; oracle timed on 100+2000 sweeps, 1 core")


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(mode, chain_sweeps):
    """HBM bytes per launch from committed PMC counters, if taken on this kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        tr = json.load(f)
    if tr.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    ent = tr.get("modes", {}).get(mode)
    if not ent:
        return None
    # counters were taken on a shorter run of the same chains: scale per chain-sweep
    return ent["bytes_per_chain_sweep"] * chain_sweeps


def cpu_baseline(sample_chains, warmup, sweeps, procs):
    """Oracle (as it stands) on the host cores over a bounded sample of the workload."""
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        pool.map(_oracle_chain, [(c, warmup, sweeps) for c in range(sample_chains)])
    dt = time.perf_counter() - t0
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(value=sample_chains * (warmup + sweeps) / dt, unit="sweeps/s", cores=procs,
                kind="oracle",
                sample="chains 0..%d of the beta=40 U=4.5 L=400 workload, %d+%d sweeps each, "
                       "FP64 rank-1 with recompute every 100, one chain per process, "
                       "%d processes x 1 BLAS thread on %s, %.1f s wall"
                       % (sample_chains - 1, warmup, sweeps, procs, model, dt))


def _oracle_chain(args):
    c, warmup, sweeps = args
    from threadpoolctl import threadpool_limits

    from oracle import bath as OB
    from oracle import hfqmc as OH
    w = WORKLOAD
    with threadpool_limits(1):
        g0 = OB.bath_to_tau(OB.semicircle_iw(w["beta"], w["t"], 20000), w["t"] ** 2, w["beta"],
                            w["L"])
        OH.run_chain(g0, w["U"], w["beta"], w["seed"], chain=c, warmup=warmup, sweeps=sweeps,
                     n_rec=100)
    return c


def calib_copy():
    """A plain device copy of known size, profiled to scale FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = 1 << 28                                   # 2 GiB of FP64 read, 2 GiB written
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read": 8 * n, "calib_copy_bytes_written": 8 * n}))


C5_DTAUS = [0.4, 0.35, 0.3, 0.25, 0.2, 0.15, 0.1, 0.05]     # L = 250 .. 2000 at beta = 100
RANGES = {"[0.2,0.5]": [0.2, 0.25, 0.3, 0.4, 0.5],
          "[0.3,0.7]": [0.3, 0.4, 0.5, 0.6, 0.7],
          "[0.35,0.8]": [0.35, 0.45, 0.55, 0.65, 0.8]}


def _cycle_opts(args, mode, balance=False):
    return dict(n_chains=args.chains, warmup=args.chain_warmup, sweeps=args.chain_sweeps,
                mode=mode, delay_k=args.delay_k if mode != "rank1" else 0, ph=not args.two_matrix,
                balance=balance)


def workload_c5(args):
    """The eight-grid multigrid DMFT cycle, resumable through a JSON state file."""
    import paper_0801_1222_amd as P
    beta, t, U = 100.0, 1.0, args.U
    n_iw, n_fine = 8192, 4001
    st = None
    if args.state and os.path.exists(args.state):
        with open(args.state) as f:
            st = json.load(f)
        if st["beta"] != beta or st["U"] != U:
            raise SystemExit("state file %s is for beta=%g U=%g" % (args.state, st["beta"], st["U"]))
        bath = np.array(st["bath_re"]) + 1j * np.array(st["bath_im"])
    else:
        bath = P.bethe_semicircle_bath(beta, t, n_iw)
        st = dict(beta=beta, U=U, iterations=0, history=[])
    ctx = P.Context(0)
    mode = args.mode
    kw = _cycle_opts(args, mode, balance=not args.no_balance)
    Ls = [int(round(beta / d)) for d in C5_DTAUS]
    # the split the library plans for one workgroup per CU (256 on MI355X)
    split = (P.hfqmc_plan_balance(Ls, kw["n_chains"], kw["warmup"], kw["sweeps"], 1, 256)["factor"]
             if kw["balance"] else [1] * len(Ls))
    progress("c5: beta=%g U=%g L=%s, %d chains x (%d+%d) sweeps per grid and iteration, mode %s%s, "
             "chain split %s" % (beta, U, Ls, kw["n_chains"], kw["warmup"], kw["sweeps"], mode,
                                 ", single-matrix form" if kw["ph"] else "", split))
    for _ in range(args.iterations):
        it = st["iterations"]
        t0 = time.perf_counter()
        r = P.dmft_solve(ctx, U, beta, t, C5_DTAUS, args.seed + (it << 32), 1, bath_iw=bath,
                         n_fine=n_fine, mixing=args.mixing, **kw)
        dt = time.perf_counter() - t0
        bath = r["bath"]
        h = r["history"][0]
        g = r["g"]
        # the change of G(tau) against the previous iteration (a call of one
        # iteration measures against the bath's own G0(tau), kept as max_dg_bath)
        prev = st.get("g_prev")
        max_dg = float(np.abs(g - np.array(prev)).max()) if prev is not None else None
        rec = dict(workload="c5", iteration=it, U=U, beta=beta, Ls=Ls, D=float(h[2]),
                   D_err=float(h[3]), max_dg=max_dg, max_dg_bath=float(h[0]),
                   max_g_err=float(h[1]),
                   g_beta_half=float(g[(n_fine - 1) // 2]),
                   g_beta_half_err=float(r["g_err"][(n_fine - 1) // 2]), seconds=dt,
                   chains=kw["n_chains"], warmup=kw["warmup"], sweeps=kw["sweeps"],
                   chain_split=split, mode=mode,
                   single_matrix=kw["ph"], mixing=args.mixing)
        st["history"].append(rec)
        st["iterations"] = it + 1
        st["bath_re"] = bath.real.tolist()
        st["bath_im"] = bath.imag.tolist()
        st["g_prev"] = g.tolist()
        if args.state:
            tmp = args.state + ".tmp"
            with open(tmp, "w") as f:
                json.dump(st, f)
            os.replace(tmp, args.state)
        print(json.dumps(rec), flush=True)
        progress("c5 iteration %d: D = %.5f(%d), max |dG| vs previous %s, %.0f s"
                 % (it, rec["D"], round(rec["D_err"] * 1e5),
                    "%.2e" % max_dg if max_dg is not None else "-", dt))
    ctx.close()
    hist = st["history"]
    print(json.dumps(dict(workload="c5", summary=True, iterations=st["iterations"],
                          D=[h_["D"] for h_ in hist], D_err=[h_["D_err"] for h_ in hist],
                          max_dg=[h_["max_dg"] for h_ in hist],
                          seconds_per_iteration=[h_["seconds"] for h_ in hist])), flush=True)


def workload_batched(args):
    """The two batched multigrid configurations at full length: one multigrid
    step each (one persistent launch over the grids, then interpolation and the
    extrapolation in dtau^2 on the host), with its time and results."""
    import paper_0801_1222_amd as P
    ctx = P.Context(0)
    cases = [("seven grids", 20.0, 4.8, [0.4, 1 / 3, 2 / 7, 0.25, 0.2, 1 / 6, 0.125], 64, "rank1", 0),
             ("three grids", 50.0, 5.0, [0.125, 0.1, 0.0625], 128, "mixed", 0)]
    for name, beta, U, dtaus, nch, mode, k in cases:
        bath = P.bethe_semicircle_bath(beta, 1.0, 8192)
        kw = dict(n_fine=200, n_chains=nch, warmup=200, sweeps=2000, mode=mode, delay_k=k)
        # a short call first: the autotuner's trials and the graph capture stay out of the timing
        P.multigrid_solve(ctx, bath, 1.0, U, beta, dtaus, 1, **dict(kw, warmup=0, sweeps=2))
        t0 = time.perf_counter()
        r = P.multigrid_solve(ctx, bath, 1.0, U, beta, dtaus, 0, **kw)
        dt = time.perf_counter() - t0
        st = r["stats"]
        mid = (kw["n_fine"] - 1) // 2
        rec = dict(workload="batched", name=name, beta=beta, U=U, Ls=r["Ls"], chains=nch,
                   warmup=kw["warmup"], sweeps=kw["sweeps"], mode=mode,
                   delay_k=st[0]["delay_k"], seconds_call=dt,
                   seconds_kernel=st[0]["seconds_kernel"],
                   D_grids=[float(x) for x in r["D_grids"]],
                   D_err_grids=[float(x) for x in r["D_err_grids"]],
                   D=r["D"], D_err=r["D_err"], g_beta_half=float(r["g"][mid]),
                   g_beta_half_err=float(r["g_err"][mid]),
                   max_drift_grids=[s_["max_drift"] for s_ in st],
                   max_drift_gtau_grids=[s_["max_drift_gtau"] for s_ in st])
        print(json.dumps(rec), flush=True)
        progress("%s: %.1f s (kernel %.1f s), D = %.4f(%d), G(beta/2) = %.4f(%d)"
                 % (name, dt, rec["seconds_kernel"], r["D"], round(r["D_err"] * 1e4),
                    rec["g_beta_half"], round(rec["g_beta_half_err"] * 1e4)))
    ctx.close()


def workload_range_scan(args):
    """Grid-range bias of the multigrid DMFT fixed point: one cycle per dtau range from a
    common start; D and its error from the last iterations of each range."""
    import paper_0801_1222_amd as P
    beta, t, U = 45.0, 1.0, args.U
    ctx = P.Context(0)
    kw = _cycle_opts(args, args.mode)
    # common start: a short cycle on the middle range
    start = P.dmft_solve(ctx, U, beta, t, RANGES["[0.3,0.7]"], args.seed, args.iterations,
                         n_iw=4096, n_fine=451, mixing=args.mixing, **kw)["bath"]
    progress("range scan: common start after %d iterations" % args.iterations)
    out = {}
    for i, (name, dts) in enumerate(RANGES.items()):
        r = P.dmft_solve(ctx, U, beta, t, dts, args.seed + ((i + 1) << 40), args.scan_iterations,
                         bath_iw=start, n_fine=451, mixing=args.mixing, **kw)
        d = r["history"][:, 2]
        tail = d[args.scan_iterations // 4:]
        rec = dict(workload="range-scan", range=name, dtaus=dts,
                   Ls=[int(round(beta / x)) for x in dts], D=float(np.mean(tail)),
                   D_err=float(np.std(tail, ddof=1) / np.sqrt(len(tail))), D_history=d.tolist(),
                   chains=kw["n_chains"], warmup=kw["warmup"], sweeps=kw["sweeps"],
                   mode=args.mode, single_matrix=kw["ph"])
        out[name] = rec
        print(json.dumps(rec), flush=True)
        progress("range %s: D = %.5f(%d)" % (name, rec["D"], round(rec["D_err"] * 1e5)))
    ref = out["[0.2,0.5]"]
    print(json.dumps(dict(workload="range-scan", summary=True, U=U, beta=beta,
                          shift_vs_0205={k: v["D"] - ref["D"] for k, v in out.items()},
                          shift_err={k: float(np.hypot(v["D_err"], ref["D_err"]))
                                     for k, v in out.items()})), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="mixed", choices=["rank1", "delayed", "mixed"])
    ap.add_argument("--delay-k", type=int, default=0,
                    help="delayed rank k (0 = autotuned over 16/32/64 and the LU panel width)")
    ap.add_argument("--chain-sweeps", type=int, default=None,
                    help="measured sweeps per chain (default: the workload's 2000)")
    ap.add_argument("--chain-warmup", type=int, default=None,
                    help="warm-up sweeps per chain (default: the workload's 200)")
    ap.add_argument("--rank1-sweeps", type=int, default=40,
                    help="sweeps per chain of the plain FP64 rank-1 comparison solve (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=300)
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("--g-fp32", action="store_true",
                    help="time the mixed path with G stored in FP32 between recomputes")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the peak probes and the small-L / three-grid workloads")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "c5", "range-scan", "batched"])
    ap.add_argument("--iterations", type=int, default=None,
                    help="c5: DMFT iterations in this call (default 1); range-scan: "
                         "iterations to the common start (default 6)")
    ap.add_argument("--scan-iterations", type=int, default=16,
                    help="range-scan: DMFT iterations per dtau range")
    ap.add_argument("--state", default=None, help="c5: JSON state file (resume and save)")
    ap.add_argument("--U", type=float, default=None,
                    help="c5: U (default 4.8); range-scan: U (default 4)")
    ap.add_argument("--chains", type=int, default=None)
    ap.add_argument("--mixing", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-balance", action="store_true",
                    help="c5: every grid runs its chains end to end (no chain split)")
    ap.add_argument("--two-matrix", action="store_true",
                    help="c5 / range-scan: both Green matrices (default: single-matrix form)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported "
              "(independent chains would shard across GPUs with one all-reduce of the "
              "accumulators per multigrid step)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy()
        return
    if args.workload != "headline":
        import torch  # noqa: F401  (PyTorch's runtime comes up before the library's)
        if args.workload == "c5":
            args.U = 4.8 if args.U is None else args.U
            args.chains = args.chains or 32
            args.chain_warmup = 100 if args.chain_warmup is None else args.chain_warmup
            args.chain_sweeps = args.chain_sweeps or 1000
            args.iterations = 1 if args.iterations is None else args.iterations
            workload_c5(args)
        elif args.workload == "batched":
            workload_batched(args)
        else:
            args.U = 4.0 if args.U is None else args.U
            args.chains = args.chains or 256
            args.chain_warmup = 100 if args.chain_warmup is None else args.chain_warmup
            args.chain_sweeps = args.chain_sweeps or 2000
            args.mode = "delayed" if args.mode == "mixed" else args.mode
            args.iterations = 6 if args.iterations is None else args.iterations
            workload_range_scan(args)
        return

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
    progress("context ready; mode %s, %d chains x (%d+%d) sweeps per step"
             % (args.mode, w["n_chains"], w["warmup"], w["sweeps"]))

    def solve(mode, warmup, sweeps):
        # host-pointer entry (bath and results cross PCIe; used for the warm-up step)
        return P.hfqmc_solve(ctx, g0, w["U"], w["beta"], w["dtau"], w["seed"],
                             n_chains=w["n_chains"], warmup=warmup, sweeps=sweeps, mode=mode,
                             delay_k=args.delay_k if mode != "rank1" else 0,
                             g_fp32=args.g_fp32 and mode == "mixed")

    # device-resident input and outputs for the timed steps
    g0_d = torch.tensor(g0, dtype=torch.float64, device="cuda")
    g_d = torch.zeros(L + 1, dtype=torch.float64, device="cuda")
    e_d = torch.zeros(L + 1, dtype=torch.float64, device="cuda")
    d_d = torch.zeros(2, dtype=torch.float64, device="cuda")

    def solve_dev():
        return P.hfqmc_solve_dev(ctx, g0_d.data_ptr(), L, w["U"], w["beta"], w["dtau"], w["seed"],
                                 g_d.data_ptr(), e_d.data_ptr(), d_d.data_ptr(),
                                 n_chains=w["n_chains"], warmup=w["warmup"], sweeps=w["sweeps"],
                                 mode=args.mode,
                                 delay_k=args.delay_k if args.mode != "rank1" else 0,
                                 g_fp32=args.g_fp32)

    chain_sweeps = w["n_chains"] * (w["warmup"] + w["sweeps"])
    host_rate = None
    tune = None
    for i in range(args.warmup):
        r = solve(args.mode, w["warmup"], w["sweeps"])
        rs = r["stats"]
        host_rate = chain_sweeps / (rs["seconds_total"] - rs["seconds_autotune"])
        if rs["autotuned"] and rs["seconds_autotune"] > 0:
            tune = dict(delay_k=rs["delay_k"], lu_panel=rs["lu_panel"],
                        seconds=rs["seconds_autotune"])
        progress("warmup step %d done, kernel %.2f s (autotune %.2f s)"
                 % (i, rs["seconds_kernel"], rs["seconds_autotune"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    step_s = []
    for i in range(args.steps):
        ts = time.perf_counter()
        stats.append(solve_dev())
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - ts)
        progress("timed step %d done, kernel %.2f s" % (i, stats[-1]["seconds_kernel"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = chain_sweeps * args.steps / elapsed
    st = stats[-1]
    # HIP events: around the whole captured launch sequence, and around the
    # persistent sweep kernel alone (the roofline's kernel)
    t_launch = float(np.mean([s_["seconds_kernel"] for s_ in stats]))
    t_k = float(np.mean([s_["seconds_sweep_kernel"] for s_ in stats]))
    rf = roofline(L, st, w["n_chains"], w["sweeps"], args.mode, t_k)
    rf["traffic"] = measured_traffic(args.mode, chain_sweeps)
    rf["kernel"] = "k_sweeps"
    rf["kernel_ms"] = t_k * 1e3
    rf["launch_ms"] = t_launch * 1e3
    g = g_d.cpu().numpy()
    ge = e_d.cpu().numpy()
    dd = d_d.cpu().numpy()
    checks = dict(
        ph_symmetry_max=float(np.abs(g[1:L] - g[1:L][::-1]).max()),
        g0_minus_half=float(abs(g[0] - 0.5)),
        max_elementwise_drift=float(st["max_drift"]),
        max_gtau_drift=float(st["max_drift_gtau"]),
        drift_sampling="first and every 8th recompute of each chain",
        acc_rate=float(st["acc_rate"]),
        bad_ratios=int(st["n_bad_ratio"]),
        singular=int(st["n_singular"]),
        docc=float(dd[0]),
        docc_err=float(dd[1]),
        g_beta_half=float(g[L // 2]),
        g_beta_half_err=float(ge[L // 2]),
    )
    peaks = None
    extra = {}
    if not args.no_extra:
        peaks = P.hfqmc_measure_peaks(ctx)
        progress("measured peaks: copy %.0f GB/s, read %.0f GB/s, FP64 MFMA %.1f TF/s, "
                 "FP32 MFMA %.1f TF/s, FP64 FMA %.1f TF/s"
                 % (peaks["hbm_copy_gbs"], peaks["hbm_read_gbs"], peaks["fp64_mfma_tflops"],
                    peaks["fp32_mfma_tflops"], peaks["fp64_fma_tflops"]))
        # small grids, FP64 rank-1, all in one launch: latency of the per-flip dependency
        small = batched_grids(P, ctx, "seven grids", 20.0, 4.8,
                              [0.4, 1 / 3, 2 / 7, 0.25, 0.2, 1 / 6, 0.125], 64, 200, 2000, "rank1")
        small["full_length"] = True
        fl = sum(4.0 * g_["L"] ** 2 * g_["accepted"] for g_ in small["grids"])
        small["fp64_update_tflops"] = fl / small["kernel_s"] / 1e12
        small["frac_of_measured_fp64_fma"] = (small["fp64_update_tflops"] / peaks["fp64_fma_tflops"]
                                              if peaks["fp64_fma_tflops"] > 0 else None)
        extra["small_grids_rank1"] = small
        progress("seven small grids (rank-1): %.0f chain-sweeps/s, %.3g accepted flips/s"
                 % (small["chain_sweeps_per_s"], small["accepted_flips_per_s"]))
        three = batched_grids(P, ctx, "three grids", 50.0, 5.0, [0.125, 0.1, 0.0625], 128, 2, 10,
                              "mixed")
        three["full_length"] = False
        three["note"] = ("shortened to 2+10 sweeps per chain (the full 200+2000 take about 80 s); "
                         "per-grid rates include the chain-initial recompute")
        extra["three_grids_mixed"] = three
        progress("three grids L=400/500/800 (mixed): %.0f L=400-equivalent chain-sweeps/s"
                 % three["l400_equiv_sweeps_per_s"])
        extra["single_chain_L20"] = single_chain_l20(P, ctx)
        progress("one chain, L=20, 1000+20000 sweeps: %.0f sweeps/s (oracle %.0f)"
                 % (extra["single_chain_L20"]["sweeps_per_s"],
                    extra["single_chain_L20"]["oracle_sweeps_per_s"]))
    add_measured_peaks(rf, peaks)
    add_measured_peaks(rf["secondary"], peaks)
    phv = None
    if not args.no_extra and args.mode != "rank1":
        # the same workload through the particle-hole symmetric single-matrix form
        # (the bath is symmetric): G_dn = 1 - G_up^T, one matrix updated and recomputed
        sp = P.hfqmc_solve_dev(ctx, g0_d.data_ptr(), L, w["U"], w["beta"], w["dtau"], w["seed"],
                               g_d.data_ptr(), e_d.data_ptr(), d_d.data_ptr(),
                               n_chains=w["n_chains"], warmup=w["warmup"], sweeps=w["sweeps"],
                               mode=args.mode, delay_k=args.delay_k, ph=True)
        torch.cuda.synchronize()
        rph = roofline(L, sp, w["n_chains"], w["sweeps"], args.mode, sp["seconds_sweep_kernel"],
                       spins=1)
        add_measured_peaks(rph, peaks)
        add_measured_peaks(rph["secondary"], peaks)
        gp_ = g_d.cpu().numpy()
        phv = dict(sweeps_per_s=chain_sweeps / sp["seconds_kernel"], kernel_s=sp["seconds_kernel"],
                  speedup_vs_two_matrix=t_launch / sp["seconds_kernel"], delay_k=sp["delay_k"],
                  lu_panel=sp["lu_panel"], acc_rate=sp["acc_rate"], max_drift=sp["max_drift"],
                  docc=float(d_d.cpu().numpy()[0]),
                  max_abs_dg_vs_two_matrix=float(np.abs(gp_ - g).max()),
                  roofline={k_: rph[k_] for k_ in ("bound", "achieved", "peak", "unit", "frac",
                                                    "composite_frac")},
                  note="same chains and sweeps; only G_up stored (G_dn = 1 - G_up^T holds for "
                       "a particle-hole symmetric bath); not the headline value")
        progress("single-matrix (particle-hole symmetric) form: %.0f sweeps/s" % phv["sweeps_per_s"])
    g32 = None
    if not args.no_extra and args.mode == "mixed" and not args.g_fp32:
        # the same workload with G stored in FP32 between recomputes
        s32 = P.hfqmc_solve_dev(ctx, g0_d.data_ptr(), L, w["U"], w["beta"], w["dtau"], w["seed"],
                                g_d.data_ptr(), e_d.data_ptr(), d_d.data_ptr(),
                                n_chains=w["n_chains"], warmup=w["warmup"], sweeps=w["sweeps"],
                                mode="mixed", delay_k=args.delay_k, g_fp32=True)
        torch.cuda.synchronize()
        r32 = roofline(L, s32, w["n_chains"], w["sweeps"], "mixed", s32["seconds_sweep_kernel"])
        g32_ = g_d.cpu().numpy()
        g32 = dict(sweeps_per_s=chain_sweeps / s32["seconds_kernel"], kernel_s=s32["seconds_kernel"],
                   speedup_vs_fp64_stored=t_launch / s32["seconds_kernel"], delay_k=s32["delay_k"],
                   lu_panel=s32["lu_panel"], acc_rate=s32["acc_rate"], max_drift=s32["max_drift"],
                   docc=float(d_d.cpu().numpy()[0]),
                   max_abs_dg_vs_fp64_stored=float(np.abs(g32_ - g).max()),
                   flop_roofline={k_: r32[k_] for k_ in ("bound", "achieved", "peak", "unit",
                                                          "frac")},
                   note="same chains and sweeps; G stored in FP32 between the FP64 recomputes "
                        "(half the G traffic); not the headline value")
        progress("FP32-stored G: %.0f sweeps/s" % g32["sweeps_per_s"])
    rank1 = None
    if args.rank1_sweeps > 0 and args.mode != "rank1":
        r = solve("rank1", 0, args.rank1_sweeps)
        rs = r["stats"]
        rr = roofline(L, rs, w["n_chains"], args.rank1_sweeps, "rank1", rs["seconds_sweep_kernel"])
        rank1 = dict(sweeps_per_s=w["n_chains"] * args.rank1_sweeps / rs["seconds_kernel"],
                     chain_sweeps=w["n_chains"] * args.rank1_sweeps,
                     kernel_s=rs["seconds_kernel"], recompute_every=rs["recompute_every"],
                     roofline={k: rr[k] for k in ("bound", "achieved", "peak", "unit", "frac")},
                     note="same 256 chains, 0+%d sweeps, FP64 Sherman-Morrison per accepted "
                          "flip, recompute every 100" % args.rank1_sweeps)
        progress("plain rank-1 comparison done: %.0f sweeps/s" % rank1["sweeps_per_s"])
    cpu = None
    if not args.no_cpu_baseline:
        aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        # one process per core of this process's CPU share: the GPU host grants one GPU's
        # job 16 cores whatever the affinity mask shows
        procs = max(1, min(aff, 16))
        cpu = cpu_baseline(procs, 0, args.cpu_sweeps, procs)
        cpu["affinity_cores"] = aff
        progress("cpu baseline done: %.2f sweeps/s on %d cores" % (cpu["value"], procs))
    ph = {k: st[k] for k in ("chain_s_sweep", "chain_s_flush", "chain_s_recompute",
                             "chain_s_measure", "chain_s_lu_build", "chain_s_lu_panel",
                             "chain_s_lu_strip", "chain_s_lu_back", "chain_s_lu_gemm",
                             "chain_s_flush_vectors", "chain_s_flush_gemm",
                             "chain_s_window_apply", "chain_s_fold")}
    line = {
        "metric": "HF-QMC sweeps/s (all chains, L=400)",
        "value": value,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "step_ms": [x * 1e3 for x in step_s],
        "median_step_sweeps_per_s": chain_sweeps / float(np.median(step_s)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f64+f32", "delayed": "f64", "rank1": "f64"}[args.mode],
        "data": "synthetic",
        "config": {"workload": "half-filled Bethe-lattice impurity (t=1) beta=40 U=4.5 "
                               "dtau=0.1 L=400, 256 chains x (%d+%d) sweeps"
                               % (w["warmup"], w["sweeps"]),
                   "mode": args.mode, "delay_k": st["delay_k"],
                   "recompute_every": st["recompute_every"], "n_chains": w["n_chains"], "L": L,
                   "workgroups": st["n_workgroups"], "lu_panel": st["lu_panel"],
                   "graph": bool(st["graph"]), "autotuned": bool(st["autotuned"]),
                   "g_fp32": bool(args.g_fp32)},
        "autotune": tune,
        "host_entry_sweeps_per_s": host_rate,
        "roofline": rf,
        "plain_fp64_rank1": rank1,
        "speedup_vs_rank1": (chain_sweeps / t_launch) / rank1["sweeps_per_s"] if rank1 else None,
        "cpu_baseline": cpu,
        "checks": checks,
        "phases_chain_s": ph,
        "kernel_sweeps_per_s": chain_sweeps / t_launch,
        "measured_peaks": peaks,
        "ph_single_matrix": phv,
        "fp32_stored_g": g32,
        "other_workloads": extra or None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
