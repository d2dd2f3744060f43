"""Python face of libhfqmc with the C-ABI's names (marshalling only).

  ctx = Context(0)
  out = hfqmc_solve(ctx, g0_tau, U, beta, dtau, seed, n_chains=..., ...)
  hfqmc_solve_dev(ctx, g0_dev, L, U, beta, dtau, seed, g_dev, ...)   # device pointers
  out = hfqmc_solve_grids(ctx, Ls, [g0_tau_i], U, beta, seed, ...)
  out = multigrid_solve(ctx, bath_iw, m3, U, beta, dtaus, seed, n_fine, ...)
  new_bath = dmft_bethe_step(g_fine, bath_iw, m3, U, beta, t)
  out = dmft_solve(ctx, U, beta, t, dtaus, seed, n_iter, ...)        # the whole DMFT cycle
  peaks = hfqmc_measure_peaks(ctx)                                    # achievable peaks
"""
import ctypes as C
import sys

import numpy as np

from . import _native as N
from ._native import HFQMCError  # noqa: F401

MODES = {"rank1": 0, "delayed": 1, "mixed": 2}


class Context:
    """Owns one hfqmc_ctx (device buffers, stream binding).

    PyTorch-ROCm ships its own HIP runtime next to the one this library links;
    both drive the same device through one HSA runtime, so device addresses are
    shared, but PyTorch's runtime must come up first: when torch is imported,
    its device is initialised before the context is created.
    """

    def __init__(self, device=0):
        torch = sys.modules.get("torch")
        if torch is not None and torch.cuda.is_available():
            torch.cuda.init()
        self._p = C.c_void_p()
        N.check(N.lib.hfqmc_create(C.byref(self._p), int(device)), "hfqmc_create")

    def set_stream(self, stream):
        """Bind a HIP stream: a raw handle of this library's runtime, None, or a
        torch.cuda.Stream that is the null stream (PyTorch's other streams belong
        to its own runtime and cannot be shared)."""
        handle = getattr(stream, "cuda_stream", stream)
        if hasattr(stream, "cuda_stream") and handle:
            raise ValueError("only PyTorch's null stream can be shared with libhfqmc")
        N.check(N.lib.hfqmc_set_stream(self._p, C.c_void_p(handle or 0)), "hfqmc_set_stream")

    @property
    def handle(self):
        return self._p

    def close(self):
        if self._p:
            N.lib.hfqmc_destroy(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _flags(eager=False, heat_bath=False, direct=False, ph=False, g_fp32=False, balance=False):
    return ((N.FLAG_EAGER if eager else 0) | (N.FLAG_HEAT_BATH if heat_bath else 0)
            | (N.FLAG_DIRECT_RECOMPUTE if direct else 0)
            | (N.FLAG_PH_SYMMETRIC if ph else 0) | (N.FLAG_G_FP32 if g_fp32 else 0)
            | (N.FLAG_BALANCE if balance else 0))


def _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit, flags=0,
          drift_every=0):
    o = N.Opts()
    o.drift_every = int(drift_every)
    o.flags = int(flags)
    o.n_chains = int(n_chains)
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.warmup = int(warmup)
    o.sweeps = int(sweeps)
    o.recompute_every = int(recompute_every)
    o.delay_k = int(delay_k)
    o.n_bins = int(n_bins)
    o.drift_limit = float(drift_limit)
    return o


class _Hooks:
    """Host buffers of the optional test hooks, kept alive for the call."""

    def __init__(self, o, n_grids, n_chains, Ls, n_bins, flip_cap, replay, want_chain, want_green,
                 spins=1):
        self.keep = []
        self.n_grids, self.n_chains, self.Ls = n_grids, n_chains, list(Ls)
        self.spins = spins   # 2: spin-resolved estimators, [..][2][L+1] per sample
        nb = n_bins if n_bins > 0 else (20 if n_chains == 1 else 1)
        self.n_bins = nb
        self.flip_log = self.flip_count = None
        if flip_cap:
            self.flip_log = np.zeros((n_grids, n_chains, flip_cap), dtype=np.int64)
            self.flip_count = np.zeros((n_grids, n_chains), dtype=np.int64)
            o.flip_log = N.ptr(self.flip_log, C.c_int64)
            o.flip_count = N.ptr(self.flip_count, C.c_int64)
            o.flip_cap = int(flip_cap)
        if replay is not None:
            # replay: nested lists [grid][chain] -> sequence of flip codes sweep*L + l
            cap = max(1, max(len(c) for g in replay for c in g))
            rl = np.zeros((n_grids, n_chains, cap), dtype=np.int64)
            rc = np.zeros((n_grids, n_chains), dtype=np.int64)
            for gi, g in enumerate(replay):
                for ci, c in enumerate(g):
                    rl[gi, ci, :len(c)] = c
                    rc[gi, ci] = len(c)
            self.keep += [rl, rc]
            o.replay_log = N.ptr(rl, C.c_int64)
            o.replay_count = N.ptr(rc, C.c_int64)
            o.replay_cap = cap
        self.chain_g = self.chain_d = self.chain_n = self.chain_drift = None
        if want_chain:
            tot = sum(spins * (L + 1) for L in Ls)
            self.chain_g = np.zeros(n_chains * nb * tot)
            self.chain_d = np.zeros((n_grids, n_chains, nb))
            self.chain_n = np.zeros((n_grids, n_chains, nb), dtype=np.int64)
            self.chain_drift = np.zeros((n_grids, n_chains))
            o.chain_g = N.ptr(self.chain_g)
            o.chain_d = N.ptr(self.chain_d)
            o.chain_n = N.ptr(self.chain_n, C.c_int64)
            o.chain_drift = N.ptr(self.chain_drift)
        self.green = None
        if want_green:
            L = Ls[0]
            self.green = np.zeros((n_chains, 2, L, L))
            o.final_green = N.ptr(self.green)

    def results(self):
        out = {}
        if self.flip_log is not None:
            out["flips"] = [[self.flip_log[g, c, :min(self.flip_count[g, c], self.flip_log.shape[2])].copy()
                             for c in range(self.n_chains)] for g in range(self.n_grids)]
            out["flip_count"] = self.flip_count.copy()
        if self.chain_g is not None:
            per = []
            off = 0
            for L in self.Ls:
                n = self.n_chains * self.n_bins * self.spins * (L + 1)
                shape = ((self.n_chains, self.n_bins, L + 1) if self.spins == 1
                         else (self.n_chains, self.n_bins, 2, L + 1))
                per.append(self.chain_g[off:off + n].reshape(shape).copy())
                off += n
            out["chain_g"] = per
            out["chain_d"] = self.chain_d.copy()
            out["chain_n"] = self.chain_n.copy()
            out["chain_drift"] = self.chain_drift.copy()
        if self.green is not None:
            out["green"] = self.green
        return out


def hfqmc_solve(ctx, g0_tau, U, beta, dtau, seed, n_chains=1, warmup=0, sweeps=1,
                mode="rank1", recompute_every=0, delay_k=0, n_bins=0, drift_limit=0.0, drift_every=0,
                flip_cap=0, replay=None, want_chain=False, want_green=False, eager=False,
                heat_bath=False, direct=False, ph=False, g_fp32=False, balance=False):
    """Fixed-dtau solve; returns dict(g, g_err, D, D_err, stats, [hooks])."""
    g0 = np.ascontiguousarray(g0_tau, dtype=np.float64)
    L = g0.shape[0]
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, ph, g_fp32, balance), drift_every=drift_every)
    hk = _Hooks(o, 1, n_chains, [L], n_bins, flip_cap,
                [replay] if replay is not None else None, want_chain, want_green)
    g = np.zeros(L + 1)
    ge = np.zeros(L + 1)
    d = np.zeros(2)
    st = N.Stats()
    rc = N.lib.hfqmc_solve(ctx.handle, N.ptr(g0), L, float(U), float(beta), float(dtau),
                           int(seed), C.byref(o), N.ptr(g), N.ptr(ge), N.ptr(d), C.byref(st))
    N.check(rc, "hfqmc_solve")
    out = dict(g=g, g_err=ge, D=d[0], D_err=d[1], stats=st.as_dict())
    r = hk.results()
    for k in ("flips", "chain_g"):
        if k in r:
            r[k] = r[k][0]
    for k in ("flip_count", "chain_d", "chain_n", "chain_drift"):
        if k in r:
            r[k] = r[k][0]
    out.update(r)
    return out


def hfqmc_solve_spin(ctx, g0_up, g0_dn, U, beta, dtau, seed, n_chains=1, warmup=0, sweeps=1,
                     mode="rank1", recompute_every=0, delay_k=0, n_bins=0, drift_limit=0.0, drift_every=0,
                     flip_cap=0, replay=None, want_chain=False, want_green=False, eager=False,
                     heat_bath=False, direct=False, balance=False):
    """Fixed-dtau solve with spin-dependent baths; returns dict(g_up, g_dn,
    err_up, err_dn, D, D_err, stats, [hooks]); chain_g is [n_chains][n_bins][2][L+1]."""
    gu = np.ascontiguousarray(g0_up, dtype=np.float64)
    gd = np.ascontiguousarray(g0_dn, dtype=np.float64)
    if gu.shape != gd.shape:
        raise ValueError("g0_up and g0_dn differ in length")
    L = gu.shape[0]
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, balance=balance), drift_every=drift_every)
    hk = _Hooks(o, 1, n_chains, [L], n_bins, flip_cap,
                [replay] if replay is not None else None, want_chain, want_green, spins=2)
    g = np.zeros(2 * (L + 1))
    ge = np.zeros(2 * (L + 1))
    d = np.zeros(2)
    st = N.Stats()
    rc = N.lib.hfqmc_solve_spin(ctx.handle, N.ptr(gu), N.ptr(gd), L, float(U), float(beta),
                                float(dtau), int(seed), C.byref(o), N.ptr(g), N.ptr(ge), N.ptr(d),
                                C.byref(st))
    N.check(rc, "hfqmc_solve_spin")
    out = dict(g_up=g[:L + 1].copy(), g_dn=g[L + 1:].copy(), err_up=ge[:L + 1].copy(),
               err_dn=ge[L + 1:].copy(), D=d[0], D_err=d[1], stats=st.as_dict())
    r = hk.results()
    for k in ("flips", "chain_g", "flip_count", "chain_d", "chain_n", "chain_drift"):
        if k in r:
            r[k] = r[k][0]
    out.update(r)
    return out


def hfqmc_solve_dev(ctx, g0_tau, L, U, beta, dtau, seed, g_tau, g_err=None, docc=None,
                    n_chains=1, warmup=0, sweeps=1, mode="rank1", recompute_every=0, delay_k=0,
                    n_bins=0, drift_limit=0.0, drift_every=0, eager=False, heat_bath=False, direct=False,
                    ph=False, g_fp32=False, balance=False):
    """hfqmc_solve on device buffers (raw device addresses as ints, e.g. a torch
    tensor's data_ptr(), on the context's device and stream); returns the stats."""
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, ph, g_fp32, balance), drift_every=drift_every)
    st = N.Stats()
    rc = N.lib.hfqmc_solve_dev(ctx.handle, C.c_void_p(int(g0_tau)), int(L), float(U), float(beta),
                               float(dtau), int(seed), C.byref(o), C.c_void_p(int(g_tau)),
                               C.c_void_p(int(g_err) if g_err else None),
                               C.c_void_p(int(docc) if docc else None), C.byref(st))
    N.check(rc, "hfqmc_solve_dev")
    return st.as_dict()


def hfqmc_solve_dev_noalloc(ctx, g0_tau, L, U, beta, dtau, seed, g_tau, g_err=None, docc=None,
                            n_chains=1, warmup=0, sweeps=1, mode="rank1", recompute_every=0,
                            delay_k=0, n_bins=0, drift_limit=0.0, drift_every=0, heat_bath=False,
                            direct=False, ph=False, g_fp32=False):
    """hfqmc_solve_dev without any allocation (the library's static per-device
    buffer; see include/hfqmc.h for its limits); returns the stats."""
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(True, heat_bath, direct, ph, g_fp32), drift_every=drift_every)
    st = N.Stats()
    rc = N.lib.hfqmc_solve_dev_noalloc(ctx.handle, C.c_void_p(int(g0_tau)), int(L), float(U),
                                       float(beta), float(dtau), int(seed), C.byref(o),
                                       C.c_void_p(int(g_tau)),
                                       C.c_void_p(int(g_err) if g_err else None),
                                       C.c_void_p(int(docc) if docc else None), C.byref(st))
    N.check(rc, "hfqmc_solve_dev_noalloc")
    return st.as_dict()


def hfqmc_plan_balance(Ls, n_chains, warmup, sweeps, n_bins, n_workgroups):
    """Chain-split factors of a batched launch (host only): dict(factor, span_before,
    span_after), spans in the planner's cost units."""
    L = np.ascontiguousarray(Ls, dtype=np.int32)
    f = np.zeros(L.shape[0], dtype=np.int32)
    sp = np.zeros(2)
    rc = N.lib.hfqmc_plan_balance(L.shape[0], N.ptr(L, C.c_int32), int(n_chains), int(warmup),
                                  int(sweeps), int(n_bins), int(n_workgroups),
                                  N.ptr(f, C.c_int32), N.ptr(sp))
    N.check(rc, "hfqmc_plan_balance")
    return dict(factor=f.tolist(), span_before=float(sp[0]), span_after=float(sp[1]))


def hfqmc_uniforms(ctx, seed, chain, grid, sweep0, n_sweeps, L, stream=0):
    """The method's uniforms as the device draws them: array [n_sweeps, L]."""
    out = np.zeros(int(n_sweeps) * int(L))
    rc = N.lib.hfqmc_uniforms(ctx.handle, int(seed), int(chain), int(grid), int(sweep0),
                              int(n_sweeps), int(L), int(stream), N.ptr(out))
    N.check(rc, "hfqmc_uniforms")
    return out.reshape(int(n_sweeps), int(L))


def hfqmc_measure_peaks(ctx):
    """Achievable HBM bandwidth (GB/s) and matrix-core / FMA rates (TFLOP/s)
    of the context's device, from the library's probe kernels."""
    pk = N.Peaks()
    N.check(N.lib.hfqmc_measure_peaks(ctx.handle, C.byref(pk)), "hfqmc_measure_peaks")
    return pk.as_dict()


def hfqmc_solve_grids(ctx, Ls, g0_taus, U, beta, seed, n_chains=1, warmup=0, sweeps=1,
                      mode="rank1", recompute_every=0, delay_k=0, n_bins=0, drift_limit=0.0, drift_every=0,
                      flip_cap=0, replay=None, want_chain=False, eager=False, heat_bath=False,
                      direct=False, ph=False, g_fp32=False, balance=False):
    """Several grids in one persistent launch; per-grid lists in the result."""
    Ls = [int(L) for L in Ls]
    n = len(Ls)
    Larr = np.array(Ls, dtype=np.int32)
    g0 = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64) for x in g0_taus]))
    assert g0.shape[0] == sum(Ls)
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, ph, g_fp32, balance), drift_every=drift_every)
    hk = _Hooks(o, n, n_chains, Ls, n_bins, flip_cap, replay, want_chain, False)
    P = sum(L + 1 for L in Ls)
    g = np.zeros(P)
    ge = np.zeros(P)
    d = np.zeros(2 * n)
    st = (N.Stats * n)()
    rc = N.lib.hfqmc_solve_grids(ctx.handle, n, N.ptr(Larr, C.c_int32), N.ptr(g0), float(U),
                                 float(beta), int(seed), C.byref(o), N.ptr(g), N.ptr(ge),
                                 N.ptr(d), st)
    N.check(rc, "hfqmc_solve_grids")
    gs, es, off = [], [], 0
    for L in Ls:
        gs.append(g[off:off + L + 1].copy())
        es.append(ge[off:off + L + 1].copy())
        off += L + 1
    out = dict(g=gs, g_err=es, D=d[0::2].copy(), D_err=d[1::2].copy(),
               stats=[st[i].as_dict() for i in range(n)])
    out.update(hk.results())
    return out


def multigrid_solve(ctx, bath_iw, bath_m3, U, beta, dtaus, seed, n_fine=200, n_chains=1,
                    warmup=0, sweeps=1, mode="rank1", recompute_every=0, delay_k=0, n_bins=0,
                    drift_limit=0.0, drift_every=0, eager=False, heat_bath=False, direct=False,
                    ph=False, g_fp32=False, balance=False):
    """dtau -> 0 extrapolated G(tau_j), tau_j = j beta/(n_fine-1)."""
    b = np.ascontiguousarray(np.asarray(bath_iw, dtype=np.complex128)).view(np.float64)
    n_iw = b.shape[0] // 2
    dt = np.ascontiguousarray(dtaus, dtype=np.float64)
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, ph, g_fp32, balance), drift_every=drift_every)
    Ls = [int(round(beta / x)) for x in dt]
    gf = np.zeros(n_fine)
    ef = np.zeros(n_fine)
    gg = np.zeros(sum(L + 1 for L in Ls))
    st = (N.Stats * len(Ls))()
    dg = np.zeros(2 * len(Ls))
    dx = np.zeros(2)
    rc = N.lib.multigrid_solve(ctx.handle, N.ptr(b), n_iw, float(bath_m3), float(U), float(beta),
                               N.ptr(dt), len(Ls), int(seed), C.byref(o), int(n_fine), N.ptr(gf),
                               N.ptr(ef), N.ptr(gg), st, N.ptr(dg), N.ptr(dx))
    N.check(rc, "multigrid_solve")
    grids, off = [], 0
    for L in Ls:
        grids.append(gg[off:off + L + 1].copy())
        off += L + 1
    return dict(g=gf, g_err=ef, tau=np.arange(n_fine) * (beta / (n_fine - 1)), Ls=Ls,
                g_grids=grids, stats=[st[i].as_dict() for i in range(len(Ls))],
                D_grids=dg[0::2].copy(), D_err_grids=dg[1::2].copy(), D=float(dx[0]),
                D_err=float(dx[1]))


def dmft_solve(ctx, U, beta, t, dtaus, seed, n_iter, bath_iw=None, n_iw=4096, n_fine=200,
               mixing=0.0, n_chains=1, warmup=0, sweeps=1, mode="rank1", recompute_every=0,
               delay_k=0, n_bins=0, drift_limit=0.0, drift_every=0, eager=False, heat_bath=False, direct=False,
               ph=False, g_fp32=False, balance=False):
    """Multigrid DMFT cycle on the Bethe lattice; starts from bath_iw (default:
    the U = 0 semicircle).  Returns dict(bath, g, g_err, tau, history) with
    history[it] = (max |g - g_prev|, max g_err, D, D_err), D the extrapolated
    double occupancy."""
    if bath_iw is None:
        bath_iw = bethe_semicircle_bath(beta, t, n_iw)
    b = np.ascontiguousarray(np.asarray(bath_iw, dtype=np.complex128)).copy().view(np.float64)
    n_iw = b.shape[0] // 2
    dt = np.ascontiguousarray(dtaus, dtype=np.float64)
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, ph, g_fp32, balance), drift_every=drift_every)
    gf = np.zeros(n_fine)
    ef = np.zeros(n_fine)
    hist = np.zeros(4 * int(n_iter))
    rc = N.lib.dmft_solve(ctx.handle, float(U), float(beta), float(t), N.ptr(dt), dt.shape[0],
                          int(seed), C.byref(o), int(n_fine), n_iw, int(n_iter), float(mixing),
                          N.ptr(b), N.ptr(gf), N.ptr(ef), N.ptr(hist))
    N.check(rc, "dmft_solve")
    return dict(bath=b.view(np.complex128), g=gf, g_err=ef,
                tau=np.arange(n_fine) * (beta / (n_fine - 1)), history=hist.reshape(-1, 4))


def multigrid_solve_spin(ctx, bath_up, bath_dn, bath_m3, U, beta, dtaus, seed, n_fine=200,
                         n_chains=1, warmup=0, sweeps=1, mode="rank1", recompute_every=0,
                         delay_k=0, n_bins=0, drift_limit=0.0, drift_every=0, eager=False, heat_bath=False,
                         direct=False, balance=False):
    """multigrid_solve with spin-dependent baths: dict(g [2, n_fine] (up, down),
    g_err, tau, D, D_err)."""
    bu = np.ascontiguousarray(np.asarray(bath_up, dtype=np.complex128)).view(np.float64)
    bd = np.ascontiguousarray(np.asarray(bath_dn, dtype=np.complex128)).view(np.float64)
    if bu.shape != bd.shape:
        raise ValueError("bath_up and bath_dn differ in length")
    dt = np.ascontiguousarray(dtaus, dtype=np.float64)
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, balance=balance), drift_every=drift_every)
    gf = np.zeros(2 * n_fine)
    ef = np.zeros(2 * n_fine)
    dx = np.zeros(2)
    rc = N.lib.multigrid_solve_spin(ctx.handle, N.ptr(bu), N.ptr(bd), bu.shape[0] // 2,
                                    float(bath_m3), float(U), float(beta), N.ptr(dt), dt.shape[0],
                                    int(seed), C.byref(o), int(n_fine), N.ptr(gf), N.ptr(ef),
                                    N.ptr(dx))
    N.check(rc, "multigrid_solve_spin")
    return dict(g=gf.reshape(2, n_fine), g_err=ef.reshape(2, n_fine),
                tau=np.arange(n_fine) * (beta / (n_fine - 1)), D=float(dx[0]), D_err=float(dx[1]))


def dmft_solve_af(ctx, U, beta, t, dtaus, seed, n_iter, bath_up, bath_dn, n_fine=200, mixing=0.0,
                  n_chains=1, warmup=0, sweeps=1, mode="rank1", recompute_every=0, delay_k=0,
                  n_bins=0, drift_limit=0.0, drift_every=0, eager=False, heat_bath=False, direct=False, balance=False):
    """Neel-order DMFT cycle on the Bethe lattice from the given spin baths;
    returns dict(baths (up, down), g [2, n_fine], g_err, tau, history [n_iter, 5])
    with history[it] = (max |g change|, max g_err, D, D_err, n_up - n_dn)."""
    bu = np.ascontiguousarray(np.asarray(bath_up, dtype=np.complex128)).copy().view(np.float64)
    bd = np.ascontiguousarray(np.asarray(bath_dn, dtype=np.complex128)).copy().view(np.float64)
    if bu.shape != bd.shape:
        raise ValueError("bath_up and bath_dn differ in length")
    dt = np.ascontiguousarray(dtaus, dtype=np.float64)
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, balance=balance), drift_every=drift_every)
    gf = np.zeros(2 * n_fine)
    ef = np.zeros(2 * n_fine)
    hist = np.zeros(5 * int(n_iter))
    rc = N.lib.dmft_solve_af(ctx.handle, float(U), float(beta), float(t), N.ptr(dt), dt.shape[0],
                             int(seed), C.byref(o), int(n_fine), bu.shape[0] // 2, int(n_iter),
                             float(mixing), N.ptr(bu), N.ptr(bd), N.ptr(gf), N.ptr(ef), N.ptr(hist))
    N.check(rc, "dmft_solve_af")
    return dict(baths=(bu.view(np.complex128), bd.view(np.complex128)), g=gf.reshape(2, n_fine),
                g_err=ef.reshape(2, n_fine), tau=np.arange(n_fine) * (beta / (n_fine - 1)),
                history=hist.reshape(-1, 5))


def dmft_bethe_step(g_fine, bath_iw_prev, bath_m3, U, beta, t):
    """New bath 1/(i w - t^2 G(i w)) on the frequencies of bath_iw_prev."""
    g = np.ascontiguousarray(g_fine, dtype=np.float64)
    b = np.ascontiguousarray(np.asarray(bath_iw_prev, dtype=np.complex128)).view(np.float64)
    n_iw = b.shape[0] // 2
    out = np.zeros(2 * n_iw)
    rc = N.lib.dmft_bethe_step(N.ptr(g), g.shape[0], N.ptr(b), n_iw, float(bath_m3), float(U),
                               float(beta), float(t), N.ptr(out))
    N.check(rc, "dmft_bethe_step")
    return out.view(np.complex128)


def bethe_semicircle_bath(beta, t, n_iw):
    out = np.zeros(2 * int(n_iw))
    N.check(N.lib.bethe_semicircle_bath(float(beta), float(t), int(n_iw), N.ptr(out)),
            "bethe_semicircle_bath")
    return out.view(np.complex128)


def bethe_atomic_bath(beta, t, U, n_iw):
    out = np.zeros(2 * int(n_iw))
    N.check(N.lib.bethe_atomic_bath(float(beta), float(t), float(U), int(n_iw), N.ptr(out)),
            "bethe_atomic_bath")
    return out.view(np.complex128)


def bath_to_tau(bath_iw, m3, beta, L):
    b = np.ascontiguousarray(np.asarray(bath_iw, dtype=np.complex128)).view(np.float64)
    out = np.zeros(int(L))
    N.check(N.lib.bath_to_tau(N.ptr(b), b.shape[0] // 2, float(m3), float(beta), int(L), N.ptr(out)),
            "bath_to_tau")
    return out


# ------------------------------------------------------ away from half filling


def bethe_lattice_bath(beta, t, mu, n_iw):
    """Noninteracting Bethe-lattice G at chemical potential mu (the U = 0 solution)."""
    out = np.zeros(2 * int(n_iw))
    N.check(N.lib.bethe_lattice_bath(float(beta), float(t), float(mu), int(n_iw), N.ptr(out)),
            "bethe_lattice_bath")
    return out.view(np.complex128)


def bath_to_tau_m2(bath_iw, m2, m3, beta, L):
    b = np.ascontiguousarray(np.asarray(bath_iw, dtype=np.complex128)).view(np.float64)
    out = np.zeros(int(L))
    N.check(N.lib.bath_to_tau_m2(N.ptr(b), b.shape[0] // 2, float(m2), float(m3), float(beta),
                                 int(L), N.ptr(out)), "bath_to_tau_m2")
    return out


def multigrid_solve_n(ctx, bath_iw, m2, m3, U, beta, dtaus, seed, n_fine=200, n_chains=1,
                      warmup=0, sweeps=1, mode="rank1", recompute_every=0, delay_k=0, n_bins=0,
                      drift_limit=0.0, drift_every=0, eager=False, heat_bath=False, direct=False, balance=False):
    """multigrid_solve at any filling: dict(g, g_err, tau, D, D_err, n_ref)."""
    b = np.ascontiguousarray(np.asarray(bath_iw, dtype=np.complex128)).view(np.float64)
    dt = np.ascontiguousarray(dtaus, dtype=np.float64)
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, balance=balance), drift_every=drift_every)
    gf = np.zeros(n_fine)
    ef = np.zeros(n_fine)
    dx = np.zeros(2)
    nr = np.zeros(1)
    rc = N.lib.multigrid_solve_n(ctx.handle, N.ptr(b), b.shape[0] // 2, float(m2), float(m3),
                                 float(U), float(beta), N.ptr(dt), dt.shape[0], int(seed),
                                 C.byref(o), int(n_fine), N.ptr(gf), N.ptr(ef), N.ptr(dx),
                                 N.ptr(nr))
    N.check(rc, "multigrid_solve_n")
    return dict(g=gf, g_err=ef, tau=np.arange(n_fine) * (beta / (n_fine - 1)), D=float(dx[0]),
                D_err=float(dx[1]), n_ref=float(nr[0]))


def dmft_bethe_step_mu(g_fine, bath_iw_prev, m2, m3, U, beta, t, mu):
    """New bath 1/(i w + mu - t^2 G(i w)) on the frequencies of bath_iw_prev."""
    g = np.ascontiguousarray(g_fine, dtype=np.float64)
    b = np.ascontiguousarray(np.asarray(bath_iw_prev, dtype=np.complex128)).view(np.float64)
    out = np.zeros(b.shape[0])
    rc = N.lib.dmft_bethe_step_mu(N.ptr(g), g.shape[0], N.ptr(b), b.shape[0] // 2, float(m2),
                                  float(m3), float(U), float(beta), float(t), float(mu), N.ptr(out))
    N.check(rc, "dmft_bethe_step_mu")
    return out.view(np.complex128)


def dmft_solve_mu(ctx, U, mu, beta, t, dtaus, seed, n_iter, bath_iw=None, n_iw=4096, n_fine=200,
                  mixing=0.0, n_chains=1, warmup=0, sweeps=1, mode="rank1", recompute_every=0,
                  delay_k=0, n_bins=0, drift_limit=0.0, drift_every=0, eager=False,
                  heat_bath=False, direct=False, balance=False):
    """Multigrid DMFT cycle at chemical potential mu, from bath_iw (default: the U = 0
    lattice at mu).  history[it] = (max |g change|, max g_err, D, D_err, n)."""
    if bath_iw is None:
        bath_iw = bethe_lattice_bath(beta, t, mu, n_iw)
    b = np.ascontiguousarray(np.asarray(bath_iw, dtype=np.complex128)).copy().view(np.float64)
    dt = np.ascontiguousarray(dtaus, dtype=np.float64)
    o = _opts(n_chains, mode, warmup, sweeps, recompute_every, delay_k, n_bins, drift_limit,
              _flags(eager, heat_bath, direct, balance=balance), drift_every=drift_every)
    gf = np.zeros(n_fine)
    ef = np.zeros(n_fine)
    hist = np.zeros(5 * int(n_iter))
    rc = N.lib.dmft_solve_mu(ctx.handle, float(U), float(mu), float(beta), float(t), N.ptr(dt),
                             dt.shape[0], int(seed), C.byref(o), int(n_fine), b.shape[0] // 2,
                             int(n_iter), float(mixing), N.ptr(b), N.ptr(gf), N.ptr(ef), N.ptr(hist))
    N.check(rc, "dmft_solve_mu")
    return dict(bath=b.view(np.complex128), g=gf, g_err=ef,
                tau=np.arange(n_fine) * (beta / (n_fine - 1)), history=hist.reshape(-1, 5))
