"""ctypes binding of libhfqmc.so (argument marshalling only).

Every computation happens in the native library; this module only converts
NumPy arrays to pointers and back.  Importing it fails loudly when the
library has not been built.
"""
import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhfqmc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libhfqmc.so is not built; run `python -m paper_0801_1222_amd.build` "
        "(the HIP library is required, there is no fallback)")

lib = C.CDLL(LIB_PATH)

_i32, _i64, _u64, _f64 = C.c_int32, C.c_int64, C.c_uint64, C.c_double
_pd = C.POINTER(C.c_double)
_pi64 = C.POINTER(C.c_int64)
_pi32 = C.POINTER(C.c_int32)


class Opts(C.Structure):
    _fields_ = [
        ("n_chains", _i32), ("mode", _i32),
        ("warmup", _i64), ("sweeps", _i64),
        ("recompute_every", _i32), ("delay_k", _i32), ("n_bins", _i32), ("flags", _i32),
        ("drift_limit", _f64),
        ("flip_log", _pi64), ("flip_count", _pi64), ("flip_cap", _i64),
        ("replay_log", _pi64), ("replay_count", _pi64), ("replay_cap", _i64),
        ("chain_g", _pd), ("chain_d", _pd), ("chain_n", _pi64), ("chain_drift", _pd),
        ("final_green", _pd), ("drift_every", _i32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("acc_rate", _f64), ("max_drift", _f64), ("seconds_total", _f64), ("seconds_kernel", _f64),
        ("n_proposed", _i64), ("n_accepted", _i64), ("n_recomputes", _i64),
        ("n_bad_ratio", _i64), ("n_singular", _i64), ("n_flushes", _i64),
        ("chain_s_sweep", _f64), ("chain_s_flush", _f64), ("chain_s_recompute", _f64),
        ("chain_s_measure", _f64),
        ("chain_s_lu_build", _f64), ("chain_s_lu_panel", _f64), ("chain_s_lu_strip", _f64),
        ("chain_s_lu_back", _f64),
        ("delay_k", _i32), ("recompute_every", _i32), ("n_workgroups", _i32), ("lu_panel", _i32),
        ("graph", _i32), ("autotuned", _i32), ("seconds_autotune", _f64),
        ("n_reduced_rows", _i64), ("recompute_reduced", _i32), ("chain_split", _i32),
        ("chain_s_lu_gemm", _f64), ("chain_s_flush_vectors", _f64), ("chain_s_flush_gemm", _f64),
        ("chain_s_window_apply", _f64), ("chain_s_fold", _f64), ("seconds_sweep_kernel", _f64),
        ("max_drift_gtau", _f64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Peaks(C.Structure):
    _fields_ = [("hbm_copy_gbs", _f64), ("hbm_read_gbs", _f64), ("fp64_mfma_tflops", _f64),
                ("fp32_mfma_tflops", _f64), ("fp64_fma_tflops", _f64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_ctx_p = C.c_void_p

lib.hfqmc_create.argtypes = [C.POINTER(_ctx_p), C.c_int]
lib.hfqmc_create.restype = C.c_int
lib.hfqmc_destroy.argtypes = [_ctx_p]
lib.hfqmc_destroy.restype = None
lib.hfqmc_set_stream.argtypes = [_ctx_p, C.c_void_p]
lib.hfqmc_set_stream.restype = C.c_int
lib.hfqmc_last_error.argtypes = []
lib.hfqmc_last_error.restype = C.c_char_p
lib.hfqmc_solve.argtypes = [_ctx_p, _pd, _i32, _f64, _f64, _f64, _u64, C.POINTER(Opts),
                            _pd, _pd, _pd, C.POINTER(Stats)]
lib.hfqmc_solve.restype = C.c_int
lib.hfqmc_solve_spin.argtypes = [_ctx_p, _pd, _pd, _i32, _f64, _f64, _f64, _u64, C.POINTER(Opts),
                                 _pd, _pd, _pd, C.POINTER(Stats)]
lib.hfqmc_solve_spin.restype = C.c_int
lib.multigrid_solve_spin.argtypes = [_ctx_p, _pd, _pd, _i32, _f64, _f64, _f64, _pd, _i32, _u64,
                                     C.POINTER(Opts), _i32, _pd, _pd, _pd]
lib.multigrid_solve_spin.restype = C.c_int
lib.dmft_solve_af.argtypes = [_ctx_p, _f64, _f64, _f64, _pd, _i32, _u64, C.POINTER(Opts), _i32, _i32,
                              _i32, _f64, _pd, _pd, _pd, _pd, _pd]
lib.dmft_solve_af.restype = C.c_int
lib.hfqmc_solve_dev.argtypes = [_ctx_p, C.c_void_p, _i32, _f64, _f64, _f64, _u64, C.POINTER(Opts),
                                C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Stats)]
lib.hfqmc_solve_dev.restype = C.c_int
lib.hfqmc_solve_dev_noalloc.argtypes = lib.hfqmc_solve_dev.argtypes
lib.hfqmc_solve_dev_noalloc.restype = C.c_int
lib.hfqmc_solve_grids.argtypes = [_ctx_p, _i32, _pi32, _pd, _f64, _f64, _u64, C.POINTER(Opts),
                                  _pd, _pd, _pd, C.POINTER(Stats)]
lib.hfqmc_solve_grids.restype = C.c_int
lib.multigrid_solve.argtypes = [_ctx_p, _pd, _i32, _f64, _f64, _f64, _pd, _i32, _u64,
                                C.POINTER(Opts), _i32, _pd, _pd, _pd, C.POINTER(Stats), _pd, _pd]
lib.multigrid_solve.restype = C.c_int
lib.dmft_bethe_step.argtypes = [_pd, _i32, _pd, _i32, _f64, _f64, _f64, _f64, _pd]
lib.dmft_bethe_step.restype = C.c_int
lib.bethe_semicircle_bath.argtypes = [_f64, _f64, _i32, _pd]
lib.bethe_semicircle_bath.restype = C.c_int
lib.bethe_atomic_bath.argtypes = [_f64, _f64, _f64, _i32, _pd]
lib.bethe_atomic_bath.restype = C.c_int
lib.bath_to_tau.argtypes = [_pd, _i32, _f64, _f64, _i32, _pd]
lib.bath_to_tau.restype = C.c_int
lib.dmft_solve.argtypes = [_ctx_p, _f64, _f64, _f64, _pd, _i32, _u64, C.POINTER(Opts), _i32, _i32,
                           _i32, _f64, _pd, _pd, _pd, _pd]
lib.dmft_solve.restype = C.c_int
lib.bethe_lattice_bath.argtypes = [_f64, _f64, _f64, _i32, _pd]
lib.bethe_lattice_bath.restype = C.c_int
lib.bath_to_tau_m2.argtypes = [_pd, _i32, _f64, _f64, _f64, _i32, _pd]
lib.bath_to_tau_m2.restype = C.c_int
lib.multigrid_solve_n.argtypes = [_ctx_p, _pd, _i32, _f64, _f64, _f64, _f64, _pd, _i32, _u64,
                                  C.POINTER(Opts), _i32, _pd, _pd, _pd, _pd]
lib.multigrid_solve_n.restype = C.c_int
lib.dmft_bethe_step_mu.argtypes = [_pd, _i32, _pd, _i32, _f64, _f64, _f64, _f64, _f64, _f64, _pd]
lib.dmft_bethe_step_mu.restype = C.c_int
lib.dmft_solve_mu.argtypes = [_ctx_p, _f64, _f64, _f64, _f64, _pd, _i32, _u64, C.POINTER(Opts),
                              _i32, _i32, _i32, _f64, _pd, _pd, _pd, _pd]
lib.dmft_solve_mu.restype = C.c_int
lib.hfqmc_plan_balance.argtypes = [_i32, _pi32, _i32, _i64, _i64, _i32, _i32, _pi32, _pd]
lib.hfqmc_plan_balance.restype = C.c_int
lib.hfqmc_uniforms.argtypes = [_ctx_p, _u64, _i32, _i32, _i64, _i64, _i32, _i32, _pd]
lib.hfqmc_uniforms.restype = C.c_int
lib.hfqmc_measure_peaks.argtypes = [_ctx_p, C.POINTER(Peaks)]
lib.hfqmc_measure_peaks.restype = C.c_int

FLAG_EAGER = 1       # launch kernels one by one (no captured graph)
FLAG_HEAT_BATH = 2   # heat-bath acceptance u < R/(1+R)
FLAG_DIRECT_RECOMPUTE = 4  # full-size LU recompute instead of the reduced system
FLAG_PH_SYMMETRIC = 8      # particle-hole symmetric bath: only G_up stored (G_dn = 1 - G_up^T)
FLAG_G_FP32 = 16           # mixed mode: G stored in FP32 between recomputes
FLAG_BALANCE = 32          # split long grids' chains over more workgroups (same measurements)

EXPORTED = ["hfqmc_create", "hfqmc_destroy", "hfqmc_set_stream", "hfqmc_last_error",
            "hfqmc_solve", "hfqmc_solve_spin", "hfqmc_solve_dev", "hfqmc_solve_grids", "multigrid_solve", "dmft_bethe_step",
            "bethe_semicircle_bath", "bethe_atomic_bath", "bath_to_tau", "hfqmc_measure_peaks", "dmft_solve",
            "multigrid_solve_spin", "dmft_solve_af", "hfqmc_solve_dev_noalloc",
            "bethe_lattice_bath", "bath_to_tau_m2", "multigrid_solve_n", "dmft_bethe_step_mu",
            "dmft_solve_mu", "hfqmc_plan_balance", "hfqmc_uniforms"]


def ptr(a, ctype=C.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def check(rc, what):
    if rc != 0:
        msg = lib.hfqmc_last_error().decode(errors="replace")
        raise HFQMCError(rc, "%s failed (%d): %s" % (what, rc, msg))


class HFQMCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code
