"""MI355X-native Hirsch-Fye QMC hot path (multigrid HF-QMC, arXiv:0801.1222).

The compute lives in libhfqmc.so (HIP kernels for gfx950 behind a C ABI,
declared in include/hfqmc.h); this package is its thin Python binding.
"""
from .api import (Context, HFQMCError, bath_to_tau, bethe_atomic_bath,  # noqa: F401
                  bethe_semicircle_bath,
                  dmft_bethe_step, dmft_solve, dmft_solve_af, hfqmc_measure_peaks, hfqmc_solve,
                  hfqmc_solve_dev, hfqmc_solve_dev_noalloc, hfqmc_solve_grids, hfqmc_solve_spin,
                  multigrid_solve, multigrid_solve_spin, bethe_lattice_bath, bath_to_tau_m2,
                  multigrid_solve_n, dmft_bethe_step_mu, dmft_solve_mu, hfqmc_plan_balance,
                  hfqmc_uniforms)
