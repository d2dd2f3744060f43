"""CPU oracle for the Hirsch-Fye QMC hot path and the multigrid/DMFT steps.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import anything here; the product package
never does, and the two share no code.  Plain, slow, FP64 NumPy written from
the method's definitions (see each module's docstring for the passage it
follows and the readings taken where the paper is silent).

Modules:
  philox     Philox4x64-10 counter-based uniforms (pinned to numpy.random.Philox)
  bath       semicircle bath, Matsubara <-> imaginary time, Bethe closure
  hfqmc      fixed-dtau HF-QMC chains, exact recompute, estimators, brute force
  multigrid  reference model, spline interpolation, dtau^2 extrapolation, DMFT step
"""
