/* hfqmc.h -- C ABI of the MI355X Hirsch-Fye QMC library (libhfqmc.so).
 *
 * Method: multigrid Hirsch-Fye quantum Monte Carlo for dynamical mean-field
 * theory (N. Bluemer, arXiv:0801.1222).  The impurity problem is solved at a
 * fixed bath on several Trotter grids dtau_i, each by Metropolis updates of the
 * Ising-like auxiliary field s_l on the time slices (Introduction; section
 * "Multigrid HF-QMC method"), the grid results are interpolated onto a common fine tau grid
 * with a reference model and extrapolated quadratically in dtau^2 to dtau -> 0
 * (same section, steps (i) and (ii)); the DMFT cycle is closed on the Bethe
 * lattice with semi-elliptic DOS, W = 4t (Fig. 1 and "Benchmark results").
 *
 * General conventions
 *  - Every pointer argument is owned by the caller and is only read or
 *    written during the call; the library never keeps it.  All pointers are
 *    HOST pointers.  Device memory is allocated inside the context.
 *  - FP64 everywhere on the interface.  Complex arrays are interleaved
 *    (re, im) doubles.
 *  - Imaginary-time Green functions use the positive convention
 *    G(tau) = <T c(tau) c^dag(0)>, 0 <= tau < beta, G(0) meaning G(0+) =
 *    1 - n; the point tau = beta means beta- and equals 1 - G(0+).
 *  - Matsubara arrays hold n = 0..n_iw-1 at w_n = (2n+1) pi / beta with the
 *    standard sign, G(i w) ~ 1/(i w).
 *  - Return value: HFQMC_OK (0) or a negative error code; on error the
 *    outputs are unspecified and hfqmc_last_error() describes the failure.
 *  - Calls on one context are not thread safe; use one context per thread.
 */
#ifndef HFQMC_H
#define HFQMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HFQMC_OK = 0,
  HFQMC_EINVAL = -1,        /* bad argument (null pointer, size, parameter range) */
  HFQMC_ENOMEM = -2,        /* device or host allocation failed */
  HFQMC_EDEVICE = -3,       /* HIP runtime error or no usable gfx950 device */
  HFQMC_ENUMERIC = -4,      /* NaN/Inf result or singular Dyson matrix */
  HFQMC_EDRIFT = -5,        /* drift at a recompute exceeded opts.drift_limit */
  HFQMC_EUNSUPPORTED = -6   /* option combination not implemented */
};

/* Opaque context: device, stream, device buffers and autotune cache. */
typedef struct hfqmc_ctx hfqmc_ctx;

/* Create a context on HIP device `device`.  EDEVICE if the device is absent
 * or is not gfx950. */
int hfqmc_create(hfqmc_ctx **out, int device);
void hfqmc_destroy(hfqmc_ctx *ctx);
/* Launch all device work on `stream` (a hipStream_t of the HIP runtime this
 * library is linked with; NULL = the null stream).  The stream must outlive
 * its use by the context.  Streams of another HIP runtime in the process
 * (PyTorch ships its own) are not valid here; the null stream is common. */
int hfqmc_set_stream(hfqmc_ctx *ctx, void *stream);
/* Message for the last nonzero return on the calling thread. */
const char *hfqmc_last_error(void);

/* Update scheme of the Metropolis sweep. */
enum {
  HFQMC_MODE_RANK1 = 0,        /* FP64 Sherman-Morrison rank-1 update per accepted flip */
  HFQMC_MODE_DELAYED_FP64 = 1, /* delayed rank-k updates, FP64 flush */
  HFQMC_MODE_MIXED = 2         /* delayed rank-k updates, flush as FP32 MFMA GEMM with
                                  FP32 accumulation; ratios, acceptance and the LU
                                  recompute stay FP64 */
};

/* Option bits (hfqmc_opts.flags). */
enum {
  HFQMC_FLAG_EAGER = 1,      /* launch the kernels one by one instead of replaying the
                                launch sequence (set-up kernels: bath matrices, fills,
                                references; the persistent sweep kernel between its two
                                timing events; the chain reduction) as one captured HIP
                                graph; the results are identical */
  HFQMC_FLAG_HEAT_BATH = 2,  /* heat-bath acceptance u < R/(1+R) instead of Metropolis u < R */
  HFQMC_FLAG_DIRECT_RECOMPUTE = 4, /* recompute with the full L x L LU of [M | G0] instead of the
                                      reduced system against the uniform-field references */
  HFQMC_FLAG_PH_SYMMETRIC = 8  /* particle-hole symmetric bath (G0(tau) = G0(beta - tau),
                                  G0(0+) = 1/2): only G_up is stored and updated, G_dn being
                                  1 - G_up^T for every field (V_dn = -V_up); R_dn, the
                                  estimators and final_green use that identity.  Halves the
                                  update, recompute and measurement work.  EINVAL unless every
                                  bath satisfies the symmetry to 1e-9 */,
  HFQMC_FLAG_G_FP32 = 16     /* mixed mode only (EINVAL otherwise): the Green matrices are
                                stored in FP32 between recomputes, halving their HBM traffic.
                                Ratios, window blocks, acceptance, estimators and the LU
                                recompute still compute in FP64, from the FP32-stored values;
                                each flush and each recompute rounds its result to FP32 when
                                storing it (the reduced recompute's product reads the solved
                                rows back in that form) */,
  HFQMC_FLAG_BALANCE = 32    /* batched launches of uneven grids: a grid whose chains would
                                set the launch's length runs n_chains * f chains of
                                sweeps / f measured sweeps each (f a power of two up to 64
                                dividing sweeps, sweeps / f >= n_bins), every chain with its
                                own warm-up: the same number of measurements per grid, spread
                                over more workgroups.  f per grid from hfqmc_plan_balance with
                                the device's workgroup count; chain c of a grid keeps the
                                Philox key (seed + c, grid), c now up to n_chains * f - 1.
                                EINVAL with any per-chain test hook (flip_log, replay_log,
                                chain_*, final_green) */
};

typedef struct {
  int32_t n_chains;         /* independent chains per grid; chain c uses Philox key (seed + c, grid) */
  int32_t mode;             /* HFQMC_MODE_* */
  int64_t warmup;           /* unmeasured sweeps per chain */
  int64_t sweeps;           /* measured sweeps per chain (>= 1) */
  int32_t recompute_every;  /* accepted flips between FP64 Dyson recomputes;
                               0 -> 100 (rank-1) or 4*k (delayed) */
  int32_t delay_k;          /* delayed modes: max pending flips k (2..64); 0 -> autotune:
                               k in {16, 32, 64} and the LU panel width are chosen by timing
                               short trial launches of the same grids and chain count, and
                               the choice is cached in the context */
  int32_t n_bins;           /* measurement bins per chain; 0 -> 20 if n_chains == 1 else 1 */
  int32_t flags;            /* HFQMC_FLAG_* bits */
  double drift_limit;       /* 0: report only; > 0: HFQMC_EDRIFT if a sampled recompute drift exceeds it
                               (max_drift or max_drift_gtau of hfqmc_stats) */
  /* Optional test hooks (NULL to disable).  Flip codes are sweep * L + l. */
  int64_t *flip_log;        /* [n_grids][n_chains][flip_cap] accepted flips, in order */
  int64_t *flip_count;      /* [n_grids][n_chains] number of accepted flips (may exceed flip_cap) */
  int64_t flip_cap;
  const int64_t *replay_log;   /* [n_grids][n_chains][replay_cap]: accept exactly these flips */
  const int64_t *replay_count; /* [n_grids][n_chains] */
  int64_t replay_cap;
  double *chain_g;          /* [n_grids][n_chains][n_bins][L_i+1] per-bin sums of G(tau_k) */
  double *chain_d;          /* [n_grids][n_chains][n_bins] per-bin sums of D */
  int64_t *chain_n;         /* [n_grids][n_chains][n_bins] measurements per bin */
  double *chain_drift;      /* [n_grids][n_chains] max elementwise drift at sampled recomputes */
  double *final_green;      /* single grid only: [n_chains][2][L][L] G_up, G_dn after the last sweep */
  int32_t drift_every;      /* the drift against the recomputed G is taken on recompute 1,
                               1 + drift_every, 1 + 2 drift_every, ... of each chain; 0 -> 8,
                               1 -> every recompute (complete drift; the delayed modes then
                               flush their pending flips before every recompute) */
} hfqmc_opts;

typedef struct {
  double acc_rate;          /* accepted / proposed */
  double max_drift;         /* max elementwise |G_updated - G_recomputed| over the sampled
                               recomputes: the first and every drift_every-th of each chain
                               (before the others the pending flips are not flushed, the
                               recompute replacing G); a non-finite G is reported at any
                               recompute.  A lower bound of the drift unless drift_every = 1 */
  double seconds_total;     /* wall time of the call */
  double seconds_kernel;    /* HIP-event time of the persistent sweep kernel */
  int64_t n_proposed, n_accepted, n_recomputes, n_bad_ratio, n_singular;
  int64_t n_flushes;        /* delayed modes: rank-m products applied to G */
  /* per-phase time inside the sweep kernel, summed over chains (chain-seconds,
     from the device wall clock): sweeping excluding flushes and recomputes,
     delayed-update flushes, Dyson recomputes (initial ones included), measurement */
  double chain_s_sweep, chain_s_flush, chain_s_recompute, chain_s_measure;
  /* recompute breakdown (chain-seconds): matrix build, panel factorizations,
     forward strip passes, back substitution (the reduced form's GEMM: chain_s_lu_gemm) */
  double chain_s_lu_build, chain_s_lu_panel, chain_s_lu_strip, chain_s_lu_back;
  int32_t delay_k;          /* k actually used (delayed modes) */
  int32_t recompute_every;  /* recompute interval actually used */
  int32_t n_workgroups;     /* persistent workgroups launched */
  int32_t lu_panel;         /* LU panel width of the recompute */
  int32_t graph;            /* 0: eager launches; 1: the whole launch sequence ran as one HIP
                               graph (the sweep kernel between two event-record nodes);
                               2: only the set-up launches were a graph (the runtime refused
                               the event nodes), the sweep kernel and reduction followed it */
  int32_t autotuned;        /* 1 if k and the panel width came from the autotuner */
  double seconds_autotune;  /* time spent in trial launches during this call (0 on a cache hit) */
  int64_t n_reduced_rows;   /* sum over reduced-form recomputes of the system size |S| */
  int32_t recompute_reduced;/* 1: reduced form (see hfqmc_solve), 0: full-size LU */
  int32_t chain_split;      /* HFQMC_FLAG_BALANCE: the grid's chain-split factor f (its
                               chains ran sweeps / f measured sweeps each, n_chains * f of
                               them; the largest f in a launch's total); 1 otherwise */
  double chain_s_lu_gemm;   /* recompute breakdown: the reduced form's GEMM (chain-seconds) */
  double chain_s_flush_vectors, chain_s_flush_gemm;  /* flush breakdown: X, Y and G += X Y */
  /* delayed-update breakdown (chain-seconds, part of chain_s_flush): opening a
     window with flips pending, and completing T, S and W = T S before a flush */
  double chain_s_window_apply, chain_s_fold;
  double seconds_sweep_kernel;  /* HIP-event time of the persistent sweep kernel alone (the
                                   launch sequence of seconds_kernel also builds the bath
                                   matrices and references and reduces the chains) */
  double max_drift_gtau;    /* drift of the result itself: max over the sampled recomputes and
                               the lags k of |G(tau_k) of G_updated - G(tau_k) of G_recomputed|,
                               the translation- and spin-averaged estimator of the output
                               (both spin-resolved estimators for spin-dependent baths) */
} hfqmc_stats;

/* Fixed-dtau solve: hfqmc_solve(G0(tau), U, beta, dtau, sweeps, seed) -> G(tau).
 * Hirsch-Fye QMC for the half-filled single-band Anderson impurity with bath
 * g0_tau[k] = G0(k dtau), k = 0..L-1, interaction U >= 0, inverse temperature
 * beta, L = beta/dtau slices (|beta/dtau - L| <= 1e-9 L), HS coupling
 * cosh(lambda) = exp(dtau U/2).  The periodic recompute
 * G = (1 + (1 - G0)(e^V - 1))^{-1} G0 (FP64) uses, unless
 * HFQMC_FLAG_DIRECT_RECOMPUTE is set, the exact block elimination against the
 * uniform-field reference
 * M_r = 1 + d_r (1 - G0) (d_r the more frequent of e^{+-lambda} - 1 in the
 * field, Q_r = M_r^{-1}(1 - G0) and H_r = M_r^{-1} G0 computed once per grid on
 * the device): an LU of size |S| <= L/2 on the slices S where the field
 * differs from the reference, then one GEMM for the other rows.
 * Outputs (host): g_tau[L+1] on tau_k = k dtau,
 * k = 0..L (tau_L = beta-); g_err[L+1] (or NULL) standard error over chains
 * (or bins); docc[2] (or NULL) double occupancy and its error; stats (or NULL).
 * Sizes: L from 2 to 4096 (EINVAL outside).  The reference solves (L-row
 * systems) keep their LU panel in LDS where it fits (160 KiB per workgroup on
 * gfx950) and in the workspace beyond (L > 3092).  HFQMC_FLAG_DIRECT_RECOMPUTE
 * stages an L-row panel in LDS in every recompute and is limited to L <= 3092:
 * beyond it returns HFQMC_EUNSUPPORTED before any device work, naming the LDS
 * it would need. */
int hfqmc_solve(hfqmc_ctx *ctx, const double *g0_tau, int32_t L, double U, double beta,
                double dtau, uint64_t seed, const hfqmc_opts *opts,
                double *g_tau, double *g_err, double *docc, hfqmc_stats *stats);

/* hfqmc_solve with device memory: g0_tau, g_tau, g_err and docc are device
 * pointers (hipMalloc'd or torch tensors on the context's device; g_err and
 * docc may be NULL) and are read and written on the context's stream.  The
 * statistics and the opts test hooks stay host pointers.  The buffers are
 * read and written by kernels, so they may also come from another HIP runtime
 * loaded in the same process (PyTorch's).  Same semantics and errors as
 * hfqmc_solve, except that g0_tau is not checked for finiteness on the host
 * (a non-finite bath surfaces as HFQMC_ENUMERIC). */
int hfqmc_solve_dev(hfqmc_ctx *ctx, const double *g0_tau, int32_t L, double U, double beta,
                    double dtau, uint64_t seed, const hfqmc_opts *opts,
                    double *g_tau, double *g_err, double *docc, hfqmc_stats *stats);

/* hfqmc_solve_dev that allocates nothing, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, semantics and results (bit for bit the
 * same kernels), but no device or host allocation.  Everything besides the
 * caller's inputs and outputs lives in one static device buffer of 128 MiB
 * per GPU, held by the library's code object from the first use of the
 * device until the process ends: the grid data (bath matrix, uniform-field
 * references, accumulators, counters) first, then as many per-workgroup
 * workspaces as fit, which sets the number of workgroups (about 18 at
 * L = 400 in the delayed modes, all chains at once for short grids).
 * Limits: one grid; L up to about 880 (the reference solves need four
 * workspaces), fewer with many chains; EINVAL names the sizes when a call
 * exceeds the buffer.  delay_k must be given in the delayed modes (EINVAL for
 * 0: the autotuner's trial launches allocate); the test hooks of hfqmc_opts
 * (flip_log, replay_log, chain_*, final_green) give EINVAL; the set-up
 * kernels run eagerly (HFQMC_FLAG_EAGER is implied).  Every call on a GPU
 * shares that GPU's buffer and clears what it reads before use: calls that
 * overlap on one GPU (another thread, another context, another stream) race
 * and give undefined results.  EDEVICE if the buffer could not be located
 * when the context was created. */
int hfqmc_solve_dev_noalloc(hfqmc_ctx *ctx, const double *g0_tau, int32_t L, double U, double beta,
                            double dtau, uint64_t seed, const hfqmc_opts *opts,
                            double *g_tau, double *g_err, double *docc, hfqmc_stats *stats);

/* hfqmc_solve with spin-dependent baths (a magnetic field, magnetic phases;
 * the paper's closing remarks on the method's generality): spin up sees the
 * bath g0_up[L], spin down g0_dn[L], both G0_sigma(k dtau) in the positive
 * convention; M_sigma = 1 + (1 - G0_sigma)(e^{V_sigma} - 1).  Outputs are
 * spin-resolved: g_tau[2 (L+1)] = G_up(tau_k), k = 0..L, then G_dn(tau_k)
 * (G_sigma(beta-) = n_sigma); g_err likewise or NULL; docc as hfqmc_solve.
 * opts.chain_g, when given, holds [n_chains][n_bins][2][L+1].  All update
 * modes; EINVAL with HFQMC_FLAG_PH_SYMMETRIC or HFQMC_FLAG_G_FP32, for a null
 * g0_dn and as hfqmc_solve otherwise.  Host buffers only. */
int hfqmc_solve_spin(hfqmc_ctx *ctx, const double *g0_up, const double *g0_dn, int32_t L,
                     double U, double beta, double dtau, uint64_t seed, const hfqmc_opts *opts,
                     double *g_tau, double *g_err, double *docc, hfqmc_stats *stats);

/* Batched solve of several grids in ONE persistent launch (the data-parallel
 * core of a multigrid step): grid i has L[i] slices, bath g0_tau (concatenated,
 * sum L[i] values), dtau_i = beta / L[i], Philox grid key i.  opts.n_chains
 * chains per grid.  Outputs are concatenated per grid: g_tau and g_err hold
 * sum (L[i]+1) values; docc holds 2 per grid; stats holds n_grids entries
 * (may be NULL). */
int hfqmc_solve_grids(hfqmc_ctx *ctx, int32_t n_grids, const int32_t *L, const double *g0_tau,
                      double U, double beta, uint64_t seed, const hfqmc_opts *opts,
                      double *g_tau, double *g_err, double *docc, hfqmc_stats *stats);

/* Chain-split plan of HFQMC_FLAG_BALANCE (host only: callable without a GPU).
 * The multigrid method averages independent impurity solutions per grid and
 * runs every grid of a step side by side (Multigrid HF-QMC method), while the
 * effort per sweep grows like dtau^-3 (Introduction): the long grids' chains
 * then set a batched launch's length.  Models the launch as units (grid i,
 * chain c) of cost (warmup + sweeps_i) L[i]^3, dispatched longest first to
 * n_workgroups workers (the sweep kernel's queue).  It scores every
 * threshold plan (for a target unit length, each grid split just enough for
 * its units to fit under it), then moves one grid's factor up or down, or
 * doubles the factors of all grids whose units are at least as long as a given
 * grid's, while the simulated makespan falls by more than 0.5 % (equal spans:
 * fewer chains); f_i stays a power of two <= 64 dividing sweeps with
 * sweeps / f_i >= n_bins, and all f_i are 1 when no split shortens the span
 * or when n_grids * n_chains exceeds 8192 (such launches already fill the
 * device; span then receives 0, 0: they are not simulated).  factor[n_grids] receives f_i; span (may be NULL)
 * receives the makespan without and with the split, in units of one sweep at
 * L = 1 (cost-model units).  EINVAL for n_grids < 1, NULL L or factor,
 * n_chains outside 1..2^20-1, warmup < 0, sweeps < 1, n_bins outside
 * 1..sweeps, n_workgroups < 1 or L outside 2..4096. */
int hfqmc_plan_balance(int32_t n_grids, const int32_t *L, int32_t n_chains, int64_t warmup,
                       int64_t sweeps, int32_t n_bins, int32_t n_workgroups, int32_t *factor,
                       double *span);

/* The uniforms the sweep kernels draw, written out on the device so that the
 * generator can be checked bit for bit.  The Hubbard-Stratonovich field is
 * sampled by Monte Carlo (Introduction); the method's draws come from the
 * counter-based Philox4x64-10 generator (Salmon et al., SC'11) with key
 * (seed + chain, grid) and counter (slice, sweep, 0, stream), u = (x0 >> 11) 2^-53
 * of the first output word: stream 0 holds the acceptance draws of slice l in
 * sweep s, stream 1 at sweep 0 the initial field (s_l = +1 iff u < 1/2).
 * out[n_sweeps * L] (host) receives u for sweeps sweep0 .. sweep0 + n_sweeps - 1
 * (row per sweep) and slices 0 .. L - 1.  Allocates and frees a device buffer
 * of the same size.  EINVAL for a NULL argument, negative chain, grid or
 * sweep0, n_sweeps or L below 1, stream outside 0..1, or more than 2^28
 * values; EDEVICE on a runtime error. */
int hfqmc_uniforms(hfqmc_ctx *ctx, uint64_t seed, int32_t chain, int32_t grid, int64_t sweep0,
                   int64_t n_sweeps, int32_t L, int32_t stream, double *out);

/* Achievable peaks of the context's device, the ceilings next to the
 * datasheet ones that the sweep kernel's roofline is quoted against (the
 * method's cost model: the update streams the L x L Green matrices through
 * memory, the recompute is a dense FP64 solve; Introduction, effort ~ dtau^-3).
 * Measured with the library's own probe kernels on the context's stream,
 * best of three timed launches each:
 *   hbm_copy_gbs      (read + written bytes) / time, device copy of 1 GiB
 *   hbm_read_gbs      read-only stream of 1 GiB
 *   fp64_mfma_tflops  v_mfma_f64_16x16x4f64 issue loop on every compute unit
 *   fp32_mfma_tflops  v_mfma_f32_16x16x4f32 issue loop
 *   fp64_fma_tflops   FP64 vector FMA loop
 * Allocates and frees 2 GiB of device memory; takes well under a second.
 * EINVAL for NULL arguments, ENOMEM, EDEVICE on a runtime error. */
typedef struct {
  double hbm_copy_gbs, hbm_read_gbs;
  double fp64_mfma_tflops, fp32_mfma_tflops, fp64_fma_tflops;
} hfqmc_peaks;
int hfqmc_measure_peaks(hfqmc_ctx *ctx, hfqmc_peaks *out);

/* Multigrid solve: multigrid_solve(list of dtau) -> G(tau) extrapolated to dtau -> 0.
 * bath_iw[2 n_iw]: bath on the Matsubara axis with high-frequency moment
 * bath_m3 (bath ~ 1/(i w) + m3/(i w)^3, particle-hole symmetric).  For each
 * dtau_i (n_grids >= 3) L_i = round(beta/dtau_i); all grids and chains run
 * in one persistent launch; each grid estimate is interpolated onto
 * tau_j = j beta/(n_fine-1), j = 0..n_fine-1, with the reference model
 * G_ref = 1/(1/bath - U^2/(4 i w)) and a natural cubic spline of G - G_ref,
 * then fitted per tau_j by weighted least squares c0 + c1 dtau^2 + c2 dtau^4.
 * Outputs: g_fine[n_fine], g_fine_err[n_fine] (or NULL); g_grids (or NULL)
 * concatenated raw grid estimates, sum (L_i+1) values; per_grid[n_grids]
 * stats (or NULL); docc_grids[2 n_grids] (or NULL) each grid's double
 * occupancy and its error; docc[2] (or NULL) the double occupancy
 * extrapolated to dtau -> 0 by the same weighted quadratic fit in dtau^2
 * (the D(dtau^2) analysis of Figs. 3 and 4) and its error. */
int multigrid_solve(hfqmc_ctx *ctx, const double *bath_iw, int32_t n_iw, double bath_m3,
                    double U, double beta, const double *dtaus, int32_t n_grids, uint64_t seed,
                    const hfqmc_opts *opts, int32_t n_fine, double *g_fine, double *g_fine_err,
                    double *g_grids, hfqmc_stats *per_grid, double *docc_grids, double *docc);

/* One Bethe-lattice DMFT self-consistency step (host only, no device):
 * G(i w) = G_ref(i w) - int_0^beta e^{i w tau} S(tau) d tau, S the natural
 * cubic spline of g_fine - G_ref on tau_j = j beta/(n_fine-1); then
 * bath_new(i w) = 1/(i w - t^2 G(i w)) on the same n_iw frequencies.
 * G_ref is built from bath_iw_prev (moment bath_m3) and U. */
int dmft_bethe_step(const double *g_fine, int32_t n_fine, const double *bath_iw_prev,
                    int32_t n_iw, double bath_m3, double U, double beta, double t,
                    double *bath_iw_new);

/* The multigrid DMFT cycle on the Bethe lattice (Fig. 1(c): impurity solve
 * on several grids, dtau -> 0 extrapolation, self-consistency), n_iter times:
 *   g_fine   = multigrid_solve(bath, dtaus, seed + (it << 32), opts)
 *   bath_new = 1/(i w - t^2 G(i w))          (dmft_bethe_step)
 *   bath     = mixing * bath + (1 - mixing) * bath_new,  0 <= mixing < 1.
 * bath_iw[2 n_iw] holds the starting bath on entry (e.g. bethe_semicircle_bath,
 * the U = 0 solution) and the last bath on return; its 1/(i w)^3 moment is t^2
 * throughout (the Bethe closure keeps it).  g_fine[n_fine] (and g_fine_err,
 * or NULL) is the last iteration's extrapolated G(tau_j), tau_j =
 * j beta/(n_fine-1).  history[4 n_iter] (or NULL): per iteration, the largest
 * |g_fine - g_fine of the previous iteration| (for the first, against the
 * starting bath's G0(tau_j)), the largest error bar of g_fine, and the
 * extrapolated double occupancy with its error (see multigrid_solve).  Each
 * iteration draws fresh Philox streams.  With HFQMC_FLAG_PH_SYMMETRIC the new
 * bath keeps only its imaginary part (exact for the symmetric G(tau) that flag
 * implies; the real part is rounding).  Errors as multigrid_solve; EINVAL for
 * n_iter < 1, mixing outside [0, 1), t <= 0. */
int dmft_solve(hfqmc_ctx *ctx, double U, double beta, double t, const double *dtaus,
               int32_t n_grids, uint64_t seed, const hfqmc_opts *opts, int32_t n_fine,
               int32_t n_iw, int32_t n_iter, double mixing, double *bath_iw, double *g_fine,
               double *g_fine_err, double *history);

/* multigrid_solve with spin-dependent baths bath_up, bath_dn (both with the
 * 1/(i w)^3 moment bath_m3): one spin-resolved batched launch (as
 * hfqmc_solve_spin, grid i with Philox grid key i), then per spin the
 * reference-model spline (that spin's bath in the reference) and the
 * quadratic fit in dtau^2.  g_fine[2 n_fine] = G_up(tau_j) then G_dn(tau_j),
 * g_fine_err likewise or NULL; docc[2] (or NULL) the extrapolated D and its
 * error.  Errors as multigrid_solve and hfqmc_solve_spin. */
int multigrid_solve_spin(hfqmc_ctx *ctx, const double *bath_up, const double *bath_dn,
                         int32_t n_iw, double bath_m3, double U, double beta, const double *dtaus,
                         int32_t n_grids, uint64_t seed, const hfqmc_opts *opts, int32_t n_fine,
                         double *g_fine, double *g_fine_err, double *docc);

/* The DMFT cycle for Neel order on the bipartite Bethe lattice (the method's
 * magnetic phases): sublattice B is sublattice A with the spins exchanged, so
 * each iteration runs multigrid_solve_spin(bath_up, bath_dn, seed + (it << 32))
 * and closes bath_up_new = 1/(i w - t^2 G_dn(i w)), bath_dn_new = 1/(i w - t^2
 * G_up(i w)) (dmft_bethe_step per spin), then mixes as dmft_solve.  bath_up,
 * bath_dn [2 n_iw] hold the starting baths (a spin-symmetric start stays
 * symmetric only up to noise; a small staggered field seeds the order) and the
 * last baths on return.  g_fine[2 n_fine] (and g_fine_err or NULL) the last
 * iteration's extrapolated G_up, G_dn; history[5 n_iter] (or NULL): max
 * |g_fine change| over both spins, max error bar, D, D error, and the
 * staggered moment m = n_up - n_dn = G_up(beta-) - G_dn(beta-).  Errors as
 * dmft_solve. */
int dmft_solve_af(hfqmc_ctx *ctx, double U, double beta, double t, const double *dtaus,
                  int32_t n_grids, uint64_t seed, const hfqmc_opts *opts, int32_t n_fine,
                  int32_t n_iw, int32_t n_iter, double mixing, double *bath_up, double *bath_dn,
                  double *g_fine, double *g_fine_err, double *history);

/* ------------------------------------------------------------------------------
 * Away from half filling (the method's generality, closing remarks of the paper).
 * Readings: the bath's tail is 1/(i w) + m2/(i w)^2 + m3/(i w)^3; the chemical
 * potential mu is measured from half filling (the interaction is the symmetric
 * U (n_up n_dn - (n_up + n_dn)/2) of every solve here); the reference model of
 * the interpolation at density n per spin is 1/(1/bath - U (n - 1/2) - U^2 n (1 - n)/(i w)),
 * the first two high-frequency terms of the self-energy (at n = 1/2 the
 * half-filled reference of multigrid_solve).  The impurity solves are the
 * two-matrix path (HFQMC_FLAG_PH_SYMMETRIC gives EINVAL).
 * ------------------------------------------------------------------------------ */

/* Noninteracting Bethe-lattice Green function at chemical potential mu (the U = 0
 * solution of dmft_solve_mu): (z - sqrt(z - 2t) sqrt(z + 2t))/(2 t^2), z = i w + mu,
 * on w_n, n = 0..n_iw-1.  Tail moments -mu, mu^2 + t^2.  EINVAL for a null
 * pointer, beta <= 0, t <= 0, non-finite mu, n_iw < 1. */
int bethe_lattice_bath(double beta, double t, double mu, int32_t n_iw, double *bath_iw);

/* bath_to_tau with the 1/(i w)^2 moment m2 of the tail handled in closed form. */
int bath_to_tau_m2(const double *bath_iw, int32_t n_iw, double m2, double m3, double beta,
                   int32_t L, double *g_tau);

/* multigrid_solve at any filling: grid i gets the bath transformed with both tail
 * moments (bath_to_tau_m2); step (i) uses the reference model at the finest grid's
 * density n = G(beta-) (returned in n_ref, or NULL); step (ii) as multigrid_solve.
 * g_fine[n_fine], g_fine_err (or NULL), docc[2] (or NULL) as multigrid_solve.
 * Errors as multigrid_solve, and EINVAL with HFQMC_FLAG_PH_SYMMETRIC. */
int multigrid_solve_n(hfqmc_ctx *ctx, const double *bath_iw, int32_t n_iw, double m2, double m3,
                      double U, double beta, const double *dtaus, int32_t n_grids, uint64_t seed,
                      const hfqmc_opts *opts, int32_t n_fine, double *g_fine, double *g_fine_err,
                      double *docc, double *n_ref);

/* The Bethe closure at chemical potential mu: G(i w) = G_ref(i w) - int_0^beta e^{i w tau}
 * S(tau) d tau, S the natural cubic spline of g_fine - G_ref, the reference at the
 * density n = g_fine[n_fine - 1] built from bath_iw_prev (tail m2, m3); then
 * bath_iw_new = 1/(i w + mu - t^2 G(i w)). */
int dmft_bethe_step_mu(const double *g_fine, int32_t n_fine, const double *bath_iw_prev,
                       int32_t n_iw, double m2, double m3, double U, double beta, double t,
                       double mu, double *bath_iw_new);

/* The multigrid DMFT cycle on the Bethe lattice at chemical potential mu (as
 * dmft_solve, with multigrid_solve_n and dmft_bethe_step_mu; the bath keeps the tail
 * moments -mu and mu^2 + t^2; a natural start is bethe_lattice_bath).
 * history[5 n_iter] (or NULL): max |g_fine change|, max error bar, D, D error, and
 * the density n = G(beta-) extrapolated.  Errors as dmft_solve. */
int dmft_solve_mu(hfqmc_ctx *ctx, double U, double mu, double beta, double t, const double *dtaus,
                  int32_t n_grids, uint64_t seed, const hfqmc_opts *opts, int32_t n_fine,
                  int32_t n_iw, int32_t n_iter, double mixing, double *bath_iw, double *g_fine,
                  double *g_fine_err, double *history);

/* U = 0 starting bath: Bethe-lattice local Green function, half-bandwidth 2t. */
int bethe_semicircle_bath(double beta, double t, int32_t n_iw, double *bath_iw);

/* Insulating starting bath (Benchmark results section, Fig. 3: the insulating
 * solution where metal and insulator coexist): the Bethe closure of the
 * half-filled Hubbard atom, bath_iw = 1/(i w - t^2 G_at(i w)) with
 * G_at(i w) = (1/(i w - U/2) + 1/(i w + U/2))/2, on w_n, n = 0..n_iw-1.  Its
 * 1/(i w)^3 moment is t^2, as for bethe_semicircle_bath.  EINVAL for a null
 * pointer, beta <= 0, t <= 0, U < 0 or n_iw < 1. */
int bethe_atomic_bath(double beta, double t, double U, int32_t n_iw, double *bath_iw);

/* Bath on a Trotter grid: g_tau[k] = G(k beta/L), k = 0..L-1, by the
 * Matsubara sum with the 1/(i w) + m3/(i w)^3 tail handled in closed form. */
int bath_to_tau(const double *bath_iw, int32_t n_iw, double m3, double beta, int32_t L,
                double *g_tau);

#ifdef __cplusplus
}
#endif

#endif /* HFQMC_H */
