// Internal interface between the C-ABI layer and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace hfqmc {

// Per-chain counters written by the sweep kernel.
enum {
  ST_PROPOSED = 0,
  ST_ACCEPTED = 1,
  ST_RECOMPUTES = 2,
  ST_BAD = 3,       // proposals whose ratio was <= 0 or NaN (rejected)
  ST_SINGULAR = 4,  // zero or non-finite pivots met in a Dyson recompute
  ST_FLIPS = 5,     // entries written to the flip log (may exceed its capacity)
  ST_REPLAYED = 6,  // replay entries consumed
  ST_FLUSHES = 7,   // delayed-update flushes (rank-m products applied to G)
  ST_T_SWEEP = 8,   // wall-clock ticks spent in sweeps, flushes and recomputes excluded
  ST_T_FLUSH = 9,   // ... in delayed-update flushes
  ST_T_REC = 10,    // ... in Dyson recomputes (initial ones included)
  ST_T_MEAS = 11,   // ... in measurements
  ST_T_LU_BUILD = 12,  // recompute breakdown: building [M | G0]
  ST_T_LU_PANEL = 13,  // ... panel factorizations
  ST_T_LU_STRIP = 14,  // ... forward strip passes (interchanges, U12, trailing update)
  ST_T_LU_BACK = 15,   // ... back substitution and the copy into G
  ST_RED_ROWS = 16,    // sum over reduced-form solves of the system size |S|
  ST_T_LU_GEMM = 17,   // recompute breakdown: the reduced form's GEMM for the rows outside S
  ST_T_FL_VEC = 18,    // flush breakdown: the full update vectors X, Y
  ST_T_FL_GEMM = 19,   // ... the rank-m product G += X Y
  ST_T_WAPPLY = 20,    // ... opening windows with flips pending (T, S update and window blocks)
  ST_T_FOLD = 21,      // ... T, S completion and W = T S before a flush
  NSTAT = 22
};

enum { MODE_RANK1 = 0, MODE_DELAYED_FP64 = 1, MODE_MIXED = 2,
       MODE_MIXED_G32 = 3 /* mixed with G stored in FP32 (the sweep kernel's mode only) */ };

// One Trotter grid of a (possibly batched) launch.  All pointers are device pointers.
struct GridDev {
  int L;
  int n_chains;           // chains of this grid (more than requested when split)
  long long sweeps;       // measured sweeps per chain of this grid
  int grid_id;            // Philox key word 1
  const double* refQ[2];  // L x L, Q_r = M_r^{-1} (1 - G0) for the uniform references
  const double* refH[2];  //   r = 0: D = e^{lambda} - 1, r = 1: D = e^{-lambda} - 1; H_r = M_r^{-1} G0
  int* ref_sing;          // set when a reference solve met a zero pivot
  int lu_nb;              // LU panel width of this grid's recomputes
  int direct;             // 1: full-size recompute (no references), 0: reduced form
  int ref_nb;             // LU panel width of this grid's reference solves
  int ref_pg;             // 1: the reference solves keep their LU panel in the workspace
  int unit_base;          // index of chain 0 of this grid in the per-launch chain arrays
  double gp, gm;          // e^{2 lambda} - 1, e^{-2 lambda} - 1  (flip factors gamma)
  double ep, em;          // e^{lambda} - 1,   e^{-lambda} - 1    (Dyson matrix diagonal)
  const double* G0;       // L x L bath matrix, row-major
  double* acc_g;          // [n_chains][n_bins][L+1] sums of G(tau_k)
  double* acc_d;          // [n_chains][n_bins] sums of D
  long long* acc_n;       // [n_chains][n_bins] measurement counts
  long long* cstats;      // [n_chains][NSTAT]
  double* cdrift;         // [n_chains] max elementwise recompute drift
  double* cdrift_gt;      // [n_chains] max drift of the G(tau) estimator at sampled recomputes
  long long* flip_log;    // [n_chains][flip_cap] or null
  const long long* replay;    // [n_chains][replay_cap] or null
  const long long* replay_n;  // [n_chains] or null
  double* g_final;        // [n_chains][2][L][L] or null
  double* g_out;          // [L+1] chain-reduced G(tau)
  double* g_err;          // [L+1]
  double* d_out;          // [2] D and its error
  const double* G0d;      // spin-down bath matrix (G0 itself unless the baths are spin-dependent)
  const double* refQd[2]; // spin-down references (refQ, refH themselves unless spin-dependent)
  const double* refHd[2];
  int spin;               // 1: spin-dependent baths; accumulators and outputs per spin,
                          //    [..][2][L+1] (up, down) in place of [..][L+1]
};

struct SweepParams {
  const GridDev* grids;
  int n_grids;
  const int* units;       // dispatch order, entry = (grid << 20) | chain
  int n_units;
  int* queue;             // work-queue counter (zeroed before launch)
  unsigned long long seed;
  long long warmup, sweeps;
  int n_rec;              // accepted flips between recomputes
  int mode;
  int delay_k;            // max pending flips (delayed modes)
  int window_b;           // max slices per window (delayed modes)
  int n_bins;
  int lu_nb;              // widest LU panel of the launch (per grid: GridDev::lu_nb)
  long long flip_cap, replay_cap;
  double* work;           // per-workgroup workspace
  long long work_stride;  // doubles per workgroup
  int Lmax;
  int lds_scratch_bytes;  // bytes of the phase-shared LDS region
  int heat_bath;          // 1: accept iff u < R/(1+R); 0: Metropolis, u < R
  int direct;             // 1: recompute with the full L x L system (no reference reduction)
  int ph;                 // 1: particle-hole symmetric bath, only G_up kept (G_dn = 1 - G_up^T)
  int spin;               // 1: spin-dependent baths (GridDev::spin)
  int pg;                 // 1: the LU panel lives in the workspace instead of LDS (large L)
  int drift_every;        // the drift is taken on recompute 1, 1 + drift_every, ... of a chain
};

constexpr int kThreads = 512;   // threads per persistent workgroup (8 wave64)
constexpr int kNBMax = 32;      // largest LU panel width
constexpr int kMaxK = 64;       // largest delayed rank

// Workspace doubles of the estimator kept across a sampled recompute (two per lag).
constexpr long long gtd_doubles(int Lmax) { return (2LL * (Lmax + 1) + 63) & ~63LL; }
// Workspace (doubles) needed per workgroup for chains of length up to Lmax.
long long workspace_doubles(int Lmax, int kmax);
// The LU panel's share of it, at its end ([Lmax + kNBMax][kNBMax + 2] doubles):
// where LDS cannot hold a 16-wide panel of the reduced system, the panel moves
// there and the recompute keeps the matrix-core path.
constexpr long long panel_doubles(int Lmax) { return (long long)(Lmax + kNBMax) * (kNBMax + 2); }
// Dynamic LDS bytes of the persistent kernel for a grid of L slices in a launch
// whose longest grid has Lmax (the head and the update buffers are sized for
// Lmax), and that grid's LU panel width (the widest that fits the LDS budget,
// at most nb_max).  direct = 0 sizes the LU for the reduced system (at most
// L/2 rows; the reduced form's product streams G[S,:] through LDS in slabs
// that fit); the reference kernel uses direct = 1.  pg = 1: the panel is in the
// workspace (panel_doubles), LDS holds the rest of the LU's state.
int lds_bytes(int Lmax, int L, int mode, int nb_max, int direct, int* lu_nb, int* scratch_bytes,
              int pg = 0);
// Sets the kernel's dynamic-LDS limit (needed above 64 KiB); call before a
// launch or a stream capture.
hipError_t prepare_sweeps(int lds);

hipError_t launch_build_g0(const double* g_tau, int L, double* G0, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, long long n, hipStream_t s);
hipError_t launch_zero(double* p, long long n, hipStream_t s);
hipError_t launch_zero_i64(long long* p, long long n, hipStream_t s);
hipError_t launch_zero_i32(int* p, long long n, hipStream_t s);
hipError_t launch_sweeps(const SweepParams& p, int n_wg, int lds, hipStream_t s);
// Uniform-field reference matrices (Q_r, H_r, r = 0, 1) of every grid: 4
// workgroups per grid, direct LU with the grid's panel width ref_nb,
// workspace slots 0..4 n_grids-1.
hipError_t prepare_reference(int lds);
hipError_t launch_reference(const SweepParams& p, int lds, int scratch, int dn, hipStream_t s);
hipError_t launch_reduce(const GridDev* grids, int n_grids, int n_bins, hipStream_t s);

// The allocation-free entry point (hfqmc_noalloc.hip): a static device buffer of
// kNoAllocBytes per GPU holds everything a single-grid solve needs besides the
// caller's inputs and outputs.
constexpr size_t kNoAllocBytes = (size_t)128 << 20;
struct NoAllocSummary {
  long long stats[NSTAT];   // per-chain counters summed over the chains
  double max_drift, max_drift_gtau;
  int nonfinite;            // a reduced output (G(tau), its error, D) is not finite
  int ref_singular;         // a uniform-field reference solve met a zero pivot
};
// Device address of device `device`'s buffer: looked up on the first call for that
// device, which must be current then (hfqmc_create makes that call).
hipError_t noalloc_scratch_lookup(int device, void** out);
hipError_t launch_put_grid(const GridDev& g, GridDev* dst, hipStream_t s);
hipError_t launch_iota(int* p, int n, hipStream_t s);
hipError_t launch_noalloc_summary(const GridDev* gd, NoAllocSummary* out, hipStream_t s);

// The method's uniforms (hfqmc_rng.hip): out[s L + l] for slices l < L and
// sweeps sweep0 .. sweep0 + n_sweeps - 1 of one (key0, grid, stream).
hipError_t launch_uniforms(uint64_t key0, uint64_t grid, long long sweep0, long long n_sweeps,
                           int L, uint64_t stream, double* out, hipStream_t s);

// Achievable-peak probes (hfqmc_peaks.hip).  Copy / read: n16 16-byte
// elements of src (and dst); out holds blocks * peak_threads() doubles.
enum { PEAK_COPY = 0, PEAK_READ = 1, PEAK_MFMA64 = 2, PEAK_MFMA32 = 3, PEAK_FMA64 = 4 };
hipError_t launch_peak(int kind, const void* src, void* dst, long long n16, int blocks, int iters,
                       double* out, hipStream_t s);
double peak_flops(int kind, int blocks, int iters);
int peak_threads();

// Chain-split planner (hfqmc_sched.cpp): grid i of a launch runs
// n_chains * factor[i] chains of sweeps / factor[i] measured sweeps each, factor[i]
// a power of two up to kMaxChainSplit dividing sweeps with sweeps / factor[i] >=
// n_bins, chosen to shorten the simulated longest-first dispatch over n_workers
// workgroups.  The spans are in the cost model's units.
constexpr int kMaxChainSplit = 64;
constexpr long long kMaxPlannedChains = 1 << 13;   // larger launches are left unsplit
double unit_cost(int L, long long warmup, long long sweeps);
double lpt_makespan(const std::vector<double>& cost, int n_workers);
int plan_chain_split(int n_grids, const int* Ls, int n_chains, long long warmup, long long sweeps,
                     int n_bins, int n_workers, int* factor, double* span_before,
                     double* span_after);

}  // namespace hfqmc
