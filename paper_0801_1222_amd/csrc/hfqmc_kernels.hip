// gfx950 kernels of the Hirsch-Fye QMC hot path.
//
// One persistent workgroup runs one Markov chain at a time (both spins,
// because the acceptance ratio is the product R_up R_dn), pulling
// (grid, chain) units from an atomic work queue in longest-first order, so
// grids of different L share one launch.  Per chain:
//   chain init      field from Philox stream 1, exact G from the Dyson recompute
//   sweep           l = 0..L-1: ratio R_sigma = 1 + gamma_sigma (1 - G_sigma(l,l)),
//                   Metropolis test u < R_up R_dn, Dyson update of both G on accept
//   recompute       every n_rec accepted flips: [1 + (1-G0)(e^V-1)] G = G0 by a
//                   blocked FP64 LU with partial pivoting inside the workgroup
//   measurement     after every measured sweep: translation/spin-averaged G(tau_k), D
// The formulas are the standard Hirsch-Fye ones that the paper relies on
// (Introduction: Trotter slices, binary HS field, MC sampling).  The sweep
// kernel comes in four instantiations (run_chain's VAR): every update mode
// chosen at run time; the mixed mode with G stored in FP32; spin-dependent
// baths; and the first with the LU panel in the workspace for long grids.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "hfqmc_internal.h"
#include "hfqmc_philox.h"

namespace hfqmc {

// ------------------------------------------------------------ utilities ----

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the workgroup; every thread gets the result.  `red` holds kThreads/64 doubles.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) s += red[i];
  return s;
}

__device__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < kThreads / 64; ++i) s = fmax(s, red[i]);
  return s;
}

// Ratio factor of one spin, evaluated in the same three roundings as
// 1 + g * (1 - G_ll) written out (no fused multiply-add), so the acceptance
// decisions are reproducible on any IEEE FP64 implementation.
__device__ __forceinline__ double ratio_factor(double g, double gll) {
#pragma clang fp contract(off)
  const double a = 1.0 - gll;
  const double b = g * a;
  return 1.0 + b;
}

__device__ __forceinline__ double mul_nc(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}

__device__ __forceinline__ double axpy_nc(double g, double x, double y) {
#pragma clang fp contract(off)
  const double p = x * y;
  return g + p;
}

// ----------------------------------------------------------- G0 build ----
// G0[i][j] = g(tau_{i-j}) for i >= j, -g(tau_{i-j+L}) for i < j.
__global__ void k_build_g0(const double* __restrict__ g, int L, double* __restrict__ G0) {
  const long long n = (long long)L * L;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(idx / L), j = (int)(idx - (long long)i * L);
    const int d = i - j;
    G0[idx] = d >= 0 ? g[d] : -g[d + L];
  }
}

// Device-to-device copy by a kernel: works on any device address of the
// process (also memory another HIP runtime in the process allocated).
__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <typename T>
__global__ void k_zero(T* p, long long n) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x)
    p[idx] = T(0);
}

// ----------------------------------------------------- chain context ----

// Global-memory views of pointers the compiler cannot place itself (loaded from
// device structs): global_load/store instead of flat accesses, which would also
// count against the LDS wait counter.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) float gfloat;
// global element type of the stored Green matrices: FP64, or FP32 where G is
// kept in single precision between recomputes
template <typename GT> struct GlobalOf;
template <> struct GlobalOf<double> { typedef gdouble type; };
template <> struct GlobalOf<float> { typedef gfloat type; };

constexpr int kStatBytes = 256;   // LDS statistics block: NSTAT counters + two drifts
static_assert(NSTAT * 8 + 16 <= kStatBytes, "statistics block too small");
constexpr int kUW = 64;           // acceptance uniforms held in LDS at a time

// Acceptance uniforms u(l, sweep) (stream 0) of slices l0 .. l0 + n - 1 into uw.
// The leading barrier orders the stores after every wave's reads of the previous
// block: a rejected proposal reaches no barrier of its own.
__device__ __forceinline__ void fill_uniforms(double* uw, uint64_t key0, uint64_t grid, long long sw,
                                              int l0, int n) {
  __syncthreads();
  if ((int)threadIdx.x < n)
    uw[threadIdx.x] = uniform53(key0, grid, (uint64_t)(l0 + threadIdx.x), (uint64_t)sw, 0ull);
  __syncthreads();
}

struct Chain {
  const double* G0;
  double ep, em;
  double* accg;    // this chain's [n_bins][L+1]
  double* accd;    // [n_bins]
  long long* accn; // [n_bins]
  int L;
  int chain;
  uint64_t key0;
  double* Gu;
  double* Gd;
  double* A;       // L x 2L LU workspace
  double* Ui;      // U11^{-1} blocks of the LU
  double* wbuf;    // delayed-update buffers
  int8_t* s;       // field, LDS
  double* uw;      // LDS [kUW]: acceptance uniforms of the current block of slices
  int grid;        // Philox key word 1
  char* scratch;   // phase-shared LDS
  int scratch_bytes;
  double* red;     // reduction scratch, LDS
  long long* st;   // per-chain statistics [NSTAT] (ST_*), LDS, written by thread 0 only
  double* drift;   // largest recompute drift so far, LDS, thread 0 only
  double* drift_gt;  // largest drift of the G(tau) estimator so far, LDS, thread 0 only
  double* gtd;     // workspace [2 (Lmax + 1)]: the estimator before a sampled recompute
  int* sr;         // LDS [L] at the start of the scratch during a reduced solve: S, then R
  const double* refQ[2];
  const double* refH[2];
  int lu_nb;       // LU panel width of this grid
  bool reduced;    // recompute against the uniform-field references
  const double* G0d;      // spin-down bath and references (spin-dependent baths)
  const double* refQd[2];
  const double* refHd[2];
  double* Pg;             // LU panel in the workspace (large L)
};

// Control state every thread keeps (uniform); the statistics live in LDS.
struct Counters {
  long long rep_i;   // next entry of the replay list
  int acc_since;     // accepted flips since the last recompute
  int n_rec;         // recomputes so far (the initial one not counted)
};

// The drift (updated G against its recompute) is sampled on the first and
// every `every`-th recompute of a chain (SweepParams::drift_every, 8 unless the
// caller asks otherwise; 1 samples all).  Before the others the pending flips
// are not flushed: the recompute replaces G by the exact G of the field, which
// already holds those flips, so the chain is unchanged.
__device__ __forceinline__ bool drift_sampled(int j, int every) { return (j - 1) % every == 0; }

// Adds v to statistic `which` (thread 0 keeps the LDS copy).
__device__ __forceinline__ void stat_add(long long* st, int which, long long v) {
  if (threadIdx.x == 0) st[which] += v;
}

// ------------------------------------------------ Dyson recompute (LU) ----
//
// Solve [1 + (1 - G0) diag(e^{V_sigma} - 1)] G_sigma = G0 for one spin with
// the augmented matrix A = [M | G0] in the workspace, padded to np = a
// multiple of the panel width NB (identity rows/columns and zero right-hand
// sides in the padding, which never become pivots).  Right-looking blocked
// LU with partial pivoting, then blocked back substitution:
//   panel   all waves; each thread keeps its panel rows in registers, one
//           pivot search (workgroup argmax) and one row exchange per column;
//           L11, U11 and L21 end in LDS, U11 also in A;
//   strip   each thread owns a column pair right of the panel: row
//           interchanges, U12 = L11^{-1} A12 in registers, then
//           A22 -= L21 U12 streamed over the trailing rows (right-hand side
//           included) in prefetched chunks;
//   back    per block from the bottom: X_b = U11^{-1} Y_b in registers, then
//           Y_above -= U01 X_b streamed the same way.
// Writes the new G into Gs and returns the largest elementwise change
// (drift) against the G it replaces.

constexpr int kRowChunk = 4;   // rows in flight per thread in the strip passes

// C[i][c] -= sum_j Q[i - qrow0][j] * u[j] for i in [r0, r1); Q in LDS (row stride qs,
// 16-byte aligned rows, read as broadcast pairs).
template <int NB>
__device__ __forceinline__ void strip_stream(double* __restrict__ A, int lda, int r0, int r1, int c,
                                             const double* __restrict__ Q, int qs, int qrow0,
                                             const double (&u)[NB]) {
  double cur[kRowChunk], nxt[kRowChunk];
#pragma unroll
  for (int b = 0; b < kRowChunk; ++b)
    if (r0 + b < r1) cur[b] = A[(r0 + b) * lda + c];
#pragma unroll 1
  for (int i0 = r0; i0 < r1; i0 += kRowChunk) {
    const int i1 = i0 + kRowChunk;
#pragma unroll
    for (int b = 0; b < kRowChunk; ++b)
      if (i1 + b < r1) nxt[b] = A[(i1 + b) * lda + c];
#pragma unroll
    for (int b = 0; b < kRowChunk; ++b) {
      const int i = i0 + b;
      if (i < r1) {
        const double2* q2 = reinterpret_cast<const double2*>(Q + (i - qrow0) * qs);
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int jj = 0; jj < NB / 2; ++jj) {
          const double2 qv = q2[jj];
          s0 = fma(qv.x, u[2 * jj], s0);
          s1 = fma(qv.y, u[2 * jj + 1], s1);
        }
        A[i * lda + c] = cur[b] - (s0 + s1);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int b = 0; b < kRowChunk; ++b) cur[b] = nxt[b];
  }
}

// Forward strip after the panel at kb: per column c right of the panel, apply
// the row interchanges, U12 = L11^{-1} A12 in registers, then A22 -= L21 U12.
// P holds the factored panel rows (stride ps).
template <int NB>
__device__ __forceinline__ void lu_strip_forward(double* __restrict__ A, int lda, int kb, int np,
                                                 int cend, const double* __restrict__ P, int ps,
                                                 const int* __restrict__ piv) {
  for (int c = kb + NB + (int)threadIdx.x; c < cend; c += kThreads) {
#pragma unroll 1
    for (int j = 0; j < NB; ++j) {
      const int pj = piv[j];
      if (pj != j) {
        double* a = A + (kb + j) * lda + c;
        double* b = A + (kb + pj) * lda + c;
        const double tmp = *a;
        *a = *b;
        *b = tmp;
      }
    }
    double u[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) u[j] = A[(kb + j) * lda + c];
#pragma unroll
    for (int j = 0; j < NB - 1; ++j) {
#pragma unroll
      for (int r = j + 1; r < NB; ++r) u[r] = fma(-P[r * ps + j], u[j], u[r]);
      // one column of L11 at a time: hoisting all its LDS reads would spill
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 1; j < NB; ++j) A[(kb + j) * lda + c] = u[j];
    strip_stream<NB>(A, lda, kb + NB, np, c, P, ps, kb, u);
  }
}

// Backward strip for the block at kb: per right-hand-side column, X_b =
// U11^{-1} Y_b in registers, then Y[0:kb] -= U01 X_b.  P rows 0..kb-1 hold
// U01, rows kb..kb+NB-1 hold U11 (stride ps).
template <int NB>
__device__ __forceinline__ void lu_strip_backward(double* __restrict__ A, int lda, int kb, int np,
                                                  int cend, const double* __restrict__ P, int ps) {
  for (int c = np + (int)threadIdx.x; c < cend; c += kThreads) {
    double u[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) u[j] = A[(kb + j) * lda + c];
#pragma unroll
    for (int j = NB - 1; j >= 0; --j) {
      u[j] = u[j] / P[(kb + j) * ps + j];
#pragma unroll
      for (int r = 0; r < j; ++r) u[r] = fma(-P[(kb + r) * ps + j], u[j], u[r]);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) A[(kb + j) * lda + c] = u[j];
    strip_stream<NB>(A, lda, 0, kb, c, P, ps, 0, u);
  }
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

// Orders a wave's global stores before its later loads of the same data by
// other lanes (the workgroup shares one L1).
__device__ __forceinline__ void wave_global_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Strip passes on the matrix cores (NB = 16 or 32).  v_mfma_f64_16x16x4f64
// operand layout, lane l = 16 q + i:  A[i][k=q], B[k=q][j=i], D[4 r + q][i]
// (register r of the accumulator; note the f32 16x16x4 variant uses D[4 q + r][i]).
// Each wave owns 16-column tiles; its B operand (NB x 16) stays in registers
// while the trailing 16-row blocks stream through the accumulators.
//
constexpr int kRB = 4;   // 16-row blocks in flight per wave

// Rows [r0, r1) (multiples of 16) of the wave's 16-column tile at column
// c = c0 + (lane & 15):  C -= Q B, Q = P rows (r - qrow0) (NB wide, stride ps),
// B = the tile's NB x 16 operand held in registers in B layout.  Row r of
// the factorization lives in physical row perm[r] of A.
template <int NB>
__device__ __forceinline__ void mfma_rows_update(double* __restrict__ A, int lda, int r0, int r1,
                                                 int c, const double* __restrict__ P, int ps,
                                                 int qrow0, const double (&b)[NB / 4],
                                                 const int* __restrict__ perm) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
#pragma unroll 1
  for (int rb = r0; rb < r1; rb += 16 * kRB) {
    // blocks past r1 re-read the last block (in bounds) and are not stored
    doublex4 acc[kRB];
    double qa[kRB][NB / 4];
    int prow[kRB][4];
#pragma unroll
    for (int g = 0; g < kRB; ++g) {
      const int rr = min(rb + 16 * g, r1 - 16);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        prow[g][r] = perm[rr + lq + 4 * r];
        acc[g][r] = A[prow[g][r] * lda + c];
      }
      const double* pa = P + (rr - qrow0 + li) * ps + lq;
#pragma unroll
      for (int m = 0; m < NB / 4; ++m) qa[g][m] = -pa[4 * m];
    }
#pragma unroll
    for (int g = 0; g < kRB; ++g) {
#pragma unroll
      for (int m = 0; m < NB / 4; ++m)
        acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[g][m], b[m], acc[g], 0, 0, 0);
    }
#pragma unroll
    for (int g = 0; g < kRB; ++g) {
      const int rr = rb + 16 * g;
      if (rr < r1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) A[prow[g][r] * lda + c] = acc[g][r];
      }
    }
  }
}

// Forward, panel at kb: U12 = L11^{-1} A12 (Li = L11^{-1} in LDS, stride ls),
// then A22 -= L21 U12 with L21 = P rows NB.. (stride ps).  Row interchanges
// must already be applied.
template <int NB>
__device__ __forceinline__ void lu_strip_forward_mfma(double* __restrict__ A, int lda, int kb,
                                                      int np, int cend16,
                                                      const double* __restrict__ P, int ps,
                                                      const double* __restrict__ Li, int ls,
                                                      const int* __restrict__ perm) {
  constexpr int KS = NB / 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  int bphys[KS];
#pragma unroll
  for (int m = 0; m < KS; ++m) bphys[m] = perm[kb + 4 * m + lq];
  for (int c0 = kb + NB + 16 * wv; c0 < cend16; c0 += 16 * (kThreads / 64)) {
    const int c = c0 + li;
    double b[KS];
#pragma unroll
    for (int m = 0; m < KS; ++m) b[m] = A[bphys[m] * lda + c];
#pragma unroll
    for (int ob = 0; ob < NB / 16; ++ob) {
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < KS; ++m)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Li[(16 * ob + li) * ls + 4 * m + lq], b[m], acc,
                                                   0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) A[perm[kb + 16 * ob + 4 * r + lq] * lda + c] = acc[r];
    }
    wave_global_sync();
#pragma unroll
    for (int m = 0; m < KS; ++m) b[m] = A[bphys[m] * lda + c];
    mfma_rows_update<NB>(A, lda, kb + NB, np, c, P, ps, kb, b, perm);
  }
}

// Backward, block at kb: X_b = U11^{-1} Y_b (Li = U11^{-1}), then
// Y[0:kb] -= U01 X_b with U01 = P rows 0..kb-1.
template <int NB, typename GT>
__device__ __forceinline__ void lu_strip_backward_mfma(double* __restrict__ A, int lda, int kb,
                                                       int np, int cend16,
                                                       const double* __restrict__ P, int ps,
                                                       const double* __restrict__ Li, int ls,
                                                       typename GlobalOf<GT>::type* __restrict__ Gs,
                                                       int ns, int L,
                                                       const int* __restrict__ rowmap,
                                                       double& dmax,
                                                       const int* __restrict__ perm,
                                                       bool drift) {
  constexpr int KS = NB / 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  int bphys[KS];
#pragma unroll
  for (int m = 0; m < KS; ++m) bphys[m] = perm[kb + 4 * m + lq];
  for (int c0 = np + 16 * wv; c0 < cend16; c0 += 16 * (kThreads / 64)) {
    const int c = c0 + li;
    const int gc = c - np;   // column of G
    double b[KS];
#pragma unroll
    for (int m = 0; m < KS; ++m) b[m] = A[bphys[m] * lda + c];
    // the updated G this block's final rows replace (for the drift); solution
    // row i is row rowmap[i] of G (identity without a map)
    double gold[NB / 16][4];
    int grow[NB / 16][4];
#pragma unroll
    for (int ob = 0; ob < NB / 16; ++ob)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = kb + 16 * ob + 4 * r + lq;
        const bool ok = row < ns && gc < L;
        grow[ob][r] = ok ? (rowmap ? rowmap[row] : row) : 0;
        gold[ob][r] = 0.0;
      }
    if (drift) {
#pragma unroll
      for (int ob = 0; ob < NB / 16; ++ob)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = kb + 16 * ob + 4 * r + lq;
          if (row < ns && gc < L) gold[ob][r] = Gs[grow[ob][r] * L + gc];
        }
    }
#pragma unroll
    for (int ob = 0; ob < NB / 16; ++ob) {
      doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < KS; ++m)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Li[(16 * ob + li) * ls + 4 * m + lq], b[m], acc,
                                                   0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = kb + 16 * ob + 4 * r + lq;
        A[perm[row] * lda + c] = acc[r];
        if (row < ns && gc < L) {
          // rows kb.. are final: write G and record the drift
          const double x = acc[r];
          if (drift) dmax = fmax(dmax, fabs(x - gold[ob][r]));
          if (!(fabs(x) < INFINITY)) dmax = INFINITY;
          Gs[grow[ob][r] * L + gc] = x;
        }
      }
    }
    wave_global_sync();
#pragma unroll
    for (int m = 0; m < KS; ++m) b[m] = A[bphys[m] * lda + c];
    mfma_rows_update<NB>(A, lda, 0, kb, c, P, ps, 0, b, perm);
  }
}

// Max of a 64-bit key over the 16 lanes of each row of the wave (xor
// butterfly on DPP: quad permutations, then half-row and row mirrors).
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

__device__ __forceinline__ unsigned long long wave_max_key(unsigned long long k) {
  unsigned long long o;
  o = dpp_u64<0xB1>(k);   // quad_perm [1,0,3,2]
  k = o > k ? o : k;
  o = dpp_u64<0x4E>(k);   // quad_perm [2,3,0,1]
  k = o > k ? o : k;
  o = dpp_u64<0x141>(k);  // row_half_mirror
  k = o > k ? o : k;
  o = dpp_u64<0x140>(k);  // row_mirror
  k = o > k ? o : k;
  unsigned long long m = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)k, 16 * r);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(k >> 32), 16 * r);
    const unsigned long long v = ((unsigned long long)hi << 32) | lo;
    m = v > m ? v : m;
  }
  return m;
}

// Panel factorization (partial pivoting) with the panel rows in registers.
// Thread t owns the physical rows t + q kThreads and tracks the position each
// one currently occupies (row interchanges only swap positions).  A row's
// registers hold a window that shifts left by one slot per eliminated column
// (slots 0..NB-1-j are its columns j..NB-1 before step j; the slots beyond
// hold values nothing reads), so the pivot column is always slot 0.  The
// multiplier of each step goes to LDS, indexed by physical row, in the P
// buffer that receives the factored rows in position order at the end.
// Pivot search: key = |a| with its 10 low mantissa bits replaced by
// 1023 - physical row (largest magnitude; ties and near-ties resolved by the
// row), reduced over the wave on DPP; each wave stages its best row with its
// position and reciprocal in LDS (double-buffered), so one barrier per
// column suffices.  U11 also goes to A; piv[j] = position exchanged with j.
template <int NB>
__device__ __forceinline__ void panel_factor_regs(double* __restrict__ A, int lda, int kb, int rows,
                                                  double* __restrict__ P, int ps,
                                                  double* __restrict__ cand,
                                                  unsigned long long* __restrict__ keys,
                                                  int* __restrict__ piv, int* sing,
                                                  int* __restrict__ perm) {
  constexpr int RPT = 512 / kThreads * (NB == 32 ? 1 : 2);
  constexpr int NW = kThreads / 64;
  constexpr int CS = NB + 2;   // staged candidate: window, reciprocal, position
  const int t = threadIdx.x, wv = t >> 6;
  double pr[RPT][NB];
  int pos[RPT], fz[RPT], phys[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = t + q * kThreads;
    pos[q] = r;
    fz[q] = NB;
    phys[q] = perm[kb + min(r, rows - 1)];
#pragma unroll
    for (int c = 0; c < NB; ++c) pr[q][c] = (r < rows) ? A[phys[q] * lda + kb + c] : 0.0;
  }
  // the old contents of P (previous panel) must have been consumed
  __syncthreads();
  // waves without rows only keep the barriers
  const int nwa = (min(rows, kThreads) + 63) >> 6;
  const bool wact = wv < nwa;
#pragma unroll 1
  for (int j = 0; j < NB; ++j) {
    if (wact) {
      unsigned long long best = 0;
      int bq = 0;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const bool act = pos[q] >= j && pos[q] < rows;
        const unsigned long long bits =
            (unsigned long long)__double_as_longlong(fabs(pr[q][0])) & ~0x3FFull;
        const unsigned long long key =
            act ? (bits | (unsigned long long)(1023 - (t + q * kThreads))) : 0ull;
        if (key > best) {
          best = key;
          bq = q;
        }
      }
      const double head = (RPT == 2 && bq) ? pr[RPT - 1][0] : pr[0][0];
      const double hinv = 1.0 / head;   // used only if this row wins
      const unsigned long long wbest = wave_max_key(best);
      if (best == wbest && wbest != 0ull) {
        double* cw = cand + wv * CS;
#pragma unroll
        for (int c = 0; c < NB; ++c) cw[c] = (RPT == 2 && bq) ? pr[RPT - 1][c] : pr[0][c];
        cw[NB] = hinv;
        cw[NB + 1] = (double)((RPT == 2 && bq) ? pos[RPT - 1] : pos[0]);
        keys[wv] = wbest;
      } else if (wbest == 0ull && (t & 63) == 0) {
        keys[wv] = 0ull;
      }
    }
    __syncthreads();
    if (wact) {
      unsigned long long gk = keys[0];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        const unsigned long long o = (w < nwa) ? keys[w] : 0ull;
        gk = o > gk ? o : gk;
      }
      const int gw = ((1023 - (int)(gk & 0x3FFull)) & (kThreads - 1)) >> 6;
      double prow[CS];
      {
        const double2* c2 = reinterpret_cast<const double2*>(cand + gw * CS);
#pragma unroll
        for (int c = 0; c < CS / 2; ++c) {
          const double2 v = c2[c];
          prow[2 * c] = v.x;
          prow[2 * c + 1] = v.y;
        }
      }
      const double pv = prow[0];
      const double rinv = prow[NB];
      const int gp = (int)prow[NB + 1];
      if (t == 0) {
        piv[j] = gp;
        if (!(fabs(pv) > 0.0 && fabs(pv) < INFINITY)) *sing = 1;
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (pos[q] == gp)
          pos[q] = j;
        else if (pos[q] == j)
          pos[q] = gp;
        if (pos[q] == j) {
          fz[q] = j;
        } else if (pos[q] > j && pos[q] < rows) {
          const double l = pr[q][0] * rinv;
          P[(t + q * kThreads) * ps + j] = l;
#pragma unroll
          for (int c = 0; c + 1 < NB; ++c) pr[q][c] = fma(-l, prow[c + 1], pr[q][c + 1]);
        }
      }
    }
    cand += (j & 1) ? -NW * CS : NW * CS;
    keys += (j & 1) ? -NW : NW;
  }
  __syncthreads();
  // multipliers (by physical row) -> registers, then every row to its position
  double lm[RPT][NB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = t + q * kThreads;
#pragma unroll
    for (int c = 0; c < NB; ++c) lm[q][c] = (r < rows) ? P[r * ps + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = pos[q];
    const int r0 = t + q * kThreads;
    if (r0 < rows) {
      const int f = fz[q];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < f) P[r * ps + c] = lm[q][c];
        if (c < NB - f) {
          P[r * ps + f + c] = pr[q][c];
          A[phys[q] * lda + kb + f + c] = pr[q][c];
        }
      }
      // the interchanges only relabel rows: position kb + r is now physical row phys
      perm[kb + r] = phys[q];
    }
  }
  __syncthreads();
}

// L11^{-1} (unit lower) and U11^{-1} of the factored panel in P, one column
// per lane, rows in registers (fully unrolled, uniform loops: the entries
// above / below the diagonal come out as exact zeros).
template <int NB>
__device__ __forceinline__ void tri_inverse_lower(const double* __restrict__ P, int ps,
                                                  double* __restrict__ Li, int ls) {
  const int j = threadIdx.x & 63;
  if (j >= NB) return;
  double x[NB];
#pragma unroll
  for (int r = 0; r < NB; ++r) {
    double acc = (r == j) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < r; ++q) acc = fma(-P[r * ps + q], x[q], acc);
    x[r] = acc;
  }
#pragma unroll
  for (int r = 0; r < NB; ++r) Li[r * ls + j] = x[r];
}

template <int NB>
__device__ __forceinline__ void tri_inverse_upper(const double* __restrict__ P, int ps,
                                                  double* __restrict__ Ui) {
  const int j = threadIdx.x & 63;
  if (j >= NB) return;
  double x[NB];
#pragma unroll
  for (int r = NB - 1; r >= 0; --r) {
    double acc = (r == j) ? 1.0 : 0.0;
#pragma unroll
    for (int q = r + 1; q < NB; ++q) acc = fma(-P[r * ps + q], x[q], acc);
    x[r] = acc / P[r * ps + r];
  }
#pragma unroll
  for (int r = 0; r < NB; ++r) Ui[r * NB + j] = x[r];
}

// Exclusive prefix sum of v over the workgroup (thread order); *total gets the
// sum.  `red` holds kThreads/64 + 1 ints.
__device__ __forceinline__ int block_exclusive_scan(int v, int* red, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) red[wv] = x;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const int r = red[w];
    before += (w < wv) ? r : 0;
    tot += r;
  }
  // the same in every lane: made uniform for the compiler (scalar control flow)
  *total = __builtin_amdgcn_readfirstlane(tot);
  return before + x - v;
}

// The reduced form's product G[R,:] = H_r[R,:] - c Q_r[R,S] G[S,:] for systems
// whose G[S,:] does not fit LDS even 16 columns wide (L beyond about 1000): K
// is streamed in slabs of kc rows through LDS (Zl), the partial sums of G[R,:]
// kept in the workspace Pq.  Kept light in registers (short operand batches,
// the drift's old values read at the store) so that it adds no pressure to
// the sweep kernel; returns this thread's largest drift (the caller reduces it).
template <typename GT>
__device__ __forceinline__ double reduced_product_slabs(
    const double* __restrict__ Aq, double* __restrict__ Pq, double* __restrict__ Zl,
    GT* __restrict__ Gs_, const double* __restrict__ Hr_, const int* __restrict__ sr, int ns,
    int nR, int kr, int L, long long lu_scr_bytes, bool drift) {
  typename GlobalOf<GT>::type* __restrict__ Gs = (typename GlobalOf<GT>::type*)Gs_;
  gcdouble* __restrict__ Hr = (gcdouble*)Hr_;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int* Rl = sr + ns;
  double dmax = 0.0;
  int zw = 64;
  while (zw > 16 && (long long)kr * (zw + 2) * 8 > lu_scr_bytes) zw >>= 1;
  int kc = kr;
  if ((long long)kr * (zw + 2) * 8 > lu_scr_bytes)
    kc = max(8, (int)((lu_scr_bytes / ((zw + 2) * 8)) & ~7LL));
  const int zs = zw + 2;
  const int li = lane & 15, lq = lane >> 4;
  const int nrb = (nR + 15) >> 4;
  for (int c0 = 0; c0 < L; c0 += zw) {
    for (int k0 = 0; k0 < kr; k0 += kc) {
      const int kcl = min(kc, kr - k0);                // rows of this slab (8 | kcl)
      const int kcs = kcl >> 2;                        // K steps of this slab (even)
      const bool first = k0 == 0, last = k0 + kcl >= kr;
      __syncthreads();
      // a wave per row, four rows in flight; lanes along the chunk
      for (int i0 = wv; i0 < kcl; i0 += 4 * (kThreads / 64)) {
        for (int j = lane; j < zw; j += 64) {
          double v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = k0 + i0 + u * (kThreads / 64);
            const int gi = sr[min(i, ns - 1)];
            const double g = Gs[gi * L + min(c0 + j, L - 1)];   // clamped: in bounds
            v[u] = (i < ns && c0 + j < L) ? g : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * (kThreads / 64);
            if (i < kcl) Zl[i * zs + j] = v[u];
          }
        }
      }
      __syncthreads();
      const int ntile = (min(zw, L - c0) + 15) >> 4;   // 16-column tiles in this chunk (<= 4)
      for (int rb = wv; rb < nrb; rb += kThreads / 64) {
        // one 16-row block of R against every tile of the chunk; the A operand
        // is prefetched a batch of kGB steps ahead (two register batches in turn)
        constexpr int kGB = 4;
        const int arow = min(rb * 16 + li, nR - 1);
        const double2* arow2 =
            reinterpret_cast<const double2*>(Aq + (long long)arow * kr + k0 + lq * kcs);
        int orow[4], oR[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          orow[r] = rb * 16 + 4 * r + lq;
          oR[r] = Rl[min(orow[r], nR - 1)];
        }
        doublex4 acc[4];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const int col = min(c0 + 16 * tt + li, L - 1);
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc[tt][r] = (tt < ntile) ? (first ? Hr[oR[r] * L + col]
                                               : Pq[(long long)min(orow[r], nR - 1) * L + col])
                                      : 0.0;
        }
        // steps q0.. of this lane's K range (clamped, in bounds: kcs is even)
        auto load_a = [&](int q0, double2 (&av)[kGB / 2]) {
#pragma unroll
          for (int u = 0; u < kGB / 2; ++u) av[u] = arow2[min(q0 / 2 + u, kcs / 2 - 1)];
        };
        auto mma = [&](int q0, const double2 (&av)[kGB / 2]) {
#pragma unroll
          for (int u = 0; u < kGB; ++u) {
            if (q0 + u < kcs) {
              const double a = (u & 1) ? av[u >> 1].y : av[u >> 1].x;
              const double* zb = Zl + (lq * kcs + q0 + u) * zs + li;
#pragma unroll
              for (int tt = 0; tt < 4; ++tt)
                if (tt < ntile)
                  acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, zb[16 * tt], acc[tt], 0, 0, 0);
            }
          }
        };
        double2 a0[kGB / 2], a1[kGB / 2];
        load_a(0, a0);
#pragma unroll 1
        for (int q0 = 0; q0 < kcs; q0 += 2 * kGB) {
          if (q0 + kGB < kcs) load_a(q0 + kGB, a1);
          mma(q0, a0);
          if (q0 + kGB >= kcs) break;
          if (q0 + 2 * kGB < kcs) load_a(q0 + 2 * kGB, a0);
          mma(q0 + kGB, a1);
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
          const int col = c0 + 16 * tt + li;
          if (tt < ntile && col < L && col < c0 + zw) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              if (orow[r] < nR) {
                const double x = acc[tt][r];
                if (last) {
                  // the drift against the updated G the final rows replace
                  if (drift) dmax = fmax(dmax, fabs(x - Gs[oR[r] * L + col]));
                  if (!(fabs(x) < INFINITY)) dmax = INFINITY;
                  Gs[oR[r] * L + col] = x;
                } else {
                  Pq[(long long)orow[r] * L + col] = x;
                }
              }
            }
          }
        }
      }
    }
  }
  return dmax;
}

// ---------------------------------------------------- the Dyson solve ----
//
// Direct form: G_sigma = M^{-1} G0 with M = 1 + K D, K = 1 - G0,
// D = diag(e^{V_sigma} - 1), by the LU of [M | G0].
//
// Reduced form (the default inside the sweep): D takes only the two values
// d_a = e^{lambda} - 1 and d_b = e^{-lambda} - 1.  With the uniform reference
// M_r = 1 + d_r K of the more frequent value d_r (shared by all chains of a
// grid, precomputed as Q_r = M_r^{-1} K and H_r = M_r^{-1} G0) and S the
// slices where D = d_s != d_r (|S| <= L/2), M = M_r + c K P_S with
// c = d_s - d_r, so that (block elimination, exact in exact arithmetic)
//   (1 + c Q_r[S,S]) G[S,:] = H_r[S,:],    G[R,:] = H_r[R,:] - c Q_r[R,S] G[S,:].
// Only the |S| x |S| system goes through the LU; the rest is one GEMM.
//
// Both share the LU below: system [A_sys | B] padded to np (identity rows and
// zero right-hand sides), right-looking with partial pivoting, solution row i
// written to G row map(i).  Returns the largest elementwise change against
// the G it replaces (the drift).
//
// rhs_k (direct form only): right-hand side K = 1 - G0 instead of G0 (the
// reference matrices Q_r).
// drift = false: the G being replaced is not read (no drift is taken)
template <typename GT, bool SPIN = false, bool PG = false>
__device__ __forceinline__ double dyson_solve(const Chain& ch, int sigma, GT* Gs_,
                                              int NB, bool reduced, bool rhs_k,
                                              bool drift = true) {
  const int L = ch.L;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const double ep = ch.ep, em = ch.em;
  const int8_t* s = ch.s;
  typename GlobalOf<GT>::type* __restrict__ Gs = (typename GlobalOf<GT>::type*)Gs_;
  // (SPIN: spin-dependent baths, spin down has a bath and references of its own)
  gcdouble* __restrict__ G0 = (gcdouble*)((SPIN && sigma < 0) ? ch.G0d : ch.G0);
  double* __restrict__ A = ch.A;
  int* sr = ch.sr;                                       // reduced form only
  char* const lu_scr = ch.scratch + (reduced ? ((4 * L + 15) & ~15) : 0);
  const int lu_scr_bytes = ch.scratch_bytes - (int)(lu_scr - ch.scratch);
  long long tc = wall_clock64();

  // ---- the system: all slices (direct) or S (reduced)
  int ns = L;
  double c = 0.0;
  gcdouble* __restrict__ Qr = nullptr;
  gcdouble* __restrict__ Hr = nullptr;
  if (reduced) {
    // slices with D = e^{lambda} - 1 (sigma s_l > 0); the other value forms S
    const int per = (L + kThreads - 1) / kThreads;
    const int l0 = min(t * per, L), l1 = min(l0 + per, L);
    int na = 0;
    for (int l = l0; l < l1; ++l) na += (sigma * s[l] > 0) ? 1 : 0;
    int n_a = 0;
    (void)block_exclusive_scan(na, reinterpret_cast<int*>(ch.red), &n_a);
    const int ref = (n_a >= L - n_a) ? 0 : 1;          // 0: reference d_a, 1: d_b
    c = ref == 0 ? (em - ep) : (ep - em);
    Qr = (gcdouble*)((SPIN && sigma < 0) ? ch.refQd[ref] : ch.refQ[ref]);
    Hr = (gcdouble*)((SPIN && sigma < 0) ? ch.refHd[ref] : ch.refH[ref]);
    const int want = ref == 0 ? -1 : 1;                // sign of sigma s_l on S
    int ms = 0;
    for (int l = l0; l < l1; ++l) ms += (sigma * s[l] == want) ? 1 : 0;
    const int sb = block_exclusive_scan(ms, reinterpret_cast<int*>(ch.red), &ns);
    // S in increasing order first, then R
    int is = sb, ir = ns + (l0 - sb);
    for (int l = l0; l < l1; ++l) {
      if (sigma * s[l] == want) sr[is++] = l;
      else sr[ir++] = l;
    }
    __syncthreads();
    if (ns == 0) {
      // D is uniform: G = H_r
      double dm = 0.0;
      for (int i = wv; i < L; i += kThreads / 64)
#pragma unroll 4
        for (int j = lane; j < L; j += 64) {
          const double x = Hr[i * L + j];
          if (drift) dm = fmax(dm, fabs(x - Gs[i * L + j]));
          if (!(fabs(x) < INFINITY)) dm = INFINITY;
          Gs[i * L + j] = x;
        }
      dm = block_max(dm, ch.red);
      __syncthreads();
      stat_add(ch.st, ST_T_LU_BUILD, wall_clock64() - tc);
      return dm;
    }
    stat_add(ch.st, ST_RED_ROWS, ns);
  }
  const int np = (ns + NB - 1) / NB * NB;
  const int rhs16 = (L + 15) & ~15;
  const int lda = np + (np > rhs16 ? np : rhs16);
  const int ps = NB + 2;              // LDS row stride of the panel (16-byte aligned rows)
  // right-hand-side columns beyond L stay zero and are skipped (up to the
  // next multiple of 16 on the matrix-core path, which works in 16-column tiles)
  const int cend = np + L;
  const int cend16 = np + rhs16;

  // ---- build [A_sys | B]: a wave per row, lanes along it
  for (int i = wv; i < np; i += kThreads / 64) {
    const int gi = reduced ? sr[min(i, ns - 1)] : i;
#pragma unroll 4
    for (int j = lane; j < np; j += 64) {
      double m;
      if (i < ns && j < ns) {
        const double dij = (i == j) ? 1.0 : 0.0;
        if (reduced) {
          m = dij + c * Qr[gi * L + sr[j]];
        } else {
          const double g0 = G0[i * L + j];
          const double f = (sigma * s[j] > 0) ? ep : em;
          m = axpy_nc(dij, dij - g0, f);
        }
      } else {
        m = (i == j) ? 1.0 : 0.0;
      }
      A[i * lda + j] = m;
    }
#pragma unroll 4
    for (int j = lane; j < lda - np; j += 64) {
      double r = 0.0;
      if (i < ns && j < L) {
        if (reduced) r = Hr[gi * L + j];
        else r = rhs_k ? ((i == j ? 1.0 : 0.0) - G0[i * L + j]) : G0[i * L + j];
      }
      A[i * lda + np + j] = r;
    }
  }

  // (PG: the panel in the workspace, the rest of the LU's state in LDS)
  double* P = PG ? ch.Pg : reinterpret_cast<double*>(lu_scr);   // [np][ps]
  const int ls = NB + 1;
  double* Li = PG ? reinterpret_cast<double*>(lu_scr) : P + np * ps;  // [NB][ls] inverted triangle
  double* redv = Li + NB * ls;                           // [kThreads/64]
  int* redi = reinterpret_cast<int*>(redv + kThreads / 64);
  int* piv = redi + kThreads / 64;                       // [NB]
  double* cand = reinterpret_cast<double*>(piv + 32);    // [2][waves][NB] staged candidate rows
  unsigned long long* pkeys =                            // [2][waves] candidate pivot keys
      reinterpret_cast<unsigned long long*>(cand + 2 * (kThreads / 64) * (NB + 2));
  // physical row of each position (the matrix-core path relabels rows instead of
  // exchanging them; the VALU path exchanges rows and keeps the identity)
  int* perm = reinterpret_cast<int*>(pkeys + 2 * (kThreads / 64));  // [np]
  double* Uinv = ch.Ui;                                  // [np / NB][NB][NB] U11^{-1} blocks (HBM)
  if (NB >= 16)
    for (int i = t; i < np; i += kThreads) perm[i] = i;
  __shared__ int s_sing;
  if (t == 0) s_sing = 0;
  __syncthreads();
  {
    const long long t1 = wall_clock64();
    stat_add(ch.st, ST_T_LU_BUILD, t1 - tc);
    tc = t1;
  }

  for (int kb = 0; kb < np; kb += NB) {
    const int rows = np - kb;
    if (NB == 32) {
      panel_factor_regs<32>(A, lda, kb, rows, P, ps, cand, pkeys, piv, &s_sing, perm);
    } else if (NB == 16) {
      panel_factor_regs<16>(A, lda, kb, rows, P, ps, cand, pkeys, piv, &s_sing, perm);
    } else {
      // ---- panel rows kb.., columns kb..kb+NB-1 into LDS, factorized by all waves
      for (int idx = t; idx < rows * NB; idx += kThreads) {
        const int r = idx / NB, cc = idx - r * NB;
        P[r * ps + cc] = A[(kb + r) * lda + kb + cc];
      }
      __syncthreads();
  #pragma unroll 1
      for (int j = 0; j < NB; ++j) {
        double best = -1.0;
        int bi = 1 << 30;
        for (int r = j + t; r < rows; r += kThreads) {
          const double v = fabs(P[r * ps + j]);
          if (v > best) {
            best = v;
            bi = r;
          }
        }
  #pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const double ob = __shfl_xor(best, o, 64);
          const int oi = __shfl_xor(bi, o, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (lane == 0) {
          redv[wv] = best;
          redi[wv] = bi;
        }
        __syncthreads();
        best = redv[0];
        bi = redi[0];
  #pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) {
          const double ob = redv[w];
          const int oi = redi[w];
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (bi >= rows) bi = j;   // no finite candidate: keep the row, flagged below
        if (t == 0) piv[j] = bi;
        if (bi != j && t < NB) {
          const double tmp = P[j * ps + t];
          P[j * ps + t] = P[bi * ps + t];
          P[bi * ps + t] = tmp;
        }
        __syncthreads();
        const double pv = P[j * ps + j];
        if (t == 0 && !(fabs(pv) > 0.0 && fabs(pv) < INFINITY)) s_sing = 1;
        for (int r = j + 1 + t; r < rows; r += kThreads) {
          double* pr = P + r * ps;
          const double l = pr[j] / pv;
          pr[j] = l;
          for (int cc = j + 1; cc < NB; ++cc) pr[cc] = fma(-l, P[j * ps + cc], pr[cc]);
        }
        __syncthreads();
      }
    }
    // U11 -> A for the back substitution (the register panel wrote it already)
    if (NB < 16) {
      for (int idx = t; idx < NB * NB; idx += kThreads) {
        const int r = idx / NB, cc = idx - r * NB;
        if (cc >= r) A[(kb + r) * lda + kb + cc] = P[r * ps + cc];
      }
    }
    {
      const long long t1 = wall_clock64();
      stat_add(ch.st, ST_T_LU_PANEL, t1 - tc);
      tc = t1;
    }
    // ---- strip: U12, trailing update (right-hand side included)
    if (NB >= 16) {
      // wave 0: Li = L11^{-1} (LDS); wave 1: U11^{-1} (kept in HBM for the back
      // substitution)
      if (wv == 0) {
        if (NB == 32) tri_inverse_lower<32>(P, ps, Li, ls);
        else tri_inverse_lower<16>(P, ps, Li, ls);
      } else if (wv == 1) {
        double* Ub = Uinv + (kb / NB) * NB * NB;
        if (NB == 32) tri_inverse_upper<32>(P, ps, Ub);
        else tri_inverse_upper<16>(P, ps, Ub);
      }
      __syncthreads();
      if (NB == 32)
        lu_strip_forward_mfma<32>(A, lda, kb, np, cend16, P, ps, Li, ls, perm);
      else
        lu_strip_forward_mfma<16>(A, lda, kb, np, cend16, P, ps, Li, ls, perm);
    } else {
      switch (NB) {
        case 8: lu_strip_forward<8>(A, lda, kb, np, cend, P, ps, piv); break;
        default: lu_strip_forward<4>(A, lda, kb, np, cend, P, ps, piv); break;
      }
    }
    __syncthreads();
    {
      const long long t1 = wall_clock64();
      stat_add(ch.st, ST_T_LU_STRIP, t1 - tc);
      tc = t1;
    }
  }

  // ---- back substitution on the right-hand-side columns, block rows from the bottom;
  // on the matrix-core path the final rows of each block go straight into G
  const int* rowmap = reduced ? sr : nullptr;
  double dmax = 0.0;
  for (int kb = np - NB; kb >= 0; kb -= NB) {
    // U01 (rows above the block; with U11 on the VALU path) into P, batched loads
    const int prow = NB >= 16 ? kb : kb + NB;
    for (int i0 = wv; i0 < prow; i0 += 4 * (kThreads / 64)) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * (kThreads / 64);
        const int pi = NB >= 16 ? perm[min(i, np - 1)] : i;
        v[u] = (i < prow && lane < NB) ? A[pi * lda + kb + lane] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * (kThreads / 64);
        if (i < prow && lane < NB) P[i * ps + lane] = v[u];
      }
    }
    if (NB >= 16) {
      const double* Ub = Uinv + (kb / NB) * NB * NB;
      for (int idx = t; idx < NB * NB; idx += kThreads) Li[(idx / NB) * ls + (idx % NB)] = Ub[idx];
    }
    __syncthreads();
    if (NB >= 16) {
      if (NB == 32)
        lu_strip_backward_mfma<32, GT>(A, lda, kb, np, cend16, P, ps, Li, ls, Gs, ns, L, rowmap,
                                       dmax, perm, drift);
      else
        lu_strip_backward_mfma<16, GT>(A, lda, kb, np, cend16, P, ps, Li, ls, Gs, ns, L, rowmap,
                                       dmax, perm, drift);
    } else {
      switch (NB) {
        case 8: lu_strip_backward<8>(A, lda, kb, np, cend, P, ps); break;
        default: lu_strip_backward<4>(A, lda, kb, np, cend, P, ps); break;
      }
    }
    __syncthreads();
  }
  if (NB < 16) {
    // G <- X, drift against the updated G (a wave per row)
    for (int i = wv; i < ns; i += kThreads / 64) {
      const int gi = rowmap ? rowmap[i] : i;
#pragma unroll 4
      for (int j = lane; j < L; j += 64) {
        const double x = A[i * lda + np + j];
        if (drift) dmax = fmax(dmax, fabs(x - Gs[gi * L + j]));
        if (!(fabs(x) < INFINITY)) dmax = INFINITY;
        Gs[gi * L + j] = x;
      }
    }
  }

  {
    const long long t1 = wall_clock64();
    stat_add(ch.st, ST_T_LU_BACK, t1 - tc);
    tc = t1;
  }
  // ---- reduced form: G[R,:] = H_r[R,:] - c Q_r[R,S] G[S,:] on the matrix cores.
  // -c Q_r[R,S] is first gathered into a dense row-major block (over the LU
  // workspace, no longer needed); G[S,:] (just written) is staged in LDS by
  // column chunks.  Lane (i, q) of the 16 x 16 x 4 MFMA walks the contiguous K
  // range [q ks, (q + 1) ks): the A operand streams as 16-byte loads.
  if (reduced && ns < L) {
    const int nR = L - ns;
    const int kr = (ns + 7) & ~7;                       // K rows (zero padded, 8 | kr)
    const int ks = kr >> 2;                             // K steps (even)
    const int* Rl = sr + ns;
    double* __restrict__ Aq = A;                        // [nR][kr]
    __syncthreads();   // every read of the LU workspace is done
    for (int j0 = wv; j0 < nR; j0 += 2 * (kThreads / 64)) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int j = j0 + u * (kThreads / 64);
        if (j < nR) {
          gcdouble* qrow = Qr + (long long)Rl[j] * L;
#pragma unroll 4
          for (int i = lane; i < kr; i += 64) Aq[j * kr + i] = (i < ns) ? -c * qrow[sr[i]] : 0.0;
        }
      }
    }
    if ((long long)kr * (16 + 2) * 8 > lu_scr_bytes) {
      // G[S,:] does not fit LDS 16 columns wide: K in slabs (large L)
      dmax = fmax(dmax, reduced_product_slabs(Aq, A + (long long)nR * kr,
                                              reinterpret_cast<double*>(lu_scr), Gs_,
                                              (const double*)Hr, sr, ns, nR, kr, L, lu_scr_bytes,
                                              drift));
    } else {
      int zw = 64;                                        // chunk width
      while (zw > 16 && (long long)kr * (zw + 2) * 8 > lu_scr_bytes) zw >>= 1;
      const int zs = zw + 2;
      double* Zl = reinterpret_cast<double*>(lu_scr);
      const int li = lane & 15, lq = lane >> 4;
      const int nrb = (nR + 15) >> 4;
      for (int c0 = 0; c0 < L; c0 += zw) {
        __syncthreads();
        // a wave per row, four rows in flight; lanes along the chunk
        for (int i0 = wv; i0 < kr; i0 += 4 * (kThreads / 64)) {
          for (int j = lane; j < zw; j += 64) {
            double v[4];
  #pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = i0 + u * (kThreads / 64);
              const int gi = sr[min(i, ns - 1)];
              v[u] = (i < ns && c0 + j < L) ? Gs[gi * L + c0 + j] : 0.0;
            }
  #pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int i = i0 + u * (kThreads / 64);
              if (i < kr) Zl[i * zs + j] = v[u];
            }
          }
        }
        __syncthreads();
        const int ntile = (min(zw, L - c0) + 15) >> 4;   // 16-column tiles in this chunk (<= 4)
        for (int rb = wv; rb < nrb; rb += kThreads / 64) {
          // one 16-row block of R against every tile of the chunk; the A operand
          // is prefetched a batch of kGB steps ahead (two register batches in turn)
          constexpr int kGB = 8;
          const int arow = min(rb * 16 + li, nR - 1);
          const double2* arow2 = reinterpret_cast<const double2*>(Aq + (long long)arow * kr + lq * ks);
          int orow[4], oR[4];
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            orow[r] = rb * 16 + 4 * r + lq;
            oR[r] = Rl[min(orow[r], nR - 1)];
          }
          doublex4 acc[4];
          double gold[4][4];
  #pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            const int col = min(c0 + 16 * tt + li, L - 1);
  #pragma unroll
            for (int r = 0; r < 4; ++r) {
              acc[tt][r] = (tt < ntile) ? Hr[oR[r] * L + col] : 0.0;
              gold[tt][r] = (drift && tt < ntile) ? Gs[oR[r] * L + col] : 0.0;
            }
          }
          // steps q0.. of this lane's K range (clamped, in bounds: ks is even)
          auto load_a = [&](int q0, double2 (&av)[kGB / 2]) {
  #pragma unroll
            for (int u = 0; u < kGB / 2; ++u) av[u] = arow2[min(q0 / 2 + u, ks / 2 - 1)];
          };
          auto mma = [&](int q0, const double2 (&av)[kGB / 2]) {
  #pragma unroll
            for (int u = 0; u < kGB; ++u) {
              if (q0 + u < ks) {
                const double a = (u & 1) ? av[u >> 1].y : av[u >> 1].x;
                const double* zb = Zl + (lq * ks + q0 + u) * zs + li;
  #pragma unroll
                for (int tt = 0; tt < 4; ++tt)
                  if (tt < ntile)
                    acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, zb[16 * tt], acc[tt], 0, 0, 0);
              }
            }
          };
          double2 a0[kGB / 2], a1[kGB / 2];
          load_a(0, a0);
  #pragma unroll 1
          for (int q0 = 0; q0 < ks; q0 += 2 * kGB) {
            if (q0 + kGB < ks) load_a(q0 + kGB, a1);
            mma(q0, a0);
            if (q0 + kGB >= ks) break;
            if (q0 + 2 * kGB < ks) load_a(q0 + 2 * kGB, a0);
            mma(q0 + kGB, a1);
          }
  #pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            const int col = c0 + 16 * tt + li;
            if (tt < ntile && col < L && col < c0 + zw) {
  #pragma unroll
              for (int r = 0; r < 4; ++r) {
                if (orow[r] < nR) {
                  const double x = acc[tt][r];
                  if (drift) dmax = fmax(dmax, fabs(x - gold[tt][r]));
                  if (!(fabs(x) < INFINITY)) dmax = INFINITY;
                  Gs[oR[r] * L + col] = x;
                }
              }
            }
          }
        }
      }
    }
  }
  dmax = block_max(dmax, ch.red);
  if (s_sing && t == 0) ch.st[ST_SINGULAR] = 1;
  __syncthreads();
  stat_add(ch.st, ST_T_LU_GEMM, wall_clock64() - tc);
  return dmax;
}

// --------------------------------------------------------- measurement ----
// Accumulate G(tau_k) = 1/(2L) sum_sigma sum_l sgn G_sigma((l+k) mod L, l)
// (sgn = -1 where l + k wraps) and D = (1/L) sum_l (1 - Gu_ll)(1 - Gd_ll)
// into the chain's bin.  Thread k walks rows i and reads G(i, (i-k) mod L),
// so every step of a wave reads one contiguous stretch of a row.
//
// With only G_up stored (ph): G_dn(i, j) = delta_ij - G_up(j, i), and the
// spin-down sum over i becomes, with j = (i - k) mod L,
//   sum_i sgn G_dn(i, j) = L delta_k0 - sum_j sgn' G_up(j, (j + k) mod L),
// sgn' = -1 where j + k wraps: again one contiguous stretch of a row per step.
// Sums of the estimator at lag k over the rows: up = sum_i sgn G_up(i, i - k),
// dn the same for G_dn (from G_up's transposed diagonals when only G_up is
// stored, see above).
template <typename GT>
__device__ __forceinline__ void lag_sums(const GT* __restrict__ Gup, const GT* __restrict__ Gdn,
                                         int L, int k, bool ph, double& up_, double& dn_) {
  // step i: every thread of a wave reads row i (one contiguous stretch):
  // G(i, i - k), with sign - where i - k wraps
  double up = 0.0, dn = 0.0;
  if (!ph) {
#pragma unroll 16
    for (int i = 0; i < L; ++i) {
      int j = i - k;
      double sg = 1.0;
      if (j < 0) {
        j += L;
        sg = -1.0;
      }
      const long long o = (long long)i * L + j;
      up += sg * Gup[o];
      dn += sg * Gdn[o];
    }
  } else {
    // and G_up(i, i + k), with sign - where i + k wraps, for the spin-down term
    double tr = 0.0;
#pragma unroll 16
    for (int i = 0; i < L; ++i) {
      int j = i - k, j2 = i + k;
      double sg = 1.0, sg2 = 1.0;
      if (j < 0) {
        j += L;
        sg = -1.0;
      }
      if (j2 >= L) {
        j2 -= L;
        sg2 = -1.0;
      }
      const GT* row = Gup + (long long)i * L;
      up += sg * row[j];
      tr += sg2 * row[j2];
    }
    dn = (k == 0 ? (double)L : 0.0) - tr;
  }
  up_ = up;
  dn_ = dn;
}

template <typename GT, bool SPIN = false>
__device__ __forceinline__ void measure(const Chain& ch, int bin, bool ph) {
  const int L = ch.L;
  double* accg = ch.accg;
  const GT* Gup = reinterpret_cast<const GT*>(ch.Gu);
  const GT* Gdn = reinterpret_cast<const GT*>(ch.Gd);
  for (int k = threadIdx.x; k < L; k += kThreads) {
    double up, dn;
    lag_sums<GT>(Gup, Gdn, L, k, ph, up, dn);
    if constexpr (SPIN) {
      // spin-resolved: [bin][up, down][L+1], G_sigma(beta-) = 1 - G_sigma(0+)
      const long long base = (long long)bin * 2 * (L + 1);
      accg[base + k] += up / L;
      accg[base + (L + 1) + k] += dn / L;
      if (k == 0) {
        accg[base + L] += 1.0 - up / L;
        accg[base + (L + 1) + L] += 1.0 - dn / L;
      }
    } else {
      const double val = (up + dn) / (2.0 * L);
      const long long base = (long long)bin * (L + 1);
      accg[base + k] += val;
      if (k == 0) accg[base + L] += 1.0 - val;
    }
  }
  double dsum = 0.0;
  for (int l = threadIdx.x; l < L; l += kThreads) {
    const long long o = (long long)l * L + l;
    const double gu = Gup[o];
    dsum += (1.0 - gu) * (ph ? gu : 1.0 - Gdn[o]);
  }
  dsum = block_sum(dsum, ch.red);
  if (threadIdx.x == 0) {
    ch.accd[bin] += dsum / L;
    ch.accn[bin] += 1;
  }
}

// Drift of the G(tau) estimator at a sampled recompute: the estimator of the
// updated G is kept (snapshot, each thread its own lags in the workspace)
// and, after the recompute, compared with the estimator of the recomputed G;
// returns the largest change over the lags (every thread gets it).  The
// spin-averaged estimator of measure(), or both spin-resolved ones for
// spin-dependent baths.
template <typename GT, bool SPIN = false>
__device__ __forceinline__ double estimator_drift(const Chain& ch, bool ph, bool snapshot) {
  const int L = ch.L;
  const GT* Gup = reinterpret_cast<const GT*>(ch.Gu);
  const GT* Gdn = reinterpret_cast<const GT*>(ch.Gd);
  gdouble* __restrict__ keep = (gdouble*)ch.gtd;
  double dm = 0.0;
  for (int k = threadIdx.x; k < L; k += kThreads) {
    double up, dn;
    lag_sums<GT>(Gup, Gdn, L, k, ph, up, dn);
    const double a = SPIN ? up / L : (up + dn) / (2.0 * L);
    const double b = SPIN ? dn / L : 0.0;
    if (snapshot) {
      keep[2 * k] = a;
      keep[2 * k + 1] = b;
    } else {
      dm = fmax(dm, fmax(fabs(a - keep[2 * k]), fabs(b - keep[2 * k + 1])));
      if (!(fabs(a) < INFINITY && fabs(b) < INFINITY)) dm = INFINITY;
    }
  }
  if (snapshot) return 0.0;
  return block_max(dm, ch.red);
}

// ---------------------------------------------------------- proposals ----


// Acceptance decision for flipping s_l (Metropolis u < R, or heat bath
// u < R/(1+R)), evaluated identically by every thread of the workgroup
// (uniform branch).  In replay mode the decision is read from the given flip
// list instead.
struct Flip {
  double g_up, g_dn, r_up, r_dn;
  bool accept;
};

__device__ __forceinline__ Flip propose(double gul, double gdl, int sl, double gp, double gm,
                                       double u, const long long* rlog, long long rlen,
                                       long long code, Counters& k, long long* st, bool hb) {
  Flip f;
  f.g_up = sl > 0 ? gm : gp;
  f.g_dn = sl > 0 ? gp : gm;
  f.r_up = ratio_factor(f.g_up, gul);
  f.r_dn = ratio_factor(f.g_dn, gdl);
  const double R = mul_nc(f.r_up, f.r_dn);
  const bool bad = !(R > 0.0);
  if (threadIdx.x == 0) {
    st[ST_PROPOSED] += 1;
    st[ST_BAD] += bad ? 1 : 0;
  }
  bool acc;
  if (rlog) {
    acc = k.rep_i < rlen && rlog[k.rep_i] == code;
  } else {
    // Metropolis min(1, R), or heat bath R / (1 + R)
    acc = !bad && (hb ? u < R / (1.0 + R) : u < R);
  }
  // every thread evaluates the same decision from the same values: stating it
  // as uniform keeps the sweep's control flow (and the counters) scalar
  f.accept = __builtin_amdgcn_readfirstlane(acc ? 1 : 0) != 0;
  if (rlog) k.rep_i += f.accept ? 1 : 0;
  return f;
}

struct ChainIO {
  long long* flog;
  const long long* rlog;
  long long rlen;
  long long flip_cap;
  double gp, gm;
  bool hb;   // heat-bath acceptance
};

__device__ __forceinline__ void log_flip(const ChainIO& io, long long* st, long long code) {
  if (threadIdx.x == 0) {
    const long long n = st[ST_FLIPS];
    if (io.flog && n < io.flip_cap) io.flog[n] = code;
    st[ST_FLIPS] = n + 1;
    st[ST_ACCEPTED] += 1;
  }
}

// Dyson recompute of both spins (the kernel's only call site of the LU, so it
// is inlined once).  The initial recompute of a chain is not counted as one.
template <typename GT, bool SPIN = false, bool PG = false>
__device__ __forceinline__ void recompute_both(const SweepParams& p, const Chain& ch, Counters& k,
                                               bool counted) {
  const long long t0 = wall_clock64();
  double d = 0.0;
  const int nsp = p.ph ? 1 : 2;
  const bool samp = counted && drift_sampled(k.n_rec + 1, p.drift_every);
  if (samp) (void)estimator_drift<GT, SPIN>(ch, p.ph != 0, true);
#pragma unroll 1
  for (int sp = 0; sp < nsp; ++sp)
    d = fmax(d, dyson_solve<GT, SPIN, PG>(ch, sp ? -1 : +1,
                                          reinterpret_cast<GT*>(sp ? ch.Gd : ch.Gu), ch.lu_nb,
                                          ch.reduced, false, samp));
  const double dg = samp ? estimator_drift<GT, SPIN>(ch, p.ph != 0, false) : 0.0;
  if (counted) {
    k.n_rec += 1;
    if (threadIdx.x == 0) {
      // (a non-finite G is reported whether or not the drift is sampled)
      if (samp || !(d < INFINITY)) *ch.drift = fmax(*ch.drift, d);
      if (samp) *ch.drift_gt = fmax(*ch.drift_gt, dg);
      ch.st[ST_RECOMPUTES] += 1;
    }
  }
  k.acc_since = 0;
  stat_add(ch.st, ST_T_REC, wall_clock64() - t0);
}

// ------------------------------------------------- plain rank-1 sweep ----
// Every accepted flip applies G <- G + (G(:,l) - e_l)(gamma/R_sigma) G(l,:) to
// both L x L matrices in HBM: 32 L^2 bytes of traffic per accepted flip.
// Processes slices l_begin.. of sweep sw; returns early (next slice) when a
// recompute is due, else L.
__device__ __forceinline__ int sweep_rank1(const SweepParams& p, const Chain& ch, long long sw,
                                           Counters& k, const ChainIO& io, int l_begin) {
  const int L = ch.L;
  const long long L2 = (long long)L * L;
  double* xu = reinterpret_cast<double*>(ch.scratch);
  double* xd = xu + p.Lmax;
  double* yu = xd + p.Lmax;
  double* yd = yu + p.Lmax;
  const bool ph = p.ph != 0;
  for (int l = l_begin; l < L; ++l) {
    const long long dl = (long long)l * L + l;
    const int sl = ch.s[l];
    if (l == l_begin || (l & (kUW - 1)) == 0) {
      const int c0 = l & ~(kUW - 1);
      fill_uniforms(ch.uw, ch.key0, (uint64_t)ch.grid, sw, c0, min(kUW, L - c0));
    }
    const double gul = ch.Gu[dl];
    const Flip f = propose(gul, ph ? 1.0 - gul : ch.Gd[dl], sl, io.gp, io.gm, ch.uw[l & (kUW - 1)],
                           io.rlog, io.rlen, sw * L + l, k, ch.st, io.hb);
    if (!f.accept) continue;
    log_flip(io, ch.st, sw * L + l);
    // update vectors x = G(:,l) - e_l and y = (gamma/R_sigma) G(l,:)
    const double cu = f.g_up / f.r_up, cd = f.g_dn / f.r_dn;
    for (int i = threadIdx.x; i < L; i += kThreads) {
      const long long ci = (long long)i * L + l;
      xu[i] = ch.Gu[ci] - (i == l ? 1.0 : 0.0);
      yu[i] = mul_nc(cu, ch.Gu[(long long)l * L + i]);
      if (!ph) {
        xd[i] = ch.Gd[ci] - (i == l ? 1.0 : 0.0);
        yd[i] = mul_nc(cd, ch.Gd[(long long)l * L + i]);
      }
    }
    __syncthreads();
    if (ph) {
      // G_up only: thread -> (column pair, row group) as below
      const int ncp = (L + 1) >> 1;
      const int rg = max(1, kThreads / ncp);
      const int t = threadIdx.x;
      if (t < ncp * rg) {
        const int cp = t % ncp, r0 = t / ncp;
        const int j = 2 * cp;
        const bool two = j + 1 < L;
        const double yu0 = yu[j];
        const double yu1 = two ? yu[j + 1] : 0.0;
        if ((L & 1) == 0) {
#pragma unroll 4
          for (int i = r0; i < L; i += rg) {
            const double xui = xu[i];
            double2* gu = reinterpret_cast<double2*>(ch.Gu + (long long)i * L + j);
            double2 a = *gu;
            a.x = axpy_nc(a.x, xui, yu0);
            a.y = axpy_nc(a.y, xui, yu1);
            *gu = a;
          }
        } else {
#pragma unroll 4
          for (int i = r0; i < L; i += rg) {
            const double xui = xu[i];
            double* gu = ch.Gu + (long long)i * L + j;
            gu[0] = axpy_nc(gu[0], xui, yu0);
            if (two) gu[1] = axpy_nc(gu[1], xui, yu1);
          }
        }
      }
    } else {
      // G += x y^T, both spins: thread -> (column pair, row group); the pair's
      // y values stay in registers, x is an LDS broadcast per row
      const int ncp = (L + 1) >> 1;
      const int rg = max(1, kThreads / ncp);
      const int t = threadIdx.x;
      if (t < ncp * rg) {
        const int cp = t % ncp, r0 = t / ncp;
        const int j = 2 * cp;
        const bool two = j + 1 < L;
        const double yu0 = yu[j], yd0 = yd[j];
        const double yu1 = two ? yu[j + 1] : 0.0, yd1 = two ? yd[j + 1] : 0.0;
        if ((L & 1) == 0) {
#pragma unroll 4
          for (int i = r0; i < L; i += rg) {
            const double xui = xu[i], xdi = xd[i];
            double2* gu = reinterpret_cast<double2*>(ch.Gu + (long long)i * L + j);
            double2* gd = reinterpret_cast<double2*>(ch.Gd + (long long)i * L + j);
            double2 a = *gu, b = *gd;
            a.x = axpy_nc(a.x, xui, yu0);
            a.y = axpy_nc(a.y, xui, yu1);
            b.x = axpy_nc(b.x, xdi, yd0);
            b.y = axpy_nc(b.y, xdi, yd1);
            *gu = a;
            *gd = b;
          }
        } else {
#pragma unroll 4
          for (int i = r0; i < L; i += rg) {
            const double xui = xu[i], xdi = xd[i];
            double* gu = ch.Gu + (long long)i * L + j;
            double* gd = ch.Gd + (long long)i * L + j;
            gu[0] = axpy_nc(gu[0], xui, yu0);
            gd[0] = axpy_nc(gd[0], xdi, yd0);
            if (two) {
              gu[1] = axpy_nc(gu[1], xui, yu1);
              gd[1] = axpy_nc(gd[1], xdi, yd1);
            }
          }
        }
      }
    }
    if (threadIdx.x == 0) ch.s[l] = (int8_t)(-sl);
    __syncthreads();
    if (++k.acc_since == p.n_rec) return l + 1;
  }
  return L;
}

// -------------------------------------------- windowed delayed update ----
//
// The sweep visits l = l0, l0+1, ... in windows of at most kWin consecutive
// slices.  Deciding and updating inside a window only needs the kWin x kWin
// diagonal blocks of G_up and G_dn, which live in LDS and get the exact
// rank-1 updates of each accepted flip.  Accepted flips stay pending across
// windows until delay_k of them are pending, a recompute is due or the sweep
// ends; then the m pending flips are applied to the full matrices as one
// rank-m update, the delayed-update form of m successive Sherman-Morrison
// steps.  With f_i the flipped slices, c_i = gamma_i / R_i, C0 = G(:,F) - I(:,F)
// and R0 = G(F,:) of the matrix before the first pending flip,
//   x_j = G(:, f_j) - e_{f_j} + sum_{i<j} x_i y_i(f_j)     ->  X = C0 T, T = (I - U)^{-1}
//   y_j = c_j (G(f_j, :) + sum_{i<j} x_i(f_j) y_i)        ->  Y = S R0, S = (I - Dc Lw)^{-1} Dc
// with U(i,j) = y_i(f_j) and Lw(j,i) = x_i(f_j) (i < j), and G += X Y = C0 (T S) R0.
// A window opened while flips are pending starts from G(B,B) + X(B,:) Y(:,B);
// X(B,:) and Y(:,B) are also the in-window parts of the pending flips' vectors,
// from which the coefficients U, Lw of the window's new flips are read.  T and
// S are built in place over U and Lw, one column / row per flip, as flips are
// added.  The rank-m product runs in FP64 (MODE_DELAYED_FP64) or with FP32
// inputs and FP32 accumulation on the matrix cores (MODE_MIXED); ratios,
// decisions, window blocks and in-window updates are FP64 in both.

constexpr int kWin = 64;        // slices per window (diagonal block edge)
constexpr int kWP = kWin + 1;   // LDS row stride of the window blocks
constexpr int kKP = kMaxK + 1;  // LDS row stride of the m x m coefficient blocks
constexpr int kSmall = 1536;    // bytes for flip positions (global slices) and coefficients
typedef float floatx4 __attribute__((ext_vector_type(4)));

// G += X Y for one spin.  X: [L][kMaxK] row-major, Y: [kMaxK][L] row-major,
// m used columns.  Y is staged once per column panel in LDS, transposed
// ([column][k], row stride kYK, as the MFMA input type), so every element of Y
// leaves memory once per flush; X rows stay in registers per 16-row strip.
// The output is walked in work items of one 16-row strip by kCW columns,
// split into contiguous ranges per wave; the next item's G is loaded while the
// current one runs on the matrix cores.
// MIXED: FP32 operands and FP32 accumulation (v_mfma_f32_16x16x4f32, output
// row 4q + r), added into the FP64 G; otherwise FP64 (v_mfma_f64_16x16x4f64,
// output row 4r + q).
constexpr int kCW = 64;          // columns per work item (4 output tiles)
constexpr int kCT = kCW / 16;
constexpr int kYK = kMaxK + 4;   // LDS stride of a staged Y column

template <bool MIXED, typename GT>
__device__ __forceinline__ void flush_gemm(
    GT* __restrict__ G, const typename std::conditional<MIXED, float, double>::type* __restrict__ X,
    const typename std::conditional<MIXED, float, double>::type* __restrict__ Y, int L, int m,
    char* __restrict__ ybuf, int ybytes) {
  typedef typename std::conditional<MIXED, float, double>::type T;
  typedef T Tx4 __attribute__((ext_vector_type(4)));
  constexpr int KS = kMaxK / 4;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int ks = (m + 3) >> 2;
  const int rows = 4 * ks;
  const int nstrip = (L + 15) >> 4;
  // panel width: a multiple of kCW whose staged columns fit the buffer
  int pw = ybytes / (kYK * (int)sizeof(T)) / kCW * kCW;
  if (pw > ((L + kCW - 1) / kCW) * kCW) pw = ((L + kCW - 1) / kCW) * kCW;
  T* __restrict__ Yl = reinterpret_cast<T*>(ybuf);
  int orow_off[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) orow_off[r] = MIXED ? 4 * lq + r : 4 * r + lq;
  // (32-bit byte offsets from the uniform base keep each address in one register)
  const char* __restrict__ Gc = reinterpret_cast<const char*>(G);
#pragma unroll 1
  for (int c0 = 0; c0 < L; c0 += pw) {
    const int w = min(pw, L - c0);
    __syncthreads();
    // a wave per Y row, four rows in flight; lanes along the panel
    for (int k0 = wv; k0 < rows; k0 += 4 * (kThreads / 64)) {
      for (int c = lane; c < pw; c += 64) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = k0 + u * (kThreads / 64);
          v[u] = (kk < m && c < w) ? Y[kk * L + c0 + c] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kk = k0 + u * (kThreads / 64);
          if (kk < rows) Yl[c * kYK + kk] = v[u];
        }
      }
    }
    __syncthreads();
    const int nchunk = (w + kCW - 1) / kCW;
    const int items = nstrip * nchunk;
    const int lo = (int)((long long)items * wv / (kThreads / 64));
    const int hi = (int)((long long)items * (wv + 1) / (kThreads / 64));
    if (lo >= hi) continue;
    // G of item `it` for this lane: 4 rows x kCT tiles (clamped, in bounds)
    auto load_g = [&](int it, GT (&g)[kCT][4]) {
      const int st = it / nchunk, chk = it - st * nchunk;
#pragma unroll
      for (int ct = 0; ct < kCT; ++ct) {
        const int col = min(c0 + chk * kCW + 16 * ct + li, L - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const unsigned o = (unsigned)(min(16 * st + orow_off[r], L - 1) * L + col)
                             << (sizeof(GT) == 8 ? 3 : 2);
          g[ct][r] = *reinterpret_cast<const GT*>(Gc + o);
        }
      }
    };
    T a[KS];
    int cur_strip = -1;
    auto process = [&](int it, const GT (&gcur)[kCT][4]) {
      const int st = it / nchunk, chk = it - st * nchunk;
      if (st != cur_strip) {
        cur_strip = st;
        const int arow = min(16 * st + li, L - 1);
        const bool arow_ok = 16 * st + li < L;
#pragma unroll
        for (int q = 0; q < KS; ++q) {
          const int kk = 4 * q + lq;
          const T v = X[arow * kMaxK + kk];
          a[q] = (arow_ok && kk < m) ? v : (T)0;
        }
      }
      Tx4 acc[kCT];
#pragma unroll
      for (int ct = 0; ct < kCT; ++ct) acc[ct] = Tx4{(T)0, (T)0, (T)0, (T)0};
      const T* yb = Yl + (chk * kCW + li) * kYK + lq;
#pragma unroll
      for (int q = 0; q < KS; ++q) {
        if (q < ks) {
#pragma unroll
          for (int ct = 0; ct < kCT; ++ct) {
            const T bv = yb[16 * ct * kYK + 4 * q];
            if constexpr (MIXED)
              acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q], bv, acc[ct], 0, 0, 0);
            else
              acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], bv, acc[ct], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int ct = 0; ct < kCT; ++ct) {
        const int col = c0 + chk * kCW + 16 * ct + li;
        const bool cok = (chk * kCW + 16 * ct + li < w);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * st + orow_off[r];
          if (cok && row < L) G[row * L + col] = (GT)((double)gcur[ct][r] + (double)acc[ct][r]);
        }
      }
    };
    // three G buffers in turn: the loads of the next two items are in flight
    // while one item runs on the matrix cores
    GT g0[kCT][4], g1[kCT][4], g2[kCT][4];
    load_g(lo, g0);
    if (lo + 1 < hi) load_g(lo + 1, g1);
#pragma unroll 1
    for (int it = lo; it < hi; it += 3) {
      if (it + 2 < hi) load_g(it + 2, g2);
      process(it, g0);
      if (it + 1 >= hi) break;
      if (it + 3 < hi) load_g(it + 3, g0);
      process(it + 1, g1);
      if (it + 2 >= hi) break;
      if (it + 4 < hi) load_g(it + 4, g1);
      process(it + 2, g2);
    }
  }
}

// The update's two factors for one spin, G += X Y with
//   X = C0 = G[:, F] - I[:, F]   (gathered, L x m)  and   Y = W R0, R0 = G[F, :],
// where W = T S (m x m, in LDS with row stride kKP) folds both triangular
// factors of the delayed update into the right factor (f_i = l0 + F[i]).
// Y on the matrix cores (FP64) in wave-independent 16 x 16 tiles whose G rows
// are loaded one tile ahead.  X and Y are stored in the product's operand
// type T (FP32 in the mixed path: the product rounds them to FP32 anyway).
template <typename T, typename GT>
__device__ __forceinline__ void flush_vectors(const GT* __restrict__ G, int L, int l0, int m,
                                              const int* __restrict__ F,
                                              const double* __restrict__ W,
                                              T* __restrict__ X, T* __restrict__ Y) {
  constexpr int KS = kMaxK / 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int ks = (m + 3) >> 2;
  const int mb = (m + 15) >> 4;
  const int nb = (L + 15) >> 4;
  // X: a wave per row, eight rows in flight, lane i gathers column f_i
  {
    constexpr int kXR = 8;
    const int fi = l0 + F[min(lane, m - 1)];
    for (int q0 = wv; q0 < L; q0 += kXR * (kThreads / 64)) {
      double v[kXR];
#pragma unroll
      for (int u = 0; u < kXR; ++u) {
        const int q = min(q0 + u * (kThreads / 64), L - 1);
        v[u] = G[q * L + fi] - (q == fi ? 1.0 : 0.0);
      }
#pragma unroll
      for (int u = 0; u < kXR; ++u) {
        const int q = q0 + u * (kThreads / 64);
        if (q < L && lane < m) X[q * kMaxK + lane] = (T)v[u];
      }
    }
  }
  // flipped slice of each k-step of this lane (clamped for k >= m; those operands are zeroed)
  int fk[KS];
#pragma unroll
  for (int q = 0; q < KS; ++q) fk[q] = l0 + F[min(4 * q + lq, m - 1)];
  const int ny = mb * nb;   // tile = jb * nb + cb
  auto load_b = [&](int tile, double (&bv)[KS]) {
    const int col = min((tile % nb) * 16 + li, L - 1);
#pragma unroll
    for (int s4 = 0; s4 < KS; ++s4) bv[s4] = (s4 < ks) ? G[fk[s4] * L + col] : 0.0;
  };
  auto tile_y = [&](int tile, const double (&bv)[KS]) {
    const int jb = tile / nb, cb = tile - jb * nb;
    const int jr = jb * 16 + li;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < KS; ++s4) {
      if (s4 < ks) {
        const int i = 4 * s4 + lq;
        const double a = (jr < m && i < m) ? W[min(jr, kMaxK - 1) * kKP + i] : 0.0;
        const double b = (i < m) ? bv[s4] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jj = jb * 16 + 4 * r + lq;
      if (jj < m && cb * 16 + li < L) Y[jj * L + cb * 16 + li] = (T)acc[r];
    }
  };
  double b0[KS], b1[KS];
  if (wv < ny) load_b(wv, b0);
#pragma unroll 1
  for (int tile = wv; tile < ny; tile += 2 * (kThreads / 64)) {
    const int t1 = tile + kThreads / 64;
    if (t1 < ny) load_b(t1, b1);
    tile_y(tile, b0);
    if (t1 >= ny) break;
    if (t1 + kThreads / 64 < ny) load_b(t1 + kThreads / 64, b0);
    tile_y(t1, b1);
  }
}

// W = T S for both spins on the matrix cores: T (upper, unit diagonal) and S
// (lower, diagonal c_j) share the m x m block TS (T[i][j] = TS[i][j] for
// i < j, S[j][i] = TS[j][i] for i <= j); W overwrites TS once every wave has
// read it.  Tiles (spin, 16 x 16 block) are spread over the waves.
__device__ __forceinline__ void flush_fold(double* __restrict__ TSu, double* __restrict__ TSd, int m,
                                           int nsp) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int mb = (m + 15) >> 4;
  const int ks = (m + 3) >> 2;
  const int nt = nsp * mb * mb;                    // at most 32 tiles: 4 per wave
  doublex4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    acc[u] = doublex4{0.0, 0.0, 0.0, 0.0};
    const int tile = wv + u * (kThreads / 64);
    if (tile < nt) {
      const int sp = tile / (mb * mb), e = tile - sp * mb * mb;
      const int ib = e / mb, jb = e - ib * mb;
      const double* TS = sp ? TSd : TSu;
      const int i = ib * 16 + li;          // A row (of T)
      const int j = jb * 16 + li;          // B column (of S)
#pragma unroll 4
      for (int s4 = 0; s4 < ks; ++s4) {
        const int k = 4 * s4 + lq;
        // unconditional LDS reads at clamped indices, then masked
        const int ic = min(i, kMaxK - 1), jc = min(j, kMaxK - 1), kc = min(k, kMaxK - 1);
        const double ta = TS[ic * kKP + kc], tb = TS[kc * kKP + jc];
        const double a = (i < m && k < m) ? ((k > i) ? ta : (k == i ? 1.0 : 0.0)) : 0.0;
        const double b = (j < m && k < m && k >= j) ? tb : 0.0;
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int tile = wv + u * (kThreads / 64);
    if (tile < nt) {
      const int sp = tile / (mb * mb), e = tile - sp * mb * mb;
      const int ib = e / mb, jb = e - ib * mb;
      double* TS = sp ? TSd : TSu;
      const int j = jb * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ib * 16 + 4 * r + lq;
        if (i < m && j < m) TS[i * kKP + j] = acc[u][r];
      }
    }
  }
  __syncthreads();
}

// LDS of the window phase (after kSmall): window blocks Wu, Wd [kWin][kWP],
// the last flip's in-window vectors, then the coefficient blocks ULu, ULd
// [kMaxK][kKP] (U above, Lw below the diagonal; the first m_inv columns and
// rows already turned into T and S).
struct WinLds {
  int* F;            // [kMaxK] flipped slices (global)
  double* cU;        // [kMaxK] gamma / R, spin up
  double* cD;
  double* Wu;
  double* Wd;
  double* xu;
  double* yu;
  double* xd;
  double* yd;
  double* ULu;
  double* ULd;
};

__device__ __forceinline__ WinLds win_lds(const Chain& ch) {
  WinLds w;
  w.F = reinterpret_cast<int*>(ch.scratch);
  w.cU = reinterpret_cast<double*>(ch.scratch + 256);
  w.cD = w.cU + kMaxK;
  w.Wu = reinterpret_cast<double*>(ch.scratch + kSmall);
  w.Wd = w.Wu + kWin * kWP;
  w.xu = w.Wd + kWin * kWP;
  w.yu = w.xu + kWin;
  w.xd = w.yu + kWin;
  w.yd = w.xd + kWin;
  w.ULu = w.yd + kWin;
  w.ULd = w.ULu + kMaxK * kKP;
  return w;
}

// Columns / rows m_inv .. m-1 of U and Lw into T and S, in place, one wave per
// triangle and spin (waves 0, 1: T; waves 2, 3: S):
//   T[r][j] = U[r][j] + sum_{r < i < j} T[r][i] U[i][j]      (T[r][r] = 1)
//   S[c][c] = c_c,  S[j][c] = c_j sum_{c <= i < j} Lw[j][i] S[i][c]
// All lanes step through j together, so every read of column / row j happens
// before any lane overwrites it at the end of the same step.
__device__ __forceinline__ void invert_ts(const WinLds& w, int m_inv, int m, int nsp) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (wv < 4 && lane < m && ((wv & 1) == 0 || nsp == 2)) {
    double* UL = (wv & 1) ? w.ULd : w.ULu;
    const double* cc = (wv & 1) ? w.cD : w.cU;
    if (wv < 2) {
      const int r = lane;
#pragma unroll 1
      for (int j = max(m_inv, 1); j < m; ++j) {
        if (r < j) {
          double acc = UL[r * kKP + j];
          // (unrolled: the LDS reads of several terms are in flight together)
#pragma unroll 8
          for (int i = r + 1; i < j; ++i) acc = fma(UL[r * kKP + i], UL[i * kKP + j], acc);
          UL[r * kKP + j] = acc;
        }
        wave_sync();
      }
    } else {
      const int c = lane;
      if (c >= m_inv) UL[c * kKP + c] = cc[c];
      wave_sync();
#pragma unroll 1
      for (int j = max(m_inv, 1); j < m; ++j) {
        if (c < j) {
          double acc = 0.0;
#pragma unroll 8
          for (int i = c; i < j; ++i) acc = fma(UL[j * kKP + i], UL[i * kKP + c], acc);
          UL[j * kKP + c] = cc[j] * acc;
        }
        wave_sync();
      }
    }
  }
  __syncthreads();
}

// Opening a window at l0 (b slices) with m flips pending (T, S complete):
// the pending flips' in-window vector parts
//   Xrec[i][r] = X(l0 + r, i) = sum_{i'} C0(l0 + r, i') T[i'][i],
//   Yrec[i][c] = Y(i, l0 + c) = sum_{i'} S[i][i'] G(f_i', l0 + c),
// then the window blocks W = G(B,B) + X(B,:) Y(:,B), all FP64 on the matrix cores.
template <typename GT>
__device__ __forceinline__ void window_apply(const Chain& ch, const WinLds& w, int l0, int b, int m,
                                             int nsp) {
  const int L = ch.L;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int ks = (m + 3) >> 2;
  const int mb = (m + 15) >> 4;
  double* Xrec = ch.wbuf;                       // [2][kMaxK][kWin]
  double* Yrec = Xrec + 2 * kMaxK * kWin;       // [2][kMaxK][kWin]
  // (1) X tiles (4 row blocks x mb) and Y tiles (mb x 4) of both spins
  const int nx = 4 * mb, ntile = nsp * (2 * nx);
  for (int tile = wv; tile < ntile; tile += kThreads / 64) {
    const int sp = tile >= 2 * nx;
    const int e = tile - sp * 2 * nx;
    const GT* G = reinterpret_cast<const GT*>(sp ? ch.Gd : ch.Gu);
    const double* TS = sp ? w.ULd : w.ULu;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    if (e < nx) {
      // X(B, :): rows rb (window), columns jb (flips); A = C0 (gathered), B = T
      const int rb = e / mb, jb = e - rb * mb;
      const int q = l0 + min(rb * 16 + li, b - 1);
      const int j = jb * 16 + li;
      // every k-step's gathered G value is loaded before the products start
      // (unconditional loads at clamped, in-bounds indices)
      double gv[kMaxK / 4];
#pragma unroll
      for (int s4 = 0; s4 < kMaxK / 4; ++s4) {
        const int fi = w.F[min(4 * s4 + lq, m - 1)];
        const double g = G[q * L + fi];
        gv[s4] = (s4 < ks) ? g - (q == fi ? 1.0 : 0.0) : 0.0;
      }
#pragma unroll
      for (int s4 = 0; s4 < kMaxK / 4; ++s4) {
        if (s4 >= ks) break;
        const int i = 4 * s4 + lq;
        const double a = (i < m) ? gv[s4] : 0.0;
        const double tv = TS[min(i, kMaxK - 1) * kKP + min(j, kMaxK - 1)];
        const double bv = (i < m && j < m) ? (i < j ? tv : (i == j ? 1.0 : 0.0)) : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = rb * 16 + 4 * r + lq;
        if (rr < b && j < m) Xrec[(sp * kMaxK + j) * kWin + rr] = acc[r];
      }
    } else {
      // Y(:, B): rows jb (flips), columns cb (window); A = S, B = G(F, B)
      const int e2 = e - nx;
      const int jb = e2 / 4, cb = e2 - jb * 4;
      const int jr = jb * 16 + li;
      const int col = l0 + min(cb * 16 + li, b - 1);
      double gv[kMaxK / 4];
#pragma unroll
      for (int s4 = 0; s4 < kMaxK / 4; ++s4) {
        const double g = G[w.F[min(4 * s4 + lq, m - 1)] * L + col];
        gv[s4] = (s4 < ks) ? g : 0.0;
      }
#pragma unroll
      for (int s4 = 0; s4 < kMaxK / 4; ++s4) {
        if (s4 >= ks) break;
        const int i = 4 * s4 + lq;
        const double sv = TS[min(jr, kMaxK - 1) * kKP + min(i, kMaxK - 1)];
        const double a = (jr < m && i < m && i <= jr) ? sv : 0.0;
        const double bv = (i < m) ? gv[s4] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jj = jb * 16 + 4 * r + lq;
        const int cc = cb * 16 + li;
        if (jj < m && cc < b) Yrec[(sp * kMaxK + jj) * kWin + cc] = acc[r];
      }
    }
  }
  __syncthreads();
  // (2) W = G(B,B) + X(B,:) Y(:,B): 4 x 4 tiles per spin, 32 tiles over the waves
  for (int tile = wv; tile < 16 * nsp; tile += kThreads / 64) {
    const int sp = tile >> 4, e = tile & 15;
    const int rb = e >> 2, cb = e & 3;
    const GT* G = reinterpret_cast<const GT*>(sp ? ch.Gd : ch.Gu);
    double* W = sp ? w.Wd : w.Wu;
    const int col = cb * 16 + li;
    doublex4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = rb * 16 + 4 * r + lq;
      acc[r] = (rr < b && col < b) ? G[(l0 + rr) * L + l0 + col] : 0.0;
    }
    const int ar = rb * 16 + li;
    double av[kMaxK / 4], bw[kMaxK / 4];
#pragma unroll
    for (int s4 = 0; s4 < kMaxK / 4; ++s4) {
      const int i = 4 * s4 + lq;
      const int ic = min(i, kMaxK - 1);
      const double xa = Xrec[(sp * kMaxK + ic) * kWin + min(ar, kWin - 1)];
      const double yb = Yrec[(sp * kMaxK + ic) * kWin + min(col, kWin - 1)];
      av[s4] = (i < m && ar < b) ? xa : 0.0;
      bw[s4] = (i < m && col < b) ? yb : 0.0;
    }
#pragma unroll
    for (int s4 = 0; s4 < kMaxK / 4; ++s4) {
      if (s4 >= ks) break;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s4], bw[s4], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = rb * 16 + 4 * r + lq;
      if (rr < b && col < b) W[rr * kWP + col] = acc[r];
    }
  }
  __syncthreads();
}

// Coefficients of the window's new flips j = m0 .. m-1 (window at l0):
// U(i, j) = y_i(f_j), Lw(j, i) = x_i(f_j) for i < j, from the window's records.
__device__ __forceinline__ void capture_coefficients(const Chain& ch, const WinLds& w, int l0,
                                                     int m0, int m, int nsp) {
  const double* Xrec = ch.wbuf;
  const double* Yrec = Xrec + 2 * kMaxK * kWin;
  const int n_new = m - m0;
  for (int idx = threadIdx.x; idx < nsp * n_new * m; idx += kThreads) {
    const int sp = idx >= n_new * m;
    const int e = idx - sp * n_new * m;
    const int j = m0 + e / m, i = e % m;
    if (i < j) {
      const int pj = w.F[j] - l0;
      double* UL = sp ? w.ULd : w.ULu;
      UL[i * kKP + j] = Yrec[(sp * kMaxK + i) * kWin + pj];
      UL[j * kKP + i] = Xrec[(sp * kMaxK + i) * kWin + pj];
    }
  }
  __syncthreads();
}

// Applies the m pending flips (T, S complete up to m) to G_up and G_dn (nsp = 2)
// or to G_up alone (nsp = 1).
template <bool MIXED, typename GT>
__device__ __forceinline__ void flush_pending(const Chain& ch, const WinLds& w, int m, int nsp) {
  typedef typename std::conditional<MIXED, float, double>::type T;
  const int L = ch.L;
  T* X = reinterpret_cast<T*>(ch.wbuf + 4 * kMaxK * kWin);   // [2][L][kMaxK]
  T* Y = X + 2LL * L * kMaxK;                                 // [2][kMaxK][L]
  const long long t0 = wall_clock64();
  flush_fold(w.ULu, w.ULd, m, nsp);
  const long long t1 = wall_clock64();
  if (threadIdx.x == 0) ch.st[ST_T_FOLD] += t1 - t0;
#pragma unroll 1
  for (int sp = 0; sp < nsp; ++sp)
    flush_vectors<T, GT>(reinterpret_cast<const GT*>(sp ? ch.Gd : ch.Gu), L, 0, m, w.F,
                         sp ? w.ULd : w.ULu, X + (long long)sp * L * kMaxK,
                         Y + (long long)sp * kMaxK * L);
  __syncthreads();
  const long long t2 = wall_clock64();
  char* un = ch.scratch + kSmall;
#pragma unroll 1
  for (int sp = 0; sp < nsp; ++sp)
    flush_gemm<MIXED, GT>(reinterpret_cast<GT*>(sp ? ch.Gd : ch.Gu), X + (long long)sp * L * kMaxK,
                          Y + (long long)sp * kMaxK * L, L, m, un, ch.scratch_bytes - kSmall);
  __syncthreads();
  if (threadIdx.x == 0) {
    ch.st[ST_T_FL_VEC] += t2 - t1;
    ch.st[ST_T_FL_GEMM] += wall_clock64() - t2;
  }
}

template <bool MIXED, typename GT>
__device__ __forceinline__ int sweep_window(const SweepParams& p, const Chain& ch, long long sw,
                                            Counters& k, const ChainIO& io, int l_begin) {
  const int L = ch.L;
  const int t = threadIdx.x;
  const WinLds w = win_lds(ch);
  double* Xrec = ch.wbuf;
  double* Yrec = Xrec + 2 * kMaxK * kWin;
  int m = 0, m_inv = 0;          // pending flips; those already in T and S
  int l0 = l_begin;
  const bool ph = p.ph != 0;     // G_up only; G_dn = 1 - G_up^T
  const int nsp = ph ? 1 : 2;
  while (l0 < L) {
    const int b = min(kWin, L - l0);
    fill_uniforms(ch.uw, ch.key0, (uint64_t)ch.grid, sw, l0, b);
    if (m > 0) {
      const long long t0 = wall_clock64();
      invert_ts(w, m_inv, m, nsp);
      m_inv = m;
      window_apply<GT>(ch, w, l0, b, m, nsp);
      if (t == 0) {
        const long long dt = wall_clock64() - t0;
        ch.st[ST_T_FLUSH] += dt;
        ch.st[ST_T_WAPPLY] += dt;
      }
    } else {
      for (int idx = t; idx < kWin * kWin; idx += kThreads) {
        const int q = idx >> 6, r = idx & 63;
        if (q < b && r < b) {
          const long long o = (long long)(l0 + q) * L + l0 + r;
          w.Wu[q * kWP + r] = reinterpret_cast<const GT*>(ch.Gu)[o];
          if (!ph) w.Wd[q * kWP + r] = reinterpret_cast<const GT*>(ch.Gd)[o];
        }
      }
      __syncthreads();
    }
    const int m0 = m;
    int pos = 0;
    bool close = false;
    while (pos < b && !close) {
      const int l = l0 + pos;
      const int sl = ch.s[l];
      const double wul = w.Wu[pos * kWP + pos];
      const Flip f = propose(wul, ph ? 1.0 - wul : w.Wd[pos * kWP + pos], sl, io.gp, io.gm,
                             ch.uw[pos], io.rlog, io.rlen, sw * L + l, k, ch.st, io.hb);
      if (f.accept) {
        log_flip(io, ch.st, sw * L + l);
        const double cu = f.g_up / f.r_up, cd = f.g_dn / f.r_dn;
        // in-window parts of x = G(:,l) - e_l and y = c G(l,:)
        if (t < b) {
          const double v = w.Wu[t * kWP + pos] - (t == pos ? 1.0 : 0.0);
          w.xu[t] = v;
          Xrec[(0 * kMaxK + m) * kWin + t] = v;
        } else if (t >= 64 && t < 64 + b) {
          const int r = t - 64;
          const double v = mul_nc(cu, w.Wu[pos * kWP + r]);
          w.yu[r] = v;
          Yrec[(0 * kMaxK + m) * kWin + r] = v;
        } else if (!ph && t >= 128 && t < 128 + b) {
          const int q = t - 128;
          const double v = w.Wd[q * kWP + pos] - (q == pos ? 1.0 : 0.0);
          w.xd[q] = v;
          Xrec[(1 * kMaxK + m) * kWin + q] = v;
        } else if (!ph && t >= 192 && t < 192 + b) {
          const int r = t - 192;
          const double v = mul_nc(cd, w.Wd[pos * kWP + r]);
          w.yd[r] = v;
          Yrec[(1 * kMaxK + m) * kWin + r] = v;
        }
        if (t == 0) {
          w.F[m] = l;
          w.cU[m] = cu;
          w.cD[m] = cd;
        }
        __syncthreads();
        // only the trailing block (rows and columns after pos) is read again in
        // this window: later proposals read its diagonal, later flips' vectors
        // and coefficients read rows / columns beyond their own slice
        for (int idx = t; idx < kWin * kWin; idx += kThreads) {
          const int q = idx >> 6, r = idx & 63;
          if (q > pos && q < b && r > pos && r < b) {
            w.Wu[q * kWP + r] = axpy_nc(w.Wu[q * kWP + r], w.xu[q], w.yu[r]);
            if (!ph) w.Wd[q * kWP + r] = axpy_nc(w.Wd[q * kWP + r], w.xd[q], w.yd[r]);
          }
        }
        if (t == 0) ch.s[l] = (int8_t)(-sl);
        ++m;
        ++k.acc_since;
        __syncthreads();
        close = (m == p.delay_k) || (k.acc_since == p.n_rec);
      }
      ++pos;
    }
    l0 += pos;
    if (m > m0) {
      const long long t0 = wall_clock64();
      capture_coefficients(ch, w, l0 - pos, m0, m, nsp);
      if (t == 0) ch.st[ST_T_FLUSH] += wall_clock64() - t0;
    }
    // a recompute that does not sample the drift needs no flush before it
    if (m > 0 && k.acc_since == p.n_rec && !drift_sampled(k.n_rec + 1, p.drift_every)) {
      m = 0;
      m_inv = 0;
    }
    // flush at delay_k pending, before a recompute and at the sweep end
    if (m > 0 && (close || l0 >= L)) {
      const long long t0 = wall_clock64();
      invert_ts(w, m_inv, m, nsp);
      if (t == 0) ch.st[ST_T_FOLD] += wall_clock64() - t0;
      flush_pending<MIXED, GT>(ch, w, m, nsp);
      if (t == 0) {
        ch.st[ST_T_FLUSH] += wall_clock64() - t0;
        ch.st[ST_FLUSHES] += 1;
      }
      m = 0;
      m_inv = 0;
    }
    if (k.acc_since == p.n_rec) return l0;
  }
  return L;
}

// ----------------------------------------------------------- the chain ----

// Pointers of one chain: workspace ws (G_up, G_dn, LU, U11^{-1} blocks,
// delayed-update buffers) and the LDS layout (field, uniforms, reduction
// slots, statistics, slice lists, then the phase-shared scratch).
__device__ __forceinline__ void setup_chain(Chain& ch, const SweepParams& p, const GridDev* gd,
                                            int chain, double* ws, char* lds, int lu_nb,
                                            int scratch_bytes) {
  ch.G0 = gd->G0;
  ch.ep = gd->ep;
  ch.em = gd->em;
  ch.L = gd->L;
  ch.chain = chain;
  ch.key0 = p.seed + (uint64_t)chain;
  ch.refQ[0] = gd->refQ[0];
  ch.refQ[1] = gd->refQ[1];
  ch.refH[0] = gd->refH[0];
  ch.refH[1] = gd->refH[1];
  ch.lu_nb = lu_nb;
  ch.reduced = gd->direct == 0;
  const int L = ch.L;
  const long long L2 = (long long)L * L;
  ch.Gu = ws;
  ch.Gd = ws + L2;
  ch.A = ws + 2 * L2;
  {
    // LU workspace for any panel width: 2 (L + kNBMax)^2 doubles (the padded
    // L x 2L system, or the reduced one with its product's operands), then the
    // U11^{-1} blocks
    const long long lp = L + kNBMax;
    ch.Ui = ch.A + 2 * lp * lp;
    ch.gtd = ch.Ui + lp * kNBMax;
    ch.wbuf = ch.gtd + gtd_doubles(p.Lmax);
  }
  ch.grid = gd->grid_id;
  ch.s = reinterpret_cast<int8_t*>(lds);
  const int s_bytes = (p.Lmax + 15) & ~15;
  ch.uw = reinterpret_cast<double*>(lds + s_bytes);
  ch.red = ch.uw + kUW;
  ch.st = reinterpret_cast<long long*>(ch.red + 64);
  ch.drift = reinterpret_cast<double*>(ch.st + NSTAT);
  ch.drift_gt = ch.drift + 1;
  ch.scratch = reinterpret_cast<char*>(ch.red + 64) + kStatBytes;
  ch.sr = reinterpret_cast<int*>(ch.scratch);
  ch.scratch_bytes = scratch_bytes;
}

// VAR 0: every mode, chosen at run time; 1: mixed with G stored in FP32;
// 2: spin-dependent baths (every mode, FP64-stored G, spin-resolved estimators);
// 3: as 0 with the LU panel in the workspace (long grids)
template <int VAR>
__device__ __forceinline__ void run_chain(const SweepParams& p, const GridDev* gd, int chain, double* ws,
                          char* lds) {
  typedef typename std::conditional<VAR == 1, float, double>::type GT;   // stored G
  constexpr bool SPIN = VAR == 2;
  constexpr bool PG = VAR == 3;
  Chain ch;
  setup_chain(ch, p, gd, chain, ws, lds, gd->lu_nb, p.lds_scratch_bytes);
  const int L = ch.L;
  const long long L2 = (long long)L * L;

  // this chain's accumulators
  const int nb = p.n_bins;
  const int ng = SPIN ? 2 * (L + 1) : L + 1;   // estimator entries per sample
  ch.accg = gd->acc_g + (long long)chain * nb * ng;
  if constexpr (PG) ch.Pg = ws + p.work_stride - panel_doubles(p.Lmax);
  if constexpr (SPIN) {
    ch.G0d = gd->G0d;
    ch.refQd[0] = gd->refQd[0];
    ch.refQd[1] = gd->refQd[1];
    ch.refHd[0] = gd->refHd[0];
    ch.refHd[1] = gd->refHd[1];
  }
  ch.accd = gd->acc_d + (long long)chain * nb;
  ch.accn = gd->acc_n + (long long)chain * nb;

  // initial field: s_l = +1 if u < 1/2 (stream 1, sweep 0)
  for (int l = threadIdx.x; l < L; l += kThreads)
    ch.s[l] = uniform53(ch.key0, (uint64_t)gd->grid_id, (uint64_t)l, 0ull, 1ull) < 0.5 ? 1 : -1;
  __syncthreads();

  if (threadIdx.x < NSTAT) ch.st[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    *ch.drift = 0.0;
    *ch.drift_gt = 0.0;
  }
  __syncthreads();
  Counters k = {0, 0, 0};

  ChainIO io;
  io.flog = gd->flip_log ? gd->flip_log + (long long)chain * p.flip_cap : nullptr;
  io.rlog = gd->replay ? gd->replay + (long long)chain * p.replay_cap : nullptr;
  io.rlen = gd->replay ? min(gd->replay_n[chain], p.replay_cap) : 0;
  io.flip_cap = p.flip_cap;
  io.gp = gd->gp;
  io.gm = gd->gm;
  io.hb = p.heat_bath != 0;

  // One loop drives the whole chain so that every phase has a single call
  // site: recompute (initial, then whenever n_rec flips have been accepted,
  // right after the flip that completes the count), sweep segments, and the
  // measurement after each measured sweep.
  const long long n_meas = gd->sweeps;   // measured sweeps of this grid's chains
  const long long total = p.warmup + n_meas;
  long long sw = 0;
  int l = 0;
  bool need_rec = true, first = true;
  for (;;) {
    if (need_rec) {
      recompute_both<GT, SPIN, PG>(p, ch, k, !first);
      first = false;
      need_rec = false;
    }
    if (l >= L) {
      if (sw >= p.warmup) {
        const long long t1 = wall_clock64();
        const long long msw = sw - p.warmup;
        const int bin = (int)((msw * nb) / n_meas);
        measure<GT, SPIN>(ch, bin, p.ph != 0);
        stat_add(ch.st, ST_T_MEAS, wall_clock64() - t1);
      }
      __syncthreads();
      ++sw;
      l = 0;
    }
    if (sw >= total) break;
    const long long t0 = wall_clock64();
    const long long f0 = threadIdx.x == 0 ? ch.st[ST_T_FLUSH] : 0;
    int nl;
    if constexpr (VAR == 1) {
      nl = sweep_window<true, float>(p, ch, sw, k, io, l);
    } else {
      if (p.mode == MODE_RANK1)
        nl = sweep_rank1(p, ch, sw, k, io, l);
      else if (p.mode == MODE_MIXED)
        nl = sweep_window<true, double>(p, ch, sw, k, io, l);
      else
        nl = sweep_window<false, double>(p, ch, sw, k, io, l);
    }
    if (threadIdx.x == 0) ch.st[ST_T_SWEEP] += (wall_clock64() - t0) - (ch.st[ST_T_FLUSH] - f0);
    need_rec = (k.acc_since == p.n_rec);
    l = nl;
  }

  if (threadIdx.x == 0) {
    long long* st = gd->cstats + (long long)chain * NSTAT;
    ch.st[ST_REPLAYED] = k.rep_i;
    for (int q = 0; q < NSTAT; ++q) st[q] = ch.st[q];
    gd->cdrift[chain] = *ch.drift;
    gd->cdrift_gt[chain] = *ch.drift_gt;
  }
  if (gd->g_final) {
    double* out = gd->g_final + (long long)chain * 2 * L2;
    const GT* Gup = reinterpret_cast<const GT*>(ch.Gu);
    const GT* Gdn = reinterpret_cast<const GT*>(ch.Gd);
    for (long long idx = threadIdx.x; idx < L2; idx += kThreads) {
      out[idx] = Gup[idx];
      if (p.ph) {
        const long long i = idx / L, j = idx - i * L;   // G_dn(i, j) = delta_ij - G_up(j, i)
        out[L2 + idx] = (i == j ? 1.0 : 0.0) - Gup[j * L + i];
      } else {
        out[L2 + idx] = Gdn[idx];
      }
    }
  }
  __syncthreads();
}

// ------------------------------------------------- persistent kernel ----

// One kernel per variant of run_chain (VAR above): the default kernel carries
// no code of the other two
template <int VAR>
__global__ void __launch_bounds__(kThreads) k_sweeps(SweepParams p) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_unit;
  double* ws = p.work + (long long)blockIdx.x * p.work_stride;
  for (;;) {
    if (threadIdx.x == 0) s_unit = atomicAdd(p.queue, 1);
    __syncthreads();
    const int unit = __builtin_amdgcn_readfirstlane(s_unit);   // uniform: scalar loads, branches
    __syncthreads();
    if (unit >= p.n_units) break;
    const int code = p.units[unit];
    const int gi = code >> 20, c = code & 0xFFFFF;
    run_chain<VAR>(p, p.grids + gi, c, ws, lds);
  }
}

// Uniform-field references of every grid: workgroup 4 g + 2 r + kind solves
// M_r X = G0 (kind 0, X = H_r) or M_r X = 1 - G0 (kind 1, X = Q_r) with the
// direct LU, M_r = 1 + d_r (1 - G0), d_0 = e^{lambda} - 1, d_1 = e^{-lambda} - 1
// (the field s = +1 everywhere, spin up for r = 0 and down for r = 1).
// dn: the spin-down references of grids with spin-dependent baths (from G0d).
__global__ void __launch_bounds__(kThreads) k_reference(SweepParams p, int scratch_bytes, int dn) {
  extern __shared__ __align__(16) char lds[];
  const int gi = blockIdx.x >> 2, r = (blockIdx.x >> 1) & 1, kind = blockIdx.x & 1;
  const GridDev* gd = p.grids + gi;
  if (gd->direct) return;   // grids recomputed in full size need no references
  if (dn && !gd->spin) return;
  const int nb = gd->ref_nb;
  Chain ch;
  double* ws = p.work + (long long)blockIdx.x * p.work_stride;
  setup_chain(ch, p, gd, 0, ws, lds, nb, scratch_bytes);
  if (dn) ch.G0 = gd->G0d;
  for (int l = threadIdx.x; l < ch.L; l += kThreads) ch.s[l] = 1;
  if (threadIdx.x < NSTAT) ch.st[threadIdx.x] = 0;
  __syncthreads();
  double* out = const_cast<double*>(dn ? (kind ? gd->refQd[r] : gd->refHd[r])
                                       : (kind ? gd->refQ[r] : gd->refH[r]));
  if (gd->ref_pg) {
    // long grids: the L-row system's panel does not fit LDS, it goes to the
    // end of the workgroup's workspace slot (sized for it)
    ch.Pg = ws + p.work_stride - panel_doubles(p.Lmax);
    (void)dyson_solve<double, false, true>(ch, r == 0 ? 1 : -1, out, nb, false, kind == 1);
  } else {
    (void)dyson_solve(ch, r == 0 ? 1 : -1, out, nb, false, kind == 1);
  }
  if (threadIdx.x == 0 && ch.st[ST_SINGULAR]) *gd->ref_sing = 1;
}

// ---------------------------------------------------- chain reduction ----
// Per grid: mean over all (chain, bin) sample means and standard error
// (sample standard deviation / sqrt(number of samples)).
__global__ void k_reduce(const GridDev* grids, int n_bins) {
  const GridDev& g = grids[blockIdx.x];
  const int L = g.L;
  const int ng = g.spin ? 2 * (L + 1) : L + 1;   // G entries per sample
  const int ns_tot = g.n_chains * n_bins;
  for (int k = threadIdx.x; k <= ng; k += blockDim.x) {
    // k == ng handles D
    double sum = 0.0;
    int ns = 0;
    for (int q = 0; q < ns_tot; ++q) {
      const long long n = g.acc_n[q];
      if (n <= 0) continue;
      const double v = (k < ng ? g.acc_g[(long long)q * ng + k] : g.acc_d[q]) / (double)n;
      sum += v;
      ++ns;
    }
    const double mean = ns > 0 ? sum / ns : 0.0;
    double var = 0.0;
    for (int q = 0; q < ns_tot; ++q) {
      const long long n = g.acc_n[q];
      if (n <= 0) continue;
      const double v = (k < ng ? g.acc_g[(long long)q * ng + k] : g.acc_d[q]) / (double)n;
      var += (v - mean) * (v - mean);
    }
    const double err = ns > 1 ? sqrt(var / (ns - 1)) / sqrt((double)ns) : 0.0;
    if (k < ng) {
      g.g_out[k] = mean;
      g.g_err[k] = err;
    } else {
      g.d_out[0] = mean;
      g.d_out[1] = err;
    }
  }
}

// ------------------------------------------------------------- host side ----

long long workspace_doubles(int Lmax, int kmax) {
  const long long L2 = (long long)Lmax * Lmax;
  const long long Lp = Lmax + kNBMax;  // LU padding
  long long w = 2 * L2 + 2 * Lp * Lp + Lp * kNBMax + gtd_doubles(Lmax) + 256;
  if (kmax > 1) w += 4LL * kMaxK * kWin + 4LL * Lmax * kMaxK;
  w += panel_doubles(Lmax);   // last: the LU panel when it leaves LDS
  return (w + 63) & ~63LL;
}

// LDS bytes of the LU besides the panel and the inverted triangle: reduction
// slots, pivots and the double-buffered staged candidate rows.
constexpr long long kLuExtra = 1024 + 2LL * (kThreads / 64) * (kNBMax + 2) * 8 + 256 + 4 * 1056;

// LU panel width: the widest of 32/16/8/4 (at most nb_max) whose padded LDS
// panel fits the budget.
static int lu_panel(int Lmax, long long budget, int nb_max, int pg) {
  const int cand[4] = {32, 16, 8, 4};
  for (int q = 0; q < 4; ++q) {
    const int nb = cand[q];
    if (nb > nb_max) continue;
    const long long np = (Lmax + nb - 1) / nb * nb;
    if (nb >= 16 && np > (long long)kThreads * (nb == 32 ? 1 : 2)) continue;  // register panel
    const long long panel = pg ? 0 : np * (nb + 2) * 8;
    if (panel + (long long)nb * (nb + 1) * 8 + kLuExtra <= budget) return nb;
  }
  return 4;
}

int lds_bytes(int Lmax, int L, int mode, int nb_max, int direct, int* lu_nb, int* scratch_bytes,
              int pg) {
  const long long head = ((Lmax + 15) & ~15) + kUW * 8 + 64 * 8 + kStatBytes;
  const long long srb = direct ? 0 : ((4LL * L + 15) & ~15);   // reduced form's slice lists
  const long long budget = 150 * 1024 - head - srb;
  const int nsys = direct ? L : (L / 2 > 0 ? L / 2 : 1);
  const int nb = lu_panel(nsys, budget, nb_max > 0 ? nb_max : kNBMax, pg);
  *lu_nb = nb;
  const long long np = (nsys + nb - 1) / nb * nb;
  const long long lu =
      srb + (pg ? 0 : np * (nb + 2) * 8) + (long long)nb * (nb + 1) * 8 + kLuExtra;
  long long sc = lu;
  if (mode == MODE_RANK1) {
    const long long r1 = 4LL * Lmax * 8;
    sc = sc > r1 ? sc : r1;
  } else if (mode == MODE_DELAYED_FP64 || mode == MODE_MIXED) {
    const long long win = kSmall + (2LL * kWin * kWP + 4LL * kWin + 2LL * kMaxK * kKP) * 8;
    // flush GEMM: at least one kCW-wide FP64 panel of Y
    const long long yp = kSmall + 1LL * kCW * kYK * 8;
    const long long w = win > yp ? win : yp;
    sc = sc > w ? sc : w;
  }
  if (!direct) {
    // reduced form: G[S,:] staged 64 columns wide where all its rows fit, else
    // narrower; where even 16 columns of all rows do not fit, the product
    // streams K in slabs through whatever the scratch holds (at least 8 rows)
    const long long kr = (nsys + 7LL) & ~7LL;
    long long z = srb + 8LL * (16 + 2) * 8;
    for (int zw = 64; zw >= 16; zw >>= 1) {
      const long long zf = srb + kr * (zw + 2) * 8;
      if (head + (sc > zf ? sc : zf) <= 150 * 1024) {
        z = zf;
        break;
      }
    }
    sc = sc > z ? sc : z;
  }
  sc = (sc + 15) & ~15LL;
  *scratch_bytes = (int)sc;
  return (int)(head + sc);
}

hipError_t launch_build_g0(const double* g_tau, int L, double* G0, hipStream_t s) {
  const long long n = (long long)L * L;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_build_g0, dim3(blocks), dim3(256), 0, s, g_tau, L, G0);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero<double>, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_i64(long long* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero<long long>, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_i32(int* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero<int>, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t prepare_sweeps(int lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_sweeps<0>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_sweeps<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_sweeps<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_sweeps<3>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  return e;
}

hipError_t launch_sweeps(const SweepParams& p, int n_wg, int lds, hipStream_t s) {
  if (p.mode == MODE_MIXED_G32)
    hipLaunchKernelGGL(k_sweeps<1>, dim3(n_wg), dim3(kThreads), lds, s, p);
  else if (p.spin)
    hipLaunchKernelGGL(k_sweeps<2>, dim3(n_wg), dim3(kThreads), lds, s, p);
  else if (p.pg)
    hipLaunchKernelGGL(k_sweeps<3>, dim3(n_wg), dim3(kThreads), lds, s, p);
  else
    hipLaunchKernelGGL(k_sweeps<0>, dim3(n_wg), dim3(kThreads), lds, s, p);
  return hipGetLastError();
}

hipError_t prepare_reference(int lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void*)k_reference, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

hipError_t launch_reference(const SweepParams& p, int lds, int scratch, int dn, hipStream_t s) {
  hipLaunchKernelGGL(k_reference, dim3(4 * p.n_grids), dim3(kThreads), lds, s, p, scratch, dn);
  return hipGetLastError();
}

hipError_t launch_reduce(const GridDev* grids, int n_grids, int n_bins, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(n_grids), dim3(256), 0, s, grids, n_bins);
  return hipGetLastError();
}

}  // namespace hfqmc
