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
// (Introduction: Trotter slices, binary HS field, MC sampling).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hfqmc_internal.h"

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

// ------------------------------------------------------ Philox4x64-10 ----
// Counter-based generator of Salmon et al. (SC'11): 10 rounds of
// (x0,x1,x2,x3) -> (hi(M1 x2)^x1^k0, lo(M1 x2), hi(M0 x0)^x3^k1, lo(M0 x0))
// with the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2,
                                                 uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

// 53-bit uniform of the method's stream layout: key (seed + chain, grid),
// counter (slice, sweep, 0, stream); stream 0 = acceptance, 1 = initial field.
__device__ __forceinline__ double uniform53(uint64_t key0, uint64_t grid, uint64_t sl,
                                            uint64_t sweep, uint64_t stream) {
  const uint64_t x0 = philox_word0(sl, sweep, 0ull, stream, key0, grid);
  return (double)(x0 >> 11) * 0x1.0p-53;
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

template <typename T>
__global__ void k_zero(T* p, long long n) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x)
    p[idx] = T(0);
}

// ----------------------------------------------------- chain context ----

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
  double* wbuf;    // delayed-update buffers
  int8_t* s;       // field, LDS
  double* u;       // uniforms, LDS
  char* scratch;   // phase-shared LDS
  double* red;     // reduction scratch, LDS
};

// ------------------------------------------------ Dyson recompute (LU) ----
//
// Solve [1 + (1 - G0) diag(e^{V_sigma} - 1)] G_sigma = G0 for one spin with
// the augmented matrix A = [M | G0] (L x 2L, row-major, in the workspace):
// right-looking blocked LU with partial pivoting (panel of width nb held in
// LDS and factorized by wave 0), forward elimination applied to the
// right-hand side columns in the same trailing updates, then blocked back
// substitution.  Writes the new G into Gs and returns the largest
// elementwise change (drift) against the G it replaces.

// C[i][c] -= sum_j P[i - prow0][j] * A[brow + j][c] for i in [r0, r1), c in [c0, c1).
// P (LDS, row stride ps) holds the left operand; the B rows must not overlap C.
__device__ void lu_gemm_sub(double* __restrict__ A, int lda, int r0, int r1, int c0, int c1,
                            const double* __restrict__ P, int ps, int prow0, int brow, int nb) {
  // each thread owns column pairs (c, c+1), all lanes walk the same rows so the
  // P reads are LDS broadcasts
  for (int c = c0 + 2 * threadIdx.x; c < c1; c += 2 * kThreads) {
    const bool two = (c + 1) < c1;
    double u0[kNBMax], u1[kNBMax];
#pragma unroll
    for (int j = 0; j < kNBMax; ++j) {
      if (j < nb) {
        const double* b = A + (long long)(brow + j) * lda + c;
        u0[j] = b[0];
        u1[j] = two ? b[1] : 0.0;
      }
    }
    for (int i = r0; i < r1; ++i) {
      const double* p = P + (i - prow0) * ps;
      double* a = A + (long long)i * lda + c;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int j = 0; j < kNBMax; ++j) {
        if (j < nb) {
          const double pj = p[j];
          s0 = fma(pj, u0[j], s0);
          s1 = fma(pj, u1[j], s1);
        }
      }
      a[0] -= s0;
      if (two) a[1] -= s1;
    }
  }
}

__device__ double dyson_recompute(const Chain& ch, int sigma, double* __restrict__ Gs,
                                  int nbmax, int* singular) {
  const int n = ch.L;
  const int lda = 2 * n;
  double* __restrict__ A = ch.A;
  const double* __restrict__ G0 = ch.G0;
  const double ep = ch.ep, em = ch.em;
  const int8_t* s = ch.s;

  // build [M | G0]; M[i][j] = delta_ij + (delta_ij - G0[i][j]) f_j, f_j = e^{V_sigma(j)} - 1
  for (long long idx = threadIdx.x; idx < (long long)n * n; idx += kThreads) {
    const int i = (int)(idx / n), j = (int)(idx - (long long)i * n);
    const double g0 = G0[idx];
    const double f = (sigma * s[j] > 0) ? ep : em;
    const double dij = (i == j) ? 1.0 : 0.0;
    A[(long long)i * lda + j] = axpy_nc(dij, dij - g0, f);
    A[(long long)i * lda + n + j] = g0;
  }
  __syncthreads();

  double* P = reinterpret_cast<double*>(ch.scratch);
  int* piv = reinterpret_cast<int*>(P + (long long)n * (nbmax + 1));
  __shared__ int s_sing;
  if (threadIdx.x == 0) s_sing = 0;

  for (int kb = 0; kb < n; kb += nbmax) {
    const int nb = min(nbmax, n - kb);
    const int rows = n - kb;
    const int ps = nb + 1;
    // panel -> LDS
    for (int idx = threadIdx.x; idx < rows * nb; idx += kThreads) {
      const int r = idx / nb, c = idx - r * nb;
      P[r * ps + c] = A[(long long)(kb + r) * lda + kb + c];
    }
    __syncthreads();
    // unblocked LU of the panel by wave 0
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      for (int j = 0; j < nb; ++j) {
        double best = -1.0;
        int bi = rows;
        for (int r = j + lane; r < rows; r += 64) {
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
        if (bi >= rows) bi = j;
        if (lane == 0) piv[j] = bi;
        if (bi != j) {
          for (int c = lane; c < nb; c += 64) {
            const double t = P[j * ps + c];
            P[j * ps + c] = P[bi * ps + c];
            P[bi * ps + c] = t;
          }
        }
        wave_sync();
        const double p = P[j * ps + j];
        if (lane == 0 && !(fabs(p) > 0.0 && fabs(p) < INFINITY)) s_sing = 1;
        for (int r = j + 1 + lane; r < rows; r += 64) {
          const double l = P[r * ps + j] / p;
          P[r * ps + j] = l;
          for (int c = j + 1; c < nb; ++c) P[r * ps + c] = fma(-l, P[j * ps + c], P[r * ps + c]);
        }
        wave_sync();
      }
    }
    __syncthreads();
    // row interchanges on the columns right of the panel, U11/L11 rows back to A
    for (int c = kb + nb + threadIdx.x; c < lda; c += kThreads) {
      for (int j = 0; j < nb; ++j) {
        const int pj = piv[j];
        if (pj != j) {
          double* a = A + (long long)(kb + j) * lda + c;
          double* b = A + (long long)(kb + pj) * lda + c;
          const double t = *a;
          *a = *b;
          *b = t;
        }
      }
    }
    for (int idx = threadIdx.x; idx < nb * nb; idx += kThreads) {
      const int r = idx / nb, c = idx - r * nb;
      A[(long long)(kb + r) * lda + kb + c] = P[r * ps + c];
    }
    __syncthreads();
    // U12 = L11^{-1} A12 (unit lower), one column per thread
    for (int c = kb + nb + threadIdx.x; c < lda; c += kThreads) {
      double v[kNBMax];
#pragma unroll
      for (int r = 0; r < kNBMax; ++r)
        if (r < nb) v[r] = A[(long long)(kb + r) * lda + c];
#pragma unroll
      for (int r = 1; r < kNBMax; ++r) {
        if (r < nb) {
          double acc = v[r];
#pragma unroll
          for (int j = 0; j < kNBMax; ++j)
            if (j < r) acc = fma(-P[r * ps + j], v[j], acc);
          v[r] = acc;
        }
      }
#pragma unroll
      for (int r = 1; r < kNBMax; ++r)
        if (r < nb) A[(long long)(kb + r) * lda + c] = v[r];
    }
    __syncthreads();
    // trailing update of M and of the right-hand side
    if (kb + nb < n)
      lu_gemm_sub(A, lda, kb + nb, n, kb + nb, lda, P, ps, kb, kb, nb);
    __syncthreads();
  }

  // back substitution U X = Y, block rows from the bottom
  const int nblk = (n + nbmax - 1) / nbmax;
  for (int bI = nblk - 1; bI >= 0; --bI) {
    const int kb = bI * nbmax;
    const int nb = min(nbmax, n - kb);
    const int ps = nb + 1;
    // U11 -> LDS
    for (int idx = threadIdx.x; idx < nb * nb; idx += kThreads) {
      const int r = idx / nb, c = idx - r * nb;
      P[r * ps + c] = A[(long long)(kb + r) * lda + kb + c];
    }
    __syncthreads();
    for (int c = n + threadIdx.x; c < lda; c += kThreads) {
      double v[kNBMax];
#pragma unroll
      for (int r = 0; r < kNBMax; ++r)
        if (r < nb) v[r] = A[(long long)(kb + r) * lda + c];
#pragma unroll
      for (int r = kNBMax - 1; r >= 0; --r) {
        if (r < nb) {
          double acc = v[r];
#pragma unroll
          for (int j = 0; j < kNBMax; ++j)
            if (j > r && j < nb) acc = fma(-P[r * ps + j], v[j], acc);
          v[r] = acc / P[r * ps + r];
        }
      }
#pragma unroll
      for (int r = 0; r < kNBMax; ++r)
        if (r < nb) A[(long long)(kb + r) * lda + c] = v[r];
    }
    __syncthreads();
    if (kb > 0) {
      // left operand U[0:kb, kb:kb+nb] -> LDS, then rows above -= U X_b
      for (int idx = threadIdx.x; idx < kb * nb; idx += kThreads) {
        const int r = idx / nb, c = idx - r * nb;
        P[r * ps + c] = A[(long long)r * lda + kb + c];
      }
      __syncthreads();
      lu_gemm_sub(A, lda, 0, kb, n, lda, P, ps, 0, kb, nb);
      __syncthreads();
    }
  }

  // G <- X, drift against the updated G
  double dmax = 0.0;
  for (long long idx = threadIdx.x; idx < (long long)n * n; idx += kThreads) {
    const int i = (int)(idx / n), j = (int)(idx - (long long)i * n);
    const double x = A[(long long)i * lda + n + j];
    dmax = fmax(dmax, fabs(x - Gs[idx]));
    if (!(fabs(x) < INFINITY)) dmax = INFINITY;
    Gs[idx] = x;
  }
  dmax = block_max(dmax, ch.red);
  if (s_sing) *singular = 1;
  __syncthreads();
  return dmax;
}

// --------------------------------------------------------- measurement ----
// Accumulate G(tau_k) = 1/(2L) sum_sigma sum_l sgn G_sigma((l+k) mod L, l)
// (sgn = -1 where l + k wraps) and D = (1/L) sum_l (1 - Gu_ll)(1 - Gd_ll)
// into the chain's bin.  Thread k walks rows i and reads G(i, (i-k) mod L),
// so every step of a wave reads one contiguous stretch of a row.
__device__ void measure(const Chain& ch, int bin) {
  const int L = ch.L;
  double* accg = ch.accg;
  for (int k = threadIdx.x; k < L; k += kThreads) {
    double acc = 0.0;
    for (int i = 0; i < L; ++i) {
      int j = i - k;
      double sg = 1.0;
      if (j < 0) {
        j += L;
        sg = -1.0;
      }
      const long long o = (long long)i * L + j;
      acc += sg * ch.Gu[o];
      acc += sg * ch.Gd[o];
    }
    const double val = acc / (2.0 * L);
    const long long base = (long long)bin * (L + 1);
    accg[base + k] += val;
    if (k == 0) accg[base + L] += 1.0 - val;
  }
  double dsum = 0.0;
  for (int l = threadIdx.x; l < L; l += kThreads) {
    const long long o = (long long)l * L + l;
    dsum += (1.0 - ch.Gu[o]) * (1.0 - ch.Gd[o]);
  }
  dsum = block_sum(dsum, ch.red);
  if (threadIdx.x == 0) {
    ch.accd[bin] += dsum / L;
    ch.accn[bin] += 1;
  }
}

// ---------------------------------------------------------- proposals ----

struct Counters {
  long long n_prop, n_acc, n_rec, n_bad, n_flips, rep_i;
  double drift;
  int acc_since;
  int singular;
};

// Metropolis decision for flipping s_l, evaluated identically by every thread
// of the workgroup (uniform branch).  In replay mode the decision is read from
// the given flip list instead of u < R.
struct Flip {
  double g_up, g_dn, r_up, r_dn;
  bool accept;
};

__device__ __forceinline__ Flip propose(double gul, double gdl, int sl, double gp, double gm,
                                       double u, const long long* rlog, long long rlen,
                                       long long code, Counters& k) {
  Flip f;
  f.g_up = sl > 0 ? gm : gp;
  f.g_dn = sl > 0 ? gp : gm;
  f.r_up = ratio_factor(f.g_up, gul);
  f.r_dn = ratio_factor(f.g_dn, gdl);
  const double R = mul_nc(f.r_up, f.r_dn);
  ++k.n_prop;
  const bool bad = !(R > 0.0);
  k.n_bad += bad ? 1 : 0;
  if (rlog) {
    f.accept = k.rep_i < rlen && rlog[k.rep_i] == code;
    k.rep_i += f.accept ? 1 : 0;
  } else {
    f.accept = !bad && u < R;
  }
  return f;
}

struct ChainIO {
  long long* flog;
  const long long* rlog;
  long long rlen;
  long long flip_cap;
  double gp, gm;
};

__device__ __forceinline__ void log_flip(const ChainIO& io, Counters& k, long long code) {
  if (io.flog && threadIdx.x == 0 && k.n_flips < io.flip_cap) io.flog[k.n_flips] = code;
  ++k.n_flips;
}

__device__ void recompute_both(const SweepParams& p, const Chain& ch, Counters& k) {
  const double d1 = dyson_recompute(ch, +1, ch.Gu, p.lu_nb, &k.singular);
  const double d2 = dyson_recompute(ch, -1, ch.Gd, p.lu_nb, &k.singular);
  k.drift = fmax(k.drift, fmax(d1, d2));
  ++k.n_rec;
  k.acc_since = 0;
}

// ------------------------------------------------- plain rank-1 sweep ----
// Every accepted flip applies G <- G + (G(:,l) - e_l)(gamma/R_sigma) G(l,:) to
// both L x L matrices in HBM: 32 L^2 bytes of traffic per accepted flip.
__device__ void sweep_rank1(const SweepParams& p, const Chain& ch, long long sw, Counters& k,
                            const ChainIO& io) {
  const int L = ch.L;
  const long long L2 = (long long)L * L;
  double* xu = reinterpret_cast<double*>(ch.scratch);
  double* xd = xu + p.Lmax;
  double* yu = xd + p.Lmax;
  double* yd = yu + p.Lmax;
  for (int l = 0; l < L; ++l) {
    const long long dl = (long long)l * L + l;
    const int sl = ch.s[l];
    const Flip f = propose(ch.Gu[dl], ch.Gd[dl], sl, io.gp, io.gm, ch.u[l], io.rlog, io.rlen,
                           sw * L + l, k);
    if (!f.accept) continue;
    ++k.n_acc;
    log_flip(io, k, sw * L + l);
    // update vectors x = G(:,l) - e_l and y = (gamma/R_sigma) G(l,:)
    const double cu = f.g_up / f.r_up, cd = f.g_dn / f.r_dn;
    for (int i = threadIdx.x; i < L; i += kThreads) {
      const long long ci = (long long)i * L + l;
      xu[i] = ch.Gu[ci] - (i == l ? 1.0 : 0.0);
      xd[i] = ch.Gd[ci] - (i == l ? 1.0 : 0.0);
      yu[i] = mul_nc(cu, ch.Gu[(long long)l * L + i]);
      yd[i] = mul_nc(cd, ch.Gd[(long long)l * L + i]);
    }
    __syncthreads();
    // G += x y^T, both spins, two consecutive elements per thread
    {
      long long idx = 2 * (long long)threadIdx.x;
      int i = (int)(idx / L), j = (int)(idx - (long long)i * L);
      const long long step = 2 * (long long)kThreads;
      const int di = (int)(step / L), dj = (int)(step - (long long)di * L);
      for (; idx < L2; idx += step) {
        int i1 = i, j1 = j + 1;
        if (j1 == L) {
          j1 = 0;
          ++i1;
        }
        ch.Gu[idx] = axpy_nc(ch.Gu[idx], xu[i], yu[j]);
        ch.Gd[idx] = axpy_nc(ch.Gd[idx], xd[i], yd[j]);
        if (idx + 1 < L2) {
          ch.Gu[idx + 1] = axpy_nc(ch.Gu[idx + 1], xu[i1], yu[j1]);
          ch.Gd[idx + 1] = axpy_nc(ch.Gd[idx + 1], xd[i1], yd[j1]);
        }
        i += di;
        j += dj;
        if (j >= L) {
          j -= L;
          ++i;
        }
      }
    }
    if (threadIdx.x == 0) ch.s[l] = (int8_t)(-sl);
    __syncthreads();
    if (++k.acc_since == p.n_rec) recompute_both(p, ch, k);
  }
}

// -------------------------------------------- windowed delayed update ----
//
// The sweep visits l = l0, l0+1, ... inside a window of at most kWin
// consecutive slices.  Deciding and updating inside the window only needs
// the kWin x kWin diagonal blocks of G_up and G_dn, which live in LDS and get
// the exact rank-1 updates of each accepted flip.  The window closes after
// delay_k accepted flips (or at the recompute point, or the sweep end); the
// m accepted flips are then applied to the full matrices as one rank-m update
//   G <- G + X Y,   X = [x_1..x_m] (L x m),  Y = [y_1..y_m]^T (m x L),
// the delayed-update form of m successive Sherman-Morrison steps.  Their full
// vectors follow from the untouched G and the in-window values:
//   x_j = G(:, f_j) - e_{f_j} + sum_{i<j} x_i y_i(f_j)
//   y_j = c_j (G(f_j, :) + sum_{i<j} x_i(f_j) y_i),  c_j = gamma_j / R_j.
// The rank-m product runs in FP64 (MODE_DELAYED_FP64) or with FP32 inputs and
// FP32 accumulation on the matrix cores (MODE_MIXED); ratios, decisions and
// the in-window updates are FP64 in both.

constexpr int kWin = 64;        // slices per window (diagonal block edge)
constexpr int kWP = kWin + 1;   // LDS row stride of the window blocks
constexpr int kKP = kMaxK + 1;  // LDS row stride of the m x m coefficient blocks
constexpr int kSmall = 1536;    // bytes for flip positions and coefficients
constexpr int kTile = 64;       // flush output tile edge
constexpr int kTP = kTile + 4;  // FP64 tile row stride
constexpr int kXS = kMaxK + 1;  // FP32 X tile row stride
constexpr int kYS = kTile + 1;  // FP32 Y tile row stride

typedef float floatx4 __attribute__((ext_vector_type(4)));

// G += X Y for one spin. X: [L][kMaxK] row-major, Y: [kMaxK][L] row-major, m used columns.
template <bool MIXED>
__device__ void flush_gemm(double* __restrict__ G, const double* __restrict__ X,
                           const double* __restrict__ Y, int L, int m, char* lds) {
  const int t = threadIdx.x;
  if constexpr (MIXED) {
    float* Xs = reinterpret_cast<float*>(lds);          // [kTile][kXS]
    float* Ys = Xs + kTile * kXS;                        // [kMaxK][kYS]
    const int m4 = (m + 3) & ~3;
    const int w = t >> 6, lane = t & 63;
    for (int r0 = 0; r0 < L; r0 += kTile) {
      for (int idx = t; idx < kTile * m4; idx += kThreads) {
        const int r = idx / m4, kk = idx - r * m4;
        const int row = r0 + r;
        Xs[r * kXS + kk] = (row < L && kk < m) ? (float)X[(long long)row * kMaxK + kk] : 0.f;
      }
      for (int c0 = 0; c0 < L; c0 += kTile) {
        for (int idx = t; idx < m4 * kTile; idx += kThreads) {
          const int kk = idx / kTile, c = idx - kk * kTile;
          const int col = c0 + c;
          Ys[kk * kYS + c] = (col < L && kk < m) ? (float)Y[(long long)kk * L + col] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int blk = 2 * w + h;
          const int br = blk >> 2, bc = blk & 3;
          floatx4 acc = {0.f, 0.f, 0.f, 0.f};
          for (int k0 = 0; k0 < m4; k0 += 4) {
            const float a = Xs[(br * 16 + (lane & 15)) * kXS + k0 + (lane >> 4)];
            const float b = Ys[(k0 + (lane >> 4)) * kYS + bc * 16 + (lane & 15)];
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
          }
          const int col = c0 + bc * 16 + (lane & 15);
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int row = r0 + br * 16 + 4 * (lane >> 4) + rr;
            if (row < L && col < L) G[(long long)row * L + col] += (double)acc[rr];
          }
        }
        __syncthreads();
      }
    }
  } else {
    double* Xt = reinterpret_cast<double*>(lds);        // [kMaxK][kTP]  (k-major)
    double* Yt = Xt + kMaxK * kTP;                      // [kMaxK][kTP]
    const int tr = t >> 4, tc = t & 15;                 // 32 x 16 threads, 2 x 4 outputs each
    for (int r0 = 0; r0 < L; r0 += kTile) {
      for (int idx = t; idx < kTile * m; idx += kThreads) {
        const int r = idx / m, kk = idx - r * m;
        const int row = r0 + r;
        Xt[kk * kTP + r] = row < L ? X[(long long)row * kMaxK + kk] : 0.0;
      }
      for (int c0 = 0; c0 < L; c0 += kTile) {
        for (int idx = t; idx < m * kTile; idx += kThreads) {
          const int kk = idx / kTile, c = idx - kk * kTile;
          const int col = c0 + c;
          Yt[kk * kTP + c] = col < L ? Y[(long long)kk * L + col] : 0.0;
        }
        __syncthreads();
        double acc[2][4] = {{0.0}};
        for (int kk = 0; kk < m; ++kk) {
          const double x0 = Xt[kk * kTP + 2 * tr], x1 = Xt[kk * kTP + 2 * tr + 1];
          const double* yv = Yt + kk * kTP + 4 * tc;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            acc[0][q] = fma(x0, yv[q], acc[0][q]);
            acc[1][q] = fma(x1, yv[q], acc[1][q]);
          }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int row = r0 + 2 * tr + a;
          if (row >= L) continue;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int col = c0 + 4 * tc + q;
            if (col < L) G[(long long)row * L + col] += acc[a][q];
          }
        }
        __syncthreads();
      }
    }
  }
}

template <bool MIXED>
__device__ void flush_window(const Chain& ch, int l0, int m) {
  const int L = ch.L;
  const int t = threadIdx.x;
  const int* F = reinterpret_cast<const int*>(ch.scratch);
  const double* cU = reinterpret_cast<const double*>(ch.scratch + 256);
  const double* cD = cU + kMaxK;
  char* un = ch.scratch + kSmall;
  double* ULu = reinterpret_cast<double*>(un);
  double* ULd = ULu + kMaxK * kKP;
  const double* Xrec = ch.wbuf;                       // [2][kMaxK][kWin]
  const double* Yrec = Xrec + 2 * kMaxK * kWin;       // [2][kMaxK][kWin]
  double* X = ch.wbuf + 4 * kMaxK * kWin;             // [2][L][kMaxK]
  double* Y = X + 2LL * L * kMaxK;                    // [2][kMaxK][L]
  // in-window coefficients: U(i,j) = y_i(f_j) (i < j) above, x_j(f_i) (i > j) below
  for (int idx = t; idx < m * m; idx += kThreads) {
    const int i = idx / m, j = idx - i * m;
    double vu = 0.0, vd = 0.0;
    if (i < j) {
      vu = Yrec[(0 * kMaxK + i) * kWin + F[j]];
      vd = Yrec[(1 * kMaxK + i) * kWin + F[j]];
    } else if (i > j) {
      vu = Xrec[(0 * kMaxK + j) * kWin + F[i]];
      vd = Xrec[(1 * kMaxK + j) * kWin + F[i]];
    }
    ULu[i * kKP + j] = vu;
    ULd[i * kKP + j] = vd;
  }
  __syncthreads();
  // full update vectors: one row of X or one column of Y per item
  for (int item = t; item < 4 * L; item += kThreads) {
    const int sp = item / (2 * L);
    const int rem = item - sp * 2 * L;
    const double* G = sp ? ch.Gd : ch.Gu;
    const double* UL = sp ? ULd : ULu;
    if (rem < L) {
      const int q = rem;
      double* xs = X + (long long)sp * L * kMaxK + (long long)q * kMaxK;
      for (int j = 0; j < m; ++j) {
        const int fj = l0 + F[j];
        double acc = G[(long long)q * L + fj] - (q == fj ? 1.0 : 0.0);
        for (int i = 0; i < j; ++i) acc = fma(xs[i], UL[i * kKP + j], acc);
        xs[j] = acc;
      }
    } else {
      const int r = rem - L;
      double* ys = Y + (long long)sp * kMaxK * L;
      const double* c = sp ? cD : cU;
      for (int j = 0; j < m; ++j) {
        const int fj = l0 + F[j];
        double acc = G[(long long)fj * L + r];
        for (int i = 0; i < j; ++i) acc = fma(UL[j * kKP + i], ys[(long long)i * L + r], acc);
        ys[(long long)j * L + r] = c[j] * acc;
      }
    }
  }
  __syncthreads();
  flush_gemm<MIXED>(ch.Gu, X, Y, L, m, un);
  flush_gemm<MIXED>(ch.Gd, X + (long long)L * kMaxK, Y + (long long)kMaxK * L, L, m, un);
  __syncthreads();
}

template <bool MIXED>
__device__ void sweep_window(const SweepParams& p, const Chain& ch, long long sw, Counters& k,
                             const ChainIO& io) {
  const int L = ch.L;
  const int t = threadIdx.x;
  int* F = reinterpret_cast<int*>(ch.scratch);
  double* cU = reinterpret_cast<double*>(ch.scratch + 256);
  double* cD = cU + kMaxK;
  char* un = ch.scratch + kSmall;
  double* Wu = reinterpret_cast<double*>(un);
  double* Wd = Wu + kWin * kWP;
  double* xu = Wd + kWin * kWP;
  double* yu = xu + kWin;
  double* xd = yu + kWin;
  double* yd = xd + kWin;
  double* Xrec = ch.wbuf;
  double* Yrec = Xrec + 2 * kMaxK * kWin;
  int l0 = 0;
  while (l0 < L) {
    const int b = min(kWin, L - l0);
    for (int idx = t; idx < kWin * kWin; idx += kThreads) {
      const int q = idx >> 6, r = idx & 63;
      if (q < b && r < b) {
        const long long o = (long long)(l0 + q) * L + l0 + r;
        Wu[q * kWP + r] = ch.Gu[o];
        Wd[q * kWP + r] = ch.Gd[o];
      }
    }
    __syncthreads();
    int m = 0, pos = 0;
    bool close = false;
    while (pos < b && !close) {
      const int l = l0 + pos;
      const int sl = ch.s[l];
      const Flip f = propose(Wu[pos * kWP + pos], Wd[pos * kWP + pos], sl, io.gp, io.gm, ch.u[l],
                             io.rlog, io.rlen, sw * L + l, k);
      if (f.accept) {
        ++k.n_acc;
        log_flip(io, k, sw * L + l);
        const double cu = f.g_up / f.r_up, cd = f.g_dn / f.r_dn;
        // in-window parts of x = G(:,l) - e_l and y = c G(l,:), kept for the flush
        if (t < b) {
          const double v = Wu[t * kWP + pos] - (t == pos ? 1.0 : 0.0);
          xu[t] = v;
          Xrec[(0 * kMaxK + m) * kWin + t] = v;
        } else if (t >= 64 && t < 64 + b) {
          const int r = t - 64;
          const double v = mul_nc(cu, Wu[pos * kWP + r]);
          yu[r] = v;
          Yrec[(0 * kMaxK + m) * kWin + r] = v;
        } else if (t >= 128 && t < 128 + b) {
          const int q = t - 128;
          const double v = Wd[q * kWP + pos] - (q == pos ? 1.0 : 0.0);
          xd[q] = v;
          Xrec[(1 * kMaxK + m) * kWin + q] = v;
        } else if (t >= 192 && t < 192 + b) {
          const int r = t - 192;
          const double v = mul_nc(cd, Wd[pos * kWP + r]);
          yd[r] = v;
          Yrec[(1 * kMaxK + m) * kWin + r] = v;
        }
        if (t == 0) {
          F[m] = pos;
          cU[m] = cu;
          cD[m] = cd;
        }
        __syncthreads();
        for (int idx = t; idx < kWin * kWin; idx += kThreads) {
          const int q = idx >> 6, r = idx & 63;
          if (q < b && r < b) {
            Wu[q * kWP + r] = axpy_nc(Wu[q * kWP + r], xu[q], yu[r]);
            Wd[q * kWP + r] = axpy_nc(Wd[q * kWP + r], xd[q], yd[r]);
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
    if (m > 0) flush_window<MIXED>(ch, l0, m);
    if (k.acc_since == p.n_rec) recompute_both(p, ch, k);
    l0 += pos;
  }
}

// ----------------------------------------------------------- the chain ----

__device__ void run_chain(const SweepParams& p, const GridDev* gd, int chain, double* ws,
                          char* lds) {
  Chain ch;
  ch.G0 = gd->G0;
  ch.ep = gd->ep;
  ch.em = gd->em;
  ch.L = gd->L;
  ch.chain = chain;
  ch.key0 = p.seed + (uint64_t)chain;
  const int L = ch.L;
  const long long L2 = (long long)L * L;
  ch.Gu = ws;
  ch.Gd = ws + L2;
  ch.A = ws + 2 * L2;
  ch.wbuf = ws + 4 * L2;
  ch.s = reinterpret_cast<int8_t*>(lds);
  const int s_bytes = (p.Lmax + 15) & ~15;
  ch.u = reinterpret_cast<double*>(lds + s_bytes);
  ch.red = ch.u + p.Lmax;
  ch.scratch = reinterpret_cast<char*>(ch.red + 64);

  // this chain's accumulators
  const int nb = p.n_bins;
  ch.accg = gd->acc_g + (long long)chain * nb * (L + 1);
  ch.accd = gd->acc_d + (long long)chain * nb;
  ch.accn = gd->acc_n + (long long)chain * nb;

  // initial field: s_l = +1 if u < 1/2 (stream 1, sweep 0)
  for (int l = threadIdx.x; l < L; l += kThreads)
    ch.s[l] = uniform53(ch.key0, (uint64_t)gd->grid_id, (uint64_t)l, 0ull, 1ull) < 0.5 ? 1 : -1;
  __syncthreads();

  Counters k = {0, 0, 0, 0, 0, 0, 0.0, 0, 0};
  dyson_recompute(ch, +1, ch.Gu, p.lu_nb, &k.singular);
  dyson_recompute(ch, -1, ch.Gd, p.lu_nb, &k.singular);

  ChainIO io;
  io.flog = gd->flip_log ? gd->flip_log + (long long)chain * p.flip_cap : nullptr;
  io.rlog = gd->replay ? gd->replay + (long long)chain * p.replay_cap : nullptr;
  io.rlen = gd->replay ? min(gd->replay_n[chain], p.replay_cap) : 0;
  io.flip_cap = p.flip_cap;
  io.gp = gd->gp;
  io.gm = gd->gm;

  const long long total = p.warmup + p.sweeps;
  for (long long sw = 0; sw < total; ++sw) {
    for (int l = threadIdx.x; l < L; l += kThreads)
      ch.u[l] = uniform53(ch.key0, (uint64_t)gd->grid_id, (uint64_t)l, (uint64_t)sw, 0ull);
    __syncthreads();
    if (p.mode == MODE_RANK1)
      sweep_rank1(p, ch, sw, k, io);
    else if (p.mode == MODE_MIXED)
      sweep_window<true>(p, ch, sw, k, io);
    else
      sweep_window<false>(p, ch, sw, k, io);
    if (sw >= p.warmup) {
      const long long msw = sw - p.warmup;
      const int bin = (int)((msw * nb) / p.sweeps);
      measure(ch, bin);
    }
    __syncthreads();
  }

  if (threadIdx.x == 0) {
    long long* st = gd->cstats + (long long)chain * NSTAT;
    st[ST_PROPOSED] = k.n_prop;
    st[ST_ACCEPTED] = k.n_acc;
    st[ST_RECOMPUTES] = k.n_rec;
    st[ST_BAD] = k.n_bad;
    st[ST_SINGULAR] = k.singular;
    st[ST_FLIPS] = k.n_flips;
    st[ST_REPLAYED] = k.rep_i;
    gd->cdrift[chain] = k.drift;
  }
  if (gd->g_final) {
    double* out = gd->g_final + (long long)chain * 2 * L2;
    for (long long idx = threadIdx.x; idx < L2; idx += kThreads) {
      out[idx] = ch.Gu[idx];
      out[L2 + idx] = ch.Gd[idx];
    }
  }
  __syncthreads();
}

// ------------------------------------------------- persistent kernel ----

__global__ void __launch_bounds__(kThreads) k_sweeps(SweepParams p) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_unit;
  double* ws = p.work + (long long)blockIdx.x * p.work_stride;
  for (;;) {
    if (threadIdx.x == 0) s_unit = atomicAdd(p.queue, 1);
    __syncthreads();
    const int unit = s_unit;
    __syncthreads();
    if (unit >= p.n_units) break;
    const int code = p.units[unit];
    const int gi = code >> 20, c = code & 0xFFFFF;
    run_chain(p, p.grids + gi, c, ws, lds);
  }
}

// ---------------------------------------------------- chain reduction ----
// Per grid: mean over all (chain, bin) sample means and standard error
// (sample standard deviation / sqrt(number of samples)).
__global__ void k_reduce(const GridDev* grids, int n_bins) {
  const GridDev& g = grids[blockIdx.x];
  const int L = g.L;
  const int ns_tot = g.n_chains * n_bins;
  for (int k = threadIdx.x; k <= L + 1; k += blockDim.x) {
    // k == L + 1 handles D
    double sum = 0.0;
    int ns = 0;
    for (int q = 0; q < ns_tot; ++q) {
      const long long n = g.acc_n[q];
      if (n <= 0) continue;
      const double v = (k <= L ? g.acc_g[(long long)q * (L + 1) + k] : g.acc_d[q]) / (double)n;
      sum += v;
      ++ns;
    }
    const double mean = ns > 0 ? sum / ns : 0.0;
    double var = 0.0;
    for (int q = 0; q < ns_tot; ++q) {
      const long long n = g.acc_n[q];
      if (n <= 0) continue;
      const double v = (k <= L ? g.acc_g[(long long)q * (L + 1) + k] : g.acc_d[q]) / (double)n;
      var += (v - mean) * (v - mean);
    }
    const double err = ns > 1 ? sqrt(var / (ns - 1)) / sqrt((double)ns) : 0.0;
    if (k <= L) {
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
  long long w = 4 * L2 + 256;
  if (kmax > 1) w += 4LL * kMaxK * kWin + 4LL * Lmax * kMaxK;
  return (w + 63) & ~63LL;
}

int lds_bytes(int Lmax, int mode, int k, int b, int* lu_nb, int* scratch_bytes) {
  (void)k;
  (void)b;
  int nb = 12288 / (Lmax > 0 ? Lmax : 1);
  if (nb > kNBMax) nb = kNBMax;
  if (nb < 4) nb = 4;
  *lu_nb = nb;
  const long long lu = (long long)Lmax * (nb + 1) * 8 + 64 * 4;
  long long sc = lu;
  if (mode == MODE_RANK1) {
    const long long r1 = 4LL * Lmax * 8;
    sc = sc > r1 ? sc : r1;
  } else {
    const long long win = kSmall + (2LL * kWin * kWP + 4LL * kWin) * 8;
    const long long ul = kSmall + 2LL * kMaxK * kKP * 8;
    const long long t64 = kSmall + 2LL * kMaxK * kTP * 8;
    const long long t32 = kSmall + (1LL * kTile * kXS + 1LL * kMaxK * kYS) * 4;
    long long w = win > ul ? win : ul;
    w = w > t64 ? w : t64;
    w = w > t32 ? w : t32;
    sc = sc > w ? sc : w;
  }
  sc = (sc + 15) & ~15LL;
  *scratch_bytes = (int)sc;
  const long long head = ((Lmax + 15) & ~15) + (long long)Lmax * 8 + 64 * 8;
  return (int)(head + sc);
}

hipError_t launch_build_g0(const double* g_tau, int L, double* G0, hipStream_t s) {
  const long long n = (long long)L * L;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_build_g0, dim3(blocks), dim3(256), 0, s, g_tau, L, G0);
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

hipError_t launch_sweeps(const SweepParams& p, int n_wg, int lds, hipStream_t s) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_sweeps,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sweeps, dim3(n_wg), dim3(kThreads), lds, s, p);
  return hipGetLastError();
}

hipError_t launch_reduce(const GridDev* grids, int n_grids, int n_bins, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(n_grids), dim3(256), 0, s, grids, n_bins);
  return hipGetLastError();
}

}  // namespace hfqmc
