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

  int singular = 0;
  dyson_recompute(ch, +1, ch.Gu, p.lu_nb, &singular);
  dyson_recompute(ch, -1, ch.Gd, p.lu_nb, &singular);

  long long n_prop = 0, n_acc = 0, n_rec = 0, n_bad = 0, n_flips = 0, rep_i = 0;
  double drift = 0.0;
  int acc_since = 0;
  const long long total = p.warmup + p.sweeps;
  long long* flog = gd->flip_log ? gd->flip_log + (long long)chain * p.flip_cap : nullptr;
  const long long* rlog = gd->replay ? gd->replay + (long long)chain * p.replay_cap : nullptr;
  const long long rlen = gd->replay ? min(gd->replay_n[chain], p.replay_cap) : 0;
  const double gp = gd->gp, gm = gd->gm;

  double* xu = reinterpret_cast<double*>(ch.scratch);
  double* xd = xu + p.Lmax;
  double* yu = xd + p.Lmax;
  double* yd = yu + p.Lmax;

  for (long long sw = 0; sw < total; ++sw) {
    for (int l = threadIdx.x; l < L; l += kThreads)
      ch.u[l] = uniform53(ch.key0, (uint64_t)gd->grid_id, (uint64_t)l, (uint64_t)sw, 0ull);
    __syncthreads();
    for (int l = 0; l < L; ++l) {
      const long long dl = (long long)l * L + l;
      const double gul = ch.Gu[dl], gdl = ch.Gd[dl];
      const int sl = ch.s[l];
      const double g_up = sl > 0 ? gm : gp;
      const double g_dn = sl > 0 ? gp : gm;
      const double r_up = ratio_factor(g_up, gul);
      const double r_dn = ratio_factor(g_dn, gdl);
      const double R = mul_nc(r_up, r_dn);
      ++n_prop;
      const bool bad = !(R > 0.0);
      n_bad += bad ? 1 : 0;
      bool accept;
      if (rlog) {
        accept = rep_i < rlen && rlog[rep_i] == sw * L + l;
        rep_i += accept ? 1 : 0;
      } else {
        accept = !bad && ch.u[l] < R;
      }
      if (!accept) continue;
      ++n_acc;
      if (flog && threadIdx.x == 0 && n_flips < p.flip_cap) flog[n_flips] = sw * L + l;
      ++n_flips;
      // update vectors x = G(:,l) - e_l and y = (gamma/R_sigma) G(l,:)
      const double cu = g_up / r_up, cd = g_dn / r_dn;
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
      if (++acc_since == p.n_rec) {
        const double d1 = dyson_recompute(ch, +1, ch.Gu, p.lu_nb, &singular);
        const double d2 = dyson_recompute(ch, -1, ch.Gd, p.lu_nb, &singular);
        drift = fmax(drift, fmax(d1, d2));
        ++n_rec;
        acc_since = 0;
      }
    }
    if (sw >= p.warmup) {
      const long long m = sw - p.warmup;
      const int bin = (int)((m * nb) / p.sweeps);
      measure(ch, bin);
    }
    __syncthreads();
  }

  if (threadIdx.x == 0) {
    long long* st = gd->cstats + (long long)chain * NSTAT;
    st[ST_PROPOSED] = n_prop;
    st[ST_ACCEPTED] = n_acc;
    st[ST_RECOMPUTES] = n_rec;
    st[ST_BAD] = n_bad;
    st[ST_SINGULAR] = singular;
    st[ST_FLIPS] = n_flips;
    st[ST_REPLAYED] = rep_i;
    gd->cdrift[chain] = drift;
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
  long long w = 4 * L2 + 4LL * Lmax * kmax + 256;
  return (w + 63) & ~63LL;
}

int lds_bytes(int Lmax, int mode, int k, int b, int* lu_nb, int* scratch_bytes) {
  (void)mode;
  (void)k;
  (void)b;
  int nb = 12288 / (Lmax > 0 ? Lmax : 1);
  if (nb > kNBMax) nb = kNBMax;
  if (nb < 4) nb = 4;
  *lu_nb = nb;
  const long long lu = (long long)Lmax * (nb + 1) * 8 + 64 * 4;
  const long long r1 = 4LL * Lmax * 8;
  long long sc = lu > r1 ? lu : r1;
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
