// Device memory of the allocation-free entry point (hfqmc_solve_dev_noalloc):
// one static buffer per GPU, and the small kernels that let that entry point
// run without host-side staging (grid record, dispatch order, statistics).
//
// `scratch` below is a file-scope device array.  In host code its name stands
// for a host-side shadow, not a device address: host code uses only the
// address noalloc_scratch_lookup() returns for a device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hfqmc_internal.h"

namespace hfqmc {

static __device__ __align__(256) char scratch[kNoAllocBytes];

// Device address of `scratch` on each GPU (each holds its own copy), looked up
// once per device with that device current and kept with the lookup's status.
namespace {
constexpr int kMaxDev = 64;
std::mutex g_mu;
void* g_ptr[kMaxDev] = {};
hipError_t g_status[kMaxDev] = {};
bool g_done[kMaxDev] = {};
}  // namespace

hipError_t noalloc_scratch_lookup(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[device]) {
    void* p = nullptr;
    g_status[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[device] = g_status[device] == hipSuccess ? p : nullptr;
    g_done[device] = true;
  }
  *out = g_ptr[device];
  return g_status[device];
}

// Stores one grid record (passed by value as a kernel argument) in device memory.
__global__ void k_put_grid(GridDev g, GridDev* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = g;
}

// Dispatch order of a single grid: unit c is chain c of grid 0.
__global__ void k_iota(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

// One record for the host: the per-chain counters summed over chains, the largest
// drifts, the reference solves' singularity flag and whether every reduced
// output (G(tau), its error, D) is finite.
__global__ void __launch_bounds__(256) k_noalloc_summary(const GridDev* gd, NoAllocSummary* out) {
  const GridDev& g = *gd;
  __shared__ long long ssum[256 / 64][NSTAT];
  __shared__ double sdr[256 / 64][2];
  __shared__ int sbad[256 / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  long long acc[NSTAT];
#pragma unroll
  for (int q = 0; q < NSTAT; ++q) acc[q] = 0;
  double d0 = 0.0, d1 = 0.0;
  int bad = 0;
  for (int c = t; c < g.n_chains; c += blockDim.x) {
#pragma unroll
    for (int q = 0; q < NSTAT; ++q) acc[q] += g.cstats[(long long)c * NSTAT + q];
    const double a = g.cdrift[c], b = g.cdrift_gt[c];
    d0 = (a == a) ? fmax(d0, a) : INFINITY;
    d1 = (b == b) ? fmax(d1, b) : INFINITY;
  }
  const int ng = g.L + 1;
  for (int k = t; k < ng; k += blockDim.x)
    if (!(fabs(g.g_out[k]) < INFINITY) || !(fabs(g.g_err[k]) < INFINITY)) bad = 1;
  if (t == 0 && !(fabs(g.d_out[0]) < INFINITY && fabs(g.d_out[1]) < INFINITY)) bad = 1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int q = 0; q < NSTAT; ++q) acc[q] += __shfl_xor(acc[q], o, 64);
    d0 = fmax(d0, __shfl_xor(d0, o, 64));
    d1 = fmax(d1, __shfl_xor(d1, o, 64));
    bad |= __shfl_xor(bad, o, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NSTAT; ++q) ssum[wv][q] = acc[q];
    sdr[wv][0] = d0;
    sdr[wv][1] = d1;
    sbad[wv] = bad;
  }
  __syncthreads();
  if (t < NSTAT) {
    long long s = 0;
    for (int w = 0; w < 256 / 64; ++w) s += ssum[w][t];
    out->stats[t] = s;
  }
  if (t == 0) {
    double a = 0.0, b = 0.0;
    int nb = 0;
    for (int w = 0; w < 256 / 64; ++w) {
      a = fmax(a, sdr[w][0]);
      b = fmax(b, sdr[w][1]);
      nb |= sbad[w];
    }
    out->max_drift = a;
    out->max_drift_gtau = b;
    out->nonfinite = nb;
    out->ref_singular = g.ref_sing ? (g.ref_sing[0] | g.ref_sing[1] | g.ref_sing[2] | g.ref_sing[3]) : 0;
  }
}

hipError_t launch_put_grid(const GridDev& g, GridDev* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_put_grid, dim3(1), dim3(64), 0, s, g, dst);
  return hipGetLastError();
}

hipError_t launch_iota(int* p, int n, hipStream_t s) {
  int blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_iota, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_noalloc_summary(const GridDev* gd, NoAllocSummary* out, hipStream_t s) {
  hipLaunchKernelGGL(k_noalloc_summary, dim3(1), dim3(256), 0, s, gd, out);
  return hipGetLastError();
}

}  // namespace hfqmc
