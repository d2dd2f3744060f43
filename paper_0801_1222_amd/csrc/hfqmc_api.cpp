// C-ABI of libhfqmc: argument checking, device memory, launch orchestration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "hfqmc.h"
#include "hfqmc_host.h"
#include "hfqmc_internal.h"

using namespace hfqmc;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(HFQMC_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need) {
    if (need <= bytes) return HFQMC_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) {
      p = nullptr;
      return fail(HFQMC_ENOMEM, "hipMalloc(%zu bytes): %s", need, hipGetErrorString(e));
    }
    bytes = need;
    return HFQMC_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// Bump allocator over a byte count (first pass sizes, second pass assigns).
struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* r = base ? (T*)(base + off) : nullptr;
    off += n * sizeof(T);
    return r;
  }
};

}  // namespace

// Autotuner choice for one (mode, chains, grids) shape.
struct TuneChoice {
  int delay_k;
  int lu_nb;
};

// A captured launch sequence and the key of everything its kernels depend on.
struct GraphEntry {
  std::vector<unsigned long long> key;
  hipGraphExec_t exec = nullptr;
  bool whole = false;   // set-up, sweep kernel and reduction; else the set-up only
};

struct hfqmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream the launch sequence is captured on
  int n_cu = 0;
  int lds_max = 0;  // bytes of LDS a workgroup may allocate
  double wall_hz = 1e8;  // device wall-clock rate
  DevBuf work;
  DevBuf arena;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr;  // around the sweep kernel (recorded inside graphs too)
  std::map<std::vector<int>, TuneChoice> tune;  // key: mode, chains, L_0, L_1, ...
  std::vector<GraphEntry> graphs;                // most recent first, at most kGraphCache
  void* na_scratch = nullptr;    // this device's allocation-free buffer (hfqmc_noalloc.hip)
  hipError_t na_status = hipSuccess;
};

namespace {
constexpr size_t kGraphCache = 4;

void drop_graphs(hfqmc_ctx* c) {
  for (auto& g : c->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}
}  // namespace

extern "C" const char* hfqmc_last_error(void) { return g_err.c_str(); }

extern "C" int hfqmc_create(hfqmc_ctx** out, int device) {
  if (!out) return fail(HFQMC_EINVAL, "hfqmc_create: out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
    return fail(HFQMC_EDEVICE, "hfqmc_create: no HIP device");
  if (device < 0 || device >= n) return fail(HFQMC_EINVAL, "hfqmc_create: device %d of %d", device, n);
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(HFQMC_EDEVICE, "hfqmc_create: device %d is %s, this library is built for gfx950",
                device, prop.gcnArchName);
  HIPCHK(hipSetDevice(device));
  hfqmc_ctx* c = new hfqmc_ctx;
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  c->lds_max = (int)prop.sharedMemPerBlock;
  {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
      c->wall_hz = khz * 1e3;
  }
  // the allocation-free entry point's buffer on this device (looked up once per
  // device; a failure is reported by that entry point only)
  c->na_status = noalloc_scratch_lookup(device, &c->na_scratch);
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreate(&c->ev_k0) != hipSuccess || hipEventCreate(&c->ev_k1) != hipSuccess ||
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(HFQMC_EDEVICE, "hfqmc_create: event or stream creation failed");
  }
  *out = c;
  return HFQMC_OK;
}

extern "C" void hfqmc_destroy(hfqmc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  (void)hipDeviceSynchronize();
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->work.release();
  c->arena.release();
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->ev_k0) (void)hipEventDestroy(c->ev_k0);
  if (c->ev_k1) (void)hipEventDestroy(c->ev_k1);
  delete c;
}

extern "C" int hfqmc_set_stream(hfqmc_ctx* c, void* stream) {
  if (!c) return fail(HFQMC_EINVAL, "hfqmc_set_stream: ctx is NULL");
  c->stream = (hipStream_t)stream;
  return HFQMC_OK;
}

namespace {

struct Resolved {
  int n_chains, mode, n_rec, delay_k, window_b, n_bins, drift_every;
  long long warmup, sweeps;
};

int resolve_opts(const hfqmc_opts* o, Resolved* r) {
  if (!o) return fail(HFQMC_EINVAL, "opts is NULL");
  if (o->n_chains < 1 || o->n_chains >= (1 << 20)) return fail(HFQMC_EINVAL, "n_chains=%d", o->n_chains);
  if (o->sweeps < 1 || o->warmup < 0) return fail(HFQMC_EINVAL, "warmup=%lld sweeps=%lld",
                                                  (long long)o->warmup, (long long)o->sweeps);
  if (o->mode < 0 || o->mode > 2) return fail(HFQMC_EINVAL, "mode=%d", o->mode);
  if (o->recompute_every < 0) return fail(HFQMC_EINVAL, "recompute_every=%d", o->recompute_every);
  if (o->n_bins < 0) return fail(HFQMC_EINVAL, "n_bins=%d", o->n_bins);
  if (o->drift_every < 0) return fail(HFQMC_EINVAL, "drift_every=%d", o->drift_every);
  if (o->drift_limit < 0) return fail(HFQMC_EINVAL, "drift_limit < 0");
  if (o->flip_log && (!o->flip_count || o->flip_cap < 1)) return fail(HFQMC_EINVAL, "flip_log needs flip_count and flip_cap >= 1");
  if (o->replay_log && (!o->replay_count || o->replay_cap < 1)) return fail(HFQMC_EINVAL, "replay_log needs replay_count and replay_cap >= 1");
  r->n_chains = o->n_chains;
  r->mode = o->mode;
  r->warmup = o->warmup;
  r->sweeps = o->sweeps;
  if (o->flags & ~(HFQMC_FLAG_EAGER | HFQMC_FLAG_HEAT_BATH | HFQMC_FLAG_DIRECT_RECOMPUTE |
                   HFQMC_FLAG_PH_SYMMETRIC | HFQMC_FLAG_G_FP32 | HFQMC_FLAG_BALANCE))
    return fail(HFQMC_EINVAL, "flags=0x%x", o->flags);
  if ((o->flags & HFQMC_FLAG_BALANCE) &&
      (o->flip_log || o->flip_count || o->replay_log || o->chain_g || o->chain_d || o->chain_n ||
       o->chain_drift || o->final_green))
    return fail(HFQMC_EINVAL, "HFQMC_FLAG_BALANCE changes the chain count: no per-chain hooks");
  if ((o->flags & HFQMC_FLAG_G_FP32) && o->mode != MODE_MIXED)
    return fail(HFQMC_EINVAL, "HFQMC_FLAG_G_FP32 needs the mixed mode (mode=%d)", o->mode);
  if (o->mode == MODE_RANK1) {
    r->delay_k = 1;
    r->window_b = 1;
  } else {
    const int k = o->delay_k;   // 0: chosen by the autotuner before the launch
    if (k != 0 && (k < 2 || k > kMaxK)) return fail(HFQMC_EINVAL, "delay_k=%d (2..%d)", k, kMaxK);
    r->delay_k = k;
    r->window_b = 64;  // slices per window; the kernel's diagonal block edge
  }
  r->n_rec = o->recompute_every > 0 ? o->recompute_every
                                    : (o->mode == MODE_RANK1 ? 100 : 4 * r->delay_k);
  r->n_bins = o->n_bins > 0 ? o->n_bins : (o->n_chains == 1 ? 20 : 1);
  r->drift_every = o->drift_every > 0 ? o->drift_every : 8;
  if (r->n_bins > r->sweeps) return fail(HFQMC_EINVAL, "n_bins=%d > sweeps", r->n_bins);
  return HFQMC_OK;
}

struct GridHost {
  int L;
  double lam;
};

// Adds per-chain counters (ST_* order) to the statistics, the phase clocks
// converted from device wall-clock ticks to seconds.
void add_counters(const long long* s, double wall_hz, hfqmc_stats* gs) {
  gs->n_proposed += s[ST_PROPOSED];
  gs->n_accepted += s[ST_ACCEPTED];
  gs->n_recomputes += s[ST_RECOMPUTES];
  gs->n_bad_ratio += s[ST_BAD];
  gs->n_singular += s[ST_SINGULAR];
  gs->n_flushes += s[ST_FLUSHES];
  const double f = 1.0 / wall_hz;
  gs->chain_s_sweep += s[ST_T_SWEEP] * f;
  gs->chain_s_flush += s[ST_T_FLUSH] * f;
  gs->chain_s_recompute += s[ST_T_REC] * f;
  gs->chain_s_measure += s[ST_T_MEAS] * f;
  gs->chain_s_lu_build += s[ST_T_LU_BUILD] * f;
  gs->chain_s_lu_panel += s[ST_T_LU_PANEL] * f;
  gs->chain_s_lu_strip += s[ST_T_LU_STRIP] * f;
  gs->chain_s_lu_back += s[ST_T_LU_BACK] * f;
  gs->n_reduced_rows += s[ST_RED_ROWS];
  gs->chain_s_lu_gemm += s[ST_T_LU_GEMM] * f;
  gs->chain_s_flush_vectors += s[ST_T_FL_VEC] * f;
  gs->chain_s_flush_gemm += s[ST_T_FL_GEMM] * f;
  gs->chain_s_window_apply += s[ST_T_WAPPLY] * f;
  gs->chain_s_fold += s[ST_T_FOLD] * f;
}

// How a solve is called: host or device buffers, a cap on the LU panel width
// (autotuner trials), and whether it is a trial launch of the autotuner.
// LU panel widths and LDS of a launch.  Where LDS forces a panel below 16 on
// some grid and every grid reaches 16 with its panel in the workspace, the
// launch moves the panels there (pg = 1): long grids keep the matrix-core LU.
struct LuPlan {
  std::vector<int> nb;
  int lds = 0, scratch = 0, lu_nb = 0, pg = 0;
};

LuPlan plan_lu(int n_grids, const int32_t* Ls, int Lmax, int mode, int nb_max, int direct,
               bool allow_pg) {
  LuPlan a;
  for (int pg = 0; pg < 2; ++pg) {
    LuPlan b;
    b.nb.resize(n_grids);
    b.pg = pg;
    bool narrow = false;
    for (int i = 0; i < n_grids; ++i) {
      int sc = 0;
      const int l = lds_bytes(Lmax, Ls[i], mode, nb_max, direct, &b.nb[i], &sc, pg);
      b.lds = std::max(b.lds, l);
      b.scratch = std::max(b.scratch, sc);
      b.lu_nb = std::max(b.lu_nb, b.nb[i]);
      narrow = narrow || b.nb[i] < 16;
    }
    if (pg == 0) {
      a = b;
      if (!narrow || direct || !allow_pg) break;
    } else if (!narrow) {
      a = b;
    }
  }
  return a;
}

struct Call {
  bool dev_io = false;
  int nb_max = 0;
  bool trial = false;
  const double* g0_dn = nullptr;   // spin-down baths (host, like g0_tau): spin-dependent solve
};

int solve_grids_impl(hfqmc_ctx* c, int n_grids, const int32_t* Ls, const double* g0_tau, double U,
                     double beta, uint64_t seed, const hfqmc_opts* opts, double* g_tau,
                     double* g_err, double* docc, hfqmc_stats* stats, const Call& call);

// Autotuner: k in {16, 32, 64} (recompute interval 4k unless given) and the
// LU panel width (the widest that fits, and 16 where 32 fits), each timed on a
// short trial launch of the caller's grids and chain count (no warm-up, two
// sweeps, one where a grid reaches L = 1000; eager launches); the fastest
// kernel time wins and is cached.
int autotune(hfqmc_ctx* c, int n_grids, const int32_t* Ls, const double* g0_tau, bool dev_io,
             double U, double beta, uint64_t seed, const hfqmc_opts* opts, int Lmax,
             TuneChoice* out, double* seconds) {
  std::vector<int> key = {opts->mode, opts->n_chains,
                          opts->flags & (HFQMC_FLAG_PH_SYMMETRIC | HFQMC_FLAG_G_FP32)};
  long long Lsum = 0;
  for (int i = 0; i < n_grids; ++i) {
    key.push_back(Ls[i]);
    Lsum += Ls[i];
  }
  *seconds = 0.0;
  auto it = c->tune.find(key);
  if (it != c->tune.end()) {
    *out = it->second;
    return HFQMC_OK;
  }
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<double> g0h;
  const double* g0 = g0_tau;
  if (dev_io) {
    // the caller's buffer may belong to another HIP runtime of the process:
    // a kernel copies it into memory of this one before it crosses to the host
    DevBuf tmp;
    if (int e = tmp.ensure(sizeof(double) * Lsum)) return e;
    g0h.resize(Lsum);
    hipError_t he = launch_copy(g0_tau, (double*)tmp.p, Lsum, c->stream);
    if (he == hipSuccess)
      he = hipMemcpyAsync(g0h.data(), tmp.p, sizeof(double) * Lsum, hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    tmp.release();
    if (he != hipSuccess) return fail(HFQMC_EDEVICE, "autotune: bath copy: %s", hipGetErrorString(he));
    g0 = g0h.data();
  }
  const int direct = (opts->flags & HFQMC_FLAG_DIRECT_RECOMPUTE) ? 1 : 0;
  const int nb_widest =
      plan_lu(n_grids, Ls, Lmax, opts->mode, 0, direct, !(opts->flags & HFQMC_FLAG_G_FP32)).lu_nb;
  std::vector<int> nbs = {nb_widest};
  if (nb_widest == 32) nbs.push_back(16);
  hfqmc_opts to;
  std::memset(&to, 0, sizeof to);
  to.n_chains = opts->n_chains;
  to.mode = opts->mode;
  to.warmup = 0;
  to.sweeps = Lmax >= 1000 ? 1 : 2;   // long grids: one sweep already takes seconds
  to.recompute_every = opts->recompute_every;
  to.drift_every = opts->drift_every;
  to.n_bins = 1;
  to.flags = (opts->flags & (HFQMC_FLAG_HEAT_BATH | HFQMC_FLAG_DIRECT_RECOMPUTE |
                             HFQMC_FLAG_PH_SYMMETRIC | HFQMC_FLAG_G_FP32)) | HFQMC_FLAG_EAGER;
  long long P = 0;
  for (int i = 0; i < n_grids; ++i) P += Ls[i] + 1;
  std::vector<double> gs(P), es(P), ds(2 * n_grids);
  std::vector<hfqmc_stats> st(n_grids);
  double best = INFINITY;
  TuneChoice choice = {32, nb_widest};
  for (int k : {16, 32, 64}) {
    for (int nb : nbs) {
      to.delay_k = k;
      Call tc;
      tc.nb_max = nb;
      tc.trial = true;
      const int rc = solve_grids_impl(c, n_grids, Ls, g0, U, beta, seed, &to, gs.data(), es.data(),
                                      ds.data(), st.data(), tc);
      if (rc != HFQMC_OK) return rc;
      const double tk = st[0].seconds_kernel;
      if (tk < best) {
        best = tk;
        choice = {k, nb};
      }
    }
  }
  c->tune[key] = choice;
  *out = choice;
  *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return HFQMC_OK;
}

// Shared implementation of every solve entry point.
int solve_grids_impl(hfqmc_ctx* c, int n_grids, const int32_t* Ls, const double* g0_tau, double U,
                     double beta, uint64_t seed, const hfqmc_opts* opts, double* g_tau,
                     double* g_err, double* docc, hfqmc_stats* stats, const Call& call) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!c) return fail(HFQMC_EINVAL, "ctx is NULL");
  if (!Ls || !g0_tau || !g_tau) return fail(HFQMC_EINVAL, "null input/output pointer");
  if (n_grids < 1) return fail(HFQMC_EINVAL, "n_grids=%d", n_grids);
  if (!(U >= 0.0) || !(beta > 0.0) || !std::isfinite(U) || !std::isfinite(beta))
    return fail(HFQMC_EINVAL, "U=%g beta=%g", U, beta);
  Resolved r;
  int rc = resolve_opts(opts, &r);
  if (rc) return rc;
  int Lmax = 0;
  long long Lsum = 0;
  for (int i = 0; i < n_grids; ++i) {
    if (Ls[i] < 2 || Ls[i] > 4096) return fail(HFQMC_EINVAL, "L[%d]=%d (2..4096)", i, Ls[i]);
    Lmax = std::max(Lmax, (int)Ls[i]);
    Lsum += Ls[i];
  }
  if (opts->final_green && n_grids != 1) return fail(HFQMC_EINVAL, "final_green needs a single grid");
  if (!call.dev_io)
    for (long long q = 0; q < Lsum; ++q)
      if (!std::isfinite(g0_tau[q])) return fail(HFQMC_EINVAL, "g0_tau[%lld] not finite", q);
  const bool spin = call.g0_dn != nullptr;
  if (spin) {
    if (call.dev_io) return fail(HFQMC_EINVAL, "spin-dependent baths: host buffers only");
    if (opts->flags & (HFQMC_FLAG_PH_SYMMETRIC | HFQMC_FLAG_G_FP32))
      return fail(HFQMC_EINVAL, "spin-dependent baths exclude HFQMC_FLAG_PH_SYMMETRIC and HFQMC_FLAG_G_FP32");
    for (long long q = 0; q < Lsum; ++q)
      if (!std::isfinite(call.g0_dn[q])) return fail(HFQMC_EINVAL, "g0_dn[%lld] not finite", q);
  }

  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  const int nch = r.n_chains, nbin = r.n_bins;

  // ---- k and the LU panel width: given, or from the autotuner
  int nb_max = call.nb_max;
  bool tuned = false;
  double t_tune = 0.0;
  if (r.mode != MODE_RANK1 && r.delay_k == 0) {
    TuneChoice tc;
    rc = autotune(c, n_grids, Ls, g0_tau, call.dev_io, U, beta, seed, opts, Lmax, &tc, &t_tune);
    if (rc) return rc;
    r.delay_k = tc.delay_k;
    if (opts->recompute_every <= 0) r.n_rec = 4 * r.delay_k;
    nb_max = tc.lu_nb;
    tuned = true;
  }

  // ---- device memory layout (two passes: size, then assign)
  // ---- launch shape (LDS, LU panel width) and the recompute form
  // per grid: the recompute form and its LU panel width; the launch's LDS
  // covers the largest need (the head and update buffers are sized for Lmax)
  const int direct = (opts->flags & HFQMC_FLAG_DIRECT_RECOMPUTE) ? 1 : 0;
  const LuPlan plan = plan_lu(n_grids, Ls, Lmax, r.mode, nb_max, direct,
                              !spin && !(opts->flags & HFQMC_FLAG_G_FP32));
  const std::vector<int>& g_nb = plan.nb;
  const int lu_nb = plan.lu_nb, scratch = plan.scratch, lds = plan.lds;
  if (lds + 1024 > c->lds_max)
    return fail(HFQMC_EUNSUPPORTED, "L=%d needs %d bytes of LDS, device allows %d", Lmax, lds, c->lds_max);
  std::vector<int> g_ref_nb(n_grids, 0), g_ref_pg(n_grids, 0);
  int ref_scratch = 0, ref_lds = 0;
  if (!direct) {
    for (int i = 0; i < n_grids; ++i) {
      // the reference solves are L-row systems: where their panel does not fit
      // LDS it goes to the workspace
      int sc = 0;
      int l = lds_bytes(Lmax, Ls[i], -1, 0, 1, &g_ref_nb[i], &sc);
      if (l + 1024 > c->lds_max) {
        g_ref_pg[i] = 1;
        l = lds_bytes(Lmax, Ls[i], -1, 0, 1, &g_ref_nb[i], &sc, 1);
      }
      ref_lds = std::max(ref_lds, l);
      ref_scratch = std::max(ref_scratch, sc);
    }
    if (ref_lds + 1024 > c->lds_max)
      return fail(HFQMC_EUNSUPPORTED, "L=%d: reference solve needs %d bytes of LDS", Lmax, ref_lds);
  }

  // workgroups per CU: limited by LDS (160 KiB per CU) and by 2048 threads per CU
  const int occ = std::max(1, std::min(c->lds_max / (lds + 1024), 2048 / kThreads));
  // chains per grid: as requested, or split where that shortens the launch
  std::vector<int> g_split(n_grids, 1), g_nch(n_grids, nch);
  if (opts->flags & HFQMC_FLAG_BALANCE)
    plan_chain_split(n_grids, Ls, nch, r.warmup, r.sweeps, nbin, c->n_cu * occ, g_split.data(),
                     nullptr, nullptr);
  long long n_chains_all = 0;
  for (int i = 0; i < n_grids; ++i) {
    g_nch[i] = nch * g_split[i];
    n_chains_all += g_nch[i];
  }

  std::vector<GridDev> gd(n_grids);
  int* d_units = nullptr;
  int* d_queue = nullptr;
  GridDev* d_grids = nullptr;
  double* d_gtau = nullptr;
  double* d_gtau_dn = nullptr;
  auto layout = [&](Bump& b) {
    d_grids = b.take<GridDev>(n_grids);
    d_units = b.take<int>((size_t)n_chains_all);
    d_queue = b.take<int>(64);
    d_gtau = b.take<double>(Lsum);
    d_gtau_dn = spin ? b.take<double>(Lsum) : nullptr;
    for (int i = 0; i < n_grids; ++i) {
      const int L = Ls[i];
      const int ng = spin ? 2 * (L + 1) : L + 1;
      const int nch = g_nch[i];   // the hooks below are excluded when it differs from the request
      GridDev& g = gd[i];
      g.G0 = b.take<double>((size_t)L * L);
      g.G0d = spin ? b.take<double>((size_t)L * L) : g.G0;
      g.acc_g = b.take<double>((size_t)nch * nbin * ng);
      g.acc_d = b.take<double>((size_t)nch * nbin);
      g.acc_n = b.take<long long>((size_t)nch * nbin);
      g.cstats = b.take<long long>((size_t)nch * NSTAT);
      g.cdrift = b.take<double>(nch);
      g.cdrift_gt = b.take<double>(nch);
      g.flip_log = opts->flip_log ? b.take<long long>((size_t)nch * opts->flip_cap) : nullptr;
      g.replay = opts->replay_log ? b.take<long long>((size_t)nch * opts->replay_cap) : nullptr;
      g.replay_n = opts->replay_log ? b.take<long long>(nch) : nullptr;
      g.g_final = opts->final_green ? b.take<double>((size_t)nch * 2 * L * L) : nullptr;
      g.g_out = b.take<double>(ng);
      g.g_err = b.take<double>(ng);
      g.d_out = b.take<double>(2);
      for (int q = 0; q < 2; ++q) {
        g.refQ[q] = direct ? nullptr : b.take<double>((size_t)L * L);
        g.refH[q] = direct ? nullptr : b.take<double>((size_t)L * L);
        g.refQd[q] = (spin && !direct) ? b.take<double>((size_t)L * L) : g.refQ[q];
        g.refHd[q] = (spin && !direct) ? b.take<double>((size_t)L * L) : g.refH[q];
      }
      g.spin = spin ? 1 : 0;
      g.ref_sing = direct ? nullptr : b.take<int>(4);
    }
  };
  Bump sizing(nullptr);
  layout(sizing);
  rc = c->arena.ensure(sizing.off + 256);
  if (rc) return rc;
  Bump assign(c->arena.p);
  layout(assign);

  // ---- per-grid constants (transcendentals on the host)
  std::vector<GridHost> gh(n_grids);
  std::vector<long long> goff0(n_grids);
  long long off = 0, unit_base = 0;
  for (int i = 0; i < n_grids; ++i) {
    const int L = Ls[i];
    const double dtau = beta / L;
    const double lam = std::acosh(std::exp(0.5 * dtau * U));
    gh[i] = {L, lam};
    GridDev& g = gd[i];
    g.L = L;
    g.n_chains = g_nch[i];
    g.sweeps = r.sweeps / g_split[i];
    g.grid_id = i;
    g.unit_base = (int)unit_base;
    unit_base += g_nch[i];
    g.lu_nb = g_nb[i];
    g.direct = direct;
    g.ref_nb = g_ref_nb[i];
    g.ref_pg = g_ref_pg[i];
    g.gp = std::expm1(2.0 * lam);
    g.gm = std::expm1(-2.0 * lam);
    g.ep = std::expm1(lam);
    g.em = std::expm1(-lam);
    goff0[i] = off;
    off += L;
  }
  // device input is copied by a kernel: the caller's buffer may come from another
  // HIP runtime of the process (PyTorch's), whose allocations this one does not track
  if (call.dev_io)
    HIPCHK(launch_copy(g0_tau, d_gtau, Lsum, st));
  else
    HIPCHK(hipMemcpyAsync(d_gtau, g0_tau, sizeof(double) * Lsum, hipMemcpyHostToDevice, st));
  if (spin)
    HIPCHK(hipMemcpyAsync(d_gtau_dn, call.g0_dn, sizeof(double) * Lsum, hipMemcpyHostToDevice, st));
  if (opts->flags & HFQMC_FLAG_PH_SYMMETRIC) {
    // G_dn = 1 - G_up^T needs G0 = 1 - G0^T: G0(0+) = 1/2 and G0(tau) = G0(beta - tau)
    std::vector<double> gh_tau;
    const double* gt = g0_tau;
    if (call.dev_io) {
      gh_tau.resize(Lsum);
      HIPCHK(hipMemcpyAsync(gh_tau.data(), d_gtau, sizeof(double) * Lsum, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      gt = gh_tau.data();
    }
    for (int i = 0; i < n_grids; ++i) {
      const double* g = gt + goff0[i];
      const int L = Ls[i];
      double dev = std::fabs(g[0] - 0.5);
      for (int q = 1; q < L; ++q) dev = std::max(dev, std::fabs(g[q] - g[L - q]));
      if (!(dev <= 1e-9))
        return fail(HFQMC_EINVAL, "HFQMC_FLAG_PH_SYMMETRIC: bath of grid %d deviates from "
                    "particle-hole symmetry by %.3e", i, dev);
    }
  }
  if (opts->replay_log) {
    for (int i = 0; i < n_grids; ++i) {
      HIPCHK(hipMemcpyAsync((void*)gd[i].replay, opts->replay_log + (size_t)i * nch * opts->replay_cap,
                            sizeof(long long) * nch * opts->replay_cap, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync((void*)gd[i].replay_n, opts->replay_count + (size_t)i * nch,
                            sizeof(long long) * nch, hipMemcpyHostToDevice, st));
    }
  }
  // ---- dispatch order: longest chains first (the planner's cost model, L^3 per
  // sweep), then grid, chain
  std::vector<int> units;
  units.reserve((size_t)n_chains_all);
  std::vector<int> order(n_grids);
  for (int i = 0; i < n_grids; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return unit_cost(Ls[a], r.warmup, gd[a].sweeps) > unit_cost(Ls[b], r.warmup, gd[b].sweeps);
  });
  for (int i : order)
    for (int ch = 0; ch < g_nch[i]; ++ch) units.push_back((i << 20) | ch);
  HIPCHK(hipMemcpyAsync(d_units, units.data(), sizeof(int) * units.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_grids, gd.data(), sizeof(GridDev) * n_grids, hipMemcpyHostToDevice, st));

  const int n_units = (int)units.size();
  int n_wg = std::min(n_units, c->n_cu * occ);
  const long long wstride = workspace_doubles(Lmax, r.mode == MODE_RANK1 ? 1 : kMaxK);
  // the reference kernel uses workspace slots 0 .. 4 n_grids - 1
  const int n_slots = direct ? n_wg : std::max(n_wg, 4 * n_grids);
  rc = c->work.ensure((size_t)n_slots * wstride * sizeof(double));
  if (rc) return rc;

  SweepParams p;
  std::memset(&p, 0, sizeof p);
  p.grids = d_grids;
  p.n_grids = n_grids;
  p.units = d_units;
  p.n_units = n_units;
  p.queue = d_queue;
  p.seed = seed;
  p.warmup = r.warmup;
  p.sweeps = r.sweeps;
  p.n_rec = r.n_rec;
  p.mode = (opts->flags & HFQMC_FLAG_G_FP32) ? MODE_MIXED_G32 : r.mode;
  p.delay_k = r.delay_k;
  p.window_b = r.window_b;
  p.n_bins = nbin;
  p.lu_nb = lu_nb;
  p.flip_cap = opts->flip_log ? opts->flip_cap : 0;
  p.replay_cap = opts->replay_log ? opts->replay_cap : 0;
  p.work = (double*)c->work.p;
  p.work_stride = wstride;
  p.Lmax = Lmax;
  p.lds_scratch_bytes = scratch;
  p.heat_bath = (opts->flags & HFQMC_FLAG_HEAT_BATH) ? 1 : 0;
  p.direct = direct;
  p.ph = (opts->flags & HFQMC_FLAG_PH_SYMMETRIC) ? 1 : 0;
  p.spin = spin ? 1 : 0;
  p.pg = plan.pg;
  p.drift_every = r.drift_every;

  // ---- the device launch sequence: bath matrices, zeroed accumulators and
  // counters (fill kernels), the persistent sweep kernel, the chain reduction
  HIPCHK(prepare_sweeps(lds));
  if (!direct) HIPCHK(prepare_reference(ref_lds));
  // The launch sequence: the set-up (bath matrices, zeroed accumulators and
  // counters, uniform-field references: many small launches), then the
  // persistent sweep kernel between two events (its own time) and the chain
  // reduction; captured once as a HIP graph and replayed unless eager.
  auto enqueue = [&](hipStream_t s) -> hipError_t {
    hipError_t e = hipSuccess;
    for (int i = 0; i < n_grids && e == hipSuccess; ++i) {
      const int L = Ls[i];
      const GridDev& g = gd[i];
      const int nch = g_nch[i];
      if ((e = launch_build_g0(d_gtau + goff0[i], L, const_cast<double*>(g.G0), s)) != hipSuccess) break;
      if (spin &&
          (e = launch_build_g0(d_gtau_dn + goff0[i], L, const_cast<double*>(g.G0d), s)) != hipSuccess)
        break;
      if ((e = launch_zero(g.acc_g, (long long)nch * nbin * (spin ? 2 * (L + 1) : L + 1), s)) !=
          hipSuccess)
        break;
      if ((e = launch_zero(g.acc_d, (long long)nch * nbin, s)) != hipSuccess) break;
      if ((e = launch_zero_i64(g.acc_n, (long long)nch * nbin, s)) != hipSuccess) break;
      if ((e = launch_zero_i64(g.cstats, (long long)nch * NSTAT, s)) != hipSuccess) break;
      if ((e = launch_zero(g.cdrift, nch, s)) != hipSuccess) break;
      e = launch_zero(g.cdrift_gt, nch, s);
      if (e == hipSuccess && !direct) e = launch_zero_i32(g.ref_sing, 4, s);
    }
    if (e == hipSuccess && !direct) e = launch_reference(p, ref_lds, ref_scratch, 0, s);
    if (e == hipSuccess && !direct && spin) e = launch_reference(p, ref_lds, ref_scratch, 1, s);
    if (e == hipSuccess) e = launch_zero_i32(d_queue, 64, s);
    return e;
  };
  auto enqueue_sweeps = [&](hipStream_t s) -> hipError_t {
    hipError_t e = hipEventRecord(c->ev_k0, s);
    if (e == hipSuccess) e = launch_sweeps(p, n_wg, lds, s);
    if (e == hipSuccess) e = hipEventRecord(c->ev_k1, s);
    if (e == hipSuccess) e = launch_reduce(d_grids, n_grids, nbin, s);
    return e;
  };
  const bool use_graph = !(opts->flags & HFQMC_FLAG_EAGER);
  bool whole = false;   // the graph holds the whole sequence, not only the set-up
  if (use_graph) {
    // key: everything the captured kernels' arguments depend on
    std::vector<unsigned long long> key;
    key.push_back((unsigned long long)(uintptr_t)c->arena.p);
    key.push_back((unsigned long long)(uintptr_t)c->work.p);
    key.push_back((unsigned long long)n_wg);
    key.push_back((unsigned long long)lds);
    for (int i = 0; i < n_grids; ++i) key.push_back((unsigned long long)Ls[i]);
    for (int i = 0; i < n_grids; ++i) key.push_back((unsigned long long)g_nch[i]);
    {
      unsigned long long w[(sizeof(SweepParams) + 7) / 8] = {0};
      std::memcpy(w, &p, sizeof p);
      key.insert(key.end(), w, w + (sizeof(SweepParams) + 7) / 8);
    }
    hipGraphExec_t exec = nullptr;
    for (size_t q = 0; q < c->graphs.size(); ++q) {
      if (c->graphs[q].key == key) {
        exec = c->graphs[q].exec;
        whole = c->graphs[q].whole;
        std::rotate(c->graphs.begin(), c->graphs.begin() + q, c->graphs.begin() + q + 1);
        break;
      }
    }
    if (!exec) {
      // three captures (set-up; the sweep kernel; the reduction) joined into one
      // graph: set-up -> event ev_k0 -> sweep kernel -> event ev_k1 -> reduction.
      // The events are explicit event-record nodes (a record under stream
      // capture only orders the capture).  If the runtime refuses them, the
      // graph holds the set-up only and the rest is launched after it.
      auto capture = [&](int part, hipGraph_t* out) -> hipError_t {
        *out = nullptr;
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        if (part == 0) e = enqueue(c->cap_stream);
        else if (part == 1) e = launch_sweeps(p, n_wg, lds, c->cap_stream);
        else e = launch_reduce(d_grids, n_grids, nbin, c->cap_stream);
        const hipError_t e2 = hipStreamEndCapture(c->cap_stream, out);
        if (e == hipSuccess) e = e2;
        if (e != hipSuccess && *out) {
          (void)hipGraphDestroy(*out);
          *out = nullptr;
        }
        return e;
      };
      hipGraph_t graph = nullptr, gsw = nullptr, gred = nullptr;
      hipError_t e = capture(0, &graph);
      if (e != hipSuccess)
        return fail(HFQMC_EDEVICE, "capturing the set-up launches: %s", hipGetErrorString(e));
      if (capture(1, &gsw) == hipSuccess && capture(2, &gred) == hipSuccess) {
        // the set-up's leaves: nodes that no edge leaves from
        size_t nn = 0, ne = 0;
        bool ok = hipGraphGetNodes(graph, nullptr, &nn) == hipSuccess &&
                  hipGraphGetEdges(graph, nullptr, nullptr, &ne) == hipSuccess;
        std::vector<hipGraphNode_t> nodes(nn), from(ne), to(ne), leaves;
        ok = ok && hipGraphGetNodes(graph, nodes.data(), &nn) == hipSuccess &&
             (ne == 0 || hipGraphGetEdges(graph, from.data(), to.data(), &ne) == hipSuccess);
        if (ok)
          for (hipGraphNode_t n : nodes)
            if (std::find(from.begin(), from.end(), n) == from.end()) leaves.push_back(n);
        hipGraphNode_t n0 = nullptr, nk = nullptr, n1 = nullptr, nr = nullptr;
        ok = ok && !leaves.empty() &&
             hipGraphAddEventRecordNode(&n0, graph, leaves.data(), leaves.size(), c->ev_k0) == hipSuccess &&
             hipGraphAddChildGraphNode(&nk, graph, &n0, 1, gsw) == hipSuccess &&
             hipGraphAddEventRecordNode(&n1, graph, &nk, 1, c->ev_k1) == hipSuccess &&
             hipGraphAddChildGraphNode(&nr, graph, &n1, 1, gred) == hipSuccess;
        if (ok) {
          whole = true;
        } else {
          // start again from a clean set-up graph
          (void)hipGraphDestroy(graph);
          e = capture(0, &graph);
          if (e != hipSuccess)
            return fail(HFQMC_EDEVICE, "capturing the set-up launches: %s", hipGetErrorString(e));
        }
      }
      (void)hipGetLastError();   // a refused node leaves no sticky state behind
      if (gsw) (void)hipGraphDestroy(gsw);
      if (gred) (void)hipGraphDestroy(gred);
      const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e3 != hipSuccess) return fail(HFQMC_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e3));
      if (c->graphs.size() >= kGraphCache) {
        (void)hipGraphExecDestroy(c->graphs.back().exec);
        c->graphs.pop_back();
      }
      GraphEntry ge;
      ge.key = key;
      ge.exec = exec;
      ge.whole = whole;
      c->graphs.insert(c->graphs.begin(), ge);
    }
    HIPCHK(hipEventRecord(c->ev0, st));
    {
      hipError_t e = hipGraphLaunch(exec, st);
      if (e == hipSuccess && !whole) e = enqueue_sweeps(st);
      if (e != hipSuccess)
        return fail(HFQMC_EDEVICE, "graph launch (%d workgroups, %d B LDS): %s", n_wg, lds,
                    hipGetErrorString(e));
    }
    HIPCHK(hipEventRecord(c->ev1, st));
  } else {
    HIPCHK(hipEventRecord(c->ev0, st));
    {
      hipError_t e = enqueue(st);
      if (e == hipSuccess) e = enqueue_sweeps(st);
      if (e != hipSuccess)
        return fail(HFQMC_EDEVICE, "launch sequence (%d workgroups, %d B LDS, device LDS %d B): %s",
                    n_wg, lds, c->lds_max, hipGetErrorString(e));
    }
    HIPCHK(hipEventRecord(c->ev1, st));
  }

  // ---- results back
  auto out_copy = [&](double* dst, const double* src, long long n) -> hipError_t {
    return call.dev_io ? launch_copy(src, dst, n, st)
                       : hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToHost, st);
  };
  std::vector<long long> cst;
  std::vector<double> cdr, cdg;
  int ref_bad = 0;
  std::vector<double> gcheck;
  long long goff = 0;
  double max_drift = 0.0, max_drift_gt = 0.0;
  bool numeric_bad = false;
  hfqmc_stats tot;
  std::memset(&tot, 0, sizeof tot);
  for (int i = 0; i < n_grids; ++i) {
    const int L = Ls[i];
    const int ng = spin ? 2 * (L + 1) : L + 1;
    const GridDev& g = gd[i];
    const int nchg = g_nch[i];
    cst.assign((size_t)nchg * NSTAT, 0);
    cdr.assign(nchg, 0.0);
    cdg.assign(nchg, 0.0);
    HIPCHK(out_copy(g_tau + goff, g.g_out, ng));
    if (g_err) HIPCHK(out_copy(g_err + goff, g.g_err, ng));
    if (docc) HIPCHK(out_copy(docc + 2 * i, g.d_out, 2));
    if (call.dev_io) {
      gcheck.resize(L + 1);
      HIPCHK(hipMemcpyAsync(gcheck.data(), g.g_out, sizeof(double) * (L + 1), hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipMemcpyAsync(cst.data(), g.cstats, sizeof(long long) * cst.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(cdr.data(), g.cdrift, sizeof(double) * nchg, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(cdg.data(), g.cdrift_gt, sizeof(double) * nchg, hipMemcpyDeviceToHost, st));
    int rs = 0;
    if (!direct) HIPCHK(hipMemcpyAsync(&rs, g.ref_sing, sizeof(int), hipMemcpyDeviceToHost, st));
    const size_t cb = (size_t)i * nch;
    if (opts->flip_log) {
      HIPCHK(hipMemcpyAsync(opts->flip_log + cb * opts->flip_cap, g.flip_log,
                            sizeof(long long) * nch * opts->flip_cap, hipMemcpyDeviceToHost, st));
    }
    if (opts->chain_g)
      HIPCHK(hipMemcpyAsync(opts->chain_g + (size_t)nch * nbin * (goff), g.acc_g,
                            sizeof(double) * nch * nbin * ng, hipMemcpyDeviceToHost, st));
    if (opts->chain_d)
      HIPCHK(hipMemcpyAsync(opts->chain_d + cb * nbin, g.acc_d, sizeof(double) * nch * nbin, hipMemcpyDeviceToHost, st));
    if (opts->chain_n)
      HIPCHK(hipMemcpyAsync((long long*)opts->chain_n + cb * nbin, g.acc_n, sizeof(long long) * nch * nbin, hipMemcpyDeviceToHost, st));
    if (opts->final_green)
      HIPCHK(hipMemcpyAsync(opts->final_green, g.g_final, sizeof(double) * nch * 2 * L * L, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ref_bad |= rs;
    hfqmc_stats gs;
    std::memset(&gs, 0, sizeof gs);
    double gdrift = 0.0, gdrift_gt = 0.0;
    for (int ch = 0; ch < nchg; ++ch) {
      const long long* s = &cst[(size_t)ch * NSTAT];
      add_counters(s, c->wall_hz, &gs);
      gdrift = std::max(gdrift, cdr[ch]);
      if (!(cdr[ch] == cdr[ch])) gdrift = INFINITY;
      gdrift_gt = std::max(gdrift_gt, cdg[ch]);
      if (!(cdg[ch] == cdg[ch])) gdrift_gt = INFINITY;
      if (opts->flip_count) opts->flip_count[cb + ch] = s[ST_FLIPS];
      if (opts->chain_drift) opts->chain_drift[cb + ch] = cdr[ch];
    }
    gs.max_drift = gdrift;
    gs.max_drift_gtau = gdrift_gt;
    gs.acc_rate = gs.n_proposed ? (double)gs.n_accepted / gs.n_proposed : 0.0;
    gs.delay_k = r.delay_k;
    gs.recompute_every = r.n_rec;
    gs.n_workgroups = n_wg;
    gs.lu_panel = lu_nb;
    gs.graph = use_graph ? (whole ? 1 : 2) : 0;
    gs.autotuned = tuned ? 1 : 0;
    gs.seconds_autotune = t_tune;
    gs.recompute_reduced = direct ? 0 : 1;
    gs.chain_split = g_split[i];
    tot.chain_split = std::max(tot.chain_split, g_split[i]);
    if (stats && n_grids > 1) stats[i] = gs;
    tot.n_proposed += gs.n_proposed;
    tot.n_accepted += gs.n_accepted;
    tot.n_recomputes += gs.n_recomputes;
    tot.n_bad_ratio += gs.n_bad_ratio;
    tot.n_singular += gs.n_singular;
    tot.n_flushes += gs.n_flushes;
    tot.chain_s_sweep += gs.chain_s_sweep;
    tot.chain_s_flush += gs.chain_s_flush;
    tot.chain_s_recompute += gs.chain_s_recompute;
    tot.chain_s_measure += gs.chain_s_measure;
    tot.chain_s_lu_build += gs.chain_s_lu_build;
    tot.chain_s_lu_panel += gs.chain_s_lu_panel;
    tot.chain_s_lu_strip += gs.chain_s_lu_strip;
    tot.chain_s_lu_back += gs.chain_s_lu_back;
    tot.n_reduced_rows += gs.n_reduced_rows;
    tot.chain_s_lu_gemm += gs.chain_s_lu_gemm;
    tot.chain_s_flush_vectors += gs.chain_s_flush_vectors;
    tot.chain_s_flush_gemm += gs.chain_s_flush_gemm;
    tot.chain_s_window_apply += gs.chain_s_window_apply;
    tot.chain_s_fold += gs.chain_s_fold;
    max_drift = std::max(max_drift, gdrift);
    max_drift_gt = std::max(max_drift_gt, gdrift_gt);
    const double* gv = call.dev_io ? gcheck.data() : g_tau + goff;
    for (int k = 0; k < (call.dev_io ? L + 1 : ng); ++k)
      if (!std::isfinite(gv[k])) numeric_bad = true;
    goff += ng;
  }
  float ms = 0.f, ms_k = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  HIPCHK(hipEventElapsedTime(&ms_k, c->ev_k0, c->ev_k1));
  const double wall =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  tot.max_drift = max_drift;
  tot.max_drift_gtau = max_drift_gt;
  tot.acc_rate = tot.n_proposed ? (double)tot.n_accepted / tot.n_proposed : 0.0;
  tot.seconds_kernel = ms * 1e-3;
  tot.seconds_sweep_kernel = ms_k * 1e-3;
  tot.seconds_total = wall;
  tot.delay_k = r.delay_k;
  tot.recompute_every = r.n_rec;
  tot.n_workgroups = n_wg;
  tot.lu_panel = lu_nb;
  tot.graph = use_graph ? (whole ? 1 : 2) : 0;
  tot.autotuned = tuned ? 1 : 0;
  tot.seconds_autotune = t_tune;
  tot.recompute_reduced = direct ? 0 : 1;
  if (stats) {
    if (n_grids == 1) {
      stats[0] = tot;
    } else {
      for (int i = 0; i < n_grids; ++i) {
        stats[i].seconds_kernel = tot.seconds_kernel;
        stats[i].seconds_sweep_kernel = tot.seconds_sweep_kernel;
        stats[i].seconds_total = wall;
      }
    }
  }
  if (ref_bad) return fail(HFQMC_ENUMERIC, "singular uniform-field reference matrix");
  if (tot.n_singular) return fail(HFQMC_ENUMERIC, "singular Dyson matrix in %lld recomputes", (long long)tot.n_singular);
  if (numeric_bad || !(max_drift < INFINITY) || !(max_drift_gt < INFINITY))
    return fail(HFQMC_ENUMERIC, "non-finite Green function");
  if (opts->drift_limit > 0 && std::max(max_drift, max_drift_gt) > opts->drift_limit)
    return fail(HFQMC_EDRIFT, "recompute drift %.3e (G(tau): %.3e) exceeds limit %.3e", max_drift,
                max_drift_gt, opts->drift_limit);
  return HFQMC_OK;
}

}  // namespace

extern "C" int hfqmc_solve(hfqmc_ctx* c, const double* g0_tau, int32_t L, double U, double beta,
                           double dtau, uint64_t seed, const hfqmc_opts* opts, double* g_tau,
                           double* g_err, double* docc, hfqmc_stats* stats) {
  if (!(dtau > 0.0) || !(beta > 0.0)) return fail(HFQMC_EINVAL, "dtau=%g beta=%g", dtau, beta);
  if (std::fabs(beta / dtau - L) > 1e-9 * L) return fail(HFQMC_EINVAL, "beta/dtau=%.12g != L=%d", beta / dtau, L);
  const int32_t Ls[1] = {L};
  return solve_grids_impl(c, 1, Ls, g0_tau, U, beta, seed, opts, g_tau, g_err, docc, stats, Call());
}

extern "C" int hfqmc_solve_spin(hfqmc_ctx* c, const double* g0_up, const double* g0_dn, int32_t L,
                                double U, double beta, double dtau, uint64_t seed,
                                const hfqmc_opts* opts, double* g_tau, double* g_err, double* docc,
                                hfqmc_stats* stats) {
  if (!g0_dn) return fail(HFQMC_EINVAL, "hfqmc_solve_spin: g0_dn is null");
  if (!(dtau > 0.0) || !(beta > 0.0)) return fail(HFQMC_EINVAL, "dtau=%g beta=%g", dtau, beta);
  if (std::fabs(beta / dtau - L) > 1e-9 * L) return fail(HFQMC_EINVAL, "beta/dtau=%.12g != L=%d", beta / dtau, L);
  const int32_t Ls[1] = {L};
  Call call;
  call.g0_dn = g0_dn;
  return solve_grids_impl(c, 1, Ls, g0_up, U, beta, seed, opts, g_tau, g_err, docc, stats, call);
}

extern "C" int hfqmc_solve_dev(hfqmc_ctx* c, const double* g0_tau, int32_t L, double U, double beta,
                               double dtau, uint64_t seed, const hfqmc_opts* opts, double* g_tau,
                               double* g_err, double* docc, hfqmc_stats* stats) {
  if (!(dtau > 0.0) || !(beta > 0.0)) return fail(HFQMC_EINVAL, "dtau=%g beta=%g", dtau, beta);
  if (std::fabs(beta / dtau - L) > 1e-9 * L) return fail(HFQMC_EINVAL, "beta/dtau=%.12g != L=%d", beta / dtau, L);
  const int32_t Ls[1] = {L};
  Call call;
  call.dev_io = true;
  return solve_grids_impl(c, 1, Ls, g0_tau, U, beta, seed, opts, g_tau, g_err, docc, stats, call);
}

// hfqmc_solve_dev without any allocation: every buffer besides the caller's
// inputs and outputs lives in this device's static buffer of kNoAllocBytes (the
// grid data first, then as many per-workgroup workspaces as fit), the grid
// record and the dispatch order are written by kernels, the statistics are
// summed on the device and read back as one record, and the set-up kernels run
// eagerly (no graph is instantiated).  The same kernels as hfqmc_solve_dev, so
// the results are the same bit for bit.
extern "C" int hfqmc_solve_dev_noalloc(hfqmc_ctx* c, const double* g0_tau, int32_t L, double U,
                                       double beta, double dtau, uint64_t seed,
                                       const hfqmc_opts* opts, double* g_tau, double* g_err,
                                       double* docc, hfqmc_stats* stats) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!c) return fail(HFQMC_EINVAL, "hfqmc_solve_dev_noalloc: ctx is NULL");
  if (!g0_tau || !g_tau) return fail(HFQMC_EINVAL, "hfqmc_solve_dev_noalloc: null input/output pointer");
  if (!(dtau > 0.0) || !(beta > 0.0) || !std::isfinite(beta))
    return fail(HFQMC_EINVAL, "dtau=%g beta=%g", dtau, beta);
  if (L < 2 || L > 4096) return fail(HFQMC_EINVAL, "L=%d (2..4096)", L);
  if (std::fabs(beta / dtau - L) > 1e-9 * L) return fail(HFQMC_EINVAL, "beta/dtau=%.12g != L=%d", beta / dtau, L);
  if (!(U >= 0.0) || !std::isfinite(U)) return fail(HFQMC_EINVAL, "U=%g", U);
  Resolved r;
  int rc = resolve_opts(opts, &r);
  if (rc) return rc;
  if (opts->flip_log || opts->replay_log || opts->chain_g || opts->chain_d || opts->chain_n ||
      opts->chain_drift || opts->final_green)
    return fail(HFQMC_EINVAL, "hfqmc_solve_dev_noalloc: the test hooks are not available here "
                "(their device copies would need allocations)");
  if (opts->flags & HFQMC_FLAG_BALANCE)
    return fail(HFQMC_EINVAL, "hfqmc_solve_dev_noalloc: HFQMC_FLAG_BALANCE is not available here "
                "(the buffer is sized for n_chains chains)");
  if (r.mode != MODE_RANK1 && r.delay_k == 0)
    return fail(HFQMC_EINVAL, "hfqmc_solve_dev_noalloc: delay_k must be given in the delayed "
                "modes (the autotuner's trial launches allocate)");
  if (!c->na_scratch)
    return fail(HFQMC_EDEVICE, "hfqmc_solve_dev_noalloc: no allocation-free buffer on device %d: %s",
                c->device, hipGetErrorString(c->na_status));
  HIPCHK(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  const int nch = r.n_chains, nbin = r.n_bins;
  const int direct = (opts->flags & HFQMC_FLAG_DIRECT_RECOMPUTE) ? 1 : 0;

  // ---- launch shape (as plan_lu for one grid) and the reference solves' LDS
  int nb = 0, sc = 0, pg = 0;
  int lds = lds_bytes(L, L, r.mode, 0, direct, &nb, &sc, 0);
  if (nb < 16 && !direct && !(opts->flags & HFQMC_FLAG_G_FP32)) {
    int nb1 = 0, sc1 = 0;
    const int l1 = lds_bytes(L, L, r.mode, 0, direct, &nb1, &sc1, 1);
    if (nb1 >= 16) {
      nb = nb1;
      sc = sc1;
      lds = l1;
      pg = 1;
    }
  }
  if (lds + 1024 > c->lds_max)
    return fail(HFQMC_EUNSUPPORTED, "L=%d needs %d bytes of LDS, device allows %d", L, lds, c->lds_max);
  int ref_nb = 0, ref_sc = 0, ref_lds = 0;
  if (!direct) {
    ref_lds = lds_bytes(L, L, -1, 0, 1, &ref_nb, &ref_sc);
    if (ref_lds + 1024 > c->lds_max)
      return fail(HFQMC_EUNSUPPORTED, "L=%d: reference solve needs %d bytes of LDS", L, ref_lds);
  }

  // ---- the buffer: grid data, then the per-workgroup workspaces
  GridDev g;
  std::memset(&g, 0, sizeof g);
  GridDev* d_grid = nullptr;
  int* d_units = nullptr;
  int* d_queue = nullptr;
  NoAllocSummary* d_sum = nullptr;
  double* d_gtau = nullptr;
  auto layout = [&](Bump& b) {
    d_grid = b.take<GridDev>(1);
    d_units = b.take<int>(nch);
    d_queue = b.take<int>(64);
    d_sum = b.take<NoAllocSummary>(1);
    d_gtau = b.take<double>(L);
    g.G0 = b.take<double>((size_t)L * L);
    g.G0d = g.G0;
    g.acc_g = b.take<double>((size_t)nch * nbin * (L + 1));
    g.acc_d = b.take<double>((size_t)nch * nbin);
    g.acc_n = b.take<long long>((size_t)nch * nbin);
    g.cstats = b.take<long long>((size_t)nch * NSTAT);
    g.cdrift = b.take<double>(nch);
    g.cdrift_gt = b.take<double>(nch);
    g.g_out = b.take<double>(L + 1);
    g.g_err = b.take<double>(L + 1);
    g.d_out = b.take<double>(2);
    for (int q = 0; q < 2; ++q) {
      g.refQ[q] = direct ? nullptr : b.take<double>((size_t)L * L);
      g.refH[q] = direct ? nullptr : b.take<double>((size_t)L * L);
      g.refQd[q] = g.refQ[q];
      g.refHd[q] = g.refH[q];
    }
    g.ref_sing = direct ? nullptr : b.take<int>(4);
  };
  Bump sizing(nullptr);
  layout(sizing);
  const size_t head = (sizing.off + 255) & ~(size_t)255;
  const long long wstride = workspace_doubles(L, r.mode == MODE_RANK1 ? 1 : kMaxK);
  const long long slots =
      head < kNoAllocBytes ? (long long)((kNoAllocBytes - head) / (sizeof(double) * wstride)) : 0;
  const int need = direct ? 1 : 4;   // the reference solves use workspace slots 0..3
  if (slots < need)
    return fail(HFQMC_EINVAL, "hfqmc_solve_dev_noalloc: L=%d with %d chains exceeds the "
                "allocation-free buffer of %zu bytes (grid data %zu bytes, then %d workspaces of "
                "%lld bytes needed)", L, nch, kNoAllocBytes, head, need,
                (long long)(sizeof(double) * wstride));
  Bump assign(c->na_scratch);
  layout(assign);
  double* work = reinterpret_cast<double*>(static_cast<char*>(c->na_scratch) + head);
  const int occ = std::max(1, std::min(c->lds_max / (lds + 1024), 2048 / kThreads));
  const int n_wg = (int)std::min<long long>(std::min(nch, c->n_cu * occ), slots);

  const double lam = std::acosh(std::exp(0.5 * dtau * U));
  g.L = L;
  g.n_chains = nch;
  g.grid_id = 0;
  g.unit_base = 0;
  g.sweeps = r.sweeps;
  g.lu_nb = nb;
  g.direct = direct;
  g.ref_nb = ref_nb;
  g.ref_pg = 0;
  g.gp = std::expm1(2.0 * lam);
  g.gm = std::expm1(-2.0 * lam);
  g.ep = std::expm1(lam);
  g.em = std::expm1(-lam);
  g.spin = 0;

  HIPCHK(launch_copy(g0_tau, d_gtau, L, st));
  if (opts->flags & HFQMC_FLAG_PH_SYMMETRIC) {
    // G0 = 1 - G0^T: G0(0+) = 1/2 and G0(tau) = G0(beta - tau) (the bath on the stack)
    double hb[4096];
    HIPCHK(hipMemcpyAsync(hb, d_gtau, sizeof(double) * L, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double dev = std::fabs(hb[0] - 0.5);
    for (int q = 1; q < L; ++q) dev = std::max(dev, std::fabs(hb[q] - hb[L - q]));
    if (!(dev <= 1e-9))
      return fail(HFQMC_EINVAL, "HFQMC_FLAG_PH_SYMMETRIC: the bath deviates from particle-hole "
                  "symmetry by %.3e", dev);
  }

  SweepParams p;
  std::memset(&p, 0, sizeof p);
  p.grids = d_grid;
  p.n_grids = 1;
  p.units = d_units;
  p.n_units = nch;
  p.queue = d_queue;
  p.seed = seed;
  p.warmup = r.warmup;
  p.sweeps = r.sweeps;
  p.n_rec = r.n_rec;
  p.mode = (opts->flags & HFQMC_FLAG_G_FP32) ? MODE_MIXED_G32 : r.mode;
  p.delay_k = r.delay_k;
  p.window_b = r.window_b;
  p.n_bins = nbin;
  p.lu_nb = nb;
  p.work = work;
  p.work_stride = wstride;
  p.Lmax = L;
  p.lds_scratch_bytes = sc;
  p.heat_bath = (opts->flags & HFQMC_FLAG_HEAT_BATH) ? 1 : 0;
  p.direct = direct;
  p.ph = (opts->flags & HFQMC_FLAG_PH_SYMMETRIC) ? 1 : 0;
  p.spin = 0;
  p.pg = pg;
  p.drift_every = r.drift_every;
  HIPCHK(prepare_sweeps(lds));
  if (!direct) HIPCHK(prepare_reference(ref_lds));

  // ---- the launch sequence, eager; everything this call reads starts cleared
  HIPCHK(hipEventRecord(c->ev0, st));
  HIPCHK(launch_put_grid(g, d_grid, st));
  HIPCHK(launch_iota(d_units, nch, st));
  HIPCHK(launch_build_g0(d_gtau, L, const_cast<double*>(g.G0), st));
  HIPCHK(launch_zero(g.acc_g, (long long)nch * nbin * (L + 1), st));
  HIPCHK(launch_zero(g.acc_d, (long long)nch * nbin, st));
  HIPCHK(launch_zero_i64(g.acc_n, (long long)nch * nbin, st));
  HIPCHK(launch_zero_i64(g.cstats, (long long)nch * NSTAT, st));
  HIPCHK(launch_zero(g.cdrift, nch, st));
  HIPCHK(launch_zero(g.cdrift_gt, nch, st));
  if (!direct) {
    HIPCHK(launch_zero_i32(g.ref_sing, 4, st));
    HIPCHK(launch_reference(p, ref_lds, ref_sc, 0, st));
  }
  HIPCHK(launch_zero_i32(d_queue, 64, st));
  HIPCHK(hipEventRecord(c->ev_k0, st));
  {
    const hipError_t e = launch_sweeps(p, n_wg, lds, st);
    if (e != hipSuccess)
      return fail(HFQMC_EDEVICE, "sweep kernel (%d workgroups, %d B LDS): %s", n_wg, lds,
                  hipGetErrorString(e));
  }
  HIPCHK(hipEventRecord(c->ev_k1, st));
  HIPCHK(launch_reduce(d_grid, 1, nbin, st));
  HIPCHK(hipEventRecord(c->ev1, st));
  HIPCHK(launch_noalloc_summary(d_grid, d_sum, st));
  HIPCHK(launch_copy(g.g_out, g_tau, L + 1, st));
  if (g_err) HIPCHK(launch_copy(g.g_err, g_err, L + 1, st));
  if (docc) HIPCHK(launch_copy(g.d_out, docc, 2, st));
  NoAllocSummary hs;
  HIPCHK(hipMemcpyAsync(&hs, d_sum, sizeof hs, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));

  float ms = 0.f, ms_k = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  HIPCHK(hipEventElapsedTime(&ms_k, c->ev_k0, c->ev_k1));
  if (stats) {
    hfqmc_stats tot;
    std::memset(&tot, 0, sizeof tot);
    add_counters(hs.stats, c->wall_hz, &tot);
    tot.max_drift = hs.max_drift;
    tot.max_drift_gtau = hs.max_drift_gtau;
    tot.acc_rate = tot.n_proposed ? (double)tot.n_accepted / tot.n_proposed : 0.0;
    tot.seconds_kernel = ms * 1e-3;
    tot.seconds_sweep_kernel = ms_k * 1e-3;
    tot.seconds_total =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    tot.delay_k = r.delay_k;
    tot.recompute_every = r.n_rec;
    tot.n_workgroups = n_wg;
    tot.lu_panel = nb;
    tot.graph = 0;
    tot.autotuned = 0;
    tot.seconds_autotune = 0.0;
    tot.recompute_reduced = direct ? 0 : 1;
    *stats = tot;
  }
  if (hs.ref_singular) return fail(HFQMC_ENUMERIC, "singular uniform-field reference matrix");
  if (hs.stats[ST_SINGULAR])
    return fail(HFQMC_ENUMERIC, "singular Dyson matrix in %lld recomputes", hs.stats[ST_SINGULAR]);
  if (hs.nonfinite || !(hs.max_drift < INFINITY) || !(hs.max_drift_gtau < INFINITY))
    return fail(HFQMC_ENUMERIC, "non-finite Green function");
  if (opts->drift_limit > 0 && std::max(hs.max_drift, hs.max_drift_gtau) > opts->drift_limit)
    return fail(HFQMC_EDRIFT, "recompute drift %.3e (G(tau): %.3e) exceeds limit %.3e",
                hs.max_drift, hs.max_drift_gtau, opts->drift_limit);
  return HFQMC_OK;
}

extern "C" int hfqmc_measure_peaks(hfqmc_ctx* c, hfqmc_peaks* out) {
  if (!c || !out) return fail(HFQMC_EINVAL, "hfqmc_measure_peaks: NULL argument");
  HIPCHK(hipSetDevice(c->device));
  std::memset(out, 0, sizeof *out);
  // streams: 1 GiB each way (four times the last-level cache); arithmetic:
  // 4 workgroups of 8 waves per compute unit
  const long long n16 = (1LL << 30) / 16;
  const int sblocks = c->n_cu * 8;
  const int ablocks = c->n_cu * 4;
  const int nthr = peak_threads();
  const size_t out_bytes = (size_t)std::max(sblocks, ablocks) * nthr * sizeof(double);
  DevBuf buf;
  if (int e = buf.ensure(2 * n16 * 16 + out_bytes)) return e;
  char* src = (char*)buf.p;
  char* dst = src + n16 * 16;
  double* o = (double*)(dst + n16 * 16);
  hipStream_t s = c->stream;
  hipError_t he = launch_zero((double*)src, 4 * n16, s);   // defined values in both buffers
  auto best_ms = [&](int kind, int blocks, int iters, float* ms) -> hipError_t {
    *ms = 1e30f;
    for (int rep = 0; rep < 4 && he == hipSuccess; ++rep) {   // first launch warms up
      he = hipEventRecord(c->ev0, s);
      if (he == hipSuccess) he = launch_peak(kind, src, dst, n16, blocks, iters, o, s);
      if (he == hipSuccess) he = hipEventRecord(c->ev1, s);
      if (he == hipSuccess) he = hipEventSynchronize(c->ev1);
      float t = 0.f;
      if (he == hipSuccess) he = hipEventElapsedTime(&t, c->ev0, c->ev1);
      if (he == hipSuccess && rep > 0 && t < *ms) *ms = t;
    }
    return he;
  };
  float ms = 0.f;
  const int it64 = 4096, it32 = 8192, itv = 16384;
  if (best_ms(PEAK_COPY, sblocks, 0, &ms) == hipSuccess) out->hbm_copy_gbs = 2.0 * n16 * 16 / (ms * 1e-3) / 1e9;
  if (best_ms(PEAK_READ, sblocks, 0, &ms) == hipSuccess) out->hbm_read_gbs = 1.0 * n16 * 16 / (ms * 1e-3) / 1e9;
  if (best_ms(PEAK_MFMA64, ablocks, it64, &ms) == hipSuccess)
    out->fp64_mfma_tflops = peak_flops(PEAK_MFMA64, ablocks, it64) / (ms * 1e-3) / 1e12;
  if (best_ms(PEAK_MFMA32, ablocks, it32, &ms) == hipSuccess)
    out->fp32_mfma_tflops = peak_flops(PEAK_MFMA32, ablocks, it32) / (ms * 1e-3) / 1e12;
  if (best_ms(PEAK_FMA64, ablocks, itv, &ms) == hipSuccess)
    out->fp64_fma_tflops = peak_flops(PEAK_FMA64, ablocks, itv) / (ms * 1e-3) / 1e12;
  const hipError_t se = hipStreamSynchronize(s);
  buf.release();
  if (he != hipSuccess) return fail(HFQMC_EDEVICE, "peak probe: %s", hipGetErrorString(he));
  if (se != hipSuccess) return fail(HFQMC_EDEVICE, "peak probe: %s", hipGetErrorString(se));
  return HFQMC_OK;
}

extern "C" int hfqmc_uniforms(hfqmc_ctx* c, uint64_t seed, int32_t chain, int32_t grid,
                              int64_t sweep0, int64_t n_sweeps, int32_t L, int32_t stream,
                              double* out) {
  if (!c || !out) return fail(HFQMC_EINVAL, "hfqmc_uniforms: NULL argument");
  if (chain < 0 || grid < 0 || sweep0 < 0 || n_sweeps < 1 || L < 1 || stream < 0 || stream > 1)
    return fail(HFQMC_EINVAL, "hfqmc_uniforms: chain=%d grid=%d sweep0=%lld n_sweeps=%lld L=%d stream=%d",
                chain, grid, (long long)sweep0, (long long)n_sweeps, L, stream);
  const long long n = (long long)n_sweeps * L;
  if (n > (1LL << 28)) return fail(HFQMC_EINVAL, "hfqmc_uniforms: %lld values (at most 2^28)", n);
  HIPCHK(hipSetDevice(c->device));
  DevBuf buf;
  if (int e = buf.ensure(sizeof(double) * n)) return e;
  hipStream_t s = c->stream;
  hipError_t he = launch_uniforms(seed + (uint64_t)chain, (uint64_t)grid, sweep0, n_sweeps, L,
                                  (uint64_t)stream, (double*)buf.p, s);
  if (he == hipSuccess) he = hipMemcpyAsync(out, buf.p, sizeof(double) * n, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  buf.release();
  if (he != hipSuccess) return fail(HFQMC_EDEVICE, "hfqmc_uniforms: %s", hipGetErrorString(he));
  return HFQMC_OK;
}

extern "C" int hfqmc_solve_grids(hfqmc_ctx* c, int32_t n_grids, const int32_t* L,
                                 const double* g0_tau, double U, double beta, uint64_t seed,
                                 const hfqmc_opts* opts, double* g_tau, double* g_err,
                                 double* docc, hfqmc_stats* stats) {
  return solve_grids_impl(c, n_grids, L, g0_tau, U, beta, seed, opts, g_tau, g_err, docc, stats, Call());
}

extern "C" int hfqmc_plan_balance(int32_t n_grids, const int32_t* L, int32_t n_chains,
                                  int64_t warmup, int64_t sweeps, int32_t n_bins,
                                  int32_t n_workgroups, int32_t* factor, double* span) {
  if (n_grids < 1 || !L || !factor) return fail(HFQMC_EINVAL, "n_grids=%d, null L or factor", n_grids);
  if (n_chains < 1 || n_chains >= (1 << 20)) return fail(HFQMC_EINVAL, "n_chains=%d", n_chains);
  if (warmup < 0 || sweeps < 1) return fail(HFQMC_EINVAL, "warmup=%lld sweeps=%lld",
                                            (long long)warmup, (long long)sweeps);
  if (n_bins < 1 || n_bins > sweeps) return fail(HFQMC_EINVAL, "n_bins=%d", n_bins);
  if (n_workgroups < 1) return fail(HFQMC_EINVAL, "n_workgroups=%d", n_workgroups);
  for (int i = 0; i < n_grids; ++i)
    if (L[i] < 2 || L[i] > 4096) return fail(HFQMC_EINVAL, "L[%d]=%d (2..4096)", i, L[i]);
  std::vector<int> f(n_grids);
  double s0 = 0.0, s1 = 0.0;
  plan_chain_split(n_grids, L, n_chains, warmup, sweeps, n_bins, n_workgroups, f.data(), &s0, &s1);
  for (int i = 0; i < n_grids; ++i) factor[i] = f[i];
  if (span) {
    span[0] = s0;
    span[1] = s1;
  }
  return HFQMC_OK;
}

extern "C" int bethe_semicircle_bath(double beta, double t, int32_t n_iw, double* bath_iw) {
  if (!bath_iw || !(beta > 0) || !(t > 0) || n_iw < 1) return fail(HFQMC_EINVAL, "bethe_semicircle_bath: bad argument");
  host::semicircle(beta, t, n_iw, bath_iw);
  return HFQMC_OK;
}

extern "C" int bethe_atomic_bath(double beta, double t, double U, int32_t n_iw, double* bath_iw) {
  if (!bath_iw || !(beta > 0) || !(t > 0) || !(U >= 0) || n_iw < 1)
    return fail(HFQMC_EINVAL, "bethe_atomic_bath: bad argument");
  host::atomic_seed(beta, t, U, n_iw, bath_iw);
  return HFQMC_OK;
}

extern "C" int bath_to_tau(const double* bath_iw, int32_t n_iw, double m3, double beta, int32_t L,
                           double* g_tau) {
  if (!bath_iw || !g_tau || n_iw < 16 || L < 2 || !(beta > 0)) return fail(HFQMC_EINVAL, "bath_to_tau: bad argument");
  std::vector<double> tau(L);
  for (int k = 0; k < L; ++k) tau[k] = k * (beta / L);
  host::iw_to_tau(bath_iw, n_iw, m3, beta, tau.data(), L, g_tau);
  return HFQMC_OK;
}

extern "C" int multigrid_solve(hfqmc_ctx* c, const double* bath_iw, int32_t n_iw, double bath_m3,
                               double U, double beta, const double* dtaus, int32_t n_grids,
                               uint64_t seed, const hfqmc_opts* opts, int32_t n_fine,
                               double* g_fine, double* g_fine_err, double* g_grids,
                               hfqmc_stats* per_grid, double* docc_grids, double* docc) {
  if (!bath_iw || !dtaus || !g_fine) return fail(HFQMC_EINVAL, "multigrid_solve: null pointer");
  if (n_grids < 3) return fail(HFQMC_EINVAL, "multigrid_solve: n_grids=%d < 3", n_grids);
  if (n_fine < 4) return fail(HFQMC_EINVAL, "multigrid_solve: n_fine=%d < 4", n_fine);
  if (n_iw < 16) return fail(HFQMC_EINVAL, "multigrid_solve: n_iw=%d < 16", n_iw);
  if (!(beta > 0) || !(U >= 0)) return fail(HFQMC_EINVAL, "multigrid_solve: U=%g beta=%g", U, beta);
  std::vector<int32_t> Ls(n_grids);
  std::vector<double> dts(n_grids);
  long long Lsum = 0, Psum = 0;
  for (int i = 0; i < n_grids; ++i) {
    if (!(dtaus[i] > 0)) return fail(HFQMC_EINVAL, "dtau[%d]=%g", i, dtaus[i]);
    Ls[i] = (int32_t)std::lround(beta / dtaus[i]);
    dts[i] = beta / Ls[i];
    Lsum += Ls[i];
    Psum += Ls[i] + 1;
  }
  std::vector<double> g0(Lsum), gg(Psum), ge(Psum), dd(2 * (size_t)n_grids);
  long long off = 0;
  for (int i = 0; i < n_grids; ++i) {
    int rc = bath_to_tau(bath_iw, n_iw, bath_m3, beta, Ls[i], g0.data() + off);
    if (rc) return rc;
    off += Ls[i];
  }
  int rc = solve_grids_impl(c, n_grids, Ls.data(), g0.data(), U, beta, seed, opts, gg.data(),
                            ge.data(), dd.data(), per_grid, Call());
  if (rc) return rc;
  // (i) interpolation onto the fine grid with the reference model
  std::vector<double> tf(n_fine), gref_f(n_fine);
  for (int j = 0; j < n_fine; ++j) tf[j] = j * (beta / (n_fine - 1));
  host::reference_tau(bath_iw, n_iw, bath_m3, U, beta, tf.data(), n_fine, gref_f.data());
  std::vector<double> gi((size_t)n_grids * n_fine), ei((size_t)n_grids * n_fine);
  off = 0;
  for (int i = 0; i < n_grids; ++i) {
    const int L = Ls[i];
    std::vector<double> tk(L + 1), gref_k(L + 1), d(L + 1);
    for (int k = 0; k <= L; ++k) tk[k] = k * (beta / L);
    host::reference_tau(bath_iw, n_iw, bath_m3, U, beta, tk.data(), L + 1, gref_k.data());
    for (int k = 0; k <= L; ++k) d[k] = gg[off + k] - gref_k[k];
    host::Spline sp(tk.data(), d.data(), L + 1);
    for (int j = 0; j < n_fine; ++j) {
      gi[(size_t)i * n_fine + j] = gref_f[j] + sp(tf[j]);
      // linear interpolation of the error bars
      const double x = tf[j] / (beta / L);
      int k0 = (int)std::floor(x);
      if (k0 < 0) k0 = 0;
      if (k0 > L - 1) k0 = L - 1;
      const double fr = x - k0;
      ei[(size_t)i * n_fine + j] = ge[off + k0] * (1.0 - fr) + ge[off + k0 + 1] * fr;
    }
    off += L + 1;
  }
  // (ii) quadratic-in-dtau^2 least squares per fine point
  std::vector<double> err(n_fine);
  host::extrapolate(dts.data(), n_grids, gi.data(), ei.data(), n_fine, g_fine, err.data());
  if (g_fine_err) std::memcpy(g_fine_err, err.data(), sizeof(double) * n_fine);
  if (g_grids) std::memcpy(g_grids, gg.data(), sizeof(double) * Psum);
  // the double occupancy of each grid and its dtau -> 0 extrapolation
  if (docc_grids) std::memcpy(docc_grids, dd.data(), sizeof(double) * 2 * n_grids);
  if (docc) {
    std::vector<double> dv(n_grids), de(n_grids);
    for (int i = 0; i < n_grids; ++i) {
      dv[i] = dd[2 * i];
      de[i] = dd[2 * i + 1];
    }
    host::extrapolate(dts.data(), n_grids, dv.data(), de.data(), 1, &docc[0], &docc[1]);
  }
  return HFQMC_OK;
}

extern "C" int dmft_bethe_step(const double* g_fine, int32_t n_fine, const double* bath_iw_prev,
                               int32_t n_iw, double bath_m3, double U, double beta, double t,
                               double* bath_iw_new) {
  if (!g_fine || !bath_iw_prev || !bath_iw_new) return fail(HFQMC_EINVAL, "dmft_bethe_step: null pointer");
  if (n_fine < 4 || n_iw < 16 || !(beta > 0) || !(t > 0) || !(U >= 0))
    return fail(HFQMC_EINVAL, "dmft_bethe_step: bad size or parameter");
  for (int j = 0; j < n_fine; ++j)
    if (!std::isfinite(g_fine[j])) return fail(HFQMC_EINVAL, "dmft_bethe_step: g_fine[%d] not finite", j);
  return host::bethe_step(g_fine, n_fine, bath_iw_prev, n_iw, bath_m3, U, beta, t, bath_iw_new);
}

extern "C" int dmft_solve(hfqmc_ctx* c, double U, double beta, double t, const double* dtaus,
                          int32_t n_grids, uint64_t seed, const hfqmc_opts* opts, int32_t n_fine,
                          int32_t n_iw, int32_t n_iter, double mixing, double* bath_iw,
                          double* g_fine, double* g_fine_err, double* history) {
  if (!bath_iw || !g_fine || !dtaus || !opts) return fail(HFQMC_EINVAL, "dmft_solve: null pointer");
  if (n_iter < 1) return fail(HFQMC_EINVAL, "dmft_solve: n_iter=%d", n_iter);
  if (!(mixing >= 0.0 && mixing < 1.0)) return fail(HFQMC_EINVAL, "dmft_solve: mixing=%g", mixing);
  if (!(t > 0)) return fail(HFQMC_EINVAL, "dmft_solve: t=%g", t);
  if (n_fine < 4 || n_iw < 16) return fail(HFQMC_EINVAL, "dmft_solve: n_fine=%d n_iw=%d", n_fine, n_iw);
  // the Bethe closure keeps the bath's 1/(i w)^3 moment at t^2
  const double m3 = t * t;
  std::vector<double> prev(n_fine), err(n_fine), nb(2 * (size_t)n_iw);
  {
    // distance of the first iteration: to the input bath's own G0(tau_j)
    std::vector<double> tf(n_fine);
    for (int j = 0; j < n_fine; ++j) tf[j] = j * (beta / (n_fine - 1));
    host::reference_tau(bath_iw, n_iw, m3, 0.0, beta, tf.data(), n_fine, prev.data());
  }
  for (int it = 0; it < n_iter; ++it) {
    // independent Philox streams per iteration: the seed moves by 2^32 (chain keys
    // are seed + chain with fewer than 2^20 chains)
    const uint64_t s_it = seed + ((uint64_t)it << 32);
    double dx[2] = {0.0, 0.0};
    int rc = multigrid_solve(c, bath_iw, n_iw, m3, U, beta, dtaus, n_grids, s_it, opts, n_fine,
                             g_fine, err.data(), nullptr, nullptr, nullptr, dx);
    if (rc) return rc;
    double dmax = 0.0, emax = 0.0;
    for (int j = 0; j < n_fine; ++j) {
      dmax = std::max(dmax, std::fabs(g_fine[j] - prev[j]));
      emax = std::max(emax, err[j]);
      prev[j] = g_fine[j];
    }
    if (history) {
      history[4 * it] = dmax;
      history[4 * it + 1] = emax;
      history[4 * it + 2] = dx[0];
      history[4 * it + 3] = dx[1];
    }
    rc = host::bethe_step(g_fine, n_fine, bath_iw, n_iw, m3, U, beta, t, nb.data());
    if (rc) return fail(rc, "dmft_solve: Bethe step failed in iteration %d", it);
    if (opts->flags & HFQMC_FLAG_PH_SYMMETRIC) {
      // a symmetric G(tau) transforms to a purely imaginary G(i w); the rounding
      // left in the real part is magnified by an insulating bath's pole near
      // zero frequency, so it is dropped
      for (int n = 0; n < n_iw; ++n) nb[2 * n] = 0.0;
    }
    for (size_t q = 0; q < nb.size(); ++q) bath_iw[q] = mixing * bath_iw[q] + (1.0 - mixing) * nb[q];
  }
  if (g_fine_err) std::memcpy(g_fine_err, err.data(), sizeof(double) * n_fine);
  return HFQMC_OK;
}

extern "C" int bethe_lattice_bath(double beta, double t, double mu, int32_t n_iw, double* bath_iw) {
  if (!bath_iw || !(beta > 0) || !(t > 0) || !std::isfinite(mu) || n_iw < 1)
    return fail(HFQMC_EINVAL, "bethe_lattice_bath: bad argument");
  host::bethe_lattice(beta, t, mu, n_iw, bath_iw);
  return HFQMC_OK;
}

extern "C" int bath_to_tau_m2(const double* bath_iw, int32_t n_iw, double m2, double m3,
                              double beta, int32_t L, double* g_tau) {
  if (!bath_iw || !g_tau || n_iw < 16 || L < 2 || !(beta > 0) || !std::isfinite(m2) ||
      !std::isfinite(m3))
    return fail(HFQMC_EINVAL, "bath_to_tau_m2: bad argument");
  std::vector<double> tau(L);
  for (int k = 0; k < L; ++k) tau[k] = k * (beta / L);
  host::iw_to_tau(bath_iw, n_iw, m3, beta, tau.data(), L, g_tau, m2);
  return HFQMC_OK;
}

// The multigrid step at any filling: the bath's tail moments m2, m3 enter its
// transform onto every grid, and the reference model of step (i) is taken at
// the finest grid's density n = G(beta-).
extern "C" int multigrid_solve_n(hfqmc_ctx* c, const double* bath_iw, int32_t n_iw, double m2,
                                 double m3, double U, double beta, const double* dtaus,
                                 int32_t n_grids, uint64_t seed, const hfqmc_opts* opts,
                                 int32_t n_fine, double* g_fine, double* g_fine_err, double* docc,
                                 double* n_ref) {
  if (!bath_iw || !dtaus || !g_fine) return fail(HFQMC_EINVAL, "multigrid_solve_n: null pointer");
  if (n_grids < 3) return fail(HFQMC_EINVAL, "multigrid_solve_n: n_grids=%d < 3", n_grids);
  if (n_fine < 4) return fail(HFQMC_EINVAL, "multigrid_solve_n: n_fine=%d < 4", n_fine);
  if (n_iw < 16) return fail(HFQMC_EINVAL, "multigrid_solve_n: n_iw=%d < 16", n_iw);
  if (!(beta > 0) || !(U >= 0) || !std::isfinite(m2) || !std::isfinite(m3))
    return fail(HFQMC_EINVAL, "multigrid_solve_n: U=%g beta=%g m2=%g m3=%g", U, beta, m2, m3);
  if (opts && (opts->flags & HFQMC_FLAG_PH_SYMMETRIC))
    return fail(HFQMC_EINVAL, "multigrid_solve_n: HFQMC_FLAG_PH_SYMMETRIC needs half filling");
  std::vector<int32_t> Ls(n_grids);
  std::vector<double> dts(n_grids);
  long long Lsum = 0, Psum = 0;
  int finest = 0;
  for (int i = 0; i < n_grids; ++i) {
    if (!(dtaus[i] > 0)) return fail(HFQMC_EINVAL, "dtau[%d]=%g", i, dtaus[i]);
    Ls[i] = (int32_t)std::lround(beta / dtaus[i]);
    dts[i] = beta / Ls[i];
    Lsum += Ls[i];
    Psum += Ls[i] + 1;
    if (Ls[i] > Ls[finest]) finest = i;
  }
  std::vector<double> g0(Lsum), gg(Psum), ge(Psum), dd(2 * (size_t)n_grids);
  long long off = 0;
  for (int i = 0; i < n_grids; ++i) {
    int rc = bath_to_tau_m2(bath_iw, n_iw, m2, m3, beta, Ls[i], g0.data() + off);
    if (rc) return rc;
    off += Ls[i];
  }
  int rc = solve_grids_impl(c, n_grids, Ls.data(), g0.data(), U, beta, seed, opts, gg.data(),
                            ge.data(), dd.data(), nullptr, Call());
  if (rc) return rc;
  off = 0;
  long long off_finest = 0;
  for (int i = 0; i < n_grids; ++i) {
    if (i == finest) off_finest = off;
    off += Ls[i] + 1;
  }
  const double n = gg[off_finest + Ls[finest]];   // G(beta-) of the finest grid
  std::vector<double> tf(n_fine), gref_f(n_fine);
  for (int j = 0; j < n_fine; ++j) tf[j] = j * (beta / (n_fine - 1));
  host::reference_tau_n(bath_iw, n_iw, m2, m3, U, beta, n, tf.data(), n_fine, gref_f.data());
  std::vector<double> gi((size_t)n_grids * n_fine), ei((size_t)n_grids * n_fine);
  off = 0;
  for (int i = 0; i < n_grids; ++i) {
    const int L = Ls[i];
    std::vector<double> tk(L + 1), gref_k(L + 1), d(L + 1);
    for (int k = 0; k <= L; ++k) tk[k] = k * (beta / L);
    host::reference_tau_n(bath_iw, n_iw, m2, m3, U, beta, n, tk.data(), L + 1, gref_k.data());
    for (int k = 0; k <= L; ++k) d[k] = gg[off + k] - gref_k[k];
    host::Spline sp(tk.data(), d.data(), L + 1);
    for (int j = 0; j < n_fine; ++j) {
      gi[(size_t)i * n_fine + j] = gref_f[j] + sp(tf[j]);
      const double x = tf[j] / (beta / L);
      int k0 = (int)std::floor(x);
      if (k0 < 0) k0 = 0;
      if (k0 > L - 1) k0 = L - 1;
      const double fr = x - k0;
      ei[(size_t)i * n_fine + j] = ge[off + k0] * (1.0 - fr) + ge[off + k0 + 1] * fr;
    }
    off += L + 1;
  }
  std::vector<double> err(n_fine);
  host::extrapolate(dts.data(), n_grids, gi.data(), ei.data(), n_fine, g_fine, err.data());
  if (g_fine_err) std::memcpy(g_fine_err, err.data(), sizeof(double) * n_fine);
  if (docc) {
    std::vector<double> dv(n_grids), de(n_grids);
    for (int i = 0; i < n_grids; ++i) {
      dv[i] = dd[2 * i];
      de[i] = dd[2 * i + 1];
    }
    host::extrapolate(dts.data(), n_grids, dv.data(), de.data(), 1, &docc[0], &docc[1]);
  }
  if (n_ref) *n_ref = n;
  return HFQMC_OK;
}

extern "C" int dmft_bethe_step_mu(const double* g_fine, int32_t n_fine, const double* bath_iw_prev,
                                  int32_t n_iw, double m2, double m3, double U, double beta,
                                  double t, double mu, double* bath_iw_new) {
  if (!g_fine || !bath_iw_prev || !bath_iw_new) return fail(HFQMC_EINVAL, "dmft_bethe_step_mu: null pointer");
  if (n_fine < 4 || n_iw < 16 || !(beta > 0) || !(t > 0) || !(U >= 0) || !std::isfinite(mu))
    return fail(HFQMC_EINVAL, "dmft_bethe_step_mu: bad size or parameter");
  for (int j = 0; j < n_fine; ++j)
    if (!std::isfinite(g_fine[j])) return fail(HFQMC_EINVAL, "dmft_bethe_step_mu: g_fine[%d] not finite", j);
  return host::bethe_step_n(g_fine, n_fine, bath_iw_prev, n_iw, m2, m3, U, beta, t, mu, bath_iw_new);
}

extern "C" int dmft_solve_mu(hfqmc_ctx* c, double U, double mu, double beta, double t,
                             const double* dtaus, int32_t n_grids, uint64_t seed,
                             const hfqmc_opts* opts, int32_t n_fine, int32_t n_iw, int32_t n_iter,
                             double mixing, double* bath_iw, double* g_fine, double* g_fine_err,
                             double* history) {
  if (!bath_iw || !g_fine || !dtaus || !opts) return fail(HFQMC_EINVAL, "dmft_solve_mu: null pointer");
  if (n_iter < 1) return fail(HFQMC_EINVAL, "dmft_solve_mu: n_iter=%d", n_iter);
  if (!(mixing >= 0.0 && mixing < 1.0)) return fail(HFQMC_EINVAL, "dmft_solve_mu: mixing=%g", mixing);
  if (!(t > 0) || !std::isfinite(mu)) return fail(HFQMC_EINVAL, "dmft_solve_mu: t=%g mu=%g", t, mu);
  if (n_fine < 4 || n_iw < 16) return fail(HFQMC_EINVAL, "dmft_solve_mu: n_fine=%d n_iw=%d", n_fine, n_iw);
  // the closure at mu keeps the bath's tail moments at -mu and mu^2 + t^2
  const double m2 = -mu, m3 = mu * mu + t * t;
  std::vector<double> prev(n_fine), err(n_fine), nb(2 * (size_t)n_iw);
  {
    std::vector<double> tf(n_fine);
    for (int j = 0; j < n_fine; ++j) tf[j] = j * (beta / (n_fine - 1));
    host::reference_tau_n(bath_iw, n_iw, m2, m3, 0.0, beta, 0.5, tf.data(), n_fine, prev.data());
  }
  for (int it = 0; it < n_iter; ++it) {
    const uint64_t s_it = seed + ((uint64_t)it << 32);
    double dx[2] = {0.0, 0.0};
    int rc = multigrid_solve_n(c, bath_iw, n_iw, m2, m3, U, beta, dtaus, n_grids, s_it, opts, n_fine,
                               g_fine, err.data(), dx, nullptr);
    if (rc) return rc;
    double dmax = 0.0, emax = 0.0;
    for (int j = 0; j < n_fine; ++j) {
      dmax = std::max(dmax, std::fabs(g_fine[j] - prev[j]));
      emax = std::max(emax, err[j]);
      prev[j] = g_fine[j];
    }
    if (history) {
      history[5 * it] = dmax;
      history[5 * it + 1] = emax;
      history[5 * it + 2] = dx[0];
      history[5 * it + 3] = dx[1];
      history[5 * it + 4] = g_fine[n_fine - 1];   // n = G(beta-)
    }
    rc = host::bethe_step_n(g_fine, n_fine, bath_iw, n_iw, m2, m3, U, beta, t, mu, nb.data());
    if (rc) return fail(rc, "dmft_solve_mu: Bethe step failed in iteration %d", it);
    for (size_t q = 0; q < nb.size(); ++q) bath_iw[q] = mixing * bath_iw[q] + (1.0 - mixing) * nb[q];
  }
  if (g_fine_err) std::memcpy(g_fine_err, err.data(), sizeof(double) * n_fine);
  return HFQMC_OK;
}

// The multigrid step with spin-dependent baths: one batched spin-resolved
// launch over the grids, then for each spin the reference-model spline onto
// the fine grid (that spin's bath in the reference) and the extrapolation.
extern "C" int multigrid_solve_spin(hfqmc_ctx* c, const double* bath_up, const double* bath_dn,
                                    int32_t n_iw, double bath_m3, double U, double beta,
                                    const double* dtaus, int32_t n_grids, uint64_t seed,
                                    const hfqmc_opts* opts, int32_t n_fine, double* g_fine,
                                    double* g_fine_err, double* docc) {
  if (!bath_up || !bath_dn || !dtaus || !g_fine)
    return fail(HFQMC_EINVAL, "multigrid_solve_spin: null pointer");
  if (n_grids < 3) return fail(HFQMC_EINVAL, "multigrid_solve_spin: n_grids=%d < 3", n_grids);
  if (n_fine < 4) return fail(HFQMC_EINVAL, "multigrid_solve_spin: n_fine=%d < 4", n_fine);
  if (n_iw < 16) return fail(HFQMC_EINVAL, "multigrid_solve_spin: n_iw=%d < 16", n_iw);
  if (!(beta > 0) || !(U >= 0)) return fail(HFQMC_EINVAL, "multigrid_solve_spin: U=%g beta=%g", U, beta);
  std::vector<int32_t> Ls(n_grids);
  std::vector<double> dts(n_grids);
  long long Lsum = 0, Psum = 0;
  for (int i = 0; i < n_grids; ++i) {
    if (!(dtaus[i] > 0)) return fail(HFQMC_EINVAL, "dtau[%d]=%g", i, dtaus[i]);
    Ls[i] = (int32_t)std::lround(beta / dtaus[i]);
    dts[i] = beta / Ls[i];
    Lsum += Ls[i];
    Psum += 2 * (Ls[i] + 1);
  }
  const double* baths[2] = {bath_up, bath_dn};
  std::vector<double> g0u(Lsum), g0d(Lsum), gg(Psum), ge(Psum), dd(2 * (size_t)n_grids);
  long long off = 0;
  for (int i = 0; i < n_grids; ++i) {
    int rc = bath_to_tau(bath_up, n_iw, bath_m3, beta, Ls[i], g0u.data() + off);
    if (!rc) rc = bath_to_tau(bath_dn, n_iw, bath_m3, beta, Ls[i], g0d.data() + off);
    if (rc) return rc;
    off += Ls[i];
  }
  Call call;
  call.g0_dn = g0d.data();
  int rc = solve_grids_impl(c, n_grids, Ls.data(), g0u.data(), U, beta, seed, opts, gg.data(),
                            ge.data(), dd.data(), nullptr, call);
  if (rc) return rc;
  std::vector<double> tf(n_fine), gref_f(n_fine);
  for (int j = 0; j < n_fine; ++j) tf[j] = j * (beta / (n_fine - 1));
  for (int sp = 0; sp < 2; ++sp) {
    host::reference_tau(baths[sp], n_iw, bath_m3, U, beta, tf.data(), n_fine, gref_f.data());
    std::vector<double> gi((size_t)n_grids * n_fine), ei((size_t)n_grids * n_fine);
    off = 0;
    for (int i = 0; i < n_grids; ++i) {
      const int L = Ls[i];
      const long long o = off + (long long)sp * (L + 1);   // [grid][spin][L+1]
      std::vector<double> tk(L + 1), gref_k(L + 1), d(L + 1);
      for (int k = 0; k <= L; ++k) tk[k] = k * (beta / L);
      host::reference_tau(baths[sp], n_iw, bath_m3, U, beta, tk.data(), L + 1, gref_k.data());
      for (int k = 0; k <= L; ++k) d[k] = gg[o + k] - gref_k[k];
      host::Spline spl(tk.data(), d.data(), L + 1);
      for (int j = 0; j < n_fine; ++j) {
        gi[(size_t)i * n_fine + j] = gref_f[j] + spl(tf[j]);
        const double x = tf[j] / (beta / L);
        int k0 = (int)std::floor(x);
        if (k0 < 0) k0 = 0;
        if (k0 > L - 1) k0 = L - 1;
        const double fr = x - k0;
        ei[(size_t)i * n_fine + j] = ge[o + k0] * (1.0 - fr) + ge[o + k0 + 1] * fr;
      }
      off += 2 * (L + 1);
    }
    std::vector<double> err(n_fine);
    host::extrapolate(dts.data(), n_grids, gi.data(), ei.data(), n_fine, g_fine + (size_t)sp * n_fine,
                      err.data());
    if (g_fine_err) std::memcpy(g_fine_err + (size_t)sp * n_fine, err.data(), sizeof(double) * n_fine);
  }
  if (docc) {
    std::vector<double> dv(n_grids), de(n_grids);
    for (int i = 0; i < n_grids; ++i) {
      dv[i] = dd[2 * i];
      de[i] = dd[2 * i + 1];
    }
    host::extrapolate(dts.data(), n_grids, dv.data(), de.data(), 1, &docc[0], &docc[1]);
  }
  return HFQMC_OK;
}

extern "C" int dmft_solve_af(hfqmc_ctx* c, double U, double beta, double t, const double* dtaus,
                             int32_t n_grids, uint64_t seed, const hfqmc_opts* opts, int32_t n_fine,
                             int32_t n_iw, int32_t n_iter, double mixing, double* bath_up,
                             double* bath_dn, double* g_fine, double* g_fine_err,
                             double* history) {
  if (!bath_up || !bath_dn || !g_fine || !dtaus || !opts)
    return fail(HFQMC_EINVAL, "dmft_solve_af: null pointer");
  if (n_iter < 1) return fail(HFQMC_EINVAL, "dmft_solve_af: n_iter=%d", n_iter);
  if (!(mixing >= 0.0 && mixing < 1.0)) return fail(HFQMC_EINVAL, "dmft_solve_af: mixing=%g", mixing);
  if (!(t > 0)) return fail(HFQMC_EINVAL, "dmft_solve_af: t=%g", t);
  if (n_fine < 4 || n_iw < 16) return fail(HFQMC_EINVAL, "dmft_solve_af: n_fine=%d n_iw=%d", n_fine, n_iw);
  const double m3 = t * t;
  std::vector<double> prev(2 * (size_t)n_fine), err(2 * (size_t)n_fine);
  std::vector<double> nb_up(2 * (size_t)n_iw), nb_dn(2 * (size_t)n_iw);
  {
    std::vector<double> tf(n_fine);
    for (int j = 0; j < n_fine; ++j) tf[j] = j * (beta / (n_fine - 1));
    host::reference_tau(bath_up, n_iw, m3, 0.0, beta, tf.data(), n_fine, prev.data());
    host::reference_tau(bath_dn, n_iw, m3, 0.0, beta, tf.data(), n_fine, prev.data() + n_fine);
  }
  for (int it = 0; it < n_iter; ++it) {
    const uint64_t s_it = seed + ((uint64_t)it << 32);
    double dx[2] = {0.0, 0.0};
    int rc = multigrid_solve_spin(c, bath_up, bath_dn, n_iw, m3, U, beta, dtaus, n_grids, s_it, opts,
                                  n_fine, g_fine, err.data(), dx);
    if (rc) return rc;
    double dmax = 0.0, emax = 0.0;
    for (size_t j = 0; j < 2 * (size_t)n_fine; ++j) {
      dmax = std::max(dmax, std::fabs(g_fine[j] - prev[j]));
      emax = std::max(emax, err[j]);
      prev[j] = g_fine[j];
    }
    if (history) {
      history[5 * it] = dmax;
      history[5 * it + 1] = emax;
      history[5 * it + 2] = dx[0];
      history[5 * it + 3] = dx[1];
      history[5 * it + 4] = g_fine[n_fine - 1] - g_fine[2 * n_fine - 1];   // n_up - n_dn
    }
    // Neel order on the bipartite lattice: spin sigma's bath closes over G_-sigma
    rc = host::bethe_step(g_fine, n_fine, bath_up, n_iw, m3, U, beta, t, nb_dn.data());
    if (!rc) rc = host::bethe_step(g_fine + n_fine, n_fine, bath_dn, n_iw, m3, U, beta, t, nb_up.data());
    if (rc) return fail(rc, "dmft_solve_af: Bethe step failed in iteration %d", it);
    for (size_t q = 0; q < nb_up.size(); ++q) {
      bath_up[q] = mixing * bath_up[q] + (1.0 - mixing) * nb_up[q];
      bath_dn[q] = mixing * bath_dn[q] + (1.0 - mixing) * nb_dn[q];
    }
  }
  if (g_fine_err) std::memcpy(g_fine_err, err.data(), sizeof(double) * 2 * n_fine);
  return HFQMC_OK;
}
