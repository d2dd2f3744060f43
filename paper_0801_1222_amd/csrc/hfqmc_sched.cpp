// Chain-split planner for launches whose grids differ widely in cost.
//
// The multigrid method runs every Trotter grid with its own independent
// impurity solutions, averaged per grid (Multigrid HF-QMC section); the work
// per sweep grows like L^3, so in a batched launch of grids spanning a factor
// 8 in L the long grid's chains are 512 times longer than the short ones and
// set the launch's length while the rest of the device idles.  Splitting the
// measured sweeps of a long grid's chain over f independent chains (each with
// its own warm-up) keeps the number of measurements per grid and spreads the
// grid over more workgroups, at the price of (f - 1) extra warm-ups.
//
// The planner picks the factors by simulating the dispatch the sweep kernel
// performs: units (grid, chain) taken longest first from an atomic queue by
// P persistent workgroups, i.e. longest-processing-time-first list scheduling.
// It scores every threshold plan (for a target unit length, each grid split
// just enough to fit under it), then improves the best by local moves.
#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
#include <vector>

#include "hfqmc_internal.h"

namespace hfqmc {

double unit_cost(int L, long long warmup, long long sweeps) {
  const double l = (double)L;
  return (double)(warmup + sweeps) * l * l * l;
}

double lpt_makespan(const std::vector<double>& cost, int n_workers) {
  if (cost.empty()) return 0.0;
  std::vector<double> c(cost);
  std::sort(c.begin(), c.end(), std::greater<double>());
  const int p = std::max(1, std::min(n_workers, (int)c.size()));
  std::priority_queue<double, std::vector<double>, std::greater<double>> fin;
  for (int w = 0; w < p; ++w) fin.push(0.0);
  double span = 0.0;
  for (double x : c) {
    const double t = fin.top() + x;
    fin.pop();
    fin.push(t);
    span = std::max(span, t);
  }
  return span;
}

namespace {

double simulate(int n_grids, const int* Ls, int n_chains, long long warmup, long long sweeps,
                const std::vector<int>& f, int n_workers) {
  std::vector<double> cost;
  for (int i = 0; i < n_grids; ++i) {
    const double u = unit_cost(Ls[i], warmup, sweeps / f[i]);
    for (int c = 0; c < n_chains * f[i]; ++c) cost.push_back(u);
  }
  return lpt_makespan(cost, n_workers);
}

}  // namespace

int plan_chain_split(int n_grids, const int* Ls, int n_chains, long long warmup, long long sweeps,
                     int n_bins, int n_workers, int* factor, double* span_before,
                     double* span_after) {
  auto allowed = [&](long long g) {
    return g <= kMaxChainSplit && sweeps % g == 0 && sweeps / g >= n_bins &&
           (long long)n_chains * g < (1LL << 20);
  };
  auto units_of = [&](const std::vector<int>& f) {
    long long u = 0;
    for (int i = 0; i < n_grids; ++i) u += f[i];
    return u;
  };
  // launches of many chains already keep every workgroup busy to the end (and
  // would make each simulation long): they are not split, nor simulated
  if ((long long)n_grids * n_chains > kMaxPlannedChains) {
    for (int i = 0; i < n_grids; ++i) factor[i] = 1;
    if (span_before) *span_before = 0.0;
    if (span_after) *span_after = 0.0;
    return 0;
  }
  std::vector<int> f(n_grids, 1);
  double span = simulate(n_grids, Ls, n_chains, warmup, sweeps, f, n_workers);
  if (span_before) *span_before = span;
  // keeps g if it is shorter by more than 0.5 %, or as short with fewer chains
  auto offer = [&](const std::vector<int>& g) {
    const double s = simulate(n_grids, Ls, n_chains, warmup, sweeps, g, n_workers);
    if (s < span * (1.0 - 5e-3) || (s <= span * (1.0 + 1e-9) && units_of(g) < units_of(f))) {
      f = g;
      span = s;
      return true;
    }
    return false;
  };
  // 1. threshold plans: for a target unit length T every grid takes the
  //    smallest allowed factor whose units fit under T; T runs over every
  //    unit length some grid can have
  std::vector<double> targets;
  for (int i = 0; i < n_grids; ++i)
    for (long long g = 1; allowed(g); g *= 2) targets.push_back(unit_cost(Ls[i], warmup, sweeps / g));
  std::sort(targets.begin(), targets.end());
  for (double T : targets) {
    std::vector<int> g(n_grids, 1);
    for (int i = 0; i < n_grids; ++i)
      while (unit_cost(Ls[i], warmup, sweeps / g[i]) > T && allowed(2LL * g[i])) g[i] *= 2;
    offer(g);
  }
  // 2. local moves from the best threshold plan, until none shortens the span:
  //    one grid's factor doubled or halved, or the factors of every grid whose
  //    units are at least as long as grid i's doubled together (a long grid's
  //    split only pays once the next grids' units no longer pile up on top)
  for (int step = 0; step < 256; ++step) {
    bool moved = false;
    for (int i = 0; i < n_grids && !moved; ++i) {
      std::vector<int> g(f);
      if (allowed(2LL * g[i])) {
        g[i] *= 2;
        moved = offer(g);
      }
      if (!moved && f[i] > 1) {
        g = f;
        g[i] /= 2;
        moved = offer(g);
      }
      if (!moved) {
        const double ui = unit_cost(Ls[i], warmup, sweeps / f[i]);
        g = f;
        bool ok = true;
        for (int j = 0; j < n_grids && ok; ++j)
          if (unit_cost(Ls[j], warmup, sweeps / f[j]) >= ui) {
            ok = allowed(2LL * g[j]);
            g[j] *= 2;
          }
        if (ok) moved = offer(g);
      }
    }
    if (!moved) break;
  }
  for (int i = 0; i < n_grids; ++i) factor[i] = f[i];
  if (span_after) *span_after = span;
  return 0;
}

}  // namespace hfqmc
