// Launch timing of the multigrid V-cycle and the launch-shape autotuner
// (aao_profile_vcycle, aao_autotune; declared in include/aao_heat.h).
//
// The V-cycle's tiled level kernels can run short tiles (more workgroups,
// shorter critical path) or tall ones (less halo work per node), and the
// register-resident tail can also take a 64 x 64 level or leave it to the
// grid kernels.  Neither choice changes the cycle's arithmetic.  Which is
// faster depends on the device and on how many blocks a launch carries: one
// block in an S-tilde step, one per coarse interval in an MGRIT relaxation,
// one per time step in Theta-tilde.  The tuner times every candidate's
// V-cycle, replayed as a captured graph, at those block counts and keeps the
// one with the least V-cycle time per application of P-tilde; results can be
// kept in a text cache keyed by the device architecture and the problem's
// shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "aao_internal.h"

namespace {

int tfail(aao_problem* h, int code, const std::string& msg) {
  h->err = msg;
  return code;
}

// Cache key: device architecture and everything that fixes the launches.
std::string tune_key(const aao_problem* h) {
  hipDeviceProp_t prop{};
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ') c = '_';
  std::ostringstream k;
  k << arch << " dim=" << h->dim << " n=" << h->n << " s=" << h->s << " nt=" << h->nt << " prec=" << h->opts.precision
    << " vark=" << (h->vark ? 1 : 0) << " nu=" << h->opts.nu1 << "," << h->opts.nu2 << " k=" << h->opts.inner_k
    << " schur=" << h->opts.schur << " cf=" << h->opts.mgrit_cf << " it=" << h->opts.mgrit_iters
    << " fcf=" << h->opts.mgrit_fcf << " coarse=" << h->opts.coarse_max << " tail=" << h->opts.mg_tail_max
    << " low=" << h->opts.mg_low_from << "," << h->opts.mg_coarse_fp32 << " sk=" << h->opts.schur_k
    << " ck=" << h->opts.mgrit_coarse_k << " orth=" << h->opts.inner_orth;
  return k.str();
}

bool cache_lookup(const char* path, const std::string& key, int& tall, int& ext) {
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    const size_t bar = line.find(" | ");
    if (bar == std::string::npos || line.compare(0, bar, key) != 0 || bar != key.size()) continue;
    std::istringstream v(line.substr(bar + 3));
    int t = 0, e = 0;
    if (v >> t >> e) {
      tall = t;
      ext = e;
      found = true;   // the last matching line wins
    }
  }
  return found;
}

}  // namespace

extern "C" {

int aao_profile_vcycle(aao_problem* h, int stage, int count, int reps, char* labels, size_t labels_cap, double* us,
                       double* us_alone, int cap, int* nlaunch, double* total_us) {
  if (!h) return AAO_INVALID_ARG;
  if (!h->ws) return tfail(h, AAO_NO_WORKSPACE, "aao_set_workspace first");
  if (stage < 0 || stage >= h->s) return tfail(h, AAO_INVALID_ARG, "stage out of range");
  if (count < 1 || count > h->nt) return tfail(h, AAO_INVALID_ARG, "count must be in [1, nt]");
  if (reps < 1 || reps > 1000) return tfail(h, AAO_INVALID_ARG, "reps must be in [1, 1000]");
  if (!nlaunch || !total_us) return tfail(h, AAO_INVALID_ARG, "null pointer");
  std::vector<std::string> lab;
  std::vector<double> t, ta;
  double total = 0.0;
  const hipError_t e = aao::profile_vcycle(h, stage, count, reps, lab, t, ta, total);
  if (e != hipSuccess) return aao::status_from_hip(h, e, "profile_vcycle");
  *nlaunch = (int)t.size();
  *total_us = total;
  for (int i = 0; i < cap && i < (int)t.size(); ++i) {
    if (us) us[i] = t[i];
    if (us_alone) us_alone[i] = ta[i];
  }
  if (labels && labels_cap > 0) {
    std::string all;
    for (const auto& s : lab) all += s + "\n";
    const size_t n = std::min(all.size(), labels_cap - 1);
    std::memcpy(labels, all.data(), n);
    labels[n] = '\0';
  }
  return AAO_OK;
}

int aao_autotune(aao_problem* h, int reps, const char* cache_path, aao_tune* out) {
  if (!h) return AAO_INVALID_ARG;
  if (!h->ws) return tfail(h, AAO_NO_WORKSPACE, "aao_set_workspace first");
  if (reps < 1 || reps > 1000) return tfail(h, AAO_INVALID_ARG, "reps must be in [1, 1000]");
  aao_tune local{};
  aao_tune& r = out ? *out : local;
  r = aao_tune{};
  // block counts per launch and V-cycles per P-tilde application at each
  // (k inner iterations x s stages x cycles per shifted-block solve; the
  // S-tilde steps take schur_k iterations, MGRIT's coarse ones mgrit_coarse_k)
  const double per_v = (double)h->s * h->opts.cycles;
  const double per_solve = per_v * (h->opts.schur_k > 0 ? h->opts.schur_k : h->opts.inner_k);
  const double per_coarse = per_v * (h->opts.mgrit_coarse_k > 0 ? h->opts.mgrit_coarse_k : h->opts.inner_k);
  const int nt = h->nt;
  int K = 1;
  if (h->opts.schur == AAO_SCHUR_MGRIT) K = (nt + h->opts.mgrit_cf - 1) / h->opts.mgrit_cf;
  r.blocks[0] = 1;
  r.blocks[1] = std::max(1, std::min(K, nt));
  r.blocks[2] = nt;
  if (h->opts.schur == AAO_SCHUR_MGRIT) {
    const int c = h->opts.mgrit_cf, it = h->opts.mgrit_iters;
    r.weight[0] = per_coarse * it * std::max(K - 2, 0);
    r.weight[1] = per_solve * ((double)it * c * (h->opts.mgrit_fcf ? 2 : 1) + (c - 1));
  } else {
    r.weight[0] = per_solve * nt;
  }
  r.weight[2] += per_v * h->opts.inner_k;
  const std::string key = tune_key(h);
  const aao_problem::Tune saved = h->tune;
  int tall = 0, ext = 0;
  if (cache_path && cache_lookup(cache_path, key, tall, ext)) {
    r.from_cache = 1;
  } else {
    const int thresholds[3] = {1, 8, 1 << 30};
    double best = 1e300;
    for (int c = 0; c < 6; ++c) {
      h->tune.tall_min_b = thresholds[c % 3];
      h->tune.tail_extend = c < 3;
      double cost = 0.0;
      for (int b = 0; b < 3; ++b) {
        if (r.weight[b] == 0.0 && b != 2) continue;
        std::vector<std::string> lab;
        std::vector<double> t, ta;
        double total = 0.0;
        const hipError_t e = aao::profile_vcycle(h, 0, r.blocks[b], reps, lab, t, ta, total);
        if (e != hipSuccess) {
          h->tune = saved;
          return aao::status_from_hip(h, e, "autotune");
        }
        r.us[c][b] = total;
        cost += r.weight[b] * total;
      }
      if (cost < best) {
        best = cost;
        tall = thresholds[c % 3];
        ext = c < 3 ? 1 : 0;
      }
    }
    if (cache_path) {
      std::ofstream f(cache_path, std::ios::app);
      f << key << " | " << tall << " " << ext << "\n";
    }
  }
  h->tune.tall_min_b = tall;
  h->tune.tail_extend = ext != 0;
  r.tall_min_b = tall;
  r.tail_extend = ext;
  // graphs captured with the old launch shapes are dropped
  if (h->tune.tall_min_b != saved.tall_min_b || h->tune.tail_extend != saved.tail_extend) aao::release_graphs(h);
  return AAO_OK;
}

int aao_set_launch_shapes(aao_problem* h, int tall_min_b, int tail_extend) {
  if (!h) return AAO_INVALID_ARG;
  if (tall_min_b < 1 || (tail_extend != 0 && tail_extend != 1))
    return tfail(h, AAO_INVALID_ARG, "tall_min_b must be >= 1 and tail_extend 0 or 1");
  if (h->tune.tall_min_b != tall_min_b || h->tune.tail_extend != (tail_extend != 0)) aao::release_graphs(h);
  h->tune.tall_min_b = tall_min_b;
  h->tune.tail_extend = tail_extend != 0;
  return AAO_OK;
}

}  // extern "C"
