// Autotuner of a case's schedule: the fill-reducing ordering's switch to the
// dense trailing block, the lanes per sparse list, and the dense backward
// solve's synchronisation.  Each candidate is a real case solved on the
// device; the median device time of `trials` solves decides.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace pfi {
pf_status validate_desc(const pf_case_desc* d);
}

using namespace pfi;

namespace {

// Median device time of `trials` converged solves under `s`; false when the
// case cannot be created or a solve does not converge.
bool time_schedule(Ctx* ctx, const pf_case_desc* d, const pf_options& o, int trials, const pf_schedule& s,
                   double* ms) {
  Case* c = nullptr;
  if (create_case(ctx, d, s, &c) != PF_OK) return false;
  bool ok = true;
  std::vector<double> t;
  for (int i = 0; i <= trials && ok; ++i) {  // the first solve warms up
    pf_result r;
    pf_status st;
    {
      std::lock_guard<std::mutex> lk(ctx->launch_mu);
      st = solve_case(c, &o, &r);
    }
    ok = st == PF_OK && r.status == PF_CONVERGED;
    if (ok && i > 0) t.push_back(r.device_ms);
  }
  pf_destroy(static_cast<pf_case*>(c));
  if (!ok) return false;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return true;
}

}  // namespace

extern "C" pf_status pf_autotune(pf_ctx* ctx, const pf_case_desc* d, const pf_options* opt, int32_t trials,
                                 pf_schedule* best, pf_tune_report* rep) {
  if (!ctx || !best) {
    set_error("pf_autotune: NULL argument");
    return PF_E_INVALID;
  }
  pf_status st = validate_desc(d);
  if (st != PF_OK) return st;
  pf_options o;
  pf_default_options(&o);
  if (opt) o = *opt;
  st = check_opts(&o);
  if (st != PF_OK) return st;
  trials = std::max(1, std::min(trials, 50));
  pf_schedule cur;
  pf_default_schedule(&cur);
  double cur_ms = 0;
  int count = 1;
  if (!time_schedule(ctx, d, o, trials, cur, &cur_ms)) {
    set_error("pf_autotune: the case does not converge under the default schedule");
    return PF_E_INVALID;
  }
  const double default_ms = cur_ms;
  auto consider = [&](pf_schedule s) {
    double ms;
    ++count;
    if (time_schedule(ctx, d, o, trials, s, &ms) && ms < 0.98 * cur_ms) {
      cur = s;
      cur_ms = ms;
    }
  };
  // dense_switch: the fastest candidate, kept when it beats the default by
  // 2 % (its effect is not monotone, so no greedy chain over the values)
  {
    const pf_schedule base = cur;
    pf_schedule fastest = cur;
    double fastest_ms = cur_ms;
    for (double ds : {0.08, 0.12, 0.2, 0.3, 0.4, 0.5, 0.65, 0.8}) {
      pf_schedule s = base;
      s.dense_switch = ds;
      double ms;
      ++count;
      if (time_schedule(ctx, d, o, trials, s, &ms) && ms < fastest_ms) {
        fastest = s;
        fastest_ms = ms;
      }
    }
    if (fastest_ms < 0.98 * cur_ms) {
      cur = fastest;
      cur_ms = fastest_ms;
    }
  }
  const pf_schedule b2 = cur;
  for (int ls : {2, 4}) {
    pf_schedule s = b2;
    s.lane_scale = ls;
    consider(s);
  }
  const pf_schedule b3 = cur;
  for (int tm : {1, 2}) {
    pf_schedule s = b3;
    s.trsv_mode = tm;
    consider(s);
  }
  {
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    ctx->tuned[topology_hash(d)] = cur;
  }
  *best = cur;
  if (rep) {
    rep->candidates = count;
    rep->trials = trials;
    rep->default_ms = default_ms;
    rep->best_ms = cur_ms;
  }
  return PF_OK;
}
