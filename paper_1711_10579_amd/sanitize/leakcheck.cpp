// Host-sanitizer harness of the library (built with AddressSanitizer and
// UndefinedBehaviorSanitizer together with the library's host code, see
// sanitize.py).  Host mode: the symbolic analysis of Sec. III-A and of the
// Krylov preconditioners replayed on seeded grids, every schedule, and the
// input validation on malformed cases, in loops; with "gpu" also context and
// case creation, LU and BiCGStab solves, a batch, served requests and
// destruction, in loops.  LeakSanitizer reports at exit whatever the library
// left allocated; a sanitizer error ends the process with a failure status.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <utility>
#include <vector>

#include "../../include/pf.h"
#include "../../include/pf_debug.h"

namespace {

// A meshed single-phase grid: a random recursive tree plus chords, branch
// admittances stamped into Ybus (an input, as a caller would give it).
struct Grid {
  int n = 0;
  std::vector<int> rp, ci;
  std::vector<double> y, pm, qm, vm, va;
  std::vector<int8_t> type;
  pf_case_desc desc() {
    pf_case_desc d;
    std::memset(&d, 0, sizeof d);
    d.model = PF_MODEL_POLAR_1PH;
    d.n = n;
    d.nnz = (int)ci.size();
    d.row_ptr = rp.data();
    d.col_idx = ci.data();
    d.y = y.data();
    d.bus_type = type.data();
    d.p_sp = pm.data();
    d.q_sp = qm.data();
    d.v_mag = vm.data();
    d.v_ang = va.data();
    return d;
  }
};

Grid make_grid(int n, int chords, unsigned seed) {
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  std::set<std::pair<int, int>> edges;
  for (int k = 1; k < n; ++k) edges.insert({(int)(U(rng) * k), k});
  for (int c = 0; c < chords;) {
    int a = (int)(U(rng) * n), b = (int)(U(rng) * n);
    if (a == b) continue;
    if (a > b) std::swap(a, b);
    if (edges.insert({a, b}).second) ++c;
  }
  std::vector<std::vector<std::pair<int, std::complex<double>>>> rows(n);
  std::vector<std::complex<double>> diag(n);
  for (auto& e : edges) {
    const std::complex<double> z(0.01 + 0.04 * U(rng), 0.05 + 0.15 * U(rng));
    const std::complex<double> yb = 1.0 / z;
    const double bsh = 0.04 * U(rng);
    diag[e.first] += yb + std::complex<double>(0, bsh / 2);
    diag[e.second] += yb + std::complex<double>(0, bsh / 2);
    rows[e.first].push_back({e.second, -yb});
    rows[e.second].push_back({e.first, -yb});
  }
  Grid g;
  g.n = n;
  g.rp.push_back(0);
  for (int i = 0; i < n; ++i) {
    rows[i].push_back({i, diag[i]});
    std::sort(rows[i].begin(), rows[i].end(), [](auto& a, auto& b) { return a.first < b.first; });
    for (auto& e : rows[i]) {
      g.ci.push_back(e.first);
      g.y.push_back(e.second.real());
      g.y.push_back(e.second.imag());
    }
    g.rp.push_back((int)g.ci.size());
  }
  g.type.assign(n, PF_PQ);
  g.type[0] = PF_SLACK;
  g.pm.assign(n, 0.0);
  g.qm.assign(n, 0.0);
  g.vm.assign(n, 1.0);
  g.va.assign(n, 0.0);
  double load = 0.0;
  for (int i = 1; i < n; ++i) {
    if (i % 10 == 0) {
      g.type[i] = PF_PV;
      g.vm[i] = 1.02;
    } else {
      g.pm[i] = -(0.05 + 0.25 * U(rng)) * 0.5;
      g.qm[i] = 0.4843 * g.pm[i];
      load -= g.pm[i];
    }
  }
  // PV buses share the load (balanced dispatch)
  int npv = 0;
  for (int i = 1; i < n; ++i) npv += g.type[i] == PF_PV;
  for (int i = 1; i < n; ++i)
    if (g.type[i] == PF_PV) g.pm[i] = load / std::max(npv, 1);
  return g;
}

int failures = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "leakcheck: FAILED %s (%s)\n", what, pf_last_error());
    ++failures;
  }
}

void host_mode(int loops) {
  pf_schedule sch[3];
  pf_default_schedule(&sch[0]);
  pf_default_schedule(&sch[1]);
  sch[1].dense_switch = 0.3;
  sch[1].lane_scale = 2;
  pf_default_schedule(&sch[2]);
  sch[2].dense_switch = 0.8;
  sch[2].min_dense = 8;
  sch[2].trsv_mode = 2;
  for (int it = 0; it < loops; ++it) {
    for (int n : {2, 30, 300, 2000}) {
      Grid g = make_grid(n, n / 3, 1000 + it * 17 + n);
      pf_case_desc d = g.desc();
      for (auto& s : sch) {
        double res = 0;
        int64_t chk = 0;
        expect(pf_debug_schedule_check(&d, &s, 7, &res, &chk) == PF_OK && res < 1e-10, "schedule replay");
      }
      double dev = 0, res = 0;
      int64_t chk = 0;
      expect(pf_debug_krylov_check(&d, 7, &dev, &res, &chk) == PF_OK && dev < 1e-12, "krylov replay");
    }
    // malformed inputs take the validation's error paths
    Grid g = make_grid(50, 20, 5 + it);
    {
      pf_case_desc d = g.desc();
      std::vector<int> ci = g.ci;
      std::swap(ci[1], ci[2]);  // unsorted row 0
      d.col_idx = ci.data();
      double res;
      int64_t chk;
      expect(pf_debug_schedule_check(&d, nullptr, 1, &res, &chk) == PF_E_INVALID, "unsorted CSR refused");
    }
    {
      pf_case_desc d = g.desc();
      std::vector<double> y = g.y;
      y[3] = std::nan("");
      d.y = y.data();
      double res;
      int64_t chk;
      expect(pf_debug_schedule_check(&d, nullptr, 1, &res, &chk) == PF_E_INVALID, "NaN refused");
    }
    {
      pf_case_desc d = g.desc();
      std::vector<int8_t> t = g.type;
      t[0] = PF_PQ;
      d.bus_type = t.data();
      double res;
      int64_t chk;
      expect(pf_debug_schedule_check(&d, nullptr, 1, &res, &chk) == PF_E_INVALID, "no slack refused");
    }
  }
}

void gpu_mode(int loops) {
  for (int it = 0; it < loops; ++it) {
    pf_ctx* ctx = nullptr;
    if (pf_ctx_create(0, nullptr, nullptr, nullptr, nullptr, &ctx) != PF_OK) {
      expect(false, "pf_ctx_create");
      return;
    }
    Grid g1 = make_grid(1000, 300, 11 + it), g2 = make_grid(400, 120, 12 + it);
    pf_case_desc d1 = g1.desc(), d2 = g2.desc();
    pf_case *c1 = nullptr, *c2 = nullptr;
    expect(pf_create(ctx, &d1, &c1) == PF_OK, "pf_create");
    expect(pf_create(ctx, &d2, &c2) == PF_OK, "pf_create");
    pf_options o;
    pf_default_options(&o);
    pf_result r;
    expect(pf_solve(c1, &o, &r) == PF_OK && r.status == PF_CONVERGED, "LU solve");
    o.solver = PF_SOLVER_BICGSTAB;
    o.max_iter = 40;
    expect(pf_solve(c1, &o, &r) == PF_OK && r.status == PF_CONVERGED, "BiCGStab solve");
    pf_default_options(&o);
    pf_case* both[2] = {c1, c2};
    pf_result rr[2];
    expect(pf_solve_batch(ctx, both, 2, &o, rr) == PF_OK && rr[1].status == PF_CONVERGED, "batch");
    size_t used = 0;
    expect(pf_solve_noalloc(c2, &o, &r, &used) == PF_OK && r.status == PF_CONVERGED, "no-alloc solve");
    expect(pf_serve_config(ctx, size_t(256) << 20, 4) == PF_OK, "pool budget");
    uint64_t t = 0;
    expect(pf_submit(ctx, c2, &o, &t) == PF_OK, "submit");
    for (int32_t done = 0; !done;) expect(pf_poll(ctx, t, &r, &done) == PF_OK, "poll");
    expect(r.status == PF_CONVERGED, "served solve");
    expect(pf_destroy(c1) == PF_OK && pf_destroy(c2) == PF_OK, "pf_destroy");
    pf_ctx_destroy(ctx);
  }
}

}  // namespace

int main(int argc, char** argv) {
  const bool gpu = argc > 1 && std::strcmp(argv[1], "gpu") == 0;
  const int loops = argc > 2 ? std::atoi(argv[2]) : 3;
  host_mode(loops);
  if (gpu) gpu_mode(loops);
  std::printf("leakcheck: %s mode, %d loops, %d failures\n", gpu ? "host+gpu" : "host", loops, failures);
  return failures == 0 ? 0 : 1;
}
