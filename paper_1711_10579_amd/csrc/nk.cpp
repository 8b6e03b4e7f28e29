// Newton-Krylov inner solve (Sec. III-B) on the host side: the case's Krylov
// storage, the batch's launch lists, and the Newton step that drives the
// batched GMRES kernels (krylov.hip).
//
// The number of Arnoldi steps an instance needs is decided on the device.
// After every step the host reads the instances' Krylov states: it ends the
// cycle of the instances that asked for it (solution update, restart or
// result) and launches the next step for the others, until none iterates.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.hpp"
#include "kernels.hpp"

namespace pfi {

namespace {

template <typename T>
size_t carve_bytes(int64_t count) {
  return ((size_t)std::max<int64_t>(count, 0) * sizeof(T) + 255) & ~(size_t)255;
}

template <typename T>
T* carve(char*& p, int64_t count) {
  T* r = (T*)p;
  p += carve_bytes<T>(count);
  return r;
}

}  // namespace

void free_krylov(Case* c) {
  if (c->kbase && c->kown) {
    c->ctx->dfree(c->kbase);
    c->bytes -= c->kbytes;
  }
  c->kbase = nullptr;
  c->kbytes = 0;
  c->kown = false;
  c->km = 0;
}

void detach_krylov(Case* c) {
  if (c->kbase && !c->kown) {
    c->kbase = nullptr;
    c->kbytes = 0;
    c->km = 0;
  }
}

namespace {

int krylov_m(int m) { return std::max(m, 30); }

}  // namespace

bool krylov_wide(const pfh::KAnalysis& ka) {
  for (size_t l = 0; l + 1 < ka.lev_ptr.size(); ++l)
    if (ka.lev_ptr[l + 1] - ka.lev_ptr[l] > 4096) return true;
  for (size_t l = 0; l + 1 < ka.ulev_ptr.size(); ++l)
    if (ka.ulev_ptr[l + 1] - ka.ulev_ptr[l] > 4096) return true;
  return false;
}

size_t krylov_bytes(const Case* c, int m) {
  if (!c->ka) return 0;
  const pfh::KAnalysis& ka = *c->ka;
  const int km = krylov_m(m);
  const int nu = ka.nu;
  const int64_t knnz = ka.nnz(), nup = ka.nup();
  const int nb = ka.nblocks();
  const int kchunks = (nu + pfd::KCH - 1) / pfd::KCH;
  const int64_t n2 = 2LL * nu;
  const int64_t nh = (int64_t)(km + 1) * km + 2LL * km + (km + 1) + km;
  const int nl = (int)ka.lev_ptr.size() - 1, nul = (int)ka.ulev_ptr.size() - 1;
  size_t total = carve_bytes<int>(nu) + carve_bytes<int>(nu + 1) + carve_bytes<int>(knnz) + carve_bytes<int>(nu) +
                 carve_bytes<int>(c->nnz) + carve_bytes<int>(knnz + 1) + 2 * carve_bytes<int>(nup) +
                 carve_bytes<int>(nb + 1) + 2 * carve_bytes<int>(nu) + carve_bytes<int64_t>(nb + 1);
  total += carve_bytes<int>(nl + 1) + carve_bytes<int>(nul + 1) + 2 * carve_bytes<int4>(nu) + carve_bytes<int>(nb);
  total += 2 * carve_bytes<double>(4 * knnz) + carve_bytes<double>(4LL * nu) + carve_bytes<double>(ka.bj_off.back()) +
           carve_bytes<double>((km + 1) * n2) + 3 * carve_bytes<double>(n2);
  total += carve_bytes<double>(nh) + carve_bytes<double>(3LL * std::max(kchunks, 1) * (km + 1)) +
           carve_bytes<pfd::KState>(1);
  return total;
}

bool attach_krylov(Case* c, int m, char* base, bool own, hipStream_t s) {
  if (c->kbase && c->kown && !own) free_krylov(c);  // too small for this request: replaced by the lent storage
  const pfh::KAnalysis& ka = *c->ka;
  const int km = krylov_m(m);
  const int nu = ka.nu;
  const int64_t knnz = ka.nnz(), nup = ka.nup();
  const int nb = ka.nblocks();
  const int kchunks = (nu + pfd::KCH - 1) / pfd::KCH;
  const int64_t n2 = 2LL * nu;
  const int64_t nh = (int64_t)(km + 1) * km + 2LL * km + (km + 1) + km;
  const int nl = (int)ka.lev_ptr.size() - 1, nul = (int)ka.ulev_ptr.size() - 1;
  const size_t total = krylov_bytes(c, m);
  char* p = base;
  pfd::Inst& h = c->hinst;
  int* kp_of_r = carve<int>(p, nu);
  int* krow_ptr = carve<int>(p, nu + 1);
  int* kcol = carve<int>(p, knnz);
  int* kdiag = carve<int>(p, nu);
  int* kmap = carve<int>(p, c->nnz);
  int* kup_ptr = carve<int>(p, knnz + 1);
  int* kup_t = carve<int>(p, nup);
  int* kup_s = carve<int>(p, nup);
  int* bj_ptr = carve<int>(p, nb + 1);
  int* bj_rows = carve<int>(p, nu);
  int* bj_loc = carve<int>(p, nu);
  int64_t* bj_off = carve<int64_t>(p, nb + 1);
  int* kl_ptr = carve<int>(p, nl + 1);
  int* ku_ptr = carve<int>(p, nul + 1);
  int4* kl_info = carve<int4>(p, nu);
  int4* ku_info = carve<int4>(p, nu);
  h.bjbad = carve<int>(p, nb);
  h.jval = carve<double>(p, 4 * knnz);
  h.pval = carve<double>(p, 4 * knnz);
  h.pdinv = carve<double>(p, 4LL * nu);
  h.bjinv = carve<double>(p, ka.bj_off.back());
  h.kv = carve<double>(p, (km + 1) * n2);
  h.kw = carve<double>(p, n2);
  h.kz = carve<double>(p, n2);
  h.kx = carve<double>(p, n2);
  h.kh = carve<double>(p, nh);
  h.kpart = carve<double>(p, 3LL * std::max(kchunks, 1) * (km + 1));
  h.ks = carve<pfd::KState>(p, 1);
  if ((size_t)(p - base) != total) {
    set_error("pf_solve: internal Krylov layout error");
    return false;
  }
  h.km = km;
  h.kchunks = kchunks;
  h.knb = nb;
  h.kp_of_r = kp_of_r;
  h.krow_ptr = krow_ptr;
  h.kcol = kcol;
  h.kdiag = kdiag;
  h.kmap = kmap;
  h.kup_ptr = kup_ptr;
  h.kup_t = kup_t;
  h.kup_s = kup_s;
  h.bj_ptr = bj_ptr;
  h.bj_rows = bj_rows;
  h.bj_loc = bj_loc;
  h.bj_off = bj_off;
  h.knl = nl;
  h.knul = nul;
  h.kwide = krylov_wide(ka) ? 1 : 0;
  h.kl_ptr = kl_ptr;
  h.kl_info = kl_info;
  h.ku_ptr = ku_ptr;
  h.ku_info = ku_info;

  // the sources stay alive with the case (the copies are asynchronous)
  if (c->k_linfo.empty() && nu > 0) {
    c->k_linfo.resize(nu);
    c->k_uinfo.resize(nu);
    for (int k = 0; k < nu; ++k) {
      const int r = ka.lev_rows[k];
      c->k_linfo[k] = make_int4(r, ka.row_ptr[r], ka.diag[r], 0);
      const int u = ka.ulev_rows[k];
      c->k_uinfo[k] = make_int4(u, ka.diag[u] + 1, ka.row_ptr[u + 1], 0);
    }
  }
  bool ok = true;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (bytes) ok &= hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  up(kp_of_r, ka.p_of_r.data(), sizeof(int) * nu);
  up(krow_ptr, ka.row_ptr.data(), sizeof(int) * (nu + 1));
  up(kcol, ka.col.data(), sizeof(int) * knnz);
  up(kdiag, ka.diag.data(), sizeof(int) * nu);
  up(kmap, c->kmap_host.data(), sizeof(int) * c->nnz);
  up(kup_ptr, ka.up_ptr.data(), sizeof(int) * (knnz + 1));
  up(kup_t, ka.up_t.data(), sizeof(int) * nup);
  up(kup_s, ka.up_s.data(), sizeof(int) * nup);
  up(bj_ptr, ka.bj_ptr.data(), sizeof(int) * (nb + 1));
  up(bj_rows, ka.bj_rows.data(), sizeof(int) * nu);
  up(bj_loc, ka.bj_loc.data(), sizeof(int) * nu);
  up(bj_off, ka.bj_off.data(), sizeof(int64_t) * (nb + 1));
  up(kl_ptr, ka.lev_ptr.data(), sizeof(int) * (nl + 1));
  up(ku_ptr, ka.ulev_ptr.data(), sizeof(int) * (nul + 1));
  up(kl_info, c->k_linfo.data(), sizeof(int4) * nu);
  up(ku_info, c->k_uinfo.data(), sizeof(int4) * nu);
  static_assert(sizeof(pfd::KState) % 4 == 0, "KState is cleared as 32-bit words");
  pfd::launch_zero_words(s, h.ks, (int64_t)(sizeof(pfd::KState) / 4));
  pfd::launch_set_inst(s, c->d_inst, h);
  if (!ok || hipGetLastError() != hipSuccess) {
    set_error("pf_solve: upload of the Krylov storage failed");
    return false;
  }
  c->kbase = base;
  c->kbytes = total;
  c->kown = own;
  c->km = km;
  if (own) c->bytes += total;
  return true;
}

bool ensure_krylov(Case* c, int m) {
  if (c->kbase && c->km >= m) return true;
  if (!c->ka) {
    set_error("pf_solve: the case has no Krylov analysis");
    return false;
  }
  Ctx* ctx = c->ctx;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
    set_error("pf_solve: device failure before the Krylov set-up");
    return false;
  }
  if (c->kbase && !c->kown) {
    set_error("pf_solve: lent Krylov storage is too small");
    return false;
  }
  free_krylov(c);
  const size_t total = krylov_bytes(c, m);
  char* base = (char*)ctx->dalloc(total);
  if (!base) {
    set_error("pf_solve: device allocation of the Krylov storage failed");
    return false;
  }
  if (!attach_krylov(c, m, base, true, ctx->stream) || hipStreamSynchronize(ctx->stream) != hipSuccess) {
    ctx->dfree(base);
    c->kbase = nullptr;
    c->kbytes = 0;
    c->km = 0;
    set_error("pf_solve: set-up of the Krylov storage failed");
    return false;
  }
  return true;
}

bool Batch::build_krylov() {
  std::vector<int2> work;
  k_lev.clear();
  k_ulev.clear();
  max_kchunks = 0;
  size_t max_l = 0, max_u = 0;
  k_min_nu = k_max_nu = 0;
  k_wide = k_narrow = false;
  // each instance takes its own path (one work-group, or one launch per
  // level when some level is too wide), whatever the batch holds
  std::vector<char> wide(nslots, 0);
  for (int s = 0; s < nslots; ++s) {
    Case* c = cases[s];
    if (!c->ka) return false;
    const pfh::KAnalysis& ka = *c->ka;
    max_kchunks = std::max(max_kchunks, (ka.nu + pfd::KCH - 1) / pfd::KCH);
    wide[s] = krylov_wide(ka);
    if (wide[s]) {
      k_wide = true;
      max_l = std::max(max_l, ka.lev_ptr.size() - 1);
      max_u = std::max(max_u, ka.ulev_ptr.size() - 1);
    } else {
      k_min_nu = k_narrow ? std::min(k_min_nu, ka.nu) : ka.nu;
      k_narrow = true;
      k_max_nu = std::max(k_max_nu, ka.nu);
    }
  }
  auto levels = [&](bool upper, size_t nl, std::vector<std::pair<int64_t, int>>* out) {
    for (size_t l = 0; l < nl; ++l) {
      const int64_t off = (int64_t)work.size();
      for (int s = 0; s < nslots; ++s) {
        if (!wide[s]) continue;
        const pfh::KAnalysis& ka = *cases[s]->ka;
        const auto& ptr = upper ? ka.ulev_ptr : ka.lev_ptr;
        const auto& rows = upper ? ka.ulev_rows : ka.lev_rows;
        if (l + 1 >= ptr.size()) continue;
        for (int k = ptr[l]; k < ptr[l + 1]; ++k) work.push_back(make_int2(s, rows[k]));
      }
      out->emplace_back(off, (int)((int64_t)work.size() - off));
    }
  };
  levels(false, max_l, &k_lev);
  levels(true, max_u, &k_ulev);
  {
    // the groups above the small size first (a work-group each), then the
    // small ones (a wave each for their inverse, four to a wave when
    // applied), in fours of one instance, padded with entries of group -1
    const int64_t off = (int64_t)work.size();
    const int small = pfd::bj_small_nodes();
    for (int pass = 0; pass < 2; ++pass) {
      for (int s = 0; s < nslots; ++s) {
        const pfh::KAnalysis& ka = *cases[s]->ka;
        for (int b = 0; b < ka.nblocks(); ++b)
          if ((ka.bj_ptr[b + 1] - ka.bj_ptr[b] > small) == (pass == 0)) work.push_back(make_int2(s, b));
        if (pass == 1)
          while (((int64_t)work.size() - off - k_blocks_big) % 4 != 0) work.push_back(make_int2(s, -1));
      }
      if (pass == 0) k_blocks_big = (int)((int64_t)work.size() - off);
    }
    k_blocks = {off, (int)((int64_t)work.size() - off)};
  }
  const size_t bw = (sizeof(int2) * std::max<size_t>(work.size(), 1) + 255) & ~(size_t)255;
  if (kmem) ctx->dfree(kmem);
  kmem = (char*)ctx->dalloc(bw);
  if (!kmem) return false;
  d_kwork = (int2*)kmem;
  hipStream_t st = stream;
  bool ok = true;
  if (!work.empty())
    ok &= hipMemcpyAsync(d_kwork, work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipStreamSynchronize(st) == hipSuccess;
  kbuilt = ok;
  return ok;
}

namespace {

template <typename T>
pf_status nk_step_t(Batch* b, const pf_options* opt) {
  Ctx* ctx = b->ctx;
  hipStream_t s = b->stream;
  const auto* I = b->d_insts;
  for (Case* c : b->cases)
    if (!ensure_krylov(c, opt->gmres_m)) return PF_E_NOMEM;
  if (!b->kbuilt && !b->build_krylov()) {
    set_error("pf_solve: Krylov batch set-up failed");
    return PF_E_NOMEM;
  }
  pfd::KOpts ko;
  ko.eta_max = opt->eta_max;
  ko.eta_floor = opt->precision == PF_PREC_MIXED ? 1e-6 : 1e-12;
  ko.m = opt->gmres_m;
  ko.max_restarts = opt->gmres_max_restarts;
  const bool ilu = opt->precond == PF_PRECOND_ILU0;
  const int ns = b->nslots, mc = b->max_kchunks;
  const int2* kw = b->d_kwork;
  {
    Prof p(ctx, PF_K_JFILL, 0.0, 0.0);
    pfd::launch_kfill<T>(s, I, ns, b->max_nnz, ilu ? 1 : 0);
  }
  {
    Prof p(ctx, PF_K_PRECOND_SETUP, 0.0, 0.0);
    if (ilu) {
      if (b->k_narrow) pfd::launch_ilu_factor_wg<T>(s, I, ns);
      for (const auto& l : b->k_lev) pfd::launch_ilu_rows<T>(s, I, kw + l.first, l.second);
    } else {
      pfd::launch_bj_inv<T>(s, I, kw + b->k_blocks.first, b->k_blocks_big, b->k_blocks.second - b->k_blocks_big);
    }
  }
  const bool bcg = opt->solver == PF_SOLVER_BICGSTAB;
  {
    Prof p(ctx, PF_K_KRYLOV, 0.0, 0.0);
    if (bcg) {
      pfd::launch_bcg_begin<T>(s, I, ns, mc, ko);
      pfd::launch_bcg_dir<T>(s, I, ns, mc);  // p = r = r0 = F
    } else
      pfd::launch_kbegin<T>(s, I, ns, mc, ko);
    pfd::launch_kfinish<T>(s, I, ns, mc);
  }
  auto apply = [&](int mode) {
    Prof p(ctx, PF_K_PRECOND_APPLY, 0.0, 0.0);
    if (ilu) {
      if (b->k_narrow) pfd::launch_ilu_apply_wg<T>(s, I, ns, mode, b->k_min_nu, b->k_max_nu);
      for (const auto& l : b->k_lev) pfd::launch_ilu_fwd<T>(s, I, kw + l.first, l.second, mode);
      for (const auto& l : b->k_ulev) pfd::launch_ilu_bwd<T>(s, I, kw + l.first, l.second, mode);
    } else {
      pfd::launch_bj_apply<T>(s, I, kw + b->k_blocks.first, b->k_blocks_big, b->k_blocks.second, mode);
    }
  };
  // Iterations (BiCGStab) or Arnoldi steps (GMRES) queued per read of the
  // instances' Krylov states: first as many as the inner solve at this
  // Newton step took in the batch's last solve, then the rest of that count
  // up to 8 at a time, or 2 at a time once it is passed.  An instance that
  // finishes within a run skips the rest of it.
  std::vector<int> st(ns), tot(ns);
  int queued = 0;
  const size_t step_k = (size_t)b->nk_step_index++;
  const int guess = step_k < b->k_inner.size() ? b->k_inner[step_k]
                    : b->k_inner.empty()       ? 8
                                               : b->k_inner.back();
  auto run_length = [&](int done) {
    if (queued == 0) return std::max(1, std::min(guess, 64));
    return guess > done ? std::min(guess - done, 8) : 2;
  };
  auto remember = [&](int most) {
    if (queued == 0) return;
    if (b->k_inner.size() <= step_k) b->k_inner.resize(step_k + 1, 8);
    b->k_inner[step_k] = std::max(1, most);
  };
  const int64_t guard_max = (int64_t)(opt->gmres_max_restarts + 1) * (opt->gmres_m + 2) + 4;
  for (int64_t guard = 0;; ++guard) {
    if (guard > guard_max) {
      set_error("pf_solve: the Krylov inner solve did not settle");
      return PF_E_DEVICE;
    }
    // the gather writes straight into pinned host memory
    pfd::launch_kgather(s, I, ns, b->h_kstate);
    if (hipStreamSynchronize(s) != hipSuccess) {
      set_error("pf_solve: device failure in the Krylov inner solve");
      return PF_E_DEVICE;
    }
    std::memcpy(st.data(), b->h_kstate, sizeof(int) * ns);
    std::memcpy(tot.data(), b->h_kstate + ns, sizeof(int) * ns);
    int most = 0;
    for (int i = 0; i < ns; ++i) most = std::max(most, tot[i]);
    if (bcg) {
      bool any = false;
      for (int v : st) any |= v == pfd::KS_BP || v == pfd::KS_BS || v == pfd::KS_BH;
      if (!any) {
        remember(most);
        break;
      }
      // a run of BiCGStab iterations between two reads of the states (each
      // kernel acts only on the instances in the state it serves)
      const int run = run_length(most);
      queued += run;
      for (int i = 0; i < run; ++i) {
        // the iteration's index in the inner solve: every instance still
        // iterating has done exactly that many
        const int it = queued - run + i;
        apply(2);
        {
          Prof p(ctx, PF_K_KRYLOV, 0.0, 0.0);
          pfd::launch_bcg_half<T>(s, I, ns, mc, it);
        }
        apply(3);
        Prof p(ctx, PF_K_KRYLOV, 0.0, 0.0);
        pfd::launch_bcg_end<T>(s, I, ns, mc, ko, it);
      }
      Prof p(ctx, PF_K_KRYLOV, 0.0, 0.0);
      pfd::launch_kfinish<T>(s, I, ns, mc);
      continue;
    }
    bool iter = false, cyc = false;
    for (int v : st) {
      iter |= v == pfd::KS_ITER;
      cyc |= v == pfd::KS_CYCLE;
    }
    if (!iter && !cyc) {
      remember(most);
      break;
    }
    // a run of Arnoldi steps, then the end of every cycle they complete,
    // between two reads of the states: each kernel acts only on the
    // instances in the state it serves, so an instance whose cycle ends
    // within the run skips its remaining steps
    // (a run ends with the current cycle: steps past it would be skipped)
    const int left = ko.m - most % std::max(ko.m, 1);
    const int run = iter ? std::max(1, std::min(run_length(most), left)) : 0;
    queued += std::max(run, 1);
    for (int i = 0; i < run; ++i) {
      apply(0);
      Prof p(ctx, PF_K_KRYLOV, 0.0, 0.0);
      pfd::launch_karnoldi<T>(s, I, ns, mc, ko);
    }
    {
      Prof p(ctx, PF_K_KRYLOV, 0.0, 0.0);
      pfd::launch_kycomb<T>(s, I, ns, mc);
    }
    apply(1);
    Prof p(ctx, PF_K_KRYLOV, 0.0, 0.0);
    pfd::launch_kcycle_end<T>(s, I, ns, mc, ko);
    pfd::launch_kfinish<T>(s, I, ns, mc);
  }
  {
    Prof p(ctx, PF_K_UPDATE, 0.0, 0.0);
    pfd::launch_update<T>(s, I, ns, b->max_nu);
  }
  return launch_status("pf_solve");
}

}  // namespace

pf_status nk_step(Batch* b, const pf_options* opt) {
  return opt->precision == PF_PREC_MIXED ? nk_step_t<float>(b, opt) : nk_step_t<double>(b, opt);
}

}  // namespace pfi
