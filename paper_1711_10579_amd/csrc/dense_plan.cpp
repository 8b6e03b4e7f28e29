// Launch plans of the dense trailing block's blocked LU and of the backward
// solve (dense.hip), shared by the batch builder and the host self-check.

#include <algorithm>
#include <map>

#include "internal.hpp"

namespace pfi {

void dense_grid(int M, int k, int* kb, int* nrt, int* nct) {
  *kb = std::min(kDenseNB, M - k);
  *nrt = (M - (k + *kb) + kDenseNB - 1) / kDenseNB;
  *nct = (M + 1 - (k + *kb) + kDenseNB - 1) / kDenseNB;
}

void dense_plan_step(const std::vector<int>& Ms, int k0, std::vector<int2>* items, int* nflag, int* npanel) {
  items->clear();
  const int ns = (int)Ms.size();
  const int p = k0 / kDenseNB;
  int kb, nrt, nct;
  // the previous step's update of the tiles right of its next block column
  // (that column was updated by the previous step's panel): pass 0 the
  // tiles of column p + 1, flagged, pass 1 the rest
  auto prev = [&](int pass) {
    if (k0 < kDenseNB) return;
    for (int s = 0; s < ns; ++s) {
      if (Ms[s] <= k0) continue;
      dense_grid(Ms[s], k0 - kDenseNB, &kb, &nrt, &nct);
      for (int t = 0; t < nrt * nct; ++t) {
        const int rb = p + t % nrt, cb = p + t / nrt;
        if (cb == p || (cb == p + 1) != (pass == 0)) continue;
        items->push_back(make_int2(s, cb | rb << 12 | (pass == 0 ? 1 : 0) << 24));
      }
    }
  };
  prev(0);
  *nflag = (int)items->size();
  for (int s = 0; s < ns; ++s) {
    if (Ms[s] <= k0) continue;
    dense_grid(Ms[s], k0, &kb, &nrt, &nct);
    for (int g = 0; g < 1 + nrt; ++g) items->push_back(make_int2(s, g));
  }
  *npanel = (int)items->size() - *nflag;
  prev(1);
}

void bwd_plan(const std::vector<BwdInput>& in, bool single, std::vector<int2>* items, int* nd, int* nrw) {
  items->clear();
  const int ns = (int)in.size();
  // dense blocks: the last block of each instance first
  for (int s = 0; s < ns; ++s) {
    if (in[s].M <= 0) continue;
    const int nblk = (in[s].M + kDenseNB - 1) / kDenseNB;
    if (single)
      items->push_back(make_int2(s, 0));
    else
      for (int w = 0; w < nblk; ++w) items->push_back(make_int2(s, w));
  }
  *nd = (int)items->size();
  // sparse rows by backward level; a work-group holds rows of one level and
  // one lane-group size only (rows of a level do not depend on each other)
  int nlev = 0;
  for (const auto& c : in) nlev = std::max(nlev, (int)c.lev_ptr->size() - 1);
  std::vector<int2> desc, rows;
  for (int l = 0; l < nlev; ++l) {
    std::map<int, std::vector<int2>> byG;
    for (int s = 0; s < ns; ++s) {
      const auto& lp = *in[s].lev_ptr;
      if (l + 1 >= (int)lp.size()) continue;
      auto& v = byG[(*in[s].g)[l]];
      for (int k = lp[l]; k < lp[l + 1]; ++k) v.push_back(make_int2(s, (*in[s].rows)[k]));
    }
    for (auto& kv : byG) {
      const int G = kv.first, per = 256 / G;
      for (size_t k = 0; k < kv.second.size(); k += per) {
        const int cnt = (int)std::min<size_t>(per, kv.second.size() - k);
        desc.push_back(make_int2((int)rows.size() + (int)k, cnt | G << 16));
      }
      rows.insert(rows.end(), kv.second.begin(), kv.second.end());
    }
  }
  *nrw = (int)desc.size();
  // offsets of the row items relative to the start of the list
  const int base = *nd + *nrw;
  for (auto& d : desc) d.x += base;
  items->insert(items->end(), desc.begin(), desc.end());
  items->insert(items->end(), rows.begin(), rows.end());
}

}  // namespace pfi
