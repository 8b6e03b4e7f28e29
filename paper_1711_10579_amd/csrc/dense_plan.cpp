// Launch plan of the dense trailing block's blocked LU (dense.hip), shared by
// the batch builder and the host self-check.

#include <algorithm>

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

}  // namespace pfi
