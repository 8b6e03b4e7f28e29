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

void dense_plan_step(const std::vector<int>& Ms, int k0, std::vector<int2>* items, int* npanel) {
  items->clear();
  const int ns = (int)Ms.size();
  int kb, nrt, nct;
  for (int s = 0; s < ns; ++s) {
    if (Ms[s] <= k0) continue;
    dense_grid(Ms[s], k0, &kb, &nrt, &nct);
    for (int g = 0; g < 1 + nrt; ++g) items->push_back(make_int2(s, g));
  }
  *npanel = (int)items->size();
  // tiles of the next panel's block row and column first (they wait for the
  // panel), then the rest of the previous step's update
  for (int pass = 0; pass < 2; ++pass)
    for (int s = 0; s < ns; ++s) {
      if (Ms[s] <= k0) continue;
      dense_grid(Ms[s], k0, &kb, &nrt, &nct);
      for (int t = 0; t < nrt * nct; ++t) {
        const bool next = t % nrt == 0 || t / nrt == 0;
        if (next != (pass == 0)) continue;
        const int mode = (k0 >= kDenseNB ? kDenseUpdPrev : 0) | (next ? kDenseUpdThis : 0);
        if (mode) items->push_back(make_int2(s, t | mode << 24));
      }
    }
}

}  // namespace pfi
