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

void dense_plan_step(const std::vector<int>& Ms, int k0, std::vector<int2>* comb, int* npanel,
                     std::vector<int2>* next) {
  comb->clear();
  next->clear();
  const int ns = (int)Ms.size();
  int kb, nrt, nct;
  for (int s = 0; s < ns; ++s) {
    if (Ms[s] <= k0) continue;
    dense_grid(Ms[s], k0, &kb, &nrt, &nct);
    for (int g = 0; g < 1 + nrt; ++g) comb->push_back(make_int2(s, g));
  }
  *npanel = (int)comb->size();
  if (k0 >= kDenseNB)
    for (int s = 0; s < ns; ++s) {
      const int k = k0 - kDenseNB;
      if (Ms[s] <= k) continue;
      dense_grid(Ms[s], k, &kb, &nrt, &nct);
      for (int t = 0; t < nrt * nct; ++t)
        if (t % nrt >= 1 && t / nrt >= 1) comb->push_back(make_int2(s, t));
    }
  for (int s = 0; s < ns; ++s) {
    if (Ms[s] <= k0) continue;
    dense_grid(Ms[s], k0, &kb, &nrt, &nct);
    for (int t = 0; t < nrt * nct; ++t)
      if (t % nrt == 0 || t / nrt == 0) next->push_back(make_int2(s, t));
  }
}

}  // namespace pfi
