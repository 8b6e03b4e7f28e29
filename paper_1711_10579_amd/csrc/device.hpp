// Device-side data layout shared by the kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pfd {

// Sparse factor schedule (device pointers).  Block ids:
//   D_j: j;  L(rowidx[colptr[j]+p], j): ns + colptr[j] + p;
//   U(j, rowidx[colptr[j]+p]): ns + nnzl + colptr[j] + p.
// Targets of column j: tb = j + 2 colptr[j]; D: tb, U(j, r_p): tb + 1 + p,
// L(r_p, j): tb + 1 + len + p; updates of target t: [uptr[t], uptr[t+1]).
struct Sched {
  const int* colptr;
  const int* rowidx;
  const int64_t* uptr;
  const int* upd_l;
  const int* upd_u;
  int ns, nt, ldt;
  int64_t nnzl;
};

// Reduction / status slots of one instance (device memory, reset per step).
struct Red {
  unsigned long long norm_bits;  // max |F| as IEEE bits (non-negative doubles order as integers)
  unsigned long long step_bits;  // max |dx|
  int singular;                  // set when a pivot is zero or non-finite
  int pad;
};

}  // namespace pfd
