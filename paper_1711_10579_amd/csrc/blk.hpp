// 2x2 blocks of the Jacobian (row-major [a b; c d]) and their arithmetic,
// shared by the factor and Krylov kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pfd {

// Pointers into device (global) memory.  Memory reached through the
// instance descriptors is otherwise accessed through generic pointers, whose
// loads the compiler issues as flat loads; flat loads are also counted by the
// LDS wait counter, so every LDS wait or barrier would wait for them too.
#define PF_AS1 __attribute__((address_space(1)))
template <typename T>
__device__ inline PF_AS1 T* gp(T* p) {
  return (PF_AS1 T*)p;
}
template <typename T>
__device__ inline const PF_AS1 T* gp(const T* p) {
  return (const PF_AS1 T*)p;
}

// work item i of a list of (instance, index) pairs, through a global pointer
__device__ inline int2 ld_item(const int2* work, int i) {
  const auto wp = (const PF_AS1 int*)work;
  return make_int2(wp[2 * i], wp[2 * i + 1]);
}

// Bound of an in-launch wait in ticks of the device's constant real-time
// counter (100 MHz): about one second.
constexpr unsigned long long kWaitTicks = 100000000ull;
__device__ inline unsigned long long rt_now() { return __builtin_amdgcn_s_memrealtime(); }
// s_waitcnt vmcnt(0): every vector memory access of the wave, stores
// included, has completed
__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Device-coherent accesses for data handed between work-groups inside a
// launch: relaxed atomics at agent scope (stores write through, loads bypass
// the caches that are not coherent across the device), issued as global
// (not generic) accesses so that they are counted by the vector-memory wait
// counter alone and LDS waits do not wait for them.  p points to device
// memory.
template <typename T>
__device__ inline T ld_dev(const T* p) {
  return __hip_atomic_load((const PF_AS1 T*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void st_dev(T* p, T v) {
  __hip_atomic_store((PF_AS1 T*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Work-groups of a launch are handed to the device's eight XCDs (each with
// its own L2) in turn.  xcd_block(b, G) renumbers block b of a grid of G so
// that each XCD takes one contiguous range of the renumbered blocks: data
// that neighbouring blocks share is then fetched into one L2, not eight.
// A permutation of [0, G).
__device__ inline int xcd_block(int b, int G) {
  constexpr int kXcd = 8;
  const int c = G / kXcd, rem = G % kXcd;
  const int x = b % kXcd, k = b / kXcd;
  return x < rem ? x * (c + 1) + k : rem * (c + 1) + (x - rem) * c + k;
}

// four ints as a native vector (loadable through any address space)
typedef int i4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Blk {
  T a, b, c, d;  // [[a b] [c d]]
};

template <typename T, typename Ptr>
__device__ inline Blk<T> ld_blk_as(Ptr p, int64_t id) {
  const auto q = p + 4 * id;
  Blk<T> r;
  r.a = q[0];
  r.b = q[1];
  r.c = q[2];
  r.d = q[3];
  return r;
}

template <typename T>
__device__ inline Blk<T> ld_blk(const PF_AS1 T* p, int64_t id) {
  return ld_blk_as<T>(p, id);
}

template <typename T>
__device__ inline void st_blk(PF_AS1 T* p, int64_t id, const Blk<T>& v) {
  PF_AS1 T* q = p + 4 * id;
  q[0] = v.a;
  q[1] = v.b;
  q[2] = v.c;
  q[3] = v.d;
}

template <typename T>
__device__ inline Blk<T> ld_blk(const T* p, int64_t id) {
  const T* q = p + 4 * id;
  Blk<T> r;
  r.a = q[0];
  r.b = q[1];
  r.c = q[2];
  r.d = q[3];
  return r;
}

template <typename T>
__device__ inline void st_blk(T* p, int64_t id, const Blk<T>& v) {
  T* q = p + 4 * id;
  q[0] = v.a;
  q[1] = v.b;
  q[2] = v.c;
  q[3] = v.d;
}

// acc -= X * Y
template <typename T>
__device__ inline void blk_msub(Blk<T>& acc, const Blk<T>& X, const Blk<T>& Y) {
  acc.a -= X.a * Y.a + X.b * Y.c;
  acc.b -= X.a * Y.b + X.b * Y.d;
  acc.c -= X.c * Y.a + X.d * Y.c;
  acc.d -= X.c * Y.b + X.d * Y.d;
}

template <typename T>
__device__ inline Blk<T> blk_mul(const Blk<T>& X, const Blk<T>& Y) {
  Blk<T> r;
  r.a = X.a * Y.a + X.b * Y.c;
  r.b = X.a * Y.b + X.b * Y.d;
  r.c = X.c * Y.a + X.d * Y.c;
  r.d = X.c * Y.b + X.d * Y.d;
  return r;
}

// inverse of a 2x2 block (determinant in FP64); false when it is zero or
// not finite
template <typename T>
__device__ inline bool blk_inv(const Blk<T>& m, Blk<T>* out) {
  const double det = (double)m.a * (double)m.d - (double)m.b * (double)m.c;
  if (!(det != 0.0) || !isfinite(det)) return false;
  const double id = 1.0 / det;
  out->a = (T)((double)m.d * id);
  out->b = (T)(-(double)m.b * id);
  out->c = (T)(-(double)m.c * id);
  out->d = (T)((double)m.a * id);
  return true;
}

// sum over the G lanes of a group (G a power of two, groups aligned to G)
template <typename T, int G>
__device__ inline Blk<T> group_sum(Blk<T> v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    v.a += __shfl_xor(v.a, off, 64);
    v.b += __shfl_xor(v.b, off, 64);
    v.c += __shfl_xor(v.c, off, 64);
    v.d += __shfl_xor(v.d, off, 64);
  }
  return v;
}

// Marker of a solution entry not yet computed: a signalling NaN with a fixed
// payload.  Arithmetic never produces a signalling NaN (its NaN results are
// quiet) and the inputs are finite, so a stored solution value never has
// these bits.
template <typename T>
struct Unsolved;
template <>
struct Unsolved<double> {
  typedef unsigned long long U;
  static constexpr U bits = 0x7FF4DEADBEEFCAFEull;
};
template <>
struct Unsolved<float> {
  typedef unsigned int U;
  static constexpr U bits = 0x7FA5DEADu;
};
template <typename T>
__device__ inline bool unsolved(T v) {
  return __builtin_bit_cast(typename Unsolved<T>::U, v) == Unsolved<T>::bits;
}
template <typename T>
__device__ inline T unsolved_value() {
  return __builtin_bit_cast(T, Unsolved<T>::bits);
}

}  // namespace pfd
