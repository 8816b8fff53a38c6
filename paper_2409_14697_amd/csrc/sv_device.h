// Device-side helpers shared by the HIP kernels of the state-vector core.
//
// Storage: amplitude i of a 2^N state is element i of an array of interleaved
// (re, im) pairs (Eq. 1 of QueenV2, Sec. II-A); qubit q is bit q of i.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sv {

typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Complex value in registers.
template <typename R>
struct cplx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc + a * b
template <typename R>
__device__ __forceinline__ cplx<R> cfma(cplx<R> acc, cplx<R> a, cplx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}

// Insert a zero bit at position b of k (bits >= b move up by one).
__device__ __forceinline__ uint64_t insert0(uint64_t k, unsigned b) {
  const uint64_t lo = k & ((1ull << b) - 1ull);
  return ((k >> b) << (b + 1)) | lo;
}

// Deposit the low bits of x into the set bits of mask, lowest first (the
// PDEP-like index map of Sec. III-B, done with shifts and masks).
__device__ __forceinline__ uint64_t deposit(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  while (mask) {
    const uint64_t low = mask & (~mask + 1ull);
    if (x & 1ull) r |= low;
    x >>= 1;
    mask &= mask - 1ull;
  }
  return r;
}

// A launch may hold at most 2^32 work-items; grids are capped at kMaxGrid
// blocks and kernels loop over the remaining work blocks.
constexpr uint64_t kMaxGrid = 1ull << 22;
inline uint64_t capped_grid(uint64_t work_blocks) { return work_blocks < kMaxGrid ? work_blocks : kMaxGrid; }

// Blocks are dispatched round-robin over the 8 XCDs of an MI355X; this index
// makes XCD x (blocks x, x+8, ...) own one contiguous range of work items.
// Identity when the grid is not a multiple of 8.
__device__ __forceinline__ uint64_t xcd_block() {
  const uint64_t b = blockIdx.x, nb = gridDim.x;
  if (nb % 8) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// A workgroup barrier without the memory fence of __syncthreads (which
// would also wait for this wave's global stores): the caller has already
// waited for the LDS traffic the barrier orders.  The empty asm statements
// keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// The barrier between the phases of a tile: every lane's LDS reads and
// writes (and scalar loads) are complete, then all waves meet.
__device__ __forceinline__ void lds_sync() {
  wait_lgkm0();
  lds_barrier();
}

// Memory element types: one load/store instruction moves one element.
//   dbl2 : one complex128 amplitude (16 B)
//   flt2 : one complex64 amplitude (8 B)
//   flt4 : two consecutive complex64 amplitudes (16 B)
template <typename E>
struct elem_traits;
template <>
struct elem_traits<dbl2> {
  typedef double R;
  static constexpr int amps = 1;
  static __device__ __forceinline__ cplx<R> get(const dbl2& e, int) { return {e.x, e.y}; }
  static __device__ __forceinline__ void put(dbl2& e, int, cplx<R> v) { e.x = v.re; e.y = v.im; }
};
template <>
struct elem_traits<flt2> {
  typedef float R;
  static constexpr int amps = 1;
  static __device__ __forceinline__ cplx<R> get(const flt2& e, int) { return {e.x, e.y}; }
  static __device__ __forceinline__ void put(flt2& e, int, cplx<R> v) { e.x = v.re; e.y = v.im; }
};
template <>
struct elem_traits<flt4> {
  typedef float R;
  static constexpr int amps = 2;
  static __device__ __forceinline__ cplx<R> get(const flt4& e, int h) {
    return h ? cplx<R>{e.z, e.w} : cplx<R>{e.x, e.y};
  }
  static __device__ __forceinline__ void put(flt4& e, int h, cplx<R> v) {
    if (h) { e.z = v.re; e.w = v.im; } else { e.x = v.re; e.y = v.im; }
  }
};

// Streaming loads/stores: every byte of a sweep is touched once, so the
// accesses are marked non-temporal.
template <typename E>
__device__ __forceinline__ E ld(const E* p) { return __builtin_nontemporal_load(p); }
template <typename E>
__device__ __forceinline__ void st(E* p, E v) { __builtin_nontemporal_store(v, p); }

}  // namespace sv
