// Gate sweeps: one pass over the state per gate (the gate-by-gate scheme of
// QueenV2 Sec. II-B, used for single gates and for fused ops that do not fit
// an in-cache pass).
//
// Each work item owns one group of amplitudes: an Eq. 2 pair, an Eq. 3 quad,
// or only the touched members of one (CNOT swaps 2 of its 4, CZ/CPHASE change
// 1 of 4).  Work item k's group base is k with zero bits inserted at the
// gate's positions (the PDEP-like index deposit of Sec. III-B), OR'd with the
// bits a control fixes to 1.  Consecutive lanes take consecutive k, so every
// load instruction of a wave reads runs of consecutive addresses.
//
// complex64 states are processed two amplitudes (16 B) per access whenever bit
// 0 is not one of the gate's positions; every group then has a twin at index
// +1 and both are updated from one 16-byte load.
//
// Launch shape (measured on MI355X at 16 GiB): one group per lane and many
// small blocks keep the most loads in flight -- more resident waves beat more
// loads per lane.  Blocks are dispatched round-robin over the 8 XCDs; the
// block index is remapped so that each XCD walks one contiguous eighth of the
// state, which keeps each XCD's DRAM stream sequential.
#include "sv_device.h"
#include "sv_kernels.h"

namespace sv {
namespace {

constexpr int kBlock = 256;
constexpr int kXcds = 8;

// Block index remapped so that XCD x (blocks x, x+8, ...) owns a contiguous
// range; identity when the grid is not a multiple of the XCD count.
__device__ __forceinline__ uint64_t xcd_block() {
  const uint64_t b = blockIdx.x, nb = gridDim.x;
  if (nb % kXcds) return b;
  return (b % kXcds) * (nb / kXcds) + b / kXcds;
}

template <int NZ, int NV>
struct Geo {
  unsigned z[NZ > 0 ? NZ : 1];
  uint64_t set;
  uint64_t off[NV];
};

// ---------------------------------------------------------------- operators
template <typename R>
struct OpDense1 {
  cplx<R> m[4];
  __device__ __forceinline__ void operator()(cplx<R>* a, uint64_t) const {
    const cplx<R> a0 = a[0], a1 = a[1];
    a[0] = cfma(cmul(m[0], a0), m[1], a1);
    a[1] = cfma(cmul(m[2], a0), m[3], a1);
  }
};

template <typename R>
struct OpDense2 {
  cplx<R> m[16];
  __device__ __forceinline__ void operator()(cplx<R>* a, uint64_t) const {
    const cplx<R> x0 = a[0], x1 = a[1], x2 = a[2], x3 = a[3];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cplx<R> y = cmul(m[4 * r + 0], x0);
      y = cfma(y, m[4 * r + 1], x1);
      y = cfma(y, m[4 * r + 2], x2);
      y = cfma(y, m[4 * r + 3], x3);
      a[r] = y;
    }
  }
};

template <typename R>
struct OpSwap {
  __device__ __forceinline__ void operator()(cplx<R>* a, uint64_t) const {
    const cplx<R> t = a[0];
    a[0] = a[1];
    a[1] = t;
  }
};

template <typename R>
struct OpPhase {
  cplx<R> p;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint64_t) const { a[0] = cmul(p, a[0]); }
};

template <typename R>
struct OpDiag {
  cplx<R> d[4];
  unsigned b0, b1;
  int nb;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint64_t i) const {
    unsigned r = (unsigned)(i >> b0) & 1u;
    if (nb == 2) r = (r << 1) | ((unsigned)(i >> b1) & 1u);
    a[0] = cmul(d[r], a[0]);
  }
};

template <typename R>
struct OpScale {
  R s;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint64_t) const {
    a[0].re *= s;
    a[0].im *= s;
  }
};

// ---------------------------------------------------------------- kernel
template <typename E, int NZ, int NV, class Op>
__global__ __launch_bounds__(kBlock) void k_group(E* __restrict__ psi, uint64_t ngroups, Geo<NZ, NV> g,
                                                  Op op) {
  typedef elem_traits<E> TR;
  typedef typename TR::R R;
  constexpr int ITEMS = 1;
  const uint64_t k0 = xcd_block() * (uint64_t)(kBlock * ITEMS) + threadIdx.x;
  E v[ITEMS][NV];
  uint64_t base[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint64_t k = k0 + (uint64_t)j * kBlock;
    uint64_t b = k;
#pragma unroll
    for (int z = 0; z < NZ; ++z) b = insert0(b, g.z[z]);
    b |= g.set;
    base[j] = b;
    if (k < ngroups) {
#pragma unroll
      for (int r = 0; r < NV; ++r) v[j][r] = ld(psi + b + g.off[r]);
    }
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint64_t k = k0 + (uint64_t)j * kBlock;
    if (k < ngroups) {
#pragma unroll
      for (int h = 0; h < TR::amps; ++h) {
        cplx<R> a[NV];
#pragma unroll
        for (int r = 0; r < NV; ++r) a[r] = TR::get(v[j][r], h);
        op(a, base[j] * TR::amps + h);
#pragma unroll
        for (int r = 0; r < NV; ++r) TR::put(v[j][r], h, a[r]);
      }
#pragma unroll
      for (int r = 0; r < NV; ++r) st(psi + base[j] + g.off[r], v[j][r]);
    }
  }
}

template <typename R>
cplx<R> to_dev(cd x) {
  return cplx<R>{(R)x.real(), (R)x.imag()};
}

template <typename E, int NZ, int NV, class Op>
hipError_t run(void* psi, uint64_t ngroups, const GroupSpec& gs, unsigned shift, const Op& op, hipStream_t s) {
  constexpr int ITEMS = 1;
  Geo<NZ, NV> g;
  for (int z = 0; z < NZ; ++z) g.z[z] = gs.z[z] - shift;
  g.set = gs.set >> shift;
  for (int r = 0; r < NV; ++r) g.off[r] = gs.off[r] >> shift;
  const uint64_t per_block = (uint64_t)kBlock * ITEMS;
  const uint64_t blocks = (ngroups + per_block - 1) / per_block;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_group<E, NZ, NV, Op>), dim3((unsigned)blocks), dim3(kBlock), 0, s, (E*)psi, ngroups, g,
                     op);
  return hipGetLastError();
}

// Dispatch on (op, nz, nv) for one element type.
template <typename E>
hipError_t dispatch(void* psi, int n, const SweepArgs& a, hipStream_t s) {
  typedef typename elem_traits<E>::R R;
  const unsigned shift = elem_traits<E>::amps == 2 ? 1u : 0u;
  const int nbits = n - (int)shift;  // index bits in element space
  const GroupSpec& gs = a.g;
  const uint64_t ngroups = 1ull << (nbits - gs.nz);
  switch (a.op) {
    case SWEEP_DENSE1: {
      OpDense1<R> op;
      for (int i = 0; i < 4; ++i) op.m[i] = to_dev<R>(a.m[i]);
      return run<E, 1, 2>(psi, ngroups, gs, shift, op, s);
    }
    case SWEEP_DENSE2: {
      OpDense2<R> op;
      for (int i = 0; i < 16; ++i) op.m[i] = to_dev<R>(a.m[i]);
      return run<E, 2, 4>(psi, ngroups, gs, shift, op, s);
    }
    case SWEEP_SWAP: {
      OpSwap<R> op;
      if (gs.nz == 1) return run<E, 1, 2>(psi, ngroups, gs, shift, op, s);
      return run<E, 2, 2>(psi, ngroups, gs, shift, op, s);
    }
    case SWEEP_PHASE: {
      OpPhase<R> op;
      op.p = to_dev<R>(a.m[0]);
      if (gs.nz == 1) return run<E, 1, 1>(psi, ngroups, gs, shift, op, s);
      return run<E, 2, 1>(psi, ngroups, gs, shift, op, s);
    }
    case SWEEP_DIAG: {
      OpDiag<R> op;
      for (int i = 0; i < 4; ++i) op.d[i] = to_dev<R>(a.m[i]);
      op.b0 = a.diag_b0;
      op.b1 = a.diag_b1;
      op.nb = a.diag_nbits;
      return run<E, 0, 1>(psi, ngroups, gs, shift, op, s);
    }
    case SWEEP_SCALE: {
      OpScale<R> op;
      op.s = (R)a.m[0].real();
      return run<E, 0, 1>(psi, ngroups, gs, shift, op, s);
    }
  }
  return hipErrorInvalidValue;
}

bool uses_bit0(const GroupSpec& g) {
  uint64_t m = g.set;
  for (int i = 0; i < g.nz; ++i) m |= 1ull << g.z[i];
  for (int i = 0; i < g.nv; ++i) m |= g.off[i];
  return (m & 1ull) != 0;
}

}  // namespace

hipError_t launch_sweep(sv_dtype dt, void* psi, int n, const SweepArgs& a, hipStream_t s) {
  if (dt == SV_C128) return dispatch<dbl2>(psi, n, a, s);
  if (n >= 1 && !uses_bit0(a.g)) return dispatch<flt4>(psi, n, a, s);
  return dispatch<flt2>(psi, n, a, s);
}

// ---------------------------------------------------------------- utilities
namespace {

template <typename E>
__global__ __launch_bounds__(kBlock) void k_init_basis(E* __restrict__ psi, uint64_t count, uint64_t index) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) {
    E v = {};
    if (i == index) v.x = 1;
    psi[i] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_copy16(flt4* __restrict__ dst, const flt4* __restrict__ src,
                                                   uint64_t count) {
  constexpr int ITEMS = 1;
  const uint64_t i0 = xcd_block() * (kBlock * ITEMS) + threadIdx.x;
  flt4 v[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint64_t i = i0 + (uint64_t)j * kBlock;
    if (i < count) v[j] = ld(src + i);
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const uint64_t i = i0 + (uint64_t)j * kBlock;
    if (i < count) st(dst + i, v[j]);
  }
}

}  // namespace

hipError_t launch_init_basis(sv_dtype dt, void* psi, int n, uint64_t index, hipStream_t s) {
  const uint64_t count = 1ull << n;
  const uint64_t blocks = (count + kBlock - 1) / kBlock;
  if (dt == SV_C128)
    hipLaunchKernelGGL(k_init_basis<dbl2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, (dbl2*)psi, count, index);
  else
    hipLaunchKernelGGL(k_init_basis<flt2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, (flt2*)psi, count, index);
  return hipGetLastError();
}

hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const uint64_t count = bytes / 16;
  const uint64_t per_block = (uint64_t)kBlock;
  const uint64_t blocks = (count + per_block - 1) / per_block;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kBlock), 0, s, (flt4*)dst, (const flt4*)src, count);
  return hipGetLastError();
}

}  // namespace sv
