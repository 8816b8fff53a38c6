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

// Renormalisation: the factor 1/sqrt(norm2) is formed in FP64 from the
// device-resident squared norm (no host round trip).
template <typename R>
struct OpScaleNorm {
  const double* norm2;
  __device__ __forceinline__ void operator()(cplx<R>* a, uint64_t) const {
    const double n2 = *norm2;
    const R s = n2 > 0.0 ? (R)(1.0 / sqrt(n2)) : R(1);  // a zero state stays as it is
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
  const uint64_t nwork = (ngroups + kBlock * ITEMS - 1) / (kBlock * ITEMS);
  for (uint64_t wb = xcd_block(); wb < nwork; wb += gridDim.x) {
  const uint64_t k0 = wb * (uint64_t)(kBlock * ITEMS) + threadIdx.x;
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
}

// ---------------------------------------------------------------- lane exchange
// Gates with a qubit inside one wave's 1 KiB row (element bit < 6, or bit 0 of
// a complex64 element pair).  A wave reads 64 consecutive 16-byte elements per
// load instruction -- whole bursts, never a strided subset -- and the partner
// amplitudes of such a qubit are fetched from the lane that holds them
// (ds_bpermute).  Each lane computes its own amplitudes y = sum_s U[rho][s] x_s
// with rho the lane's row of the gate matrix.  A matrix qubit is INTRA (the
// other half of a complex64 pair), LANE (lane bit = element bit p < 6), or REG
// (a high target held in a second register, loaded from +2^p).  The kinds are
// template parameters, so sources and coefficients resolve at compile time
// except for the lane's own LANE bits, which select among kernel-argument
// coefficients.  High controls are fixed to 1 by the group geometry.
enum { QK_NONE = -1, QK_INTRA = LOW_INTRA, QK_LANE = LOW_LANE, QK_REG = LOW_REG };

template <int NZ>
struct LowGeo {
  unsigned z[NZ > 0 ? NZ : 1];  // element-space zero positions (ascending)
  uint64_t set;                 // element-space bits fixed to 1
  uint64_t off1;                // element offset of register 1
  unsigned lanebit[2];          // lane bit of a LANE qubit
};

template <typename R, int K>
struct LowMat {
  cplx<R> u[(1 << K) * (1 << K)];
};

__device__ __forceinline__ dbl2 shfl_xor_e(dbl2 v, unsigned m) {
  dbl2 r;
  r.x = __shfl_xor(v.x, (int)m);
  r.y = __shfl_xor(v.y, (int)m);
  return r;
}
__device__ __forceinline__ flt4 shfl_xor_e(flt4 v, unsigned m) {
  flt4 r;
  r.x = __shfl_xor(v.x, (int)m);
  r.y = __shfl_xor(v.y, (int)m);
  r.z = __shfl_xor(v.z, (int)m);
  r.w = __shfl_xor(v.w, (int)m);
  return r;
}

template <typename E, int K, int KA, int KB, int NZ>
__global__ __launch_bounds__(kBlock) void k_low(E* __restrict__ psi, uint64_t ngroups, LowGeo<NZ> g,
                                                LowMat<typename elem_traits<E>::R, K> u) {
  typedef elem_traits<E> TR;
  typedef typename TR::R R;
  constexpr int D = 1 << K;
  constexpr int A = TR::amps;
  constexpr int kinds[2] = {KA, KB};
  constexpr int NV = (KA == QK_REG || (K == 2 && KB == QK_REG)) ? 2 : 1;
  // LANE qubits, in matrix order
  constexpr int NL = (KA == QK_LANE) + (K == 2 && KB == QK_LANE);
  const uint64_t nwork = (ngroups + kBlock - 1) / kBlock;
  for (uint64_t wb = xcd_block(); wb < nwork; wb += gridDim.x) {
  const uint64_t k = wb * (uint64_t)kBlock + threadIdx.x;
  const bool active = k < ngroups;
  uint64_t b = k;
#pragma unroll
  for (int z = 0; z < NZ; ++z) b = insert0(b, g.z[z]);
  b |= g.set;
  E x[NV];
#pragma unroll
  for (int r = 0; r < NV; ++r) {
    E v = {};
    if (active) v = ld(psi + b + (r ? g.off1 : 0ull));
    x[r] = v;
  }
  const unsigned lane = threadIdx.x & 63u;
  // lane-bit values of the LANE qubits packed in matrix order, and the xor
  // masks that flip each subset of them
  unsigned lv = 0, lmask[4] = {0, 0, 0, 0};
  {
    int j = 0;
#pragma unroll
    for (int m = 0; m < K; ++m)
      if (kinds[m] == QK_LANE) {
        lv |= ((lane >> g.lanebit[m]) & 1u) << (NL - 1 - j);
        ++j;
      }
#pragma unroll
    for (int f = 0; f < (1 << NL); ++f) {
      int jj = 0;
#pragma unroll
      for (int m = 0; m < K; ++m)
        if (kinds[m] == QK_LANE) {
          if ((f >> (NL - 1 - jj)) & 1) lmask[f] |= 1u << g.lanebit[m];
          ++jj;
        }
    }
  }
  // registers as seen from the lane that differs in each subset of LANE bits
  E xs[1 << NL][NV];
#pragma unroll
  for (int f = 0; f < (1 << NL); ++f)
#pragma unroll
    for (int r = 0; r < NV; ++r) xs[f][r] = f ? shfl_xor_e(x[r], lmask[f]) : x[r];
  E out[NV];
#pragma unroll
  for (int r = 0; r < NV; ++r) {
#pragma unroll
    for (int h = 0; h < A; ++h) {
      cplx<R> y = {0, 0};
#pragma unroll
      for (int d = 0; d < D; ++d) {
        int rs = r, hs = h, f = 0, jj = 0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
          const int bit = (d >> (K - 1 - m)) & 1;
          if (kinds[m] == QK_REG) rs ^= bit;
          else if (kinds[m] == QK_INTRA) hs ^= bit;
          if (kinds[m] == QK_LANE) {
            f |= bit << (NL - 1 - jj);
            ++jj;
          }
        }
        // coefficient U[rho][rho ^ d]; rho's LANE bits come from lv
        cplx<R> c = {0, 0};
#pragma unroll
        for (int v = 0; v < (1 << NL); ++v) {
          int rho = 0, j2 = 0;
#pragma unroll
          for (int m = 0; m < K; ++m) {
            int bit;
            if (kinds[m] == QK_REG) bit = r;
            else if (kinds[m] == QK_INTRA) bit = h;
            else {
              bit = (v >> (NL - 1 - j2)) & 1;
              ++j2;
            }
            rho |= bit << (K - 1 - m);
          }
          const cplx<R> cand = u.u[rho * D + (rho ^ d)];
          if (v == 0 || lv == (unsigned)v) c = cand;
        }
        y = cfma(y, c, TR::get(xs[f][rs], hs));
      }
      TR::put(out[r], h, y);
    }
  }
  if (active) {
#pragma unroll
    for (int r = 0; r < NV; ++r) st(psi + b + (r ? g.off1 : 0ull), out[r]);
  }
  }
}

template <typename R>
cplx<R> to_dev(cd x) {
  return cplx<R>{(R)x.real(), (R)x.imag()};
}

template <typename E, int K, int KA, int KB, int NZ>
hipError_t run_low(void* psi, uint64_t ngroups, const LowGeo<NZ>& g, const cd* m, hipStream_t s) {
  typedef typename elem_traits<E>::R R;
  LowMat<R, K> u;
  for (int i = 0; i < (1 << K) * (1 << K); ++i) u.u[i] = to_dev<R>(m[i]);
  const uint64_t blocks = capped_grid((ngroups + kBlock - 1) / kBlock);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_low<E, K, KA, KB, NZ>), dim3((unsigned)blocks), dim3(kBlock), 0, s, (E*)psi, ngroups, g,
                     u);
  return hipGetLastError();
}

template <typename E, int K, int KA, int KB>
hipError_t run_low_nz(void* psi, uint64_t ngroups, int nz, const unsigned* zs, uint64_t set, uint64_t off1,
                      const unsigned* lanebit, const cd* m, hipStream_t s) {
  if (nz == 0) {
    LowGeo<0> g{};
    g.set = set; g.off1 = off1; g.lanebit[0] = lanebit[0]; g.lanebit[1] = lanebit[1];
    return run_low<E, K, KA, KB, 0>(psi, ngroups, g, m, s);
  }
  LowGeo<1> g{};
  g.z[0] = zs[0]; g.set = set; g.off1 = off1; g.lanebit[0] = lanebit[0]; g.lanebit[1] = lanebit[1];
  return run_low<E, K, KA, KB, 1>(psi, ngroups, g, m, s);
}

// Instantiate the lane-exchange kernel for the layout plan_low() chose.
template <typename E>
hipError_t dispatch_low(void* psi, int n, const SweepArgs& a, hipStream_t s) {
  constexpr bool pair = elem_traits<E>::amps == 2;
  const int nbits = n - (pair ? 1 : 0);
  const int K = a.low_k;
  const int* kind = a.low_kind;
  const int nz = a.low_nz;
  const unsigned* zs = a.low_z;
  const uint64_t set = a.low_set, off1 = a.low_off1;
  const unsigned* lanebit = a.low_lanebit;
  const uint64_t ngroups = 1ull << (nbits - nz);
#define SV_LOW(KK, A_, B_) return run_low_nz<E, KK, A_, B_>(psi, ngroups, nz, zs, set, off1, lanebit, a.m, s)
  if (K == 1) {
    if (kind[0] == QK_LANE) SV_LOW(1, QK_LANE, QK_NONE);
    if constexpr (pair) {
      if (kind[0] == QK_INTRA) SV_LOW(1, QK_INTRA, QK_NONE);
    }
    return hipErrorInvalidValue;
  }
  if (kind[0] == QK_LANE && kind[1] == QK_LANE) SV_LOW(2, QK_LANE, QK_LANE);
  if (kind[0] == QK_LANE && kind[1] == QK_REG) SV_LOW(2, QK_LANE, QK_REG);
  if (kind[0] == QK_REG && kind[1] == QK_LANE) SV_LOW(2, QK_REG, QK_LANE);
  if constexpr (pair) {
    if (kind[0] == QK_INTRA && kind[1] == QK_LANE) SV_LOW(2, QK_INTRA, QK_LANE);
    if (kind[0] == QK_LANE && kind[1] == QK_INTRA) SV_LOW(2, QK_LANE, QK_INTRA);
    if (kind[0] == QK_INTRA && kind[1] == QK_REG) SV_LOW(2, QK_INTRA, QK_REG);
    if (kind[0] == QK_REG && kind[1] == QK_INTRA) SV_LOW(2, QK_REG, QK_INTRA);
  }
#undef SV_LOW
  return hipErrorInvalidValue;
}

template <typename E, int NZ, int NV, class Op>
hipError_t run(void* psi, uint64_t ngroups, const GroupSpec& gs, unsigned shift, const Op& op, hipStream_t s) {
  Geo<NZ, NV> g;
  for (int z = 0; z < NZ; ++z) g.z[z] = gs.z[z] - shift;
  g.set = gs.set >> shift;
  for (int r = 0; r < NV; ++r) g.off[r] = gs.off[r] >> shift;
  const uint64_t blocks = capped_grid((ngroups + kBlock - 1) / kBlock);
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
    case SWEEP_SCALE_NORM: {
      OpScaleNorm<R> op;
      op.norm2 = a.norm2_dev;
      return run<E, 0, 1>(psi, ngroups, gs, shift, op, s);
    }
    default:
      break;
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
  if (a.op == SWEEP_LOW) return dt == SV_C128 ? dispatch_low<dbl2>(psi, n, a, s) : dispatch_low<flt4>(psi, n, a, s);
  if (dt == SV_C128) return dispatch<dbl2>(psi, n, a, s);
  if (n >= 1 && !uses_bit0(a.g)) return dispatch<flt4>(psi, n, a, s);
  return dispatch<flt2>(psi, n, a, s);
}

// ---------------------------------------------------------------- utilities
namespace {

template <typename E>
__global__ __launch_bounds__(kBlock) void k_init_basis(E* __restrict__ psi, uint64_t count, uint64_t index) {
  for (uint64_t i = xcd_block() * kBlock + threadIdx.x; i < count; i += (uint64_t)gridDim.x * kBlock) {
    E v = {};
    if (i == index) v.x = 1;
    st(psi + i, v);
  }
}

__global__ __launch_bounds__(kBlock) void k_copy16(flt4* __restrict__ dst, const flt4* __restrict__ src,
                                                   uint64_t count) {
  constexpr int ITEMS = 1;
  for (uint64_t i0 = xcd_block() * (kBlock * ITEMS) + threadIdx.x; i0 < count;
       i0 += (uint64_t)gridDim.x * kBlock * ITEMS) {
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
}

}  // namespace

hipError_t launch_init_basis(sv_dtype dt, void* psi, int n, uint64_t index, hipStream_t s) {
  const uint64_t count = 1ull << n;
  const uint64_t blocks = capped_grid((count + kBlock - 1) / kBlock);
  if (dt == SV_C128)
    hipLaunchKernelGGL(k_init_basis<dbl2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, (dbl2*)psi, count, index);
  else
    hipLaunchKernelGGL(k_init_basis<flt2>, dim3((unsigned)blocks), dim3(kBlock), 0, s, (flt2*)psi, count, index);
  return hipGetLastError();
}

hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const uint64_t count = bytes / 16;
  const uint64_t per_block = (uint64_t)kBlock;
  const uint64_t blocks = capped_grid((count + per_block - 1) / per_block);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(kBlock), 0, s, (flt4*)dst, (const flt4*)src, count);
  return hipGetLastError();
}

}  // namespace sv
