// In-cache tile pass: the block-by-block all-in-cache execution of QueenV2
// (Sec. II-B "In-cache Operations", Sec. III-B) on gfx950 LDS.
//
// One block owns one tile of 2^m amplitudes: the indices that agree with the
// tile base on every non-local bit.  The tile is gathered from HBM with the
// PDEP-like deposit of its local index into the pass's local bit positions
// (Sec. III-B), so the low pinned positions give contiguous runs.  The pass's
// stages then run in LDS: a stage gives each lane a group of 32 (complex64)
// or 16 (complex128) amplitudes (5 or 4 local bits held in registers) and
// applies a list of ops to them in registers; ops whose controls or phase
// bits lie outside the register bits read those bits from the group's local
// index or from the tile base.  A fused run of diagonal gates (Sec. III-A) is
// a phase function of the index bits: its fixed-point angle words are summed
// per lane from both, with the tile part summed once per tile and stage.
// The tile is written back with local bit j at physical position wpos[j],
// which fuses qubit reordering (Sec. II-B) into the store.
//
// LDS rows are 128 bytes; the element index is XOR-swizzled (low bits folded
// with every higher group of bits) so that power-of-two strides between the
// lanes of a wave fall into distinct banks.
#include "sv_device.h"
#include "sv_kernels.h"
#include "sv_tile_kernels.h"

namespace sv {
namespace {

constexpr int kBlock = 256;

// Register bits of a stage: 32 complex64 or 16 complex128 amplitudes per lane.
template <typename R>
struct Regs {
  static constexpr int RB = sizeof(R) == 4 ? 5 : 4;
  static constexpr int NR = 1 << RB;
};

template <int WB>
__device__ __forceinline__ uint32_t swz(uint32_t x) {
  uint32_t y = x >> WB, h = 0;
#pragma unroll
  for (int k = 0; k * WB < 16; ++k) h ^= y >> (k * WB);
  return x ^ (h & ((1u << WB) - 1u));
}

template <typename R>
struct dev_elem;
template <>
struct dev_elem<double> {
  typedef dbl2 E;
};
template <>
struct dev_elem<float> {
  typedef flt2 E;
};

// Program memory (pass descriptors, stages, ops, matrices, batch items) is
// read-only while a pass kernel runs.  Reading it through the constant
// address space lets uniform reads go through scalar loads even where the
// compiler cannot prove that the state's stores do not alias it (the batched
// kernel takes the state and program pointers from one descriptor array).
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
// The state lives in global memory; saying so keeps its loads and stores
// global (not flat) after its pointer passed through scalar registers.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}
template <typename T>
__device__ __forceinline__ T ldg(gptr<const T> p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void stg(gptr<T> p, T v) {
  __builtin_nontemporal_store(v, p);
}

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)p;
}
// A value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}
template <typename P>
__device__ __forceinline__ P uniform_ptr(P p) {
  return (P)uniform64((uint64_t)p);
}

template <typename R>
__device__ __forceinline__ cplx<R> cget(cptr<cplx<R>> M, uint32_t i) {
  return cplx<R>{M[i].re, M[i].im};
}
// Copy a program struct out of constant memory (dword by dword: the
// implicit copy constructor cannot read another address space).
template <typename T>
__device__ __forceinline__ T cload(cptr<T> p) {
  static_assert(sizeof(T) % 4 == 0, "program structs are dword multiples");
  T out;
  const __attribute__((address_space(4))) uint32_t* src = (const __attribute__((address_space(4))) uint32_t*)p;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) dst[i] = src[i];
  return out;
}

template <int B, typename R>
__device__ __forceinline__ void op_u1(cplx<R>* v, cptr<cplx<R>> M) {
  constexpr int NR = Regs<R>::NR;
  const cplx<R> m0 = cget(M, 0), m1 = cget(M, 1), m2 = cget(M, 2), m3 = cget(M, 3);
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (!((r >> B) & 1)) {
      const cplx<R> a0 = v[r], a1 = v[r | (1 << B)];
      v[r] = cfma(cmul(m0, a0), m1, a1);
      v[r | (1 << B)] = cfma(cmul(m2, a0), m3, a1);
    }
}

template <int B0, int B1, typename R>
__device__ __forceinline__ void op_u2(cplx<R>* v, cptr<cplx<R>> M) {
  constexpr int NR = Regs<R>::NR;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (!((r >> B0) & 1) && !((r >> B1) & 1)) {
      const int i[4] = {r, r | (1 << B1), r | (1 << B0), r | (1 << B0) | (1 << B1)};
      const cplx<R> x0 = v[i[0]], x1 = v[i[1]], x2 = v[i[2]], x3 = v[i[3]];
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        cplx<R> y = cmul(cget(M, 4 * o), x0);
        y = cfma(y, cget(M, 4 * o + 1), x1);
        y = cfma(y, cget(M, 4 * o + 2), x2);
        y = cfma(y, cget(M, 4 * o + 3), x3);
        v[i[o]] = y;
      }
    }
}

// Real 2x2 (H, RY): two real scalars per output, 4 multiply-adds per amplitude.
template <int B, typename R>
__device__ __forceinline__ void op_ur(cplx<R>* v, cptr<cplx<R>> M) {
  constexpr int NR = Regs<R>::NR;
  const R m0 = cget(M, 0).re, m1 = cget(M, 1).re, m2 = cget(M, 2).re, m3 = cget(M, 3).re;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (!((r >> B) & 1)) {
      const cplx<R> a0 = v[r], a1 = v[r | (1 << B)];
      v[r] = cplx<R>{fma(m1, a1.re, m0 * a0.re), fma(m1, a1.im, m0 * a0.im)};
      v[r | (1 << B)] = cplx<R>{fma(m3, a1.re, m2 * a0.re), fma(m3, a1.im, m2 * a0.im)};
    }
}

// Real diagonal, imaginary off-diagonal (RX): (x + i y) * (i s) = -s y + i s x.
template <int B, typename R>
__device__ __forceinline__ void op_ui(cplx<R>* v, cptr<cplx<R>> M) {
  constexpr int NR = Regs<R>::NR;
  const R m0 = cget(M, 0).re, s1 = cget(M, 1).im, s2 = cget(M, 2).im, m3 = cget(M, 3).re;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (!((r >> B) & 1)) {
      const cplx<R> a0 = v[r], a1 = v[r | (1 << B)];
      v[r] = cplx<R>{fma(-s1, a1.im, m0 * a0.re), fma(s1, a1.re, m0 * a0.im)};
      v[r | (1 << B)] = cplx<R>{fma(-s2, a0.im, m3 * a1.re), fma(s2, a0.re, m3 * a1.im)};
    }
}

// Phase on the amplitudes whose register bit B is 1 (controlled phases).
template <int B, typename R>
__device__ __forceinline__ void op_p1(cplx<R>* v, cplx<R> p) {
  constexpr int NR = Regs<R>::NR;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if ((r >> B) & 1) v[r] = cmul(p, v[r]);
}

template <int B0, int B1, typename R>
__device__ __forceinline__ void op_p2(cplx<R>* v, cplx<R> p) {
  constexpr int NR = Regs<R>::NR;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (((r >> B0) & 1) && ((r >> B1) & 1)) v[r] = cmul(p, v[r]);
}

// Angle words of the phase ladder: fixed-point turns, summed modulo one turn.
template <typename R>
struct lp_word;
template <>
struct lp_word<float> {
  typedef uint32_t W;
  typedef int32_t S;
  static __device__ __forceinline__ cplx<float> phase(W t) {
    float s, c;
    sincospif((float)(S)t * 0x1p-31f, &s, &c);  // angle 2 pi t / 2^32, as (-1, 1] half turns
    return cplx<float>{c, s};
  }
};
template <>
struct lp_word<double> {
  typedef uint64_t W;
  typedef int64_t S;
  static __device__ __forceinline__ cplx<double> phase(W t) {
    double s, c;
    sincospi((double)(S)t * 0x1p-63, &s, &c);
    return cplx<double>{c, s};
  }
};

template <int B, typename R>
__device__ __forceinline__ void op_x(cplx<R>* v) {
  constexpr int NR = Regs<R>::NR;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (!((r >> B) & 1)) {
      const cplx<R> t = v[r];
      v[r] = v[r | (1 << B)];
      v[r | (1 << B)] = t;
    }
}

template <int BC, int BT, typename R>
__device__ __forceinline__ void op_cx(cplx<R>* v) {
  constexpr int NR = Regs<R>::NR;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (((r >> BC) & 1) && !((r >> BT) & 1)) {
      const cplx<R> t = v[r];
      v[r] = v[r | (1 << BT)];
      v[r | (1 << BT)] = t;
    }
}

template <int B, typename R>
__device__ __forceinline__ void op_d1(cplx<R>* v, const cplx<R>* M) {
  constexpr int NR = Regs<R>::NR;
  const cplx<R> d0 = M[0], d1 = M[1];
#pragma unroll
  for (int r = 0; r < NR; ++r) v[r] = cmul(((r >> B) & 1) ? d1 : d0, v[r]);
}

template <int B0, int B1, typename R>
__device__ __forceinline__ void op_d2(cplx<R>* v, cptr<cplx<R>> M) {
  constexpr int NR = Regs<R>::NR;
  const cplx<R> d[4] = {cget(M, 0), cget(M, 1), cget(M, 2), cget(M, 3)};
#pragma unroll
  for (int r = 0; r < NR; ++r) v[r] = cmul(d[(((r >> B0) & 1) << 1) | ((r >> B1) & 1)], v[r]);
}

// Dispatch on register bits; bit 4 exists only with 5 register bits (H5).
#define SV_PAIR_SWITCH(code, F, H5)                                                          \
  switch (code) {                                                                            \
    case 1: F(0, 1); break;   case 2: F(0, 2); break;   case 3: F(0, 3); break;             \
    case 8: F(1, 0); break;   case 10: F(1, 2); break;  case 11: F(1, 3); break;            \
    case 16: F(2, 0); break;  case 17: F(2, 1); break;  case 19: F(2, 3); break;            \
    case 24: F(3, 0); break;  case 25: F(3, 1); break;  case 26: F(3, 2); break;            \
    case 4: if constexpr (H5) F(0, 4); break;   case 12: if constexpr (H5) F(1, 4); break;  \
    case 20: if constexpr (H5) F(2, 4); break;  case 28: if constexpr (H5) F(3, 4); break;  \
    case 32: if constexpr (H5) F(4, 0); break;  case 33: if constexpr (H5) F(4, 1); break;  \
    case 34: if constexpr (H5) F(4, 2); break;  case 35: if constexpr (H5) F(4, 3); break;  \
    default: break;                                                                          \
  }
#define SV_BIT_SWITCH(b, F, H5)                                                              \
  switch (b) {                                                                               \
    case 0: F(0); break; case 1: F(1); break; case 2: F(2); break; case 3: F(3); break;     \
    case 4: if constexpr (H5) F(4); break;                                                   \
    default: break;                                                                          \
  }

// Sum of the local words (ladder layout) of the lane's set local bits.
template <typename R>
__device__ __forceinline__ typename lp_word<R>::W lp_local(cptr<typename lp_word<R>::W> words, uint32_t lsel) {
  typedef typename lp_word<R>::W W;
  // words in chunks of 8 (one scalar load each; the loop stays rolled so
  // that only one chunk is live in scalar registers)
  constexpr int CH = 8;
  static_assert(kPassLPLocalBits % CH == 0, "local words come in whole chunks");
  W t = 0;
#pragma unroll 1
  for (int c = 0; c < kPassLPLocalBits / CH; ++c, lsel >>= CH) {
#pragma unroll
    for (int b = 0; b < CH; ++b) {
      const W w = words[CH * c + b];
      t += ((lsel >> b) & 1) ? w : W(0);
    }
  }
  return t;
}

// Tile rows of a phase op (entries of the stage's row table).
__device__ __forceinline__ uint32_t op_rows(const PassOpDev& op) {
  if (op.type == POP_LP) return 1u;
  if (op.type == POP_QG) return 1u + __builtin_popcount(op.b0) + __builtin_popcountll(((uint64_t)op.pad << 32) | op.b1);
  return 0u;
}

// POP_LP: the phase of the lane's amplitudes whose register bit b0 is 1:
// the constant word, the row's tile sum (ts[0], the same in every lane) and
// the words of the lane's set local group bits (xg has zeros at the
// register positions).
template <typename R>
__device__ __forceinline__ cplx<R> lp_phase(const PassOpDev& op, cptr<cplx<R>> M, uint32_t xg,
                                            const typename lp_word<R>::W* ts) {
  typedef typename lp_word<R>::W W;
  const cptr<W> words = (cptr<W>)M;
  return lp_word<R>::phase(words[kPassLPConst] + ts[0] + lp_local<R>(words, xg & op.lmask));
}

// POP_QG: row 0 and the constant, then the rows of the local targets set in
// the lane (tile sum ts[k] plus the row's local words), then the tile-target
// rows (their tile sums are zero unless the target bit is set).
template <typename R>
__device__ __forceinline__ cplx<R> qg_phase(const PassOpDev& op, cptr<cplx<R>> M, uint32_t xg,
                                            const typename lp_word<R>::W* ts) {
  typedef typename lp_word<R>::W W;
  cptr<W> words = (cptr<W>)M;
  const uint32_t lsel = xg & op.lmask;
  W t = words[kPassLPConst] + ts[0] + lp_local<R>(words, lsel);
  uint32_t k = 1;
#pragma unroll 1
  for (uint32_t lt = op.b0; lt; lt &= lt - 1u, ++k) {
    words += kPassLPWords;
    const W h = ts[k] + lp_local<R>(words, lsel);
    t += ((xg >> __builtin_ctz(lt)) & 1u) ? h : W(0);
  }
  const uint32_t end = op_rows(op);
#pragma unroll 1
  for (; k < end; ++k) t += ts[k];
  return lp_word<R>::phase(t);
}

// Tile sums of the stage's phase-op rows into ts[] (all threads; ends with a
// barrier).  Each thread sums whole rows: its 34 tile words are independent
// loads, so they are in flight together.
template <typename R>
__device__ __forceinline__ void stage_rows(const PassStageDev& S, cptr<cplx<R>> mats, uint64_t base,
                                           typename lp_word<R>::W* ts) {
  typedef typename lp_word<R>::W W;
  const cptr<cplx<R>> sm = mats + S.mat_base;
  const cptr<uint32_t> rt = (cptr<uint32_t>)(sm + S.rows);
  for (uint32_t j = threadIdx.x; j < S.row_count; j += kBlock) {
    const uint32_t word = rt[4 * j], pred = rt[4 * j + 1];
    const uint64_t sel = base & (rt[4 * j + 2] | ((uint64_t)rt[4 * j + 3] << 32));
    const cptr<W> w = (cptr<W>)sm + word;
    W acc = 0;
#pragma unroll
    for (int i = 0; i < kPassLPTileBits; ++i) acc += ((sel >> i) & 1) ? w[i] : W(0);
    ts[j] = (pred == kPassNoSel || ((base >> pred) & 1)) ? acc : W(0);
  }
  __syncthreads();
}

// M points at the op's first matrix entry (the same address in every lane, so
// the entries come through scalar loads); `var` selects a variant per lane.
template <typename R, bool LP>
__device__ __forceinline__ void apply_op(const PassOpDev& op, cptr<cplx<R>> M, uint32_t var,
                                         cplx<R>* v, uint32_t xg, const typename lp_word<R>::W* ts) {
  const uint32_t pair = op.b0 * 8 + op.b1;
  constexpr bool H5 = Regs<R>::RB > 4;
  switch (op.type) {
    case POP_U1: {
#define F(B) op_u1<B>(v, M)
      SV_BIT_SWITCH(op.b0, F, H5)
#undef F
      break;
    }
    case POP_U2: {
#define F(A, B) op_u2<A, B>(v, M)
      SV_PAIR_SWITCH(pair, F, H5)
#undef F
      break;
    }
    case POP_X: {
#define F(B) op_x<B>(v)
      SV_BIT_SWITCH(op.b0, F, H5)
#undef F
      break;
    }
    case POP_CX: {
#define F(A, B) op_cx<A, B>(v)
      SV_PAIR_SWITCH(pair, F, H5)
#undef F
      break;
    }
    case POP_D1: {
      cplx<R> d[2] = {cget(M, 0), cget(M, 1)};
      if (op.sa != kPassNoSel) {  // two variants, picked per lane (value selects: the loads stay uniform)
        const cplx<R> e0 = cget(M, 2), e1 = cget(M, 3);
        d[0].re = var ? e0.re : d[0].re;
        d[0].im = var ? e0.im : d[0].im;
        d[1].re = var ? e1.re : d[1].re;
        d[1].im = var ? e1.im : d[1].im;
      }
#define F(B) op_d1<B>(v, d)
      SV_BIT_SWITCH(op.b0, F, H5)
#undef F
      break;
    }
    case POP_D2: {
#define F(A, B) op_d2<A, B>(v, M)
      SV_PAIR_SWITCH(pair, F, H5)
#undef F
      break;
    }
    case POP_UR: {
#define F(B) op_ur<B>(v, M)
      SV_BIT_SWITCH(op.b0, F, H5)
#undef F
      break;
    }
    case POP_UI: {
#define F(B) op_ui<B>(v, M)
      SV_BIT_SWITCH(op.b0, F, H5)
#undef F
      break;
    }
    case POP_P1:
    case POP_LP: {  // one phase per lane on the amplitudes whose bit b0 is 1
      cplx<R> p;
      if (LP && op.type == POP_LP) {
        p = lp_phase<R>(op, M, xg, ts);
      } else {
        p = cget(M, 0);
        if (op.sa != kPassNoSel) {  // two variants, picked per lane
          const cplx<R> p1 = cget(M, 1);
          p.re = var ? p1.re : p.re;
          p.im = var ? p1.im : p.im;
        }
      }
#define F(B) op_p1<B>(v, p)
      SV_BIT_SWITCH(op.b0, F, H5)
#undef F
      break;
    }
    case POP_P2: {
      const cplx<R> p = cget(M, 0);
#define F(A, B) op_p2<A, B>(v, p)
      SV_PAIR_SWITCH(pair, F, H5)
#undef F
      break;
    }
    case POP_DR: {
#pragma unroll
      for (int r = 0; r < Regs<R>::NR; ++r) v[r] = cmul(cget(M, r), v[r]);
      break;
    }
    case POP_QG: {
      if constexpr (LP) {
        const cplx<R> p = qg_phase<R>(op, M, xg, ts);
#pragma unroll
        for (int r = 0; r < Regs<R>::NR; ++r) v[r] = cmul(p, v[r]);
      }
      break;
    }
    case POP_DG: {
      cplx<R> p = cget(M, 0);
      if (op.sa != kPassNoSel) {
        const cplx<R> p1 = cget(M, 1);
        if (op.sb != kPassNoSel) {
          const cplx<R> p2 = cget(M, 2), p3 = cget(M, 3);
          // two-level select on the variant bits (kept as selects, not a table)
          const bool hi = (var >> 1) & 1u, lo = var & 1u;
          const R re0 = lo ? p1.re : p.re, im0 = lo ? p1.im : p.im;
          const R re1 = lo ? p3.re : p2.re, im1 = lo ? p3.im : p2.im;
          p.re = hi ? re1 : re0;
          p.im = hi ? im1 : im0;
        } else if (var) {
          p = p1;
        }
      }
#pragma unroll
      for (int r = 0; r < Regs<R>::NR; ++r) v[r] = cmul(p, v[r]);
      break;
    }
    default:
      break;
  }
}

// Global memory is moved in 16-byte elements: one complex128 amplitude, or a
// pair of complex64 amplitudes whose local bit 0 (always physical bit 0: the
// low bits are pinned) lies inside the element.
template <typename R>
struct gelem;
template <>
struct gelem<double> {
  typedef dbl2 G;
  static constexpr int LB = 0;  // local bits inside one element
};
template <>
struct gelem<float> {
  typedef flt4 G;
  static constexpr int LB = 1;
};

// Uniform physical offsets of the per-lane element counter: bit b of the
// counter is local bit LB + 8 + b; h[0..3] cover a batch of 16, the rest the
// batch number.
struct PassOffsets {
  uint64_t in[4], out[4];
};

template <int LB>
__device__ __forceinline__ void pass_offsets(cptr<PassDescDev> P, PassOffsets* po) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t l = LB + 8 + b;
    po->in[b] = l < P->m ? 1ull << P->lpos[l] : 0ull;
    po->out[b] = l < P->m ? 1ull << P->wpos[l] : 0ull;
  }
}

template <int U>
__device__ __forceinline__ uint64_t batch_bits(const uint64_t* h) {
  return ((U & 1) ? h[0] : 0ull) | ((U & 2) ? h[1] : 0ull) | ((U & 4) ? h[2] : 0ull) | ((U & 8) ? h[3] : 0ull);
}

template <int U>
__device__ __forceinline__ uint32_t batch_bits32(const uint32_t* h) {
  return ((U & 1) ? h[0] : 0u) | ((U & 2) ? h[1] : 0u) | ((U & 4) ? h[2] : 0u) | ((U & 8) ? h[3] : 0u);
}

// Everything a lane needs to move one tile: the pass, the state, the tile's
// base index and the uniform offsets of its element counter.
template <typename R>
struct TileRef {
  typename dev_elem<R>::E* psi;
  cptr<PassDescDev> P;
  cptr<PassStageDev> stages;
  cptr<PassOpDev> ops;
  cptr<cplx<R>> mats;
  uint64_t base;
};

template <typename R>
__device__ __forceinline__ TileRef<R> tile_ref(typename dev_elem<R>::E* psi, int n, cptr<PassDescDev> P,
                                               cptr<PassStageDev> stages, cptr<PassOpDev> ops,
                                               cptr<cplx<R>> mats, uint64_t tile_id) {
  TileRef<R> r;
  r.psi = uniform_ptr(psi);
  r.P = uniform_ptr(P);
  r.stages = uniform_ptr(stages);
  r.ops = uniform_ptr(ops);
  r.mats = uniform_ptr(mats);
  r.base = uniform64(deposit(tile_id, ((1ull << n) - 1ull) & ~r.P->lmask));
  return r;
}

constexpr int kBatch = 16;  // 16-byte loads in flight per lane

// Lane geometry of a tile: element e = t + 256 j holds local index
// x = e << LB; local bits LB .. LB+7 come from the lane, the rest from j.
struct LaneGeo {
  uint32_t per;
  bool on;
};

template <int LB>
__device__ __forceinline__ LaneGeo lane_geo(uint32_t m) {
  const uint32_t elems = (1u << m) >> LB;
  return {elems >= (uint32_t)kBlock ? elems / kBlock : 1u, threadIdx.x < elems};
}

template <int LB>
__device__ __forceinline__ uint64_t lane_bits(cptr<uint32_t> pos, uint32_t m) {
  uint64_t r = 0;
  for (uint32_t j = 0; j < 8 && LB + j < m; ++j)
    if ((threadIdx.x >> j) & 1u) r |= 1ull << pos[LB + j];
  return r;
}

// Issue the loads of the whole tile into buf (no wait).
template <typename R>
__device__ __forceinline__ void tile_load(const TileRef<R>& T, typename gelem<R>::G* buf) {
  typedef typename gelem<R>::G G;
  constexpr int LB = gelem<R>::LB;
  const cptr<PassDescDev> P = T.P;
  const LaneGeo lg = lane_geo<LB>(P->m);
  const gptr<const G> gpsi = as_global(reinterpret_cast<const G*>(T.psi));
  const uint64_t a0 = T.base | lane_bits<LB>(P->lpos, P->m);
  PassOffsets po;
  pass_offsets<LB>(P, &po);
  // unpredicated: elements past the tile (small tiles) re-read the tile base,
  // so the loads need no branches (and no waits between them)
#define SV_LD(U)                                                                        \
  {                                                                                     \
    const uint64_t ad = (U < lg.per && lg.on) ? (a0 | batch_bits<U>(po.in)) : T.base;  \
    buf[U] = ldg<G>(gpsi + (ad >> LB));                                                 \
  }
  SV_LD(0) SV_LD(1) SV_LD(2) SV_LD(3) SV_LD(4) SV_LD(5) SV_LD(6) SV_LD(7)
  SV_LD(8) SV_LD(9) SV_LD(10) SV_LD(11) SV_LD(12) SV_LD(13) SV_LD(14) SV_LD(15)
#undef SV_LD
}

template <typename R, int WB>
__device__ __forceinline__ void batch_to_lds(const typename gelem<R>::G* buf, uint32_t j0, const LaneGeo& lg,
                                             typename dev_elem<R>::E* tile) {
  typedef typename dev_elem<R>::E E;
  constexpr int LB = gelem<R>::LB;
#pragma unroll
  for (int u = 0; u < kBatch; ++u)
    if (j0 + u < lg.per && lg.on) {
      const uint32_t x = (threadIdx.x + (j0 + u) * kBlock) << LB;
      if constexpr (LB == 1) {
        tile[swz<WB>(x)] = E{buf[u].x, buf[u].y};
        tile[swz<WB>(x | 1u)] = E{buf[u].z, buf[u].w};
      } else {
        tile[swz<WB>(x)] = buf[u];
      }
    }
}

// Write the loaded tile (at most 16 elements per lane: 64 KiB tiles) to LDS.
template <typename R, int WB>
__device__ __forceinline__ void tile_fill(const TileRef<R>& T, const typename gelem<R>::G* buf,
                                          typename dev_elem<R>::E* tile) {
  const LaneGeo lg = lane_geo<gelem<R>::LB>(T.P->m);
  batch_to_lds<R, WB>(buf, 0, lg, tile);
}

// The pass's register stages on the tile in LDS (ends with a barrier).
template <typename R, int WB, bool LP>
__device__ __forceinline__ void tile_stages(const TileRef<R>& T, typename dev_elem<R>::E* tile) {
  typedef typename dev_elem<R>::E E;
  const cptr<PassDescDev> P = T.P;
  const cptr<PassStageDev> stages = T.stages;
  const cptr<PassOpDev> ops = T.ops;
  const cptr<cplx<R>> mats = T.mats;
  const uint64_t base = T.base;
  const uint32_t size = 1u << P->m;
  const uint32_t t = threadIdx.x;
  constexpr int RB = Regs<R>::RB, NR = Regs<R>::NR;
  typedef typename lp_word<R>::W W;
  __shared__ W tsum[LP ? kPassStageRowsMax : 1];  // tile sums of the stage's phase-op rows
  for (uint32_t si = 0; si < P->stage_count; ++si) {
    const PassStageDev S = cload(stages + (P->stage_first + si));
    if constexpr (LP) {
      if (S.row_count) stage_rows<R>(S, mats, base, tsum);
    }
    const uint32_t groups = size >> RB;
    // swz is linear over XOR and xg shares no bit with a register offset, so
    // swz(xg | off) = swz(xg) ^ (XOR of swz(bit) over the offset's bits): only
    // the swizzled register bits are kept, not one offset per register
    uint32_t sbit[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) sbit[b] = swz<WB>(1u << S.q[b]);
    for (uint32_t gi = t; gi < groups; gi += kBlock) {
      uint32_t xg = gi;
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const uint32_t q = S.qsort[b];
        xg = ((xg >> q) << (q + 1)) | (xg & ((1u << q) - 1u));
      }
      const uint32_t sx = swz<WB>(xg);
      cplx<R> v[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        uint32_t o = sx;
#pragma unroll
        for (int b = 0; b < RB; ++b)
          if ((r >> b) & 1) o ^= sbit[b];
        const E e = tile[o];
        v[r] = cplx<R>{e.x, e.y};
      }
      uint32_t row = 0;  // the op's first row in tsum
      for (uint32_t o = 0; o < S.op_count; ++o) {
        const PassOpDev op = cload(ops + (S.op_first + o));
        if (!(LP && (op.type == POP_LP || op.type == POP_QG)) &&
            ((xg & op.lmask) != op.lmask || (base & op.tmask) != op.tmask))
          continue;
        uint32_t var = 0;
        if (op.sa != kPassNoSel) {
          var = op.sa < kPassTileSel ? (xg >> op.sa) & 1u : (uint32_t)(base >> (op.sa - kPassTileSel)) & 1u;
          if (op.sb != kPassNoSel)
            var = (var << 1) |
                  (op.sb < kPassTileSel ? (xg >> op.sb) & 1u : (uint32_t)(base >> (op.sb - kPassTileSel)) & 1u);
        }
        apply_op<R, LP>(op, mats + op.mat, var, v, xg, tsum + row);
        if constexpr (LP) row += op_rows(op);
      }
      // The store recomputes the offsets from opaque copies of the inputs, so
      // the compiler cannot keep the load's NR offsets live across the ops
      // (they would take NR scalar registers and push the kernel into spills).
      uint32_t sxs = sx;
      asm volatile("" : "+v"(sxs));
#pragma unroll
      for (int b = 0; b < RB; ++b) asm volatile("" : "+s"(sbit[b]));
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        E e;
        e.x = v[r].re;
        e.y = v[r].im;
        uint32_t o = sxs;
#pragma unroll
        for (int b = 0; b < RB; ++b)
          if ((r >> b) & 1) o ^= sbit[b];
        tile[o] = e;
      }
    }
    __syncthreads();
  }

}

// Store the tile: local bit j goes to physical position wpos[j], a
// permutation of the positions the tile was loaded from.  When the lowest
// element bits keep their positions lanes walk the tile in load order;
// otherwise they walk the destination addresses in the load's order (the
// same coalesced runs and 16-byte elements whatever the permutation) and
// gather each element from LDS: the element's k-th address bit holds local
// bit winv[k].
template <typename R, int WB>
__device__ __forceinline__ void tile_store(const TileRef<R>& T, const typename dev_elem<R>::E* tile) {
  typedef typename dev_elem<R>::E E;
  typedef typename gelem<R>::G G;
  constexpr int LB = gelem<R>::LB;
  const cptr<PassDescDev> P = T.P;
  const uint32_t m = P->m;
  const LaneGeo lg = lane_geo<LB>(m);
  const gptr<G> gpsi = as_global(reinterpret_cast<G*>(T.psi));
  const uint64_t a0 = T.base | lane_bits<LB>(P->lpos, m);
  PassOffsets po;
  pass_offsets<LB>(P, &po);
  if (P->flags & kPassStoreLaneOrder) {  // load order: the low element bits stay in place
    const uint64_t w0 = T.base | lane_bits<LB>(P->wpos, m);
#define SV_ST(U)                                                                       \
    if (U < lg.per && lg.on) {                                                         \
      const uint32_t x = (threadIdx.x + U * kBlock) << LB;                             \
      G g;                                                                             \
      if constexpr (LB == 1) {                                                         \
        const E e0 = tile[swz<WB>(x)], e1 = tile[swz<WB>(x | 1u)];                     \
        g = G{e0.x, e0.y, e1.x, e1.y};                                                 \
      } else {                                                                         \
        g = tile[swz<WB>(x)];                                                          \
      }                                                                                \
      stg<G>(gpsi + ((w0 | batch_bits<U>(po.out)) >> LB), g);                          \
    }
    SV_ST(0) SV_ST(1) SV_ST(2) SV_ST(3) SV_ST(4) SV_ST(5) SV_ST(6) SV_ST(7)
    SV_ST(8) SV_ST(9) SV_ST(10) SV_ST(11) SV_ST(12) SV_ST(13) SV_ST(14) SV_ST(15)
#undef SV_ST
    return;
  }
  // LDS index of the lane's element: lane bit j is address bit LB + j
  uint32_t xl = 0;
  for (uint32_t jb = 0; jb < 8 && LB + jb < m; ++jb)
    if ((threadIdx.x >> jb) & 1u) xl |= 1u << P->winv[LB + jb];
  uint32_t xo[4];  // LDS offsets of the batch bits
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t k = LB + 8 + b;
    xo[b] = k < m ? 1u << P->winv[k] : 0u;
  }
  const uint32_t xp = LB ? 1u << P->winv[0] : 0u;  // the element's second amplitude (complex64)
#define SV_ST(U)                                                                       \
  if (U < lg.per && lg.on) {                                                           \
    const uint32_t x = xl | batch_bits32<U>(xo);                                       \
    G g;                                                                               \
    if constexpr (LB == 1) {                                                           \
      const E e0 = tile[swz<WB>(x)], e1 = tile[swz<WB>(x | xp)];                       \
      g = G{e0.x, e0.y, e1.x, e1.y};                                                   \
    } else {                                                                           \
      g = tile[swz<WB>(x)];                                                            \
    }                                                                                  \
    stg<G>(gpsi + ((a0 | batch_bits<U>(po.in)) >> LB), g);                             \
  }
  SV_ST(0) SV_ST(1) SV_ST(2) SV_ST(3) SV_ST(4) SV_ST(5) SV_ST(6) SV_ST(7)
  SV_ST(8) SV_ST(9) SV_ST(10) SV_ST(11) SV_ST(12) SV_ST(13) SV_ST(14) SV_ST(15)
#undef SV_ST
}

// Persistent loop over tiles, software-pipelined: the next tile's loads are
// in flight while the current tile runs its stages and is stored.  `next`
// maps a global tile number to its TileRef.
template <typename R, int WB, bool LP, typename Src>
__device__ __forceinline__ void tile_loop(uint64_t total, const Src& src, typename dev_elem<R>::E* tile) {
  typedef typename gelem<R>::G G;
  uint64_t g = xcd_block();
  if (g >= total) return;
  G buf[kBatch];
  tile_load<R>(src(g), buf);
  while (true) {
    const uint64_t ng = g + gridDim.x;
    const TileRef<R> cur = src(g);  // recomputed, not carried: fewer live registers
    __syncthreads();  // the previous tile's store has read the buffer
    tile_fill<R, WB>(cur, buf, tile);
    __syncthreads();
    if (ng < total) tile_load<R>(src(ng), buf);
    tile_stages<R, WB, LP>(cur, tile);
    tile_store<R, WB>(cur, tile);
    if (ng >= total) break;
    g = ng;
  }
}

template <typename R>
struct SingleSrc {
  typename dev_elem<R>::E* psi;
  int n;
  cptr<PassDescDev> P;
  cptr<PassStageDev> stages;
  cptr<PassOpDev> ops;
  cptr<cplx<R>> mats;
  __device__ __forceinline__ TileRef<R> operator()(uint64_t g) const {
    return tile_ref<R>(psi, n, P, stages, ops, mats, g);
  }
};

template <typename R, int WB, bool LP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_pass(typename dev_elem<R>::E* __restrict__ psi, int n,
                                                 const PassDescDev* __restrict__ passes, int pi,
                                                 const PassStageDev* __restrict__ stages,
                                                 const PassOpDev* __restrict__ ops,
                                                 const cplx<R>* __restrict__ mats) {
  typedef typename dev_elem<R>::E E;
  extern __shared__ __align__(16) unsigned char smem[];
  E* tile = reinterpret_cast<E*>(smem);
  const cptr<PassDescDev> P = as_const(passes + pi);
  const SingleSrc<R> src{psi, n, P, as_const(stages), as_const(ops), as_const(mats)};
  tile_loop<R, WB, LP>(1ull << (n - P->m), src, tile);
}

// Many states in one launch: work item i runs pass `pass` of its own program
// over its own tiles; global tile g belongs to the item whose [tile_begin,
// tile_begin + tiles) range holds g.  No item reads another's state, so each
// result is independent of the batch it ran in.
template <typename R>
struct BatchSrc {
  cptr<BatchItemDev> items;
  int count;
  __device__ __forceinline__ TileRef<R> operator()(uint64_t g) const {
    int lo = 0, hi = count - 1;  // last item with tile_begin <= g
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].tile_begin <= g) lo = mid;
      else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);  // the same in every lane
    const cptr<BatchItemDev> it = items + lo;  // fields read one by one: scalar loads
    return tile_ref<R>((typename dev_elem<R>::E*)it->psi, it->n, as_const(it->passes + it->pass),
                       as_const(it->stages), as_const(it->ops), as_const((const cplx<R>*)it->mats),
                       g - it->tile_begin);
  }
};

template <typename R, int WB, bool LP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_pass_batch(const BatchItemDev* __restrict__ items, int count,
                                                       uint64_t total_tiles) {
  typedef typename dev_elem<R>::E E;
  extern __shared__ __align__(16) unsigned char smem[];
  E* tile = reinterpret_cast<E*>(smem);
  const BatchSrc<R> src{as_const(items), count};
  tile_loop<R, WB, LP>(total_tiles, src, tile);
}

// Blocks that fit on the device at once for `kernel` with `lds` bytes of
// dynamic LDS (the persistent grid of the pipelined tile loop).
template <typename F>
uint64_t resident_blocks(F kernel, size_t lds, uint64_t* cache) {
  int nb = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, lds) != hipSuccess || nb < 1) nb = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  *cache = (uint64_t)nb * (uint64_t)cus;
  return *cache;
}

template <typename R, int WB, bool LP>
hipError_t run(void* psi, int n, int m, const PassDescDev* passes, int pass, const PassStageDev* stages,
               const PassOpDev* ops, const void* mats, hipStream_t s) {
  typedef typename dev_elem<R>::E E;
  const size_t lds = ((size_t)1 << m) * sizeof(E);
  static size_t attr = 0;            // largest dynamic LDS size requested so far
  static uint64_t resident[17] = {};  // per tile size
  if (lds > attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_pass<R, WB, LP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = lds;
  }
  if (!resident[m]) resident_blocks(k_pass<R, WB, LP>, lds, &resident[m]);
  const uint64_t tiles = 1ull << (n - m);
  const uint64_t blocks = tiles < resident[m] ? tiles : resident[m];
  hipLaunchKernelGGL((k_pass<R, WB, LP>), dim3((unsigned)blocks), dim3(kBlock), lds, s, (E*)psi, n, passes, pass, stages,
                     ops, (const cplx<R>*)mats);
  return hipGetLastError();
}

template <typename R, int WB, bool LP>
hipError_t run_batch(const BatchItemDev* items, int count, uint64_t total_tiles, int max_m, hipStream_t s) {
  typedef typename dev_elem<R>::E E;
  const size_t lds = ((size_t)1 << max_m) * sizeof(E);
  static size_t attr = 0;
  static uint64_t resident[17] = {};
  if (lds > attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_pass_batch<R, WB, LP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = lds;
  }
  if (total_tiles == 0) return hipSuccess;
  if (!resident[max_m]) resident_blocks(k_pass_batch<R, WB, LP>, lds, &resident[max_m]);
  const uint64_t blocks = total_tiles < resident[max_m] ? total_tiles : resident[max_m];
  hipLaunchKernelGGL((k_pass_batch<R, WB, LP>), dim3((unsigned)blocks), dim3(kBlock), lds, s, items, count, total_tiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pass(sv_dtype dt, void* psi, int n, int m, const PassDescDev* passes, int pass,
                       const PassStageDev* stages, const PassOpDev* ops, const void* mats, bool ladders,
                       hipStream_t s) {
  if (dt == SV_C128)
    return ladders ? run<double, 3, true>(psi, n, m, passes, pass, stages, ops, mats, s)
                   : run<double, 3, false>(psi, n, m, passes, pass, stages, ops, mats, s);
  return ladders ? run<float, 4, true>(psi, n, m, passes, pass, stages, ops, mats, s)
                 : run<float, 4, false>(psi, n, m, passes, pass, stages, ops, mats, s);
}

hipError_t launch_pass_batch(sv_dtype dt, const BatchItemDev* items, int count, uint64_t total_tiles, int max_m,
                             bool ladders, hipStream_t s) {
  if (dt == SV_C128)
    return ladders ? run_batch<double, 3, true>(items, count, total_tiles, max_m, s)
                   : run_batch<double, 3, false>(items, count, total_tiles, max_m, s);
  return ladders ? run_batch<float, 4, true>(items, count, total_tiles, max_m, s)
                 : run_batch<float, 4, false>(items, count, total_tiles, max_m, s);
}

}  // namespace sv
