// In-cache tile pass: the block-by-block all-in-cache execution of QueenV2
// (Sec. II-B "In-cache Operations", Sec. III-B) on gfx950 LDS.
//
// One block owns one tile of 2^m amplitudes: the indices that agree with the
// tile base on every non-local bit.  The tile is gathered from HBM with the
// PDEP-like deposit of its local index into the pass's local bit positions
// (Sec. III-B), so the low pinned positions give contiguous runs.  The pass's
// register stages then run in LDS: a stage gives each lane a group of 32
// (complex64) or 16 (complex128) amplitudes (5 or 4 local bits held in
// registers) and applies, as straight-line code with the bit positions
// fixed at compile time,
//   - the tensor product of one 2x2 per register bit (a layer of
//     single-qubit gates: the tensor product booster of Sec. III-A), in the
//     cheapest of four forms that holds all of them;
//   - a diagonal: one factor per register index, times per-lane factors for
//     the gates that involve bits outside the registers (a fused run of
//     phase gates, Sec. III-A, is a fixed-point phase function of the index
//     bits; its tile part is summed once per tile and stage);
//   - a permutation of the register index (X, CNOT, SWAP) at no cost: the
//     stage's LDS store writes each amplitude to its permuted address.
// The tile is written back with local bit j at physical position wpos[j],
// which fuses qubit reordering (Sec. II-B) into the store.
//
// LDS rows are 128 bytes; the element index is XOR-swizzled (low bits folded
// with every higher group of bits) so that power-of-two strides between the
// lanes of a wave fall into distinct banks.
#include <stddef.h>

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

// LDS index of local amplitude x.  Global memory moves 16-byte elements (LB
// amplitude bits inside one: 1 for complex64, 0 for complex128); the three
// element bits above them (one 128-byte row of LDS) are XORed with every
// higher group of three element bits, so that power-of-two strides between
// the lanes of a wave spread over the banks.  The map is linear over GF(2)
// and its own inverse, and keeps the amplitudes of one element together.
template <int LB>
__device__ __forceinline__ uint32_t swz(uint32_t x) {
  uint32_t y = x >> (LB + 3), h = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) h ^= y >> (3 * k);
  return x ^ ((h & 7u) << LB);
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

// Program memory (pass descriptors, stages, items, matrices, batch items) is
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

// ---- the 2x2 part: one gate per register bit, in the stage's form ----------
// Each applies the 2x2 at M[0..3] to every pair of register amplitudes that
// differ in bit B (Eq. 2 on the register bits).

// General complex 2x2: 8 multiply-adds per amplitude.
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

// Real 2x2 (H, RY): 4 per amplitude.
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

// Real diagonal, imaginary off-diagonal (RX, Y): (x + i y) * (i s) = -s y + i s x.
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

// Real diagonal, complex off-diagonal (a layer mixing the two kinds above): 6.
template <int B, typename R>
__device__ __forceinline__ void op_rc(cplx<R>* v, cptr<cplx<R>> M) {
  constexpr int NR = Regs<R>::NR;
  const R m0 = cget(M, 0).re, m3 = cget(M, 3).re;
  const cplx<R> m1 = cget(M, 1), m2 = cget(M, 2);
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (!((r >> B) & 1)) {
      const cplx<R> a0 = v[r], a1 = v[r | (1 << B)];
      cplx<R> o0 = cmul(m1, a1), o1 = cmul(m2, a0);
      o0.re = fma(m0, a0.re, o0.re);
      o0.im = fma(m0, a0.im, o0.im);
      o1.re = fma(m3, a1.re, o1.re);
      o1.im = fma(m3, a1.im, o1.im);
      v[r] = o0;
      v[r | (1 << B)] = o1;
    }
}

// Dense 4x4 on register bits (1 = most significant bit of its index, 0).
template <typename R>
__device__ __forceinline__ void op_u2(cplx<R>* v, cptr<cplx<R>> M) {
  constexpr int NR = Regs<R>::NR;
#pragma unroll
  for (int r = 0; r < NR; r += 4) {
    const cplx<R> x0 = v[r], x1 = v[r | 1], x2 = v[r | 2], x3 = v[r | 3];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      cplx<R> y = cmul(cget(M, 4 * o), x0);
      y = cfma(y, cget(M, 4 * o + 1), x1);
      y = cfma(y, cget(M, 4 * o + 2), x2);
      y = cfma(y, cget(M, 4 * o + 3), x3);
      v[r | o] = y;
    }
  }
}

// The tensor product of one 2x2 per register bit (4 entries per bit, bit 0
// first): bit B in its own form (three bits of `forms` each); bits without a
// gate are skipped.
template <int B, typename R>
__device__ __forceinline__ void slot(cplx<R>* v, cptr<cplx<R>> M, uint32_t forms) {
  const uint32_t f = pass_form_of(forms, B);
  if (f == PFORM_NONE) return;
  if (f == PFORM_UR) op_ur<B>(v, M + 4 * B);
  else if (f == PFORM_UI) op_ui<B>(v, M + 4 * B);
  else if (f == PFORM_RC) op_rc<B>(v, M + 4 * B);
  else op_u1<B>(v, M + 4 * B);
}
template <typename R>
__device__ __forceinline__ void layer(cplx<R>* v, cptr<cplx<R>> M, uint32_t forms) {
  slot<0>(v, M, forms);
  slot<1>(v, M, forms);
  slot<2>(v, M, forms);
  slot<3>(v, M, forms);
  if constexpr (Regs<R>::RB > 4) slot<4>(v, M, forms);
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

// Tile rows of a fixed-point item (entries of the stage's row table).
__device__ __forceinline__ uint32_t item_rows(const PassItemDev& it) {
  if (it.type == PIT_LP) return 1u;
  if (it.type == PIT_QG) return 1u + __builtin_popcount(it.a) + __builtin_popcountll(it.tt);
  return 0u;
}

// PIT_LP: the phase of the lane's amplitudes whose register bit `a` is 1:
// the constant word and the words of the lane's set local group bits (xg
// has zeros at the register positions) -- the lane's part, the same for
// every tile -- plus the row's tile sum (ts[0], the same in every lane).
template <typename R>
__device__ __forceinline__ typename lp_word<R>::W lp_lane_part(const PassItemDev& it, cptr<cplx<R>> M, uint32_t xg) {
  typedef typename lp_word<R>::W W;
  const cptr<W> words = (cptr<W>)M;
  return words[kPassLPConst] + lp_local<R>(words, xg & it.lmask);
}

// PIT_QG: row 0 and the constant, then the rows of the local targets set in
// the lane, then the tile-target rows (their tile sums are zero unless the
// target bit is set).  The lane's part is the constant and the local words
// of row 0 and of the set local targets' rows; the tile part is the tile
// sums of row 0, of those rows and of the tile-target rows.
template <typename R>
__device__ __forceinline__ typename lp_word<R>::W qg_lane_part(const PassItemDev& it, cptr<cplx<R>> M, uint32_t xg) {
  typedef typename lp_word<R>::W W;
  cptr<W> words = (cptr<W>)M;
  const uint32_t lsel = xg & it.lmask;
  W t = words[kPassLPConst] + lp_local<R>(words, lsel);
#pragma unroll 1
  for (uint32_t lt = it.a; lt; lt &= lt - 1u) {
    words += kPassLPWords;
    const W h = lp_local<R>(words, lsel);
    t += ((xg >> __builtin_ctz(lt)) & 1u) ? h : W(0);
  }
  return t;
}
template <typename R>
__device__ __forceinline__ typename lp_word<R>::W qg_tile_part(const PassItemDev& it, uint32_t xg,
                                                                const typename lp_word<R>::W* ts) {
  typedef typename lp_word<R>::W W;
  W t = ts[0];
  uint32_t k = 1;
#pragma unroll 1
  for (uint32_t lt = it.a; lt; lt &= lt - 1u, ++k) t += ((xg >> __builtin_ctz(lt)) & 1u) ? ts[k] : W(0);
  const uint32_t end = item_rows(it);
#pragma unroll 1
  for (; k < end; ++k) t += ts[k];
  return t;
}

// Fixed-point phase items whose lane parts a block computes once, before its
// tiles (k_pass): pre[k][t] holds the lane part of the pass's k-th such item
// for thread t.  Later items compute theirs per tile.
template <typename R>
struct pre_cap {
  static constexpr int N = sizeof(R) == 4 ? 14 : 6;
};

// Tile sums of the stage's fixed-point rows into ts[] (all threads; ends
// with a barrier).  Each thread sums whole rows: its 34 tile words are
// independent loads, so they are in flight together.
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
    ts[j] = (pred == kPassRowAlways || ((base >> pred) & 1)) ? acc : W(0);
  }
  lds_sync();
}

// Value of selector code c for the lane: local bit c of its group index, or
// tile physical bit c - 64 of the tile base.
__device__ __forceinline__ uint32_t sel_bit(uint32_t c, uint32_t xg, uint64_t base) {
  return c < kPassTileSel ? (xg >> c) & 1u : (uint32_t)(base >> (c - kPassTileSel)) & 1u;
}
__device__ __forceinline__ uint32_t item_var(uint32_t sel, uint32_t xg, uint64_t base) {
  const uint32_t a = sel & 0xffu, b = (sel >> 8) & 0xffu;
  uint32_t var = a == kPassNoSel ? 0u : sel_bit(a, xg, base);
  if (b != kPassNoSel) var = (var << 1) | sel_bit(b, xg, base);
  return var;
}

// Entry `var` of a table of n <= 4 entries, loaded uniformly (scalar loads)
// and selected per lane.
template <typename R>
__device__ __forceinline__ cplx<R> pick(cptr<cplx<R>> T, uint32_t var, int n) {
  cplx<R> x = cget(T, 0);
  if (n > 1) {
    const cplx<R> y = cget(T, 1);
    x.re = (var & 1u) ? y.re : x.re;
    x.im = (var & 1u) ? y.im : x.im;
  }
  if (n > 2) {
    const cplx<R> z = cget(T, 2), w = cget(T, 3);
    const R zr = (var & 1u) ? w.re : z.re, zi = (var & 1u) ? w.im : z.im;
    x.re = (var & 2u) ? zr : x.re;
    x.im = (var & 2u) ? zi : x.im;
  }
  return x;
}

// The diagonal part with lane items: per lane a factor G on all amplitudes
// and, per register bit a, factors f0[a] / f1[a] on the amplitudes whose bit
// a is 0 / 1; amplitude r is multiplied by G * prod_a f_{r_a}[a] * dr[r].
template <typename R, bool LP>
__device__ __forceinline__ void lane_diag(const PassStageDev& S, cptr<PassItemDev> items, cptr<cplx<R>> mats,
                                          uint32_t xg, uint64_t base, const typename lp_word<R>::W* ts,
                                          const typename lp_word<R>::W* pre, uint32_t npre, uint32_t* kfix,
                                          cplx<R>* v) {
  typedef typename lp_word<R>::W W;
  constexpr int RB = Regs<R>::RB, NR = Regs<R>::NR, HALF = NR / 2;
  const cplx<R> one = {R(1), R(0)};
  cplx<R> G = one, f0[RB], f1[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) f0[b] = f1[b] = one;
  uint32_t row = 0;  // the item's first row in ts
  for (uint32_t i = 0; i < S.item_count; ++i) {
    const PassItemDev it = cload(items + (S.item_first + i));
    const cptr<cplx<R>> T = mats + it.mat;
    if (it.type == PIT_DG) {
      const uint32_t sb = (it.sel >> 8) & 0xffu;
      G = cmul(G, pick<R>(T, item_var(it.sel, xg, base), sb == kPassNoSel ? 2 : 4));
    } else if (it.type == PIT_D1) {
      const uint32_t var = item_var(it.sel, xg, base);
      const cplx<R> e0 = pick<R>(T, var << 1, 4), e1 = pick<R>(T, (var << 1) | 1u, 4);
#pragma unroll
      for (int b = 0; b < RB; ++b)
        if (it.a == (uint32_t)b) {
          f0[b] = cmul(f0[b], e0);
          f1[b] = cmul(f1[b], e1);
        }
    } else if (LP && it.type == PIT_LP) {
      const W lane = *kfix < npre ? pre[*kfix * kBlock + threadIdx.x] : lp_lane_part<R>(it, T, xg);
      ++*kfix;
      const cplx<R> p = lp_word<R>::phase(lane + ts[row]);
#pragma unroll
      for (int b = 0; b < RB; ++b)
        if (it.a == (uint32_t)b) f1[b] = cmul(f1[b], p);
      row += 1;
    } else if (LP && it.type == PIT_QG) {
      const W lane = *kfix < npre ? pre[*kfix * kBlock + threadIdx.x] : qg_lane_part<R>(it, T, xg);
      ++*kfix;
      G = cmul(G, lp_word<R>::phase(lane + qg_tile_part<R>(it, xg, ts + row)));
      row += item_rows(it);
    }
  }
  // factors of the register index over the bits below the top one, by doubling
  cplx<R> H[HALF];
  H[0] = G;
  if (S.flags & PSF_F0) {
#pragma unroll
    for (int a = 0; a < RB - 1; ++a)
#pragma unroll
      for (int k = 0; k < (1 << a); ++k) {
        H[k | (1 << a)] = cmul(H[k], f1[a]);
        H[k] = cmul(H[k], f0[a]);
      }
  } else {
#pragma unroll
    for (int a = 0; a < RB - 1; ++a)
#pragma unroll
      for (int k = 0; k < (1 << a); ++k) H[k | (1 << a)] = cmul(H[k], f1[a]);
  }
  const cptr<cplx<R>> D = mats + S.dr;
#pragma unroll
  for (int r = 0; r < HALF; ++r) {
    const cplx<R> lo = cmul(cmul(H[r], f0[RB - 1]), cget(D, r));
    const cplx<R> hi = cmul(cmul(H[r], f1[RB - 1]), cget(D, r + HALF));
    v[r] = cmul(lo, v[r]);
    v[r + HALF] = cmul(hi, v[r + HALF]);
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

// Everything a lane needs to move one tile: the pass, the state and the
// tile's base index.
template <typename R>
struct TileRef {
  typename dev_elem<R>::E* psi;
  cptr<PassDescDev> P;
  cptr<PassStageDev> stages;
  cptr<PassItemDev> items;
  cptr<cplx<R>> mats;
  uint64_t base;
};

template <typename R>
__device__ __forceinline__ TileRef<R> tile_ref(typename dev_elem<R>::E* psi, int n, cptr<PassDescDev> P,
                                               cptr<PassStageDev> stages, cptr<PassItemDev> items,
                                               cptr<cplx<R>> mats, uint64_t tile_id) {
  TileRef<R> r;
  r.psi = uniform_ptr(psi);
  r.P = uniform_ptr(P);
  r.stages = uniform_ptr(stages);
  r.items = uniform_ptr(items);
  r.mats = uniform_ptr(mats);
  r.base = uniform64(deposit(tile_id, ((1ull << n) - 1ull) & ~r.P->lmask));
  return r;
}

constexpr int kBatch = 16;  // 16-byte elements per lane: 64 KiB tiles

// Thread geometry of a block of NT threads moving a 64 KiB tile (4096
// 16-byte elements): TB lane bits, BATCH elements per lane (UB bits).
template <int NT>
struct TileThreads {
  static_assert(NT == 256 || NT == 512, "256 or 512 threads");
  static constexpr int TB = NT == 512 ? 9 : 8;
  static constexpr int BATCH = 4096 / NT;
  static constexpr int UB = 12 - TB;
};

// Lane geometry of a tile: LDS element slot e = t + NT u (u < per) of lane t.
struct LaneGeo {
  uint32_t per;
  bool on;
};

template <int LB, int NT = kBlock>
__device__ __forceinline__ LaneGeo lane_geo(uint32_t m) {
  const uint32_t elems = (1u << m) >> LB;
  return {elems >= (uint32_t)NT ? elems / NT : 1u, threadIdx.x < elems};
}

// Physical offset of element slot bit i when the load fills slot e with tile
// element swz(e) (amplitude index swz(e) << LB): the swizzle is linear, so
// the address of a slot is the XOR of the offsets of its set bits.  pos =
// local bit positions (lpos for the load).
template <int LB>
__device__ __forceinline__ uint64_t slot_offset(cptr<uint32_t> pos, uint32_t m, uint32_t i) {
  if (LB + i >= m) return 0ull;
  uint64_t o = 1ull << pos[LB + i];
  if (i >= 3) o ^= 1ull << pos[LB + (i - 3) % 3];
  return o;
}

// Offsets of the slot bits a lane owns (bits 0..TB-1 of its slot index).
template <int LB, int NT = kBlock>
__device__ __forceinline__ uint64_t lane_slot_bits(cptr<uint32_t> pos, uint32_t m) {
  uint64_t r = 0;
  for (uint32_t j = 0; j < (uint32_t)TileThreads<NT>::TB; ++j)
    if ((threadIdx.x >> j) & 1u) r ^= slot_offset<LB>(pos, m, j);
  return r;
}

// Issue the tile's loads straight into LDS (global_load_lds_dwordx4): slot e
// of the tile receives tile element swz(e), so the tile lands in LDS in its
// swizzled layout without passing through registers.  Each instruction of a
// wave writes 1 KiB of consecutive slots; its 64 lanes read whole 128-byte
// lines (the swizzle permutes elements within a line).  No wait.
template <typename R>
__device__ __forceinline__ void tile_load_lds(const TileRef<R>& T, typename dev_elem<R>::E* tile) {
  typedef typename gelem<R>::G G;
  constexpr int LB = gelem<R>::LB;
  const cptr<PassDescDev> P = T.P;
  const uint32_t m = P->m;
  const LaneGeo lg = lane_geo<LB>(m);
  const gptr<const G> gpsi = as_global(reinterpret_cast<const G*>(T.psi));
  const uint64_t a0 = T.base | lane_slot_bits<LB>(P->lpos, m);
  uint64_t hb[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) hb[b] = slot_offset<LB>(P->lpos, m, 8 + b);
  // the wave's first slot of instruction u: uniform (the LDS destination of
  // the instruction is wave-uniform; lanes land at consecutive 16 bytes)
  const uint32_t wslot = (threadIdx.x & ~63u);
  __attribute__((address_space(3))) G* lds = (__attribute__((address_space(3))) G*)tile;
#pragma unroll
  for (int u = 0; u < kBatch; ++u)
    if ((uint32_t)u < lg.per && lg.on) {
      uint64_t ad = a0;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if ((u >> b) & 1) ad ^= hb[b];
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(gpsi + (ad >> LB)),
                                       (__attribute__((address_space(3))) void*)(lds + wslot + u * kBlock), 16, 0,
                                       0);
    }
}

// The pass's register stages on the tile in LDS (ends with a barrier).
// The lane's group index in a stage: thread t's group with zeros inserted at
// the register bits (ascending positions qsort).
template <int RB>
__device__ __forceinline__ uint32_t group_bits(uint32_t gi, const uint32_t* qsort) {
  uint32_t xg = gi;
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const uint32_t q = qsort[b];
    xg = ((xg >> q) << (q + 1)) | (xg & ((1u << q) - 1u));
  }
  return xg;
}

// Lane parts of the pass's first fixed-point phase items (at most cap) into
// pre[k * kBlock + t]; returns how many.  Valid when every thread owns at
// most one group per stage (tiles of at most kBlock groups), as in k_pass.
template <typename R>
__device__ __forceinline__ uint32_t pre_fill(cptr<PassDescDev> P, cptr<PassStageDev> stages, cptr<PassItemDev> items,
                                             cptr<cplx<R>> mats, typename lp_word<R>::W* pre, uint32_t cap) {
  constexpr int RB = Regs<R>::RB;
  const uint32_t groups = (1u << P->m) >> RB, t = threadIdx.x;
  uint32_t k = 0;
  for (uint32_t si = 0; si < P->stage_count && k < cap; ++si) {
    const PassStageDev S = cload(stages + (P->stage_first + si));
    if (!(S.flags & PSF_LANE)) continue;
    const uint32_t xg = group_bits<RB>(t, S.qsort);
    for (uint32_t i = 0; i < S.item_count && k < cap; ++i) {
      const PassItemDev it = cload(items + (S.item_first + i));
      if (it.type != PIT_LP && it.type != PIT_QG) continue;
      if (t < groups)
        pre[k * kBlock + t] = it.type == PIT_LP ? lp_lane_part<R>(it, mats + it.mat, xg)
                                                : qg_lane_part<R>(it, mats + it.mat, xg);
      ++k;
    }
  }
  return k;
}

template <typename R, bool LP>
__device__ __forceinline__ void tile_stages(const TileRef<R>& T, typename dev_elem<R>::E* tile,
                                            const typename lp_word<R>::W* pre, uint32_t npre) {
  typedef typename dev_elem<R>::E E;
  constexpr int LB = gelem<R>::LB;
  const cptr<PassDescDev> P = T.P;
  const cptr<PassStageDev> stages = T.stages;
  const cptr<PassItemDev> items = T.items;
  const cptr<cplx<R>> mats = T.mats;
  const uint64_t base = T.base;
  const uint32_t size = 1u << P->m;
  const uint32_t t = threadIdx.x;
  constexpr int RB = Regs<R>::RB, NR = Regs<R>::NR;
  typedef typename lp_word<R>::W W;
  __shared__ W tsum[LP ? kPassStageRowsMax : 1];  // tile sums of the stage's fixed-point rows
  uint32_t kfix = 0;  // fixed-point phase items of the pass so far
  for (uint32_t si = 0; si < P->stage_count; ++si) {
    const PassStageDev S = cload(stages + (P->stage_first + si));
    if constexpr (LP) {
      if (S.row_count) stage_rows<R>(S, mats, base, tsum);
    }
    const uint32_t groups = size >> RB;
    // swz is linear over XOR and xg shares no bit with a register offset, so
    // swz(xg | off) = swz(xg) ^ (XOR of swz(bit) over the offset's bits): only
    // the swizzled register bits are kept, not one offset per register
    uint32_t sbit[RB], cbit[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) sbit[b] = swz<LB>(1u << S.q[b]);
    // the store writes local index x to M x ^ c: register bit j of an
    // amplitude moves its address by the swizzled image of column q[j]
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      uint32_t img = 0;
#pragma unroll
      for (int l = 0; l < kPassLocalMax; ++l) img = (uint32_t)l == S.q[j] ? S.colimg[l] : img;
      cbit[j] = __builtin_amdgcn_readfirstlane(swz<LB>(img));
    }
    // the constant of the map for this tile (the terms selected by tile bits)
    uint32_t cmap = S.pconst;
    for (uint32_t k = 0; k < S.px_count; ++k) {
      const PassItemDev it = cload(items + (S.px_first + k));
      if (sel_bit(it.sel & 0xffu, 0u, base)) cmap ^= it.a;
    }
    const bool xperm = (S.flags & PSF_XPERM) != 0;
    // fixed-point items of this stage (every group of the stage walks them)
    uint32_t nfix = 0;
    if constexpr (LP) {
      if (S.flags & PSF_LANE)
        for (uint32_t i = 0; i < S.item_count; ++i) {
          const uint32_t ty = items[S.item_first + i].type;
          nfix += ty == PIT_LP || ty == PIT_QG;
        }
    }
    // a tile holds at most kBlock groups: one per thread
    const bool own = t < groups;
    {
      const uint32_t xg = own ? group_bits<RB>(t, S.qsort) : 0u;
      const uint32_t sx = swz<LB>(xg);
      cplx<R> v[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        uint32_t o = sx;
#pragma unroll
        for (int b = 0; b < RB; ++b)
          if ((r >> b) & 1) o ^= sbit[b];
        const E e = own ? tile[o] : E{};
        v[r] = cplx<R>{e.x, e.y};
      }
      if (S.flags & PSF_U2) op_u2<R>(v, mats + S.u2);
      // the earlier layers (2x2s, then register factors), then the last one;
      // one copy of the layer code serves all of them
      const cptr<PassSubDev> subs = (cptr<PassSubDev>)((cptr<uint32_t>)(stages + (P->stage_first + si)) +
                                                      offsetof(PassStageDev, sub) / 4);
      for (uint32_t li = 0; li <= S.nsub; ++li) {
        const bool last = li == S.nsub;
        const PassSubDev L = last ? PassSubDev{S.form, S.slot_mask, S.slots, kPassNoTable} : cload(subs + li);
        if (L.form) layer<R>(v, mats + L.slots, L.form);
        if (L.dr != kPassNoTable) {
          const cptr<cplx<R>> D = mats + L.dr;
#pragma unroll
          for (int r = 0; r < NR; ++r) v[r] = cmul(cget(D, r), v[r]);
        }
      }
      if (S.flags & PSF_LANE) {
        uint32_t kf = kfix;
        lane_diag<R, LP>(S, items, mats, xg, base, tsum, pre, npre, &kf, v);
      } else if (S.flags & PSF_DR) {
        const cptr<cplx<R>> D = mats + S.dr;
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = cmul(cget(D, r), v[r]);
      }
      // address of the group's register index 0 after the map: M xg ^ c
      uint32_t so = sx;
      if (S.flags & PSF_PERM) {
        uint32_t y = cmap;
#pragma unroll
        for (int l = 0; l < kPassLocalMax; ++l)
          if ((xg >> l) & 1u) y ^= S.colimg[l];
        so = swz<LB>(y);
      }
      // a map that moves amplitudes between groups writes after every
      // group has been read
      if (xperm) lds_sync();
      // The store recomputes the offsets from opaque copies of the inputs, so
      // the compiler cannot keep NR offsets live across the stage's work.
      asm volatile("" : "+v"(so));
#pragma unroll
      for (int b = 0; b < RB; ++b) asm volatile("" : "+s"(cbit[b]));
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        E e;
        e.x = v[r].re;
        e.y = v[r].im;
        uint32_t o = so;
#pragma unroll
        for (int b = 0; b < RB; ++b)
          if ((r >> b) & 1) o ^= cbit[b];
        if (own) tile[o] = e;
      }
    }
    kfix += nfix;
    lds_sync();
  }
}

// Read the tile for its store into registers: local bit j goes to physical
// position wpos[j], a permutation of the positions the tile was loaded from.
// When the lowest element bits keep their positions lanes walk the tile in
// load order (element x = t + 256 u); otherwise they walk the destination
// addresses in the load's order (the same coalesced runs and 16-byte
// elements whatever the permutation) and gather each element from LDS: the
// element's k-th address bit holds local bit winv[k].
template <typename R, int NT = kBlock>
__device__ __forceinline__ void tile_gather(const TileRef<R>& T, const typename dev_elem<R>::E* tile,
                                            typename gelem<R>::G* out) {
  typedef typename dev_elem<R>::E E;
  typedef typename gelem<R>::G G;
  typedef TileThreads<NT> TT;
  constexpr int LB = gelem<R>::LB;
  const cptr<PassDescDev> P = T.P;
  const uint32_t m = P->m;
  const LaneGeo lg = lane_geo<LB, NT>(m);
  // an opaque copy of the thread index: the addresses below are recomputed
  // per tile instead of being kept live (or spilled) across the whole loop
  uint32_t tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  if (P->flags & kPassStoreLaneOrder) {
#pragma unroll
    for (int u = 0; u < TT::BATCH; ++u)
      if ((uint32_t)u < lg.per && lg.on) {
        const uint32_t x = (tid + u * NT) << LB;
        if constexpr (LB == 1) {
          // both amplitudes of the element sit in one 16-byte LDS slot
          out[u] = *reinterpret_cast<const G*>(tile + swz<LB>(x));
        } else {
          out[u] = tile[swz<LB>(x)];
        }
      }
    return;
  }
  // LDS index of the lane's element: lane bit j is address bit LB + j
  uint32_t xl = 0;
  for (uint32_t jb = 0; jb < (uint32_t)TT::TB && LB + jb < m; ++jb)
    if ((tid >> jb) & 1u) xl |= 1u << P->winv[LB + jb];
  uint32_t xo[TT::UB];  // LDS offsets of the batch bits
#pragma unroll
  for (int b = 0; b < TT::UB; ++b) {
    const uint32_t k = LB + TT::TB + b;
    xo[b] = k < m ? 1u << P->winv[k] : 0u;
  }
  const uint32_t xp = LB ? 1u << P->winv[0] : 0u;  // the element's second amplitude (complex64)
#pragma unroll
  for (int u = 0; u < TT::BATCH; ++u)
    if ((uint32_t)u < lg.per && lg.on) {
      uint32_t x = xl;
#pragma unroll
      for (int b = 0; b < TT::UB; ++b)
        if ((u >> b) & 1) x |= xo[b];
      if constexpr (LB == 1) {
        const E e0 = tile[swz<LB>(x)], e1 = tile[swz<LB>(x | xp)];
        out[u] = G{e0.x, e0.y, e1.x, e1.y};
      } else {
        out[u] = tile[swz<LB>(x)];
      }
    }
}

// Store the gathered elements: in load order to the wpos addresses of the
// lane's element, or in destination order to the lpos addresses.
template <typename R, int NT = kBlock>
__device__ __forceinline__ void tile_put(const TileRef<R>& T, const typename gelem<R>::G* g) {
  typedef typename gelem<R>::G G;
  typedef TileThreads<NT> TT;
  constexpr int LB = gelem<R>::LB;
  const cptr<PassDescDev> P = T.P;
  const uint32_t m = P->m;
  const LaneGeo lg = lane_geo<LB, NT>(m);
  const gptr<G> gpsi = as_global(reinterpret_cast<G*>(T.psi));
  const cptr<uint32_t> pos = (P->flags & kPassStoreLaneOrder) ? P->wpos : P->lpos;
  uint64_t a0 = T.base;
  for (uint32_t j = 0; j < (uint32_t)TT::TB && LB + j < m; ++j)
    if ((threadIdx.x >> j) & 1u) a0 |= 1ull << pos[LB + j];
  uint64_t hb[TT::UB];
#pragma unroll
  for (int b = 0; b < TT::UB; ++b) hb[b] = LB + TT::TB + b < (int)m ? 1ull << pos[LB + TT::TB + b] : 0ull;
#pragma unroll
  for (int u = 0; u < TT::BATCH; ++u)
    if ((uint32_t)u < lg.per && lg.on) {
      uint64_t ad = a0;
#pragma unroll
      for (int b = 0; b < TT::UB; ++b)
        if ((u >> b) & 1) ad |= hb[b];
      stg<G>(gpsi + (ad >> LB), g[u]);
    }
}

// s_waitcnt with only the vector-memory counter (gfx9 encoding: expcnt and
// lgkmcnt at their no-wait values).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Persistent loop over tiles.  Per tile: the tile's loads land in LDS, the
// stages run, the result is read back into registers, and after a barrier
// the next tile's loads are issued before this tile's stores, so that the
// wait for a tile's data never waits for the previous tile's stores (the
// vector-memory counter retires in issue order).  The two blocks a CU holds
// overlap one block's memory phase with the other's stages.
template <typename R, bool LP, typename Src>
__device__ __forceinline__ void tile_loop(uint64_t total, const Src& src, typename dev_elem<R>::E* tile,
                                          const typename lp_word<R>::W* pre, uint32_t npre) {
  typedef typename gelem<R>::G G;
  uint64_t g = xcd_block();
  if (g >= total) return;
  tile_load_lds<R>(src(g), tile);
  bool full_prev = false;  // the previous tile stored kBatch elements per lane
  while (true) {
    const uint64_t ng = g + gridDim.x;
    const TileRef<R> cur = src(g);
    // this tile's loads are older than the previous tile's stores: when that
    // tile issued kBatch stores per lane, waiting until at most kBatch
    // operations remain waits for exactly the loads
    if (full_prev) wait_vm<kBatch>();
    else wait_vm<0>();
    lds_barrier();
    tile_stages<R, LP>(cur, tile, pre, npre);
    G out[kBatch];
    tile_gather<R>(cur, tile, out);
    wait_lgkm0();  // this lane's LDS reads are done
    lds_barrier();
    if (ng < total) tile_load_lds<R>(src(ng), tile);
    asm volatile("" ::: "memory");  // the loads stay ahead of the stores
    tile_put<R>(cur, out);
    full_prev = lane_geo<gelem<R>::LB>(cur.P->m).per == (uint32_t)kBatch;
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
  cptr<PassItemDev> items;
  cptr<cplx<R>> mats;
  __device__ __forceinline__ TileRef<R> operator()(uint64_t g) const {
    return tile_ref<R>(psi, n, P, stages, items, mats, g);
  }
};

template <typename R, bool LP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_pass(typename dev_elem<R>::E* __restrict__ psi, int n,
                                                 const PassDescDev* __restrict__ passes, int pi,
                                                 const PassStageDev* __restrict__ stages,
                                                 const PassItemDev* __restrict__ items,
                                                 const cplx<R>* __restrict__ mats) {
  typedef typename dev_elem<R>::E E;
  extern __shared__ __align__(16) unsigned char smem[];
  E* tile = reinterpret_cast<E*>(smem);
  const cptr<PassDescDev> P = as_const(passes + pi);
  const SingleSrc<R> src{psi, n, P, as_const(stages), as_const(items), as_const(mats)};
  typedef typename lp_word<R>::W W;
  // lane parts of the fixed-point phase items, computed once for all tiles
  __shared__ W pre[LP ? pre_cap<R>::N * kBlock : 1];
  uint32_t npre = 0;
  if constexpr (LP) {
    npre = pre_fill<R>(P, as_const(stages), as_const(items), as_const(mats), pre, pre_cap<R>::N);
    wait_lgkm0();  // the table is complete before the first tile's barrier
  }
  tile_loop<R, LP>(1ull << (n - P->m), src, tile, pre, npre);
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
                       as_const(it->stages), as_const(it->items), as_const((const cplx<R>*)it->mats),
                       g - it->tile_begin);
  }
};

template <typename R, bool LP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_pass_batch(const BatchItemDev* __restrict__ items, int count,
                                                       uint64_t total_tiles) {
  typedef typename dev_elem<R>::E E;
  extern __shared__ __align__(16) unsigned char smem[];
  E* tile = reinterpret_cast<E*>(smem);
  const BatchSrc<R> src{as_const(items), count};
  tile_loop<R, LP>(total_tiles, src, tile, nullptr, 0);
}

template <typename R, bool LP>
hipError_t run(void* psi, int n, int m, const PassDescDev* passes, int pass, const PassStageDev* stages,
               const PassItemDev* items, const void* mats, hipStream_t s) {
  typedef typename dev_elem<R>::E E;
  const size_t lds = ((size_t)1 << m) * sizeof(E);
  static KernelLaunchCache cache;
  uint64_t resident = 0;
  hipError_t e = prepare_launch(cache, (const void*)k_pass<R, LP>, kBlock, lds, &resident);
  if (e != hipSuccess) return e;
  const uint64_t tiles = 1ull << (n - m);
  const uint64_t blocks = tiles < resident ? tiles : resident;
  hipLaunchKernelGGL((k_pass<R, LP>), dim3((unsigned)blocks), dim3(kBlock), lds, s, (E*)psi, n, passes, pass, stages,
                     items, (const cplx<R>*)mats);
  return hipGetLastError();
}

template <typename R, bool LP>
hipError_t run_batch(const BatchItemDev* items, int count, uint64_t total_tiles, int max_m, hipStream_t s) {
  typedef typename dev_elem<R>::E E;
  const size_t lds = ((size_t)1 << max_m) * sizeof(E);
  static KernelLaunchCache cache;
  uint64_t resident = 0;
  hipError_t e = prepare_launch(cache, (const void*)k_pass_batch<R, LP>, kBlock, lds, &resident);
  if (e != hipSuccess) return e;
  if (total_tiles == 0) return hipSuccess;
  const uint64_t blocks = total_tiles < resident ? total_tiles : resident;
  hipLaunchKernelGGL((k_pass_batch<R, LP>), dim3((unsigned)blocks), dim3(kBlock), lds, s, items, count, total_tiles);
  return hipGetLastError();
}

// ---------------------------------------------------------------- matrix passes
// A matrix pass runs dense fused ops (general gate fusion, Sec. II-B) inside
// the tiles of one pass (in-cache operation, Sec. II-B / III-B), on the
// matrix cores.  Stage s views the tile as a 2^K x 2^(m-K) matrix X: rows
// ("members") are the K local bits of the stage (member bit b = local bit
// q[b]), columns the other local bits in the stage's column order (lane
// bits, wave bits, the rest).  It computes Y = U X with three real products
// (Gauss's complex multiplication):
//   P1 = Ur Xr,  P2 = Ui Xi,  P3 = (Ur + Ui)(Xr + Xi),  Yr = P1 - P2,
//   Yi = P3 - P1 - P2.
// Every wave owns whole column blocks (those whose wave bits spell its
// index), so a stage reads and overwrites its columns in place; a barrier
// separates two stages only when their wave bits differ.  A-operand
// fragments and address tables of all stages sit in LDS beside the tile
// (filled once per block).  The next tile's loads go to registers while the
// stages run and are written to LDS once the current tile has been read
// back; a tile's stores go out after the next tile's first stage.  A block
// (eight waves, two per SIMD) is the only one on its CU.
typedef float mx_f32x16 __attribute__((ext_vector_type(16)));
typedef double mx_f64x4 __attribute__((ext_vector_type(4)));

template <typename R>
struct mx_shape;
template <>
struct mx_shape<float> {
  // v_mfma_f32_32x32x2f32: lane l holds A[l % 32][l / 32] and B[l / 32][l % 32];
  // accumulator register r of lane l is C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
  static constexpr int BM = 32, BN = 32, BK = 2, NACC = 16;
  typedef mx_f32x16 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  static constexpr uint32_t out_u(int r) { return 8 * (r / 4) + r % 4; }  // row: register part
  static __device__ __forceinline__ uint32_t out_l(uint32_t l) { return 4 * (l / 32); }  // row: lane part
};
template <>
struct mx_shape<double> {
  // v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
  // accumulator register r of lane l is C[l / 16 + 4 r][l % 16]
  static constexpr int BM = 16, BN = 16, BK = 4, NACC = 4;
  typedef mx_f64x4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static constexpr uint32_t out_u(int r) { return 4 * r; }
  static __device__ __forceinline__ uint32_t out_l(uint32_t l) { return l / 16; }
};

template <typename R, int K>
struct mx_plan {
  static constexpr int D = 1 << K;
  static constexpr int RBK = D / mx_shape<R>::BM;  // row blocks
  static constexpr int KS = D / mx_shape<R>::BK;   // k-steps
  static constexpr int AF = RBK * KS * 64;         // A-fragment entries of one stage
  static_assert(RBK >= 1, "a stage fills at least one row block");
  static_assert(AF == D * D, "one A-fragment entry per matrix entry (matrix_pass_max_stages)");
};

// Swizzled LDS offset of a member: the XOR of the offsets of its set bits
// (swz is linear, and members and columns occupy disjoint local bits).
template <int K>
__device__ __forceinline__ uint32_t mx_member(uint32_t mem, const uint32_t* sm) {
  uint32_t o = 0;
#pragma unroll
  for (int b = 0; b < K; ++b)
    if ((mem >> b) & 1u) o ^= sm[b];
  return o;
}

// Threads of a matrix-pass block: eight waves, two per SIMD, so that one
// wave's LDS and vector work overlaps the other's matrix-core products.
constexpr int kMxThreads = 512;

// Per-stage address table of a matrix pass (uint32 words, byte offsets into
// the tile; every offset is an XOR of swizzled bit offsets, so offsets of
// disjoint bit sets combine by XOR), filled once per block:
//   [kMxBoff + ks]           member BK ks (operand reads, uniform part)
//   [kMxOoff + rb NACC + r]  member BM rb + out_u(r) (results, uniform part)
//   [kMxCol + cb]            column BN cb
//   [kMxLane + 2 l (+ 1)]    lane l: column l % BN with member l / BN (with
//                            the lane part out_l(l) of the result member)
constexpr int kMxBoff = 0, kMxOoff = 16, kMxCol = 48, kMxLane = 64, kMxTab = 192;
static_assert(kMxTab * 4 == kMatrixStageTable, "table size shared with the planner");

template <typename R, int K>
__device__ __forceinline__ void mx_table(cptr<uint32_t> sd, uint32_t m, uint32_t* tab) {
  typedef mx_shape<R> MS;
  typedef mx_plan<R, K> MP;
  constexpr int LB = gelem<R>::LB;
  constexpr uint32_t EB = sizeof(typename dev_elem<R>::E);
  constexpr int LBN = MS::BN == 32 ? 5 : 4;  // lane bits of a column block
  const cptr<uint32_t> q = sd + offsetof(PassStageDev, q) / 4;
  const cptr<uint32_t> col = sd + offsetof(PassStageDev, colimg) / 4;  // column bit j: local bit col[j]
  uint32_t sm[K];
#pragma unroll
  for (int b = 0; b < K; ++b) sm[b] = swz<LB>(1u << q[b]) * EB;
  const uint32_t nc = m - K;  // column bits
  const uint32_t cblocks = (1u << nc) / MS::BN;
  // offset of the column bits `v` taken from column bit `first` on
  auto cols = [&](uint32_t v, uint32_t first, uint32_t nbits) {
    uint32_t o = 0;
    for (uint32_t j = 0; j < nbits; ++j)
      if ((v >> j) & 1u) o ^= swz<LB>(1u << col[first + j]) * EB;
    return o;
  };
  for (uint32_t t = threadIdx.x; t < (uint32_t)kMxTab; t += kMxThreads) {
    uint32_t v = 0;
    if (t < (uint32_t)kMxBoff + MP::KS) {
      v = mx_member<K>(MS::BK * (t - kMxBoff), sm);
    } else if (t >= (uint32_t)kMxOoff && t < (uint32_t)kMxOoff + MP::RBK * MS::NACC) {
      const uint32_t i = t - kMxOoff;
      v = mx_member<K>(MS::BM * (i / MS::NACC) + MS::out_u((int)(i % MS::NACC)), sm);
    } else if (t >= (uint32_t)kMxCol && t < (uint32_t)kMxCol + cblocks) {
      v = cols(t - kMxCol, LBN, nc - LBN);
    } else if (t >= (uint32_t)kMxLane) {
      const uint32_t l = (t - kMxLane) / 2;
      v = cols(l % MS::BN, 0, LBN) ^ mx_member<K>(((t - kMxLane) & 1u) ? MS::out_l(l) : l / MS::BN, sm);
    }
    tab[t] = v;
  }
}

// One stage on the tile in LDS (no barrier inside).  tab: the stage's
// address table; am: its A fragments, entry (rb KS + ks) 64 + l =
// U[BM rb + l % BM][BK ks + l / BM].  Each wave owns whole column blocks.
template <typename R, int K>
__device__ __forceinline__ void mx_stage(typename dev_elem<R>::E* tile, const uint32_t* tab, const cplx<R>* am,
                                         uint32_t m) {
  typedef mx_shape<R> MS;
  typedef mx_plan<R, K> MP;
  typedef typename dev_elem<R>::E E;
  unsigned char* tb = reinterpret_cast<unsigned char*>(tile);
  const uint32_t l = threadIdx.x & 63u;
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t cblocks = (1u << (m - K)) / MS::BN;
  const uint32_t lb = tab[kMxLane + 2 * l], lo = tab[kMxLane + 2 * l + 1];
  // the result offsets are read with the operands' and held in registers:
  // read next to their stores, each would cost a wait on the LDS queue
  constexpr int NO = MP::RBK * MS::NACC;
  uint32_t oo[NO];
#pragma unroll
  for (int j = 0; j < NO; ++j) oo[j] = tab[kMxOoff + j];
#pragma unroll
  for (int j = 0; j < NO; ++j) asm volatile("" : "+v"(oo[j]));
  for (uint32_t cb = w; cb < cblocks; cb += kMxThreads / 64) {
    const uint32_t cu = tab[kMxCol + cb];
    const uint32_t bb = lb ^ cu, bo = lo ^ cu;
    typename MS::acc_t p1[MP::RBK], p2[MP::RBK], p3[MP::RBK];
#pragma unroll
    for (int rb = 0; rb < MP::RBK; ++rb) p1[rb] = p2[rb] = p3[rb] = typename MS::acc_t{};
#pragma unroll
    for (int ks = 0; ks < MP::KS; ++ks) {
      const E x = *reinterpret_cast<const E*>(tb + (bb ^ tab[kMxBoff + ks]));
      const R xs = x.x + x.y;
#pragma unroll
      for (int rb = 0; rb < MP::RBK; ++rb) {
        const cplx<R> a = am[(rb * MP::KS + ks) * 64 + l];
        p1[rb] = MS::mma(a.re, x.x, p1[rb]);
        p2[rb] = MS::mma(a.im, x.y, p2[rb]);
        p3[rb] = MS::mma(a.re + a.im, xs, p3[rb]);
      }
    }
    // this wave has read every member of its columns: overwrite them
#pragma unroll
    for (int rb = 0; rb < MP::RBK; ++rb)
#pragma unroll
      for (int r = 0; r < MS::NACC; ++r) {
        E y;
        y.x = p1[rb][r] - p2[rb][r];
        y.y = p3[rb][r] - p1[rb][r] - p2[rb][r];
        *reinterpret_cast<E*>(tb + (bo ^ oo[rb * MS::NACC + r])) = y;
      }
  }
}

// Global addresses of a lane's tile elements: register u of lane t is
// element slot e = t + NT u, which holds tile element swz(e) (the layout
// tile_load_lds produces).  The same for every tile of a pass but the base.
template <int NT>
struct MoveGeo {
  uint64_t lane;
  uint64_t hb[TileThreads<NT>::UB];
  LaneGeo lg;
};

template <typename R, int NT>
__device__ __forceinline__ MoveGeo<NT> move_geo(cptr<PassDescDev> P) {
  constexpr int LB = gelem<R>::LB;
  typedef TileThreads<NT> TT;
  MoveGeo<NT> g;
  const uint32_t m = P->m;
  g.lane = lane_slot_bits<LB, NT>(P->lpos, m);
#pragma unroll
  for (int b = 0; b < TT::UB; ++b) g.hb[b] = slot_offset<LB>(P->lpos, m, TT::TB + b);
  g.lg = lane_geo<LB, NT>(m);
  return g;
}

// Move the tile's elements between HBM and registers.  STORE: write them
// back to the addresses they were loaded from (a pass whose write positions
// are its load positions).
template <typename R, int NT, bool STORE>
__device__ __forceinline__ void tile_move(const TileRef<R>& T, const MoveGeo<NT>& mg, typename gelem<R>::G* v) {
  typedef typename gelem<R>::G G;
  typedef TileThreads<NT> TT;
  constexpr int LB = gelem<R>::LB;
  const gptr<G> gpsi = as_global(reinterpret_cast<G*>(T.psi));
  const uint64_t a0 = T.base | mg.lane;
  // Loads are not predicated: a lane without element u reads the tile's
  // first element instead, so that no load result merges with an older value
  // (which would wait for the load right away).
#pragma unroll
  for (int u = 0; u < TT::BATCH; ++u) {
    uint64_t ad = a0;
#pragma unroll
    for (int b = 0; b < TT::UB; ++b)
      if ((u >> b) & 1) ad ^= mg.hb[b];
    const bool ok = (uint32_t)u < mg.lg.per && mg.lg.on;
    if constexpr (STORE) {
      if (ok) stg<G>(gpsi + (ad >> LB), v[u]);
    } else {
      v[u] = ldg<G>((gptr<const G>)(gpsi + ((ok ? ad : T.base) >> LB)));
    }
  }
}

// The tile's element slots to or from registers (register u of lane t = slot t + NT u).
template <typename R, int NT, bool TO_LDS>
__device__ __forceinline__ void tile_slots(typename gelem<R>::G* v, typename dev_elem<R>::E* tile, const LaneGeo& lg) {
  typedef typename gelem<R>::G G;
  G* slots = reinterpret_cast<G*>(tile);
#pragma unroll
  for (int u = 0; u < TileThreads<NT>::BATCH; ++u)
    if ((uint32_t)u < lg.per && lg.on) {
      if constexpr (TO_LDS) slots[threadIdx.x + u * NT] = v[u];
      else v[u] = slots[threadIdx.x + u * NT];
    }
}

template <typename R, int K>
__global__ __launch_bounds__(kMxThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mpass(
    typename dev_elem<R>::E* __restrict__ psi, int n, const PassDescDev* __restrict__ passes, int pi,
    const PassStageDev* __restrict__ stages, const cplx<R>* __restrict__ mats) {
  typedef typename dev_elem<R>::E E;
  typedef typename gelem<R>::G G;
  typedef mx_shape<R> MS;
  typedef mx_plan<R, K> MP;
  extern __shared__ __align__(16) unsigned char smem[];
  const cptr<PassDescDev> P = as_const(passes + pi);
  const uint32_t m = P->m, ns = P->stage_count;
  E* tile = reinterpret_cast<E*>(smem);
  cplx<R>* am = reinterpret_cast<cplx<R>*>(tile + (1u << m));
  uint32_t* tab = reinterpret_cast<uint32_t*>(am + ns * MP::AF);
  const cptr<PassStageDev> st = as_const(stages) + P->stage_first;
  constexpr int NT = kMxThreads, BATCH = TileThreads<NT>::BATCH;
  for (uint32_t s = 0; s < ns; ++s) {
    const uint32_t at = ((cptr<uint32_t>)(st + s))[offsetof(PassStageDev, u2) / 4];
#pragma unroll
    for (int j = 0; j < (MP::AF + NT - 1) / NT; ++j) {
      const uint32_t f = threadIdx.x + j * NT, l = f % 64, ks = (f / 64) % MP::KS, rb = f / (64 * MP::KS);
      const uint32_t row = MS::BM * rb + l % MS::BM, col = MS::BK * ks + l / MS::BM;
      if (f < (uint32_t)MP::AF) am[s * MP::AF + f] = mats[at + row * MP::D + col];
    }
    mx_table<R, K>((cptr<uint32_t>)(st + s), m, tab + s * kMxTab);
  }
  const SingleSrc<R> src{psi, n, P, as_const(stages), as_const((const PassItemDev*)nullptr), as_const(mats)};
  const MoveGeo<NT> mg = move_geo<R, NT>(P);
  const uint64_t total = 1ull << (n - m);
  uint64_t g = xcd_block();
  // Per tile: the next tile's loads go out first, the previous tile's
  // stores after the first stage, so neither burst waits behind the other in
  // the memory queue while the stages could run.
  G nx[BATCH], out[BATCH];
  if (g < total) tile_move<R, NT, false>(src(g), mg, nx);
  __syncthreads();  // the A fragments and tables are in LDS
  if (g >= total) return;
  tile_slots<R, NT, true>(nx, tile, mg.lg);
  uint64_t prev = total;  // tile whose results wait in `out` (none yet)
  while (true) {
    const uint64_t ng = g + gridDim.x;
    lds_sync();  // the tile is in LDS
    if (ng < total) tile_move<R, NT, false>(src(ng), mg, nx);
    for (uint32_t s = 0; s < ns; ++s) {
      if (s > 0) {
        const uint32_t fl = ((cptr<uint32_t>)(st + s))[offsetof(PassStageDev, flags) / 4];
        if (fl & kMatrixStageSync) {
          lds_sync();
        } else {
          // the stage reads only what this wave wrote: its own LDS writes
          // are done, no other wave is waited for
          wait_lgkm0();
          asm volatile("" ::: "memory");
        }
      }
      mx_stage<R, K>(tile, tab + s * kMxTab, am + s * MP::AF, m);
      if (s == 0 && prev < total) tile_move<R, NT, true>(src(prev), mg, out);
    }
    lds_sync();  // every wave's results are in LDS
    if (ns == 0 && prev < total) tile_move<R, NT, true>(src(prev), mg, out);  // (a pass has stages)
    tile_slots<R, NT, false>(out, tile, mg.lg);
    lds_sync();  // every lane has read the tile
    prev = g;
    if (ng >= total) break;
    tile_slots<R, NT, true>(nx, tile, mg.lg);
    g = ng;
  }
  tile_move<R, NT, true>(src(prev), mg, out);
}

template <typename R, int K>
hipError_t run_mpass(void* psi, int n, int m, const PassDescDev* passes, int pass, int n_stages,
                     const PassStageDev* stages, const void* mats, hipStream_t s) {
  typedef typename dev_elem<R>::E E;
  const size_t lds = ((size_t)1 << m) * sizeof(E) +
                     (size_t)n_stages * (mx_plan<R, K>::AF * sizeof(cplx<R>) + kMxTab * sizeof(uint32_t));
  if (lds > (size_t)kMatrixPassLds) return hipErrorInvalidValue;
  static KernelLaunchCache cache;
  uint64_t resident = 0;
  hipError_t e = prepare_launch(cache, (const void*)k_mpass<R, K>, kMxThreads, lds, &resident);
  if (e != hipSuccess) return e;
  const uint64_t tiles = 1ull << (n - m);
  const uint64_t blocks = tiles < resident ? tiles : resident;
  hipLaunchKernelGGL((k_mpass<R, K>), dim3((unsigned)blocks), dim3(kMxThreads), lds, s, (E*)psi, n, passes, pass,
                     stages, (const cplx<R>*)mats);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_matrix_pass(sv_dtype dt, int k, void* psi, int n, int m, const PassDescDev* passes, int pass,
                              int n_stages, const PassStageDev* stages, const void* mats, hipStream_t s) {
  if (dt == SV_C64) {
    if (k != 5) return hipErrorInvalidValue;
    return run_mpass<float, 5>(psi, n, m, passes, pass, n_stages, stages, mats, s);
  }
  if (k == 4) return run_mpass<double, 4>(psi, n, m, passes, pass, n_stages, stages, mats, s);
  if (k == 5) return run_mpass<double, 5>(psi, n, m, passes, pass, n_stages, stages, mats, s);
  return hipErrorInvalidValue;
}

hipError_t launch_pass(sv_dtype dt, void* psi, int n, int m, const PassDescDev* passes, int pass,
                       const PassStageDev* stages, const PassItemDev* items, const void* mats, bool ladders,
                       hipStream_t s) {
  if (dt == SV_C128)
    return ladders ? run<double, true>(psi, n, m, passes, pass, stages, items, mats, s)
                   : run<double, false>(psi, n, m, passes, pass, stages, items, mats, s);
  return ladders ? run<float, true>(psi, n, m, passes, pass, stages, items, mats, s)
                 : run<float, false>(psi, n, m, passes, pass, stages, items, mats, s);
}

hipError_t launch_pass_batch(sv_dtype dt, const BatchItemDev* items, int count, uint64_t total_tiles, int max_m,
                             bool ladders, hipStream_t s) {
  if (dt == SV_C128)
    return ladders ? run_batch<double, true>(items, count, total_tiles, max_m, s)
                   : run_batch<double, false>(items, count, total_tiles, max_m, s);
  return ladders ? run_batch<float, true>(items, count, total_tiles, max_m, s)
                 : run_batch<float, false>(items, count, total_tiles, max_m, s);
}

}  // namespace sv
