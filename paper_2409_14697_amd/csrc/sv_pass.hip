// In-cache tile pass: the block-by-block all-in-cache execution of QueenV2
// (Sec. II-B "In-cache Operations", Sec. III-B) on gfx950 LDS.
//
// One block owns one tile of 2^m amplitudes: the indices that agree with the
// tile base on every non-local bit.  The tile is gathered from HBM with the
// PDEP-like deposit of its local index into the pass's local bit positions
// (Sec. III-B), so the low pinned positions give contiguous runs.  The pass's
// stages then run in LDS: a stage gives each lane groups of 16 amplitudes
// (4 local bits held in registers) and applies a list of ops to them in
// registers; ops whose controls or phase bits lie outside the register bits
// read those bits from the group's local index or from the tile base.  The
// tile is written back with local bit j at physical position wpos[j], which
// fuses qubit reordering (Sec. II-B) into the store.
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
constexpr int RB = kPassRegBits;
constexpr int NR = 1 << RB;
constexpr int kBatchBits = 3;
constexpr int kBatch = 1 << kBatchBits;  // global loads in flight per lane while gathering a tile

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

template <int B, typename R>
__device__ __forceinline__ void op_u1(cplx<R>* v, const cplx<R>* M) {
  const cplx<R> m0 = M[0], m1 = M[1], m2 = M[2], m3 = M[3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (!((r >> B) & 1)) {
      const cplx<R> a0 = v[r], a1 = v[r | (1 << B)];
      v[r] = cfma(cmul(m0, a0), m1, a1);
      v[r | (1 << B)] = cfma(cmul(m2, a0), m3, a1);
    }
}

template <int B0, int B1, typename R>
__device__ __forceinline__ void op_u2(cplx<R>* v, const cplx<R>* M) {
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (!((r >> B0) & 1) && !((r >> B1) & 1)) {
      const int i[4] = {r, r | (1 << B1), r | (1 << B0), r | (1 << B0) | (1 << B1)};
      const cplx<R> x0 = v[i[0]], x1 = v[i[1]], x2 = v[i[2]], x3 = v[i[3]];
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        cplx<R> y = cmul(M[4 * o], x0);
        y = cfma(y, M[4 * o + 1], x1);
        y = cfma(y, M[4 * o + 2], x2);
        y = cfma(y, M[4 * o + 3], x3);
        v[i[o]] = y;
      }
    }
}

template <int B, typename R>
__device__ __forceinline__ void op_x(cplx<R>* v) {
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
  const cplx<R> d0 = M[0], d1 = M[1];
#pragma unroll
  for (int r = 0; r < NR; ++r) v[r] = cmul(((r >> B) & 1) ? d1 : d0, v[r]);
}

template <int B0, int B1, typename R>
__device__ __forceinline__ void op_d2(cplx<R>* v, const cplx<R>* M) {
  const cplx<R> d[4] = {M[0], M[1], M[2], M[3]};
#pragma unroll
  for (int r = 0; r < NR; ++r) v[r] = cmul(d[(((r >> B0) & 1) << 1) | ((r >> B1) & 1)], v[r]);
}

#define SV_PAIR_SWITCH(code, F)                                         \
  switch (code) {                                                       \
    case 1: F(0, 1); break;  case 2: F(0, 2); break;  case 3: F(0, 3); break; \
    case 4: F(1, 0); break;  case 6: F(1, 2); break;  case 7: F(1, 3); break; \
    case 8: F(2, 0); break;  case 9: F(2, 1); break;  case 11: F(2, 3); break; \
    case 12: F(3, 0); break; case 13: F(3, 1); break; case 14: F(3, 2); break; \
    default: break;                                                     \
  }
#define SV_BIT_SWITCH(b, F)                                             \
  switch (b) {                                                          \
    case 0: F(0); break; case 1: F(1); break; case 2: F(2); break; case 3: F(3); break; \
    default: break;                                                     \
  }

// M points at the op's first matrix entry (the same address in every lane, so
// the entries come through scalar loads); `var` selects a variant per lane.
template <typename R>
__device__ __forceinline__ void apply_op(const PassOpDev& op, const cplx<R>* __restrict__ M, uint32_t var,
                                         cplx<R>* v) {
  const uint32_t pair = op.b0 * 4 + op.b1;
  switch (op.type) {
    case POP_U1: {
#define F(B) op_u1<B>(v, M)
      SV_BIT_SWITCH(op.b0, F)
#undef F
      break;
    }
    case POP_U2: {
#define F(A, B) op_u2<A, B>(v, M)
      SV_PAIR_SWITCH(pair, F)
#undef F
      break;
    }
    case POP_X: {
#define F(B) op_x<B>(v)
      SV_BIT_SWITCH(op.b0, F)
#undef F
      break;
    }
    case POP_CX: {
#define F(A, B) op_cx<A, B>(v)
      SV_PAIR_SWITCH(pair, F)
#undef F
      break;
    }
    case POP_D1: {
      cplx<R> d[2] = {M[0], M[1]};
      if (op.sa != kPassNoSel) {  // two variants, picked per lane
        const cplx<R> e0 = M[2], e1 = M[3];
        if (var) {
          d[0] = e0;
          d[1] = e1;
        }
      }
#define F(B) op_d1<B>(v, d)
      SV_BIT_SWITCH(op.b0, F)
#undef F
      break;
    }
    case POP_D2: {
#define F(A, B) op_d2<A, B>(v, M)
      SV_PAIR_SWITCH(pair, F)
#undef F
      break;
    }
    case POP_DG: {
      cplx<R> p = M[0];
      if (op.sa != kPassNoSel) {
        const cplx<R> p1 = M[1];
        if (op.sb != kPassNoSel) {
          const cplx<R> p2 = M[2], p3 = M[3];
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
      for (int r = 0; r < NR; ++r) v[r] = cmul(p, v[r]);
      break;
    }
    default:
      break;
  }
}

// Per-lane physical offsets of the batch index u (local bits 8 .. 8 + log2(kBatch) - 1).
struct BatchOffsets {
  uint64_t in[kBatch], out[kBatch];
};

__device__ __forceinline__ void batch_offsets(const PassDescDev& P, BatchOffsets* bo) {
#pragma unroll
  for (int u = 0; u < kBatch; ++u) {
    bo->in[u] = bo->out[u] = 0;
#pragma unroll
    for (int b = 0; b < kBatchBits; ++b)
      if (((u >> b) & 1) && 8u + b < P.m) {
        bo->in[u] |= 1ull << P.lpos[8 + b];
        bo->out[u] |= 1ull << P.wpos[8 + b];
      }
  }
}

// One tile of one pass: gather, run the stages, scatter.  `tile` is the LDS
// buffer of 2^m elements; every thread of the block calls this.
template <typename R, int WB>
__device__ __forceinline__ void tile_pass(typename dev_elem<R>::E* __restrict__ psi, int n, const PassDescDev& P,
                                          const PassStageDev* __restrict__ stages,
                                          const PassOpDev* __restrict__ ops, const cplx<R>* __restrict__ mats,
                                          uint64_t tile_id, typename dev_elem<R>::E* tile,
                                          const BatchOffsets& bo) {
  typedef typename dev_elem<R>::E E;
  const uint32_t m = P.m;
  const uint32_t size = 1u << m;
  const uint64_t all = (1ull << n) - 1ull;
  const uint32_t t = threadIdx.x;
  const uint32_t per = size >= (uint32_t)kBlock ? size / kBlock : 1u;  // elements per lane
  const bool lane_on = t < size;
  const uint64_t base = deposit(tile_id, all & ~P.lmask);

  // gather: x = t + 256 j; the low 8 local bits come from t, the rest from j.
  // kBatch loads per lane are issued before any of them is written to LDS.
  uint64_t lo_in = 0, lo_out = 0;
  for (uint32_t j = 0; j < m && j < 8; ++j)
    if ((t >> j) & 1u) {
      lo_in |= 1ull << P.lpos[j];
      lo_out |= 1ull << P.wpos[j];
    }
  for (uint32_t j0 = 0; j0 < per; j0 += kBatch) {
    // local bits 8 + log2(kBatch) .. m-1 come from j0 (the same in every lane)
    uint64_t hi_in = 0;
    for (uint32_t b = 8 + kBatchBits; b < m; ++b)
      if ((j0 >> (b - 8)) & 1u) hi_in |= 1ull << P.lpos[b];
    E buf[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (j0 + u < per && lane_on) buf[u] = ld(psi + (base | lo_in | hi_in | bo.in[u]));
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (j0 + u < per && lane_on) tile[swz<WB>(t + (j0 + u) * kBlock)] = buf[u];
  }
  __syncthreads();

  for (uint32_t si = 0; si < P.stage_count; ++si) {
    const PassStageDev& S = stages[P.stage_first + si];
    const uint32_t groups = size >> RB;
    uint32_t off[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      uint32_t o = 0;
#pragma unroll
      for (int b = 0; b < RB; ++b)
        if ((r >> b) & 1) o |= 1u << S.q[b];
      off[r] = o;
    }
    for (uint32_t gi = t; gi < groups; gi += kBlock) {
      uint32_t xg = gi;
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const uint32_t q = S.qsort[b];
        xg = ((xg >> q) << (q + 1)) | (xg & ((1u << q) - 1u));
      }
      cplx<R> v[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const E e = tile[swz<WB>(xg | off[r])];
        v[r] = cplx<R>{e.x, e.y};
      }
      for (uint32_t o = 0; o < S.op_count; ++o) {
        const PassOpDev op = ops[S.op_first + o];
        if ((xg & op.lmask) != op.lmask || (base & op.tmask) != op.tmask) continue;
        uint32_t var = 0;
        if (op.sa != kPassNoSel) {
          var = op.sa < kPassTileSel ? (xg >> op.sa) & 1u : (uint32_t)(base >> (op.sa - kPassTileSel)) & 1u;
          if (op.sb != kPassNoSel)
            var = (var << 1) |
                  (op.sb < kPassTileSel ? (xg >> op.sb) & 1u : (uint32_t)(base >> (op.sb - kPassTileSel)) & 1u);
        }
        apply_op<R>(op, mats + op.mat, var, v);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        E e;
        e.x = v[r].re;
        e.y = v[r].im;
        tile[swz<WB>(xg | off[r])] = e;
      }
    }
    __syncthreads();
  }

  for (uint32_t j0 = 0; j0 < per; j0 += kBatch) {
    uint64_t hi_out = 0;
    for (uint32_t b = 8 + kBatchBits; b < m; ++b)
      if ((j0 >> (b - 8)) & 1u) hi_out |= 1ull << P.wpos[b];
    E buf[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (j0 + u < per && lane_on) buf[u] = tile[swz<WB>(t + (j0 + u) * kBlock)];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (j0 + u < per && lane_on) st(psi + (base | lo_out | hi_out | bo.out[u]), buf[u]);
  }
  __syncthreads();  // the tile buffer is reused by the next tile
}

template <typename R, int WB>
__global__ __launch_bounds__(kBlock) void k_pass(typename dev_elem<R>::E* __restrict__ psi, int n,
                                                 const PassDescDev* __restrict__ passes, int pi,
                                                 const PassStageDev* __restrict__ stages,
                                                 const PassOpDev* __restrict__ ops,
                                                 const cplx<R>* __restrict__ mats) {
  typedef typename dev_elem<R>::E E;
  extern __shared__ __align__(16) unsigned char smem[];
  E* tile = reinterpret_cast<E*>(smem);
  const PassDescDev& P = passes[pi];
  BatchOffsets bo;
  batch_offsets(P, &bo);
  const uint64_t ntiles = 1ull << (n - P.m);
  for (uint64_t tile_id = xcd_block(); tile_id < ntiles; tile_id += gridDim.x)
    tile_pass<R, WB>(psi, n, P, stages, ops, mats, tile_id, tile, bo);
}

// Many states in one launch: work item i runs pass `pass` of its own program
// over its own tiles; global tile g belongs to the item whose [tile_begin,
// tile_begin + tiles) range holds g.  No item reads another's state, so each
// result is independent of the batch it ran in.
template <typename R, int WB>
__global__ __launch_bounds__(kBlock) void k_pass_batch(const BatchItemDev* __restrict__ items, int count,
                                                       uint64_t total_tiles) {
  typedef typename dev_elem<R>::E E;
  extern __shared__ __align__(16) unsigned char smem[];
  E* tile = reinterpret_cast<E*>(smem);
  int cur = -1;
  BatchOffsets bo;
  for (uint64_t g = xcd_block(); g < total_tiles; g += gridDim.x) {
    int lo = 0, hi = count - 1;  // last item with tile_begin <= g
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].tile_begin <= g) lo = mid;
      else hi = mid - 1;
    }
    const BatchItemDev& it = items[lo];
    const PassDescDev& P = it.passes[it.pass];
    if (lo != cur) {
      batch_offsets(P, &bo);
      cur = lo;
    }
    tile_pass<R, WB>((E*)it.psi, it.n, P, it.stages, it.ops, (const cplx<R>*)it.mats, g - it.tile_begin, tile, bo);
  }
}

template <typename R, int WB>
hipError_t run(void* psi, int n, int m, const PassDescDev* passes, int pass, const PassStageDev* stages,
               const PassOpDev* ops, const void* mats, hipStream_t s) {
  typedef typename dev_elem<R>::E E;
  const size_t lds = ((size_t)1 << m) * sizeof(E);
  static size_t attr = 0;  // largest dynamic LDS size requested so far
  if (lds > attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_pass<R, WB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = lds;
  }
  const uint64_t tiles = capped_grid(1ull << (n - m));
  hipLaunchKernelGGL((k_pass<R, WB>), dim3((unsigned)tiles), dim3(kBlock), lds, s, (E*)psi, n, passes, pass, stages,
                     ops, (const cplx<R>*)mats);
  return hipGetLastError();
}

template <typename R, int WB>
hipError_t run_batch(const BatchItemDev* items, int count, uint64_t total_tiles, int max_m, hipStream_t s) {
  typedef typename dev_elem<R>::E E;
  const size_t lds = ((size_t)1 << max_m) * sizeof(E);
  static size_t attr = 0;
  if (lds > attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_pass_batch<R, WB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = lds;
  }
  const uint64_t blocks = capped_grid(total_tiles);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_pass_batch<R, WB>), dim3((unsigned)blocks), dim3(kBlock), lds, s, items, count, total_tiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pass(sv_dtype dt, void* psi, int n, int m, const PassDescDev* passes, int pass,
                       const PassStageDev* stages, const PassOpDev* ops, const void* mats, hipStream_t s) {
  if (dt == SV_C128) return run<double, 3>(psi, n, m, passes, pass, stages, ops, mats, s);
  return run<float, 4>(psi, n, m, passes, pass, stages, ops, mats, s);
}

hipError_t launch_pass_batch(sv_dtype dt, const BatchItemDev* items, int count, uint64_t total_tiles, int max_m,
                             hipStream_t s) {
  if (dt == SV_C128) return run_batch<double, 3>(items, count, total_tiles, max_m, s);
  return run_batch<float, 4>(items, count, total_tiles, max_m, s);
}

}  // namespace sv
