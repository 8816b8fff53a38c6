// Dense k-qubit gate sweep (3 <= k <= 6), the "generic gate" that general gate
// fusion produces (QueenV2 Sec. II-B, Sec. III-A tier 5).
//
// For every group of 2^k amplitudes that differ only in the gate's bits the
// new amplitudes are U times the old ones (Eq. 2/3 generalised; q[0] is the
// most significant bit of the local index).  Viewed as a matrix product
// Y = U X, column c of X is group c.
//
// A block works on tiles of C consecutive groups (2^k x C amplitudes).  A
// tile is a set of 2^(k + log2 C) indices: the gate's bits plus the lowest
// log2 C other bits vary, the remaining bits are the tile's base (the
// PDEP-like deposit of Sec. III-B).  Lanes walk a tile in address order, so
// every load and store instruction covers whole 128-byte lines whatever the
// gate's qubits are; LDS holds the tile as X[member][column].
#include "sv_device.h"
#include "sv_kernels.h"
#include "sv_tile_kernels.h"

namespace sv {
namespace {

constexpr int kBlock = 256;

// Address map of a tile: tile-local index e has bit j at physical position
// pos[j] (ascending; 64 = a column bit beyond the state, for states with
// fewer groups than a tile has columns) and contributes lds[j] (XOR) to the
// tile's LDS index member * C + column.  The tile's base deposits the
// work-block number into `rest`.
// The matrix-core kernels swizzle LDS: the column index is XORed with
// fm(member) ^ fc[column >> es] (es = log2 of the LDS entries in 256 bytes;
// fm(member) = XOR of fmb[b] over the set bits b of the member),
// chosen per gate so that the 64 lanes of a wave, which walk the tile in
// address order, spread over all banks; a run of 2^es aligned columns of one
// member stays a permutation of itself, so the matrix-core operand reads and
// result writes stay conflict-free.  lds[] already holds the swizzle.
struct DenseGeo {
  uint64_t rest;
  uint32_t nbits;
  uint32_t inv;       // tile-local bits with no physical position
  uint32_t pos[16];
  uint32_t lds[16];
  uint32_t fmb[6];    // swizzle of member bit b
  uint32_t fc[16];    // swizzle of column block c (columns c * 2^es ..)
};

// Per-lane part of the map: tile-local bits LB .. LB+7 come from the lane.
// LB = 1 moves complex64 amplitudes in 16-byte pairs: tile-local bit 0 is
// always physical bit 0 (the lowest bit is a gate bit or a column bit), so
// an element and its bit-0 partner are adjacent in memory.
struct LaneMap {
  uint64_t addr;
  uint32_t lds;
  bool on;
};

// X: the LDS weights carry a swizzle and combine by XOR (plain maps have
// disjoint weights and combine by OR).
template <int LB, int TB = 8, bool X = false>
__device__ __forceinline__ LaneMap lane_map(uint32_t t, const DenseGeo& g) {
  LaneMap m{0, 0, ((t << LB) & g.inv) == 0};
#pragma unroll
  for (int j = 0; j < TB; ++j)
    if ((t >> j) & 1u) {
      if (g.pos[LB + j] < 64) m.addr |= 1ull << g.pos[LB + j];
      if constexpr (X) m.lds ^= g.lds[LB + j];
      else m.lds |= g.lds[LB + j];
    }
  return m;
}

// Uniform part for element u of a lane (tile-local bits LB+TB ..; TB lane bits).
template <int LB, int U, int TB = 8, bool X = false>
__device__ __forceinline__ void elem_map(const DenseGeo& g, uint64_t* addr, uint32_t* lds, bool* on) {
  uint64_t a = 0;
  uint32_t l = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b)
    if ((U >> b) & 1) {
      if (g.pos[LB + TB + b] < 64) a |= 1ull << g.pos[LB + TB + b];
      if constexpr (X) l ^= g.lds[LB + TB + b];
      else l |= g.lds[LB + TB + b];
    }
  *addr = a;
  *lds = l;
  *on = (((uint32_t)U << (TB + LB)) & g.inv) == 0;
}

#define SV_FOR_U(PER, F)                                                  \
  F(0) if constexpr (PER > 1) { F(1) } if constexpr (PER > 2) { F(2) F(3) } \
  if constexpr (PER > 4) { F(4) F(5) F(6) F(7) }                           \
  if constexpr (PER > 8) { F(8) F(9) F(10) F(11) F(12) F(13) F(14) F(15) }

// Tile columns of the VALU kernel: the tile holds 2048 amplitudes.
template <int K>
constexpr int tile_cols() {
  return 2048 >> K;
}

template <typename E, int K>
__global__ __launch_bounds__(kBlock) void k_dense(E* __restrict__ psi, uint64_t nwork, DenseGeo g,
                                                  const typename elem_traits<E>::R* __restrict__ um) {
  typedef typename elem_traits<E>::R R;
  constexpr int D = 1 << K;
  constexpr int C = tile_cols<K>();
  constexpr int PER = D * C / kBlock / 2;  // 16-byte pairs per lane
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* us = reinterpret_cast<cplx<R>*>(smem);  // D x D
  cplx<R>* xs = us + D * D;                          // D x C, row r = member r
  flt4* pairs = reinterpret_cast<flt4*>(psi);
  const int t = threadIdx.x;
  for (int e = t; e < D * D; e += kBlock) us[e] = cplx<R>{um[2 * e], um[2 * e + 1]};
  const LaneMap lm = lane_map<1>((uint32_t)t, g);
  const uint32_t l0 = g.lds[0];  // LDS offset of the bit-0 partner
  for (uint64_t wb = xcd_block(); wb < nwork; wb += gridDim.x) {
    const uint64_t base = deposit(wb, g.rest) | lm.addr;
    flt4 buf[PER];
#define SV_LD(U)                                                  \
    {                                                             \
      uint64_t a;                                                 \
      uint32_t l;                                                 \
      bool on;                                                    \
      elem_map<1, U>(g, &a, &l, &on);                             \
      if (on && lm.on) buf[U] = ld(pairs + ((base | a) >> 1));    \
    }
    SV_FOR_U(PER, SV_LD)
#undef SV_LD
    __syncthreads();  // U is staged and the previous tile's readers are done
#define SV_LDS(U)                                                 \
    {                                                             \
      uint64_t a;                                                 \
      uint32_t l;                                                 \
      bool on;                                                    \
      elem_map<1, U>(g, &a, &l, &on);                             \
      if (on && lm.on) {                                          \
        xs[lm.lds | l] = cplx<R>{buf[U].x, buf[U].y};             \
        xs[lm.lds | l | l0] = cplx<R>{buf[U].z, buf[U].w};        \
      }                                                           \
    }
    SV_FOR_U(PER, SV_LDS)
#undef SV_LDS
    __syncthreads();
#define SV_OUT(U)                                                 \
    {                                                             \
      uint64_t a;                                                 \
      uint32_t l;                                                 \
      bool on;                                                    \
      elem_map<1, U>(g, &a, &l, &on);                             \
      if (on && lm.on) {                                          \
        flt4 o;                                                   \
        _Pragma("unroll")                                         \
        for (int h = 0; h < 2; ++h) {                             \
          const uint32_t li = lm.lds | l | (h ? l0 : 0u), r = li / C, c = li % C; \
          cplx<R> y = {0, 0};                                     \
          const cplx<R>* urow = us + r * D;                       \
          _Pragma("unroll 8")                                     \
          for (int s = 0; s < D; ++s) y = cfma(y, urow[s], xs[s * C + c]); \
          if (h) { o.z = y.re; o.w = y.im; } else { o.x = y.re; o.y = y.im; } \
        }                                                         \
        st(pairs + ((base | a) >> 1), o);                         \
      }                                                           \
    }
    SV_FOR_U(PER, SV_OUT)
#undef SV_OUT
  }
}

template <typename E, int K>
hipError_t run(void* psi, int n, const DenseGeo& g, const void* m, hipStream_t s) {
  typedef typename elem_traits<E>::R R;
  constexpr int D = 1 << K;
  constexpr int C = tile_cols<K>();
  const size_t lds = (size_t)(D * D + D * C) * sizeof(cplx<R>);
  static KernelLaunchCache cache;
  hipError_t e = prepare_launch(cache, (const void*)k_dense<E, K>, kBlock, lds, nullptr);
  if (e != hipSuccess) return e;
  const uint64_t ngroups = 1ull << (n - K);
  const uint64_t nwork = (ngroups + C - 1) / C;
  hipLaunchKernelGGL((k_dense<E, K>), dim3((unsigned)capped_grid(nwork)), dim3(kBlock), lds, s, (E*)psi, nwork, g,
                     (const R*)m);
  return hipGetLastError();
}

// ---------------------------------------------------------------- MFMA
// Y = U X as a real GEMM on the interleaved storage: with rows of Y and X
// indexed 2*member + (0: re, 1: im), the operator is the real 2D x 2D matrix
// A[2i+a][2j+b] = (Ur, -Ui; Ui, Ur)[a][b] of U[i][j], so the state is never
// de-interleaved.  Matrix-core tiles (operand layouts of the instructions):
//   FP32 (complex64):  v_mfma_f32_32x32x2_f32, BM = BN = 32, BK = 2
//   FP64 (complex128): v_mfma_f64_16x16x4_f64, BM = BN = 16, BK = 4
// A operand: lane l holds A[l % BM][l / BM]; B operand: lane l holds
// B[l / BN][l % BN]; accumulator (BM x BN), column l % BN: FP32 register r of
// lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, FP64 register r holds row
// (l / 16) + 4 r (measured on gfx950 with one-hot operands).  The rows of a
// block are assigned to (member, re/im) so that registers r, r + 1 of a lane
// are the re and im parts of one output amplitude: FP32 blocks take real rows
// in order; an FP64 block row rho = g + 4 r holds member 2 g + r / 2, part r % 2
// of its 8 members.  Accumulation is in the input precision.
// A block stages U (rows padded by one entry against LDS bank conflicts) once
// and loops over column tiles of NC groups: each tile is gathered with all of
// a lane's loads in flight, then the 4 waves share its (row block, column
// block) output tiles.
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename R>
struct mfma_shape;
template <>
struct mfma_shape<float> {
  static constexpr int BM = 32, BN = 32, BK = 2, NACC = 16;
  typedef floatx16 acc_t;
  typedef flt2 E;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  // block row -> (member within the block's 16, re/im)
  static __device__ __forceinline__ void row_of(int rho, int* mem, int* part) {
    *mem = rho >> 1;
    *part = rho & 1;
  }
  // member (within the block) written by registers r, r + 1 of lane l (r even)
  static __device__ __forceinline__ int out_member(int l, int r) { return (8 * (r / 4) + 4 * (l / 32) + (r % 4)) >> 1; }
  // the same for even r, as uniform and per-lane parts (disjoint bits)
  static __device__ __forceinline__ int out_member_u(int r) { return 4 * (r / 4) + (r % 4) / 2; }
  static __device__ __forceinline__ int out_member_l(int l) { return 2 * (l / 32); }
  static constexpr int MPB = 16;  // members per row block
  static constexpr int ES = 5;    // log2 of the LDS entries (8 bytes) in 256 bytes
  // global 16-byte element: a complex64 pair (LDS entries li and li | l0;
  // li ^ l0 in a swizzled map)
  typedef flt4 G;
  static __device__ __forceinline__ void to_lds(E* xs, uint32_t li, uint32_t l0, G v) {
    xs[li] = E{v.x, v.y};
    xs[li | l0] = E{v.z, v.w};
  }
  static __device__ __forceinline__ void to_lds_x(E* xs, uint32_t li, uint32_t l0, G v) {
    xs[li] = E{v.x, v.y};
    xs[li ^ l0] = E{v.z, v.w};
  }
  static __device__ __forceinline__ G from_lds(const E* xs, uint32_t li, uint32_t l0) {
    const E a = xs[li], b = xs[li | l0];
    return G{a.x, a.y, b.x, b.y};
  }
  static __device__ __forceinline__ G from_lds_x(const E* xs, uint32_t li, uint32_t l0) {
    const E a = xs[li], b = xs[li ^ l0];
    return G{a.x, a.y, b.x, b.y};
  }
};
template <>
struct mfma_shape<double> {
  static constexpr int BM = 16, BN = 16, BK = 4, NACC = 4;
  typedef doublex4 acc_t;
  typedef dbl2 E;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void row_of(int rho, int* mem, int* part) {
    *mem = 2 * (rho % 4) + (rho / 4) / 2;
    *part = (rho / 4) % 2;
  }
  static __device__ __forceinline__ int out_member(int l, int r) { return 2 * (l / 16) + r / 2; }
  static __device__ __forceinline__ int out_member_u(int r) { return r / 2; }
  static __device__ __forceinline__ int out_member_l(int l) { return 2 * (l / 16); }
  static constexpr int MPB = 8;
  static constexpr int ES = 4;  // log2 of the LDS entries (16 bytes) in 256 bytes
  typedef dbl2 G;  // one complex128 amplitude
  static __device__ __forceinline__ void to_lds(E* xs, uint32_t li, uint32_t, G v) { xs[li] = v; }
  static __device__ __forceinline__ G from_lds(const E* xs, uint32_t li, uint32_t) { return xs[li]; }
  static __device__ __forceinline__ void to_lds_x(E* xs, uint32_t li, uint32_t, G v) { xs[li] = v; }
  static __device__ __forceinline__ G from_lds_x(const E* xs, uint32_t li, uint32_t) { return xs[li]; }
};

// groups per column tile: the X tile holds 4096 complex64 / 2048 complex128
// amplitudes (32 KiB), and at least one column block
template <typename R, int K>
constexpr int mfma_cols() {
  constexpr int target = (sizeof(R) == 4 ? 4096 : (K == 6 ? 4096 : 2048)) >> K;
  return target < mfma_shape<R>::BN ? mfma_shape<R>::BN : target;
}

template <typename R, int K>
constexpr size_t mfma_lds() {
  return (size_t)(1 << K) * mfma_cols<R, K>() * 2 * sizeof(R);
}

// Waves own row blocks: wave w computes the output tiles w, w + W, ... of
// the (row block, column block) grid, tile = rb + RBLK * cb, so it only ever
// needs the row blocks (w + W i) mod RBLK.  Their A fragments (the embedded
// U) are loop-invariant over column tiles and stay in registers.  W = 4
// waves per block, 8 for complex128 k = 6 (one row block of A per wave, so a
// block fits two waves per SIMD).
template <typename R, int K>
struct mfma_plan {
  typedef mfma_shape<R> MS;
  static constexpr int D = 1 << K;
  static constexpr int NC = mfma_cols<R, K>();
  static constexpr int W = (sizeof(R) == 8 && K == 6) ? 8 : 4;
  static constexpr int THREADS = 64 * W, TB = W == 8 ? 9 : 8;
  static constexpr int RBLK = 2 * D / MS::BM, CBLK = NC / MS::BN, TILES = RBLK * CBLK;
  static constexpr int TPW = (TILES + W - 1) / W;              // output tiles per wave
  static constexpr int NRB = RBLK >= W ? RBLK / W : 1;         // distinct row blocks per wave
  static constexpr int KSTEPS = 2 * D / MS::BK;
  static_assert(RBLK < W || RBLK % W == 0, "row blocks split evenly over the waves");
  static_assert(NC / MS::BN <= 16, "column blocks fit the swizzle table");
};

template <typename R, int K>
__global__ __launch_bounds__((mfma_plan<R, K>::THREADS)) void k_dense_mfma(typename mfma_shape<R>::E* __restrict__ psi, uint64_t nwork,
                                                       DenseGeo g, const R* __restrict__ um) {
  typedef mfma_shape<R> MS;
  typedef mfma_plan<R, K> MP;
  typedef typename MS::E E;
  constexpr int D = MP::D, NC = MP::NC, RBLK = MP::RBLK, TILES = MP::TILES, TPW = MP::TPW, NRB = MP::NRB;
  constexpr int KSTEPS = MP::KSTEPS, W = MP::W, TB = MP::TB;
  // global memory moves in 16-byte elements: complex128 amplitudes, or
  // complex64 pairs on tile-local bit 0 (LB = 1)
  constexpr int LB = sizeof(R) == 4 ? 1 : 0;
  typedef typename mfma_shape<R>::G G;
  constexpr int PER = (D * NC / MP::THREADS) >> LB;  // 16-byte elements per lane
  extern __shared__ __align__(16) unsigned char smem[];
  E* xs = reinterpret_cast<E*>(smem);  // [member][NC]
  const int t = threadIdx.x, w = t / 64, l = t % 64;
  // A fragments of this wave's row blocks: lane l supplies A[l % BM][BK ks + l / BM]
  R afrag[NRB][KSTEPS];
#pragma unroll
  for (int i = 0; i < NRB; ++i) {
    const int rb = (w + W * i) % RBLK;
    int ai, aa;  // output member and re/im of the A row this lane supplies
    MS::row_of(l % MS::BM, &ai, &aa);
    ai += MS::MPB * rb;
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
      const int ak = MS::BK * ks + l / MS::BM;  // real column of A (= real row of B)
      const R ur = um[2 * (ai * D + (ak >> 1))], ui = um[2 * (ai * D + (ak >> 1)) + 1];
      afrag[i][ks] = aa == 0 ? ((ak & 1) == 0 ? ur : -ui) : ((ak & 1) == 0 ? ui : ur);
    }
  }
  const LaneMap lm = lane_map<LB, TB>((uint32_t)t, g);
  const uint32_t l0 = g.lds[0];  // LDS offset of the bit-0 partner (LB = 1)
  G* gp = reinterpret_cast<G*>(psi);
  // software-pipelined over column tiles: the next tile's loads are in flight
  // while the current tile runs on the matrix cores and is stored
  uint64_t wb = xcd_block();
  if (wb >= nwork) return;
  G buf[PER];
#define SV_LD(U)                                                      \
  {                                                                   \
    uint64_t a;                                                       \
    uint32_t li;                                                      \
    bool on;                                                          \
    elem_map<LB, U, TB>(g, &a, &li, &on);                                 \
    buf[U] = ld(gp + (((on && lm.on) ? (ldbase | a) : ldbase) >> LB)); \
  }
  {
    const uint64_t ldbase = deposit(wb, g.rest) | lm.addr;
    SV_FOR_U(PER, SV_LD)
  }
  while (true) {
    const uint64_t nb = wb + gridDim.x;
    const uint64_t base = deposit(wb, g.rest) | lm.addr;
    __syncthreads();  // the previous tile's store phase is done with LDS
#define SV_LDS(U)                                                     \
    {                                                                 \
      uint64_t a;                                                     \
      uint32_t li;                                                    \
      bool on;                                                        \
      elem_map<LB, U, TB>(g, &a, &li, &on);                               \
      if (on && lm.on) mfma_shape<R>::to_lds(xs, lm.lds | li, l0, buf[U]); \
    }
    SV_FOR_U(PER, SV_LDS)
#undef SV_LDS
    __syncthreads();
    if (nb < nwork) {
      const uint64_t ldbase = deposit(nb, g.rest) | lm.addr;
      SV_FOR_U(PER, SV_LD)
    }
    typename MS::acc_t acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int tile = w + W * i;
      acc[i] = typename MS::acc_t{};
      if (tile >= TILES) continue;
      const int bcol = MS::BN * (tile / RBLK) + l % MS::BN;
#pragma unroll
      for (int ks = 0; ks < KSTEPS; ++ks) {
        const int bk = MS::BK * ks + l / MS::BN;
        const E xv = xs[(bk >> 1) * NC + bcol];
        const R b = (bk & 1) ? xv.y : xv.x;
        acc[i] = MS::mma(afrag[i % NRB][ks], b, acc[i]);  // row block (w + W i) % RBLK
      }
    }
    __syncthreads();  // every wave has read X: the outputs replace it in LDS
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int tile = w + W * i;
      if (tile >= TILES) continue;
      const int rb = tile % RBLK, cb = tile / RBLK;
      const int bcol = MS::BN * cb + l % MS::BN;
#pragma unroll
      for (int r = 0; r < MS::NACC; r += 2) {
        const int mem = MS::MPB * rb + MS::out_member(l, r);
        E y;
        y.x = acc[i][r];
        y.y = acc[i][r + 1];
        xs[mem * NC + bcol] = y;
      }
    }
    __syncthreads();
    // store in address order
#define SV_ST(U)                                                      \
    {                                                                 \
      uint64_t a;                                                     \
      uint32_t li;                                                    \
      bool on;                                                        \
      elem_map<LB, U, TB>(g, &a, &li, &on);                               \
      if (on && lm.on) st(gp + ((base | a) >> LB), mfma_shape<R>::from_lds(xs, lm.lds | li, l0)); \
    }
    SV_FOR_U(PER, SV_ST)
#undef SV_ST
    if (nb >= nwork) break;
    wb = nb;
  }
#undef SV_LD
}

// Swizzle of member mu from those of its single bits (the swizzle is linear).
template <int K>
__device__ __forceinline__ uint32_t member_swizzle(int mu, const uint32_t* fmb) {
  uint32_t f = 0;
#pragma unroll
  for (int b = 0; b < K; ++b)
    if ((mu >> b) & 1) f ^= fmb[b];
  return f;
}

// The same contraction on a swizzled tile (see DenseGeo): operand and result
// addresses take the member's and column block's swizzle.
template <typename R, int K>
__global__ __launch_bounds__((mfma_plan<R, K>::THREADS)) void k_dense_mfma_swz(typename mfma_shape<R>::E* __restrict__ psi, uint64_t nwork,
                                                       DenseGeo g, const R* __restrict__ um) {
  typedef mfma_shape<R> MS;
  typedef mfma_plan<R, K> MP;
  typedef typename MS::E E;
  constexpr int D = MP::D, NC = MP::NC, RBLK = MP::RBLK, TILES = MP::TILES, TPW = MP::TPW, NRB = MP::NRB;
  constexpr int KSTEPS = MP::KSTEPS, W = MP::W, TB = MP::TB;
  // global memory moves in 16-byte elements: complex128 amplitudes, or
  // complex64 pairs on tile-local bit 0 (LB = 1)
  constexpr int LB = sizeof(R) == 4 ? 1 : 0;
  typedef typename mfma_shape<R>::G G;
  constexpr int PER = (D * NC / MP::THREADS) >> LB;  // 16-byte elements per lane
  extern __shared__ __align__(16) unsigned char smem[];
  E* xs = reinterpret_cast<E*>(smem);  // [member][NC]
  const int t = threadIdx.x, l = t % 64;
  const int w = __builtin_amdgcn_readfirstlane(t / 64);  // uniform per wave
  // A fragments of this wave's row blocks: lane l supplies A[l % BM][BK ks + l / BM]
  R afrag[NRB][KSTEPS];
#pragma unroll
  for (int i = 0; i < NRB; ++i) {
    const int rb = (w + W * i) % RBLK;
    int ai, aa;  // output member and re/im of the A row this lane supplies
    MS::row_of(l % MS::BM, &ai, &aa);
    ai += MS::MPB * rb;
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
      const int ak = MS::BK * ks + l / MS::BM;  // real column of A (= real row of B)
      const R ur = um[2 * (ai * D + (ak >> 1))], ui = um[2 * (ai * D + (ak >> 1)) + 1];
      afrag[i][ks] = aa == 0 ? ((ak & 1) == 0 ? ur : -ui) : ((ak & 1) == 0 ? ui : ur);
    }
  }
  const LaneMap lm = lane_map<LB, TB, true>((uint32_t)t, g);
  const uint32_t l0 = g.lds[0];  // LDS offset of the bit-0 partner (LB = 1)
  G* gp = reinterpret_cast<G*>(psi);
  const R* xr = reinterpret_cast<const R*>(smem);
  // per-lane parts of the operand and result members (the swizzle is linear)
  const int bml = (l / MS::BN) >> 1, bpart = (l / MS::BN) & 1, oml = MS::out_member_l(l);
  uint32_t fmb0[K];
#pragma unroll
  for (int b = 0; b < K; ++b) fmb0[b] = g.fmb[b];
  const uint32_t bfl = member_swizzle<K>(bml, fmb0), ofl = member_swizzle<K>(oml, fmb0);
  // software-pipelined over column tiles: the next tile's loads are in flight
  // while the current tile runs on the matrix cores and is stored
  uint64_t wb = xcd_block();
  if (wb >= nwork) return;
  G buf[PER];
#define SV_LD(U)                                                      \
  {                                                                   \
    uint64_t a;                                                       \
    uint32_t li;                                                      \
    bool on;                                                          \
    elem_map<LB, U, TB, true>(g, &a, &li, &on);                                 \
    buf[U] = ld(gp + (((on && lm.on) ? (ldbase | a) : ldbase) >> LB)); \
  }
  {
    const uint64_t ldbase = deposit(wb, g.rest) | lm.addr;
    SV_FOR_U(PER, SV_LD)
  }
  while (true) {
    const uint64_t nb = wb + gridDim.x;
    const uint64_t base = deposit(wb, g.rest) | lm.addr;
    __syncthreads();  // the previous tile's store phase is done with LDS
#define SV_LDS(U)                                                     \
    {                                                                 \
      uint64_t a;                                                     \
      uint32_t li;                                                    \
      bool on;                                                        \
      elem_map<LB, U, TB, true>(g, &a, &li, &on);                               \
      if (on && lm.on) mfma_shape<R>::to_lds_x(xs, lm.lds ^ li, l0, buf[U]); \
    }
    SV_FOR_U(PER, SV_LDS)
#undef SV_LDS
    __syncthreads();
    if (nb < nwork) {
      const uint64_t ldbase = deposit(nb, g.rest) | lm.addr;
      SV_FOR_U(PER, SV_LD)
    }
    typename MS::acc_t acc[TPW];
    uint32_t fmb[K];
    {
      // swizzles of the single member bits, opaque per tile: the compiler then
      // derives each k-step's swizzle with a few scalar XORs instead of
      // holding one value per k-step in registers
#pragma unroll
      for (int b = 0; b < K; ++b) {
        fmb[b] = g.fmb[b];
        asm volatile("" : "+s"(fmb[b]));
      }
      const uint32_t blane = 2 * ((uint32_t)(bml * NC + l % MS::BN) ^ bfl) + bpart;
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int tile = w + W * i;
        acc[i] = typename MS::acc_t{};
        if (tile >= TILES) continue;
        const int cb = tile / RBLK;
        const uint32_t bl = blane ^ (2u * (uint32_t)(MS::BN * cb ^ g.fc[cb]));
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
          // B[bk][bcol], real row bk = 2 member + part: one float per lane at
          // LDS entry ((mu + bml) NC + bcol) ^ fm(mu + bml) ^ fc[cb]
          const int mu = (MS::BK * ks) >> 1;  // uniform part of the member (bits disjoint from bml)
          const R b = xr[2 * mu * NC + (bl ^ (2u * member_swizzle<K>(mu, fmb)))];
          acc[i] = MS::mma(afrag[i % NRB][ks], b, acc[i]);  // row block (w + W i) % RBLK
        }
      }
    }
    __syncthreads();  // every wave has read X: the outputs replace it in LDS
    const uint32_t olane = (uint32_t)(oml * NC + l % MS::BN) ^ ofl;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int tile = w + W * i;
      if (tile >= TILES) continue;
      const int rb = tile % RBLK, cb = tile / RBLK;
#pragma unroll
      for (int r = 0; r < MS::NACC; r += 2) {
        // result member mu + oml, column BN cb + l % BN
        const int mu = MS::MPB * rb + MS::out_member_u(r);
        E y;
        y.x = acc[i][r];
        y.y = acc[i][r + 1];
        const uint32_t ol = olane ^ (uint32_t)(MS::BN * cb ^ g.fc[cb]);
        xs[mu * NC + (ol ^ member_swizzle<K>(mu, fmb))] = y;
      }
    }
    __syncthreads();
    // store in address order
#define SV_ST(U)                                                      \
    {                                                                 \
      uint64_t a;                                                     \
      uint32_t li;                                                    \
      bool on;                                                        \
      elem_map<LB, U, TB, true>(g, &a, &li, &on);                               \
      if (on && lm.on) st(gp + ((base | a) >> LB), mfma_shape<R>::from_lds_x(xs, lm.lds ^ li, l0)); \
    }
    SV_FOR_U(PER, SV_ST)
#undef SV_ST
    if (nb >= nwork) break;
    wb = nb;
  }
#undef SV_LD
}

// ---------------------------------------------------------------- 3M
// The same product with three real matrix products instead of the four of
// the real embedding (Gauss's complex multiplication): with U = Ur + i Ui and
// X = Xr + i Xi,
//   P1 = Ur Xr,  P2 = Ui Xi,  P3 = (Ur + Ui)(Xr + Xi),
//   Yr = P1 - P2,  Yi = P3 - P1 - P2,
// so the matrix cores do 6 D^2 real multiply-adds per column instead of 8.
// Real rows of each product are members, so a gate needs D >= BM (complex64
// k >= 5, complex128 k >= 4).  The tile, its gather and its store are those
// of the embedding kernels; a lane reads one complex operand per k-step and
// feeds its real part, imaginary part and their sum to the three products.
// SWZ: the tile is swizzled (member and column-block masks, see DenseGeo).
template <typename R, int K>
struct m3_plan {
  typedef mfma_shape<R> MS;
  static constexpr int D = 1 << K;
  static constexpr int NC = mfma_cols<R, K>();
  static constexpr int W = (sizeof(R) == 8 && K == 6) ? 8 : 4;
  static constexpr int THREADS = 64 * W, TB = W == 8 ? 9 : 8;
  static constexpr int RB = D / MS::BM;             // row blocks (members)
  static constexpr int CBLK = NC / MS::BN, TILES = RB * CBLK;
  static constexpr int TPW = TILES / W;             // output tiles per wave
  static constexpr int KS = D / MS::BK;             // k-steps (members)
  static_assert(D >= MS::BM, "3M products need a full row block of members");
  static_assert(TILES % W == 0 && W % RB == 0, "each wave keeps one row block");
};

// Output member (within a row block) of accumulator register r of lane l.
template <typename R>
__device__ __forceinline__ int m3_out_member(int l, int r) {
  if constexpr (sizeof(R) == 4) return 8 * (r / 4) + 4 * (l / 32) + r % 4;
  else return l / 16 + 4 * r;
}

template <typename R, int K, bool SWZ>
__global__ __launch_bounds__((m3_plan<R, K>::THREADS)) void k_dense_3m(typename mfma_shape<R>::E* __restrict__ psi,
                                                                      uint64_t nwork, DenseGeo g,
                                                                      const R* __restrict__ um) {
  typedef mfma_shape<R> MS;
  typedef m3_plan<R, K> MP;
  typedef typename MS::E E;
  constexpr int D = MP::D, NC = MP::NC, RB = MP::RB, TPW = MP::TPW, KS = MP::KS, W = MP::W, TB = MP::TB;
  constexpr int LB = sizeof(R) == 4 ? 1 : 0;
  typedef typename mfma_shape<R>::G G;
  constexpr int PER = (D * NC / MP::THREADS) >> LB;  // 16-byte elements per lane
  extern __shared__ __align__(16) unsigned char smem[];
  E* xs = reinterpret_cast<E*>(smem);  // [member][NC]
  const int t = threadIdx.x, l = t % 64;
  const int w = __builtin_amdgcn_readfirstlane(t / 64);
  const int rb = w % RB;  // this wave's row block (tiles w, w + W, ... share it)
  // A fragments: lane l supplies row l % BM, column BK ks + l / BM of Ur, Ui
  // and Ur + Ui (rows and columns are members)
  R a1[KS], a2[KS], a3[KS];
  {
    const int row = MS::BM * rb + l % MS::BM;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int col = MS::BK * ks + l / MS::BM;
      const R ur = um[2 * (row * D + col)], ui = um[2 * (row * D + col) + 1];
      a1[ks] = ur;
      a2[ks] = ui;
      a3[ks] = ur + ui;
    }
  }
  const LaneMap lm = lane_map<LB, TB, SWZ>((uint32_t)t, g);
  const uint32_t l0 = g.lds[0];
  G* gp = reinterpret_cast<G*>(psi);
  // lane parts of the operand member (l / BN) and of the result members
  const int bml = l / MS::BN;
  uint32_t fmb0[K];
#pragma unroll
  for (int b = 0; b < K; ++b) fmb0[b] = SWZ ? g.fmb[b] : 0u;
  const uint32_t bfl = member_swizzle<K>(bml, fmb0);
  uint64_t wb = xcd_block();
  if (wb >= nwork) return;
  G buf[PER];
#define SV_LD(U)                                                        \
  {                                                                     \
    uint64_t a;                                                         \
    uint32_t li;                                                        \
    bool on;                                                            \
    elem_map<LB, U, TB, SWZ>(g, &a, &li, &on);                          \
    buf[U] = ld(gp + (((on && lm.on) ? (ldbase | a) : ldbase) >> LB));  \
  }
  {
    const uint64_t ldbase = deposit(wb, g.rest) | lm.addr;
    SV_FOR_U(PER, SV_LD)
  }
  while (true) {
    const uint64_t nb = wb + gridDim.x;
    const uint64_t base = deposit(wb, g.rest) | lm.addr;
    __syncthreads();  // the previous tile's store phase is done with LDS
#define SV_LDS(U)                                                       \
    {                                                                   \
      uint64_t a;                                                       \
      uint32_t li;                                                      \
      bool on;                                                          \
      elem_map<LB, U, TB, SWZ>(g, &a, &li, &on);                        \
      if (on && lm.on) {                                                \
        if constexpr (SWZ) mfma_shape<R>::to_lds_x(xs, lm.lds ^ li, l0, buf[U]); \
        else mfma_shape<R>::to_lds(xs, lm.lds | li, l0, buf[U]);        \
      }                                                                 \
    }
    SV_FOR_U(PER, SV_LDS)
#undef SV_LDS
    __syncthreads();
    if (nb < nwork) {
      const uint64_t ldbase = deposit(nb, g.rest) | lm.addr;
      SV_FOR_U(PER, SV_LD)
    }
    typename MS::acc_t p1[TPW], p2[TPW], p3[TPW];
    uint32_t fmb[K];
#pragma unroll
    for (int b = 0; b < K; ++b) {
      fmb[b] = SWZ ? g.fmb[b] : 0u;
      asm volatile("" : "+s"(fmb[b]));
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int cb = (w + W * i) / RB;
      const uint32_t bl = (uint32_t)(bml * NC) + ((uint32_t)(MS::BN * cb + l % MS::BN) ^ bfl ^ (SWZ ? g.fc[cb] : 0u));
      p1[i] = p2[i] = p3[i] = typename MS::acc_t{};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        // operand member BK ks + bml, column BN cb + l % BN
        const int mu = MS::BK * ks;  // uniform part (bits disjoint from bml)
        const E xv = xs[mu * NC + (bl ^ member_swizzle<K>(mu, fmb))];
        p1[i] = MS::mma(a1[ks], xv.x, p1[i]);
        p2[i] = MS::mma(a2[ks], xv.y, p2[i]);
        p3[i] = MS::mma(a3[ks], xv.x + xv.y, p3[i]);
      }
    }
    __syncthreads();  // every wave has read X: the outputs replace it in LDS
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int cb = (w + W * i) / RB;
      const uint32_t col = (uint32_t)(MS::BN * cb + l % MS::BN) ^ (SWZ ? g.fc[cb] : 0u);
#pragma unroll
      for (int r = 0; r < MS::NACC; ++r) {
        const int mu = MS::BM * rb + m3_out_member<R>(l, r);
        E y;
        y.x = p1[i][r] - p2[i][r];
        y.y = p3[i][r] - p1[i][r] - p2[i][r];
        xs[mu * NC + (col ^ member_swizzle<K>(mu, fmb))] = y;
      }
    }
    __syncthreads();
#define SV_ST(U)                                                        \
    {                                                                   \
      uint64_t a;                                                       \
      uint32_t li;                                                      \
      bool on;                                                          \
      elem_map<LB, U, TB, SWZ>(g, &a, &li, &on);                        \
      if (on && lm.on) {                                                \
        if constexpr (SWZ) st(gp + ((base | a) >> LB), mfma_shape<R>::from_lds_x(xs, lm.lds ^ li, l0)); \
        else st(gp + ((base | a) >> LB), mfma_shape<R>::from_lds(xs, lm.lds | li, l0)); \
      }                                                                 \
    }
    SV_FOR_U(PER, SV_ST)
#undef SV_ST
    if (nb >= nwork) break;
    wb = nb;
  }
#undef SV_LD
}

template <typename R, int K, bool SWZ>
hipError_t launch_3m(void* psi, uint64_t nwork, const DenseGeo& g, const void* m, hipStream_t s) {
  constexpr size_t lds = mfma_lds<R, K>();
  static KernelLaunchCache cache;
  hipError_t e = prepare_launch(cache, (const void*)k_dense_3m<R, K, SWZ>, m3_plan<R, K>::THREADS, lds, nullptr);
  if (e != hipSuccess) return e;
  const uint64_t blocks = nwork < 4096 ? nwork : 4096;
  hipLaunchKernelGGL((k_dense_3m<R, K, SWZ>), dim3((unsigned)blocks), dim3(m3_plan<R, K>::THREADS), lds, s,
                     (typename mfma_shape<R>::E*)psi, nwork, g, (const R*)m);
  return hipGetLastError();
}

DenseGeo make_geo(int n, int k, const int* q, int nc, int es, int lb);

template <typename R, int K, bool SWZ>
hipError_t launch_mfma(void* psi, uint64_t nwork, const DenseGeo& g, const void* m, hipStream_t s) {
  constexpr size_t lds = mfma_lds<R, K>();
  const void* fn = SWZ ? (const void*)k_dense_mfma_swz<R, K> : (const void*)k_dense_mfma<R, K>;
  static KernelLaunchCache cache;
  hipError_t e = prepare_launch(cache, fn, mfma_plan<R, K>::THREADS, lds, nullptr);
  if (e != hipSuccess) return e;
  // persistent blocks: enough to fill the chip several times over, each
  // amortising its A fragments (loaded once) over many column tiles
  const uint64_t blocks = nwork < 4096 ? nwork : 4096;
  if constexpr (SWZ)
    hipLaunchKernelGGL((k_dense_mfma_swz<R, K>), dim3((unsigned)blocks), dim3(mfma_plan<R, K>::THREADS), lds, s,
                       (typename mfma_shape<R>::E*)psi, nwork, g, (const R*)m);
  else
    hipLaunchKernelGGL((k_dense_mfma<R, K>), dim3((unsigned)blocks), dim3(mfma_plan<R, K>::THREADS), lds, s,
                       (typename mfma_shape<R>::E*)psi, nwork, g, (const R*)m);
  return hipGetLastError();
}

DenseGeo make_geo(int n, int k, const int* q, int nc, int es, int lb);

// The swizzled kernel runs when the plain layout would put a wave's 64 lanes
// on at most a quarter (complex64 k = 6: a sixteenth) of the LDS bank groups
// they could use (member bits among the lanes: low qubit placements); the
// plain kernel addresses its operands more cheaply and runs otherwise.
template <typename R, int K>
hipError_t run_mfma(void* psi, int n, const int* q, const void* m, hipStream_t s) {
  constexpr int NC = mfma_cols<R, K>();
  constexpr int LB = sizeof(R) == 4 ? 1 : 0;
  const uint64_t ngroups = 1ull << (n - K);
  const uint64_t nwork = (ngroups + NC - 1) / NC;
  const DenseGeo plain = make_geo(n, K, q, NC, 0, LB);
  // distinct bank groups (LDS index mod 2^ES) the 64 lanes of a wave touch
  uint32_t seen[2] = {0, 0};
  for (uint32_t t = 0; t < 64; ++t) {
    uint32_t x = 0;
    for (int j = 0; j < 6 && LB + j < (int)plain.nbits; ++j)
      if ((t >> j) & 1u) x |= plain.lds[LB + j];
    x &= (1u << mfma_shape<R>::ES) - 1u;
    seen[x >> 5] |= 1u << (x & 31u);
  }
  const int distinct = __builtin_popcount(seen[0]) + __builtin_popcount(seen[1]);
  // the complex64 k = 6 kernel is matrix-bound: the swizzle's extra address
  // arithmetic pays only against the worst conflicts
  const int factor = (sizeof(R) == 4 && K == 6) ? 16 : 4;
  const bool swz = distinct * factor <= (1 << mfma_shape<R>::ES);
  if constexpr ((1 << K) >= mfma_shape<R>::BM) {
    if (swz) return launch_3m<R, K, true>(psi, nwork, make_geo(n, K, q, NC, mfma_shape<R>::ES, LB), m, s);
    return launch_3m<R, K, false>(psi, nwork, plain, m, s);
  }
  if (swz) return launch_mfma<R, K, true>(psi, nwork, make_geo(n, K, q, NC, mfma_shape<R>::ES, LB), m, s);
  return launch_mfma<R, K, false>(psi, nwork, plain, m, s);
}

// Tile map of a k-qubit gate q[0..k-1] (q[0] = MSB of the member index)
// with nc columns per tile (a power of two), for an n-qubit state.  es > 0
// adds the LDS swizzle for a kernel whose lanes take tile-local bits lb ..
// (es = log2 of the LDS entries in 256 bytes); es = 0 leaves LDS unswizzled.
DenseGeo make_geo(int n, int k, const int* q, int nc, int es, int lb) {
  int cb = 0;
  while ((1 << cb) < nc) ++cb;
  struct Bit {
    uint32_t pos, lds;
    int member, col;  // member bit or column bit (-1: not)
  } bits[16];
  int nb = 0;
  uint64_t gate = 0;
  for (int i = 0; i < k; ++i) {
    bits[nb++] = {(uint32_t)q[i], (1u << (k - 1 - i)) << cb, k - 1 - i, -1};
    gate |= 1ull << q[i];
  }
  int col = 0;
  for (int p = 0; p < n && col < cb; ++p)
    if (!((gate >> p) & 1)) {
      bits[nb++] = {(uint32_t)p, 1u << col, -1, col};
      ++col;
    }
  uint64_t tilemask = gate;
  for (int i = k; i < nb; ++i) tilemask |= 1ull << bits[i].pos;
  for (; col < cb; ++col) bits[nb++] = {64u, 1u << col, -1, col};  // beyond the state
  for (int i = 1; i < nb; ++i)
    for (int j = i; j > 0 && bits[j - 1].pos > bits[j].pos; --j) {
      const Bit tmp = bits[j];
      bits[j] = bits[j - 1];
      bits[j - 1] = tmp;
    }
  DenseGeo g{};
  g.nbits = (uint32_t)nb;
  uint32_t f[16] = {};
  if (es > 0) {
    // the wave's lanes take tile-local bits lb .. lb + 5: low column bits
    // already select distinct banks; give each other bit (a member bit or a
    // column bit >= es) a free bank bit until all es bank bits are used
    const uint32_t low = (1u << es) - 1u;
    uint32_t used = 0;
    for (int j = lb; j < lb + 6 && j < nb; ++j)
      if (bits[j].lds <= low) used |= bits[j].lds;
    for (int j = lb; j < lb + 6 && j < nb; ++j) {
      if (bits[j].lds <= low) continue;
      for (int u = 0; u < es; ++u)
        if (!((used >> u) & 1u)) {
          f[j] = 1u << u;
          used |= f[j];
          break;
        }
    }
  }
  uint32_t fmem[8] = {}, fcol[16] = {};
  for (int j = 0; j < nb; ++j) {
    g.pos[j] = bits[j].pos;
    g.lds[j] = bits[j].lds ^ f[j];
    if (bits[j].pos == 64u) g.inv |= 1u << j;
    if (bits[j].member >= 0) fmem[bits[j].member] = f[j];
    if (bits[j].col >= 0) fcol[bits[j].col] = f[j];
  }
  for (int b = 0; b < k; ++b) g.fmb[b] = fmem[b];
  for (int c = 0; es > 0 && c < 16 && (c << es) < nc; ++c) {
    uint32_t v = 0;
    for (int b = 0; es + b < cb; ++b)
      if ((c >> b) & 1) v ^= fcol[es + b];
    g.fc[c] = v;
  }
  const uint64_t all = n >= 64 ? ~0ull : (1ull << n) - 1ull;
  g.rest = all & ~tilemask;
  return g;
}

}  // namespace

hipError_t launch_dense_kq(sv_dtype dt, void* psi, int n, int k, const int* q, const void* m_dev, bool mfma,
                           hipStream_t s) {
  if (dt == SV_C128) {
    switch (k) {
      case 3: return run_mfma<double, 3>(psi, n, q, m_dev, s);
      case 4: return run_mfma<double, 4>(psi, n, q, m_dev, s);
      case 5: return run_mfma<double, 5>(psi, n, q, m_dev, s);
      case 6: return run_mfma<double, 6>(psi, n, q, m_dev, s);
    }
    return hipErrorInvalidValue;
  }
  if (mfma && k >= 4) {
    switch (k) {
      case 4: return run_mfma<float, 4>(psi, n, q, m_dev, s);
      case 5: return run_mfma<float, 5>(psi, n, q, m_dev, s);
      case 6: return run_mfma<float, 6>(psi, n, q, m_dev, s);
    }
  }
  switch (k) {
    case 3: return run<flt2, 3>(psi, n, make_geo(n, k, q, tile_cols<3>(), 0, 0), m_dev, s);
    case 4: return run<flt2, 4>(psi, n, make_geo(n, k, q, tile_cols<4>(), 0, 0), m_dev, s);
    case 5: return run<flt2, 5>(psi, n, make_geo(n, k, q, tile_cols<5>(), 0, 0), m_dev, s);
    case 6: return run<flt2, 6>(psi, n, make_geo(n, k, q, tile_cols<6>(), 0, 0), m_dev, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace sv
