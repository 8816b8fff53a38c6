// Dense k-qubit gate sweep (3 <= k <= 6), the "generic gate" that general gate
// fusion produces (QueenV2 Sec. II-B, Sec. III-A tier 5).
//
// For every group of 2^k amplitudes that differ only in the gate's bits the
// new amplitudes are U times the old ones (Eq. 2/3 generalised; q[0] is the
// most significant bit of the local index).  Viewed as a matrix product
// Y = U X, column c of X is group c.
//
// A block stages U and a tile of C columns (2^k x C amplitudes) in LDS, then
// every lane produces output elements straight from LDS.  Lanes load the tile
// column-fastest, so consecutive lanes read consecutive groups.
#include "sv_device.h"
#include "sv_kernels.h"
#include "sv_tile_kernels.h"

namespace sv {
namespace {

constexpr int kBlock = 256;

struct DenseGeo {
  unsigned zs[SV_MAX_GATE_QUBITS];  // gate bits, ascending (zero-insert order)
  unsigned q[SV_MAX_GATE_QUBITS];   // gate bits in local order (q[0] = MSB)
};

template <int K>
__device__ __forceinline__ uint64_t group_base(uint64_t c, const DenseGeo& g) {
#pragma unroll
  for (int z = 0; z < K; ++z) c = insert0(c, g.zs[z]);
  return c;
}

template <int K>
__device__ __forceinline__ uint64_t member_off(int r, const DenseGeo& g) {
  uint64_t o = 0;
#pragma unroll
  for (int m = 0; m < K; ++m) o |= (uint64_t)((r >> (K - 1 - m)) & 1) << g.q[m];
  return o;
}

// Tile columns per block: the tile holds 2048 amplitudes.
template <int K>
constexpr int tile_cols() {
  return 2048 >> K;
}

template <typename E, int K>
__global__ __launch_bounds__(kBlock) void k_dense(E* __restrict__ psi, uint64_t ngroups, DenseGeo g,
                                                  const typename elem_traits<E>::R* __restrict__ um) {
  typedef typename elem_traits<E>::R R;
  constexpr int D = 1 << K;
  constexpr int C = tile_cols<K>();
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* us = reinterpret_cast<cplx<R>*>(smem);  // D x D
  cplx<R>* xs = us + D * D;                          // D x C, row r = member r
  const int t = threadIdx.x;
  for (int e = t; e < D * D; e += kBlock) us[e] = cplx<R>{um[2 * e], um[2 * e + 1]};
  const uint64_t c0 = (uint64_t)blockIdx.x * C;
  for (int e = t; e < D * C; e += kBlock) {
    const int c = e % C, r = e / C;
    const uint64_t col = c0 + c;
    if (col < ngroups) {
      const E v = psi[group_base<K>(col, g) + member_off<K>(r, g)];
      xs[e] = cplx<R>{v.x, v.y};
    }
  }
  __syncthreads();
  for (int e = t; e < D * C; e += kBlock) {
    const int c = e % C, r = e / C;
    const uint64_t col = c0 + c;
    if (col >= ngroups) continue;
    cplx<R> y = {0, 0};
    const cplx<R>* urow = us + r * D;
#pragma unroll 8
    for (int s = 0; s < D; ++s) y = cfma(y, urow[s], xs[s * C + c]);
    E out;
    out.x = y.re;
    out.y = y.im;
    psi[group_base<K>(col, g) + member_off<K>(r, g)] = out;
  }
}

template <typename E, int K>
hipError_t run(void* psi, int n, const DenseGeo& g, const void* m, hipStream_t s) {
  typedef typename elem_traits<E>::R R;
  constexpr int D = 1 << K;
  constexpr int C = tile_cols<K>();
  const size_t lds = (size_t)(D * D + D * C) * sizeof(cplx<R>);
  static bool attr_set = false;  // per process; the attribute is per function
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dense<E, K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const uint64_t ngroups = 1ull << (n - K);
  const uint64_t blocks = (ngroups + C - 1) / C;
  hipLaunchKernelGGL((k_dense<E, K>), dim3((unsigned)blocks), dim3(kBlock), lds, s, (E*)psi, ngroups, g,
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
  static constexpr int MPB = 16;  // members per row block
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
  static constexpr int MPB = 8;
};

// groups per column tile: the X tile holds 2048 complex64 / 1024 complex128
// amplitudes, and at least one column block
template <typename R, int K>
constexpr int mfma_cols() {
  constexpr int target = (sizeof(R) == 4 ? 2048 : 1024) >> K;
  return target < mfma_shape<R>::BN ? mfma_shape<R>::BN : target;
}

template <typename R, int K>
constexpr size_t mfma_lds() {
  return ((size_t)(1 << K) * ((1 << K) + 1) + (size_t)(1 << K) * mfma_cols<R, K>()) * 2 * sizeof(R);
}

template <typename R, int K>
__global__ __launch_bounds__(kBlock) void k_dense_mfma(typename mfma_shape<R>::E* __restrict__ psi,
                                                       uint64_t ngroups, DenseGeo g, const R* __restrict__ um) {
  typedef mfma_shape<R> MS;
  typedef typename MS::E E;
  constexpr int D = 1 << K, DP = D + 1;
  constexpr int NC = mfma_cols<R, K>();
  constexpr int RBLK = 2 * D / MS::BM, CBLK = NC / MS::BN, TILES = RBLK * CBLK;
  constexpr int KSTEPS = 2 * D / MS::BK;
  constexpr int PER = D * NC / kBlock;  // tile elements gathered per lane
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* us = reinterpret_cast<cplx<R>*>(smem);  // D x DP
  E* xs = reinterpret_cast<E*>(us + D * DP);       // [member][NC]
  const int t = threadIdx.x, w = t / 64, l = t % 64;
  for (int e = t; e < D * D; e += kBlock) us[(e / D) * DP + (e % D)] = cplx<R>{um[2 * e], um[2 * e + 1]};
  const uint64_t nwork = (ngroups + NC - 1) / NC;
  for (uint64_t wb = xcd_block(); wb < nwork; wb += gridDim.x) {
    const uint64_t c0 = wb * NC;
    E buf[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = t + u * kBlock, c = e % NC, r = e / NC;
      const uint64_t col = c0 + c;
      E v = {};
      if (col < ngroups) v = ld(psi + group_base<K>(col, g) + member_off<K>(r, g));
      buf[u] = v;
    }
    __syncthreads();  // U is staged and the previous tile's readers are done
#pragma unroll
    for (int u = 0; u < PER; ++u) xs[t + u * kBlock] = buf[u];
    __syncthreads();
    for (int tile = w; tile < TILES; tile += 4) {
      const int rb = tile % RBLK, cb = tile / RBLK;
      int ai, aa;  // output member and re/im of the A row this lane supplies
      MS::row_of(l % MS::BM, &ai, &aa);
      ai += MS::MPB * rb;
      const int bcol = MS::BN * cb + l % MS::BN;
      typename MS::acc_t acc = {};
#pragma unroll 8
      for (int ks = 0; ks < KSTEPS; ++ks) {
        const int ak = MS::BK * ks + l / MS::BM;  // real column of A (= real row of B)
        const cplx<R> u = us[ai * DP + (ak >> 1)];
        const R a = aa == 0 ? ((ak & 1) == 0 ? u.re : -u.im) : ((ak & 1) == 0 ? u.im : u.re);
        const int bk = MS::BK * ks + l / MS::BN;
        const E xv = xs[(bk >> 1) * NC + bcol];
        const R b = (bk & 1) ? xv.y : xv.x;
        acc = MS::mma(a, b, acc);
      }
      const uint64_t gcol = c0 + bcol;
      if (gcol < ngroups) {
        const uint64_t gb = group_base<K>(gcol, g);
#pragma unroll
        for (int r = 0; r < MS::NACC; r += 2) {
          const int mem = MS::MPB * rb + MS::out_member(l, r);
          E y;
          y.x = acc[r];
          y.y = acc[r + 1];
          st(psi + gb + member_off<K>(mem, g), y);
        }
      }
    }
  }
}

template <typename R, int K>
hipError_t run_mfma(void* psi, int n, const DenseGeo& g, const void* m, hipStream_t s) {
  constexpr int NC = mfma_cols<R, K>();
  constexpr size_t lds = mfma_lds<R, K>();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_dense_mfma<R, K>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const uint64_t ngroups = 1ull << (n - K);
  const uint64_t tiles = (ngroups + NC - 1) / NC;
  // persistent blocks: enough to fill the chip several times over, each
  // amortising its staged U over many column tiles
  const uint64_t blocks = tiles < 4096 ? tiles : 4096;
  hipLaunchKernelGGL((k_dense_mfma<R, K>), dim3((unsigned)blocks), dim3(kBlock), lds, s,
                     (typename mfma_shape<R>::E*)psi, ngroups, g, (const R*)m);
  return hipGetLastError();
}

template <typename E>
hipError_t dispatch(void* psi, int n, int k, const DenseGeo& g, const void* m, hipStream_t s) {
  switch (k) {
    case 3: return run<E, 3>(psi, n, g, m, s);
    case 4: return run<E, 4>(psi, n, g, m, s);
    case 5: return run<E, 5>(psi, n, g, m, s);
    case 6: return run<E, 6>(psi, n, g, m, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_dense_kq(sv_dtype dt, void* psi, int n, int k, const int* q, const void* m_dev, bool mfma,
                           hipStream_t s) {
  DenseGeo g{};
  int sorted[SV_MAX_GATE_QUBITS];
  for (int i = 0; i < k; ++i) {
    g.q[i] = (unsigned)q[i];
    sorted[i] = q[i];
  }
  for (int i = 1; i < k; ++i)
    for (int j = i; j > 0 && sorted[j - 1] > sorted[j]; --j) {
      int tmp = sorted[j];
      sorted[j] = sorted[j - 1];
      sorted[j - 1] = tmp;
    }
  for (int i = 0; i < k; ++i) g.zs[i] = (unsigned)sorted[i];
  if (dt == SV_C128) {
    switch (k) {
      case 3: return run_mfma<double, 3>(psi, n, g, m_dev, s);
      case 4: return run_mfma<double, 4>(psi, n, g, m_dev, s);
      case 5: return run_mfma<double, 5>(psi, n, g, m_dev, s);
      case 6: return run_mfma<double, 6>(psi, n, g, m_dev, s);
    }
    return hipErrorInvalidValue;
  }
  if (mfma && k >= 4) {
    switch (k) {
      case 4: return run_mfma<float, 4>(psi, n, g, m_dev, s);
      case 5: return run_mfma<float, 5>(psi, n, g, m_dev, s);
      case 6: return run_mfma<float, 6>(psi, n, g, m_dev, s);
    }
  }
  return dispatch<flt2>(psi, n, k, g, m_dev, s);
}

}  // namespace sv
