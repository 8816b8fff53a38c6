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

// ---------------------------------------------------------------- FP32 MFMA
// complex64 states, 4 <= k <= 6: Y = U X as a real GEMM on the interleaved
// storage.  With rows of Y and X indexed 2*member + (0: re, 1: im), the
// operator is the real 2D x 2D matrix A[2i+a][2j+b] = (Ur, -Ui; Ui, Ur)[a][b]
// of U[i][j], so no de-interleaving is needed.  v_mfma_f32_32x32x2_f32 tiles:
// A operand (32 x 2): lane l holds A[l % 32][l / 32]; B operand (2 x 32):
// lane l holds B[l / 32][l % 32]; accumulator (32 x 32, 16 registers): lane l,
// register r holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
// FP32 inputs, FP32 accumulation.  A block of 4 waves covers all 2D rows and
// 32 * 4 / (2D / 32) columns (groups); each wave keeps its 32 rows of A in
// registers and streams X fragments from an LDS tile.
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int K>
__global__ __launch_bounds__(kBlock) void k_dense_mfma(flt2* __restrict__ psi, uint64_t ngroups, DenseGeo g,
                                                       const float* __restrict__ um) {
  constexpr int D = 1 << K;          // members per group
  constexpr int RB = (2 * D) / 32;   // 32-row blocks of the real operator
  constexpr int CB = 4 / RB;         // 32-column blocks per block iteration
  constexpr int NC = 32 * CB;        // groups per block iteration
  __shared__ flt2 xs[D * NC];        // [member][column]
  const int t = threadIdx.x, w = t / 64, l = t % 64;
  const int rb = w % RB, cb = w / RB;
  // this wave's rows of A for every k-step (K-dimension pairs = input members)
  float a[D];
#pragma unroll
  for (int kk = 0; kk < D; ++kk) {
    const int i = 32 * rb + (l % 32);  // real output row
    const int oi = i >> 1, ar = i & 1, bi = l / 32;
    const float ur = um[2 * (oi * D + kk)], ui = um[2 * (oi * D + kk) + 1];
    a[kk] = ar == 0 ? (bi == 0 ? ur : -ui) : (bi == 0 ? ui : ur);
  }
  const uint64_t nwork = (ngroups + NC - 1) / NC;
  for (uint64_t wb = xcd_block(); wb < nwork; wb += gridDim.x) {
    const uint64_t c0 = wb * NC;
    __syncthreads();  // previous iteration's readers are done with xs
    for (int e = t; e < D * NC; e += kBlock) {
      const int c = e % NC, r = e / NC;
      const uint64_t col = c0 + c;
      flt2 v = {0.f, 0.f};
      if (col < ngroups) v = psi[group_base<K>(col, g) + member_off<K>(r, g)];
      xs[e] = v;
    }
    __syncthreads();
    floatx16 acc = {};
    const int col = cb * 32 + (l % 32);
#pragma unroll
    for (int kk = 0; kk < D; ++kk) {
      const flt2 xv = xs[kk * NC + col];
      const float b = (l / 32) ? xv.y : xv.x;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[kk], b, acc, 0, 0, 0);
    }
    const uint64_t gcol = c0 + col;
    if (gcol < ngroups) {
      const uint64_t gb = group_base<K>(gcol, g);
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const int i = 32 * rb + 8 * (r / 4) + 4 * (l / 32) + (r % 4);  // even real row: re, i + 1: im
        flt2 y;
        y.x = acc[r];
        y.y = acc[r + 1];
        psi[gb + member_off<K>(i >> 1, g)] = y;
      }
    }
  }
}

template <int K>
hipError_t run_mfma(void* psi, int n, const DenseGeo& g, const void* m, hipStream_t s) {
  constexpr int D = 1 << K;
  constexpr int NC = 32 * (4 / ((2 * D) / 32));
  const uint64_t ngroups = 1ull << (n - K);
  const uint64_t blocks = capped_grid((ngroups + NC - 1) / NC);
  hipLaunchKernelGGL((k_dense_mfma<K>), dim3((unsigned)blocks), dim3(kBlock), 0, s, (flt2*)psi, ngroups, g,
                     (const float*)m);
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
  if (dt == SV_C128) return dispatch<dbl2>(psi, n, k, g, m_dev, s);
  if (mfma && k >= 4) {
    switch (k) {
      case 4: return run_mfma<4>(psi, n, g, m_dev, s);
      case 5: return run_mfma<5>(psi, n, g, m_dev, s);
      case 6: return run_mfma<6>(psi, n, g, m_dev, s);
    }
  }
  return dispatch<flt2>(psi, n, k, g, m_dev, s);
}

}  // namespace sv
