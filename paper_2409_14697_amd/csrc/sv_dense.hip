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

hipError_t launch_dense_kq(sv_dtype dt, void* psi, int n, int k, const int* q, const void* m_dev, hipStream_t s) {
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
  return dispatch<flt2>(psi, n, k, g, m_dev, s);
}

}  // namespace sv
