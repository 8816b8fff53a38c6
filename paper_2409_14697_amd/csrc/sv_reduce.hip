// Readout reductions: marginal probabilities (Eq. 1: the probability of |i>
// is |a_i|^2) over an ordered qubit subset, and the squared norm (subset of
// size 0; the normalisation condition of Sec. II-A).
//
// Accumulation is FP64 for both precisions and the summation order is fixed
// (it depends only on N and the qubit list), so a result is bitwise
// reproducible no matter what else runs on the device.
//
// Layout of the work.  Index bits below L = min(8, N) are covered by the 256
// lanes of a block (lane t reads index t + ...), so each load instruction of
// a wave reads consecutive amplitudes.  A block fixes the values of the
// measured bits at or above L ("qhi", blockIdx.x) and walks a contiguous chunk
// (blockIdx.y) of the remaining high bits ("rest"); every lane therefore
// accumulates exactly one output bin.  Lanes that share a bin (they differ
// only in unmeasured low bits) are combined in a fixed order through LDS, and
// the per-chunk partial sums are added in chunk order by a second kernel.
#include <mutex>

#include "sv_device.h"
#include "sv_kernels.h"

namespace sv {
namespace {

constexpr int kBlock = 256;
constexpr uint64_t kMaxPartialDoubles = 1ull << 23;  // 64 MiB of partials at most

struct ProbGeo {
  int L;                 // low bits covered by lanes
  int m;                 // number of measured qubits
  uint64_t qhi_mask;     // measured bits >= L
  uint64_t rest_mask;    // unmeasured bits >= L
  uint64_t restlo_mask;  // unmeasured bits < L
  uint64_t chunk;        // rest values per block
  uint64_t qhi_blocks;   // values of the measured high bits
  int qpos[SV_MAX_QUBITS];  // qubits[r]
};


__device__ __forceinline__ double absq(dbl2 v) { return v.x * v.x + v.y * v.y; }
__device__ __forceinline__ double absq(flt2 v) {
  const double re = v.x, im = v.y;
  return re * re + im * im;
}

template <typename E>
__global__ __launch_bounds__(kBlock) void k_probs_partial(const E* __restrict__ psi, ProbGeo g,
                                                          double* __restrict__ partial) {
  __shared__ double red[kBlock];
  const unsigned t = threadIdx.x;
  const bool active = t < (1u << g.L);
  for (uint64_t qb = blockIdx.x; qb < g.qhi_blocks; qb += gridDim.x) {
  const uint64_t qhi_bits = deposit(qb, g.qhi_mask);
  uint64_t cur = deposit((uint64_t)blockIdx.y * g.chunk, g.rest_mask);
  double acc = 0.0;
  if (active) {
    const uint64_t fixed = (uint64_t)t | qhi_bits;
    uint64_t j = 0;
    // eight loads in flight, added in index order
    for (; j + 8 <= g.chunk; j += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = absq(psi[fixed | cur]);
        cur = ((cur | ~g.rest_mask) + 1ull) & g.rest_mask;  // next value under the mask
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; j < g.chunk; ++j) {
      acc += absq(psi[fixed | cur]);
      cur = ((cur | ~g.rest_mask) + 1ull) & g.rest_mask;
    }
  }
  red[t] = acc;
  __syncthreads();
  // lanes with zero unmeasured-low bits collect their bin in a fixed order
  if (active && ((uint64_t)t & g.restlo_mask) == 0) {
    double s = 0.0;
    const uint64_t nlo = 1ull << __popcll(g.restlo_mask);
    for (uint64_t j = 0; j < nlo; ++j) s += red[t | (unsigned)deposit(j, g.restlo_mask)];
    const uint64_t i = (uint64_t)t | qhi_bits;
    uint64_t bin = 0;
    for (int r = 0; r < g.m; ++r) bin |= ((i >> g.qpos[r]) & 1ull) << (g.m - 1 - r);
    partial[(uint64_t)blockIdx.y * (1ull << g.m) + bin] = s;
  }
  __syncthreads();  // red[] is reused by the next qhi value
  }
}

__global__ __launch_bounds__(kBlock) void k_probs_final(const double* __restrict__ partial, uint64_t nbins,
                                                        unsigned chunks, double* __restrict__ out) {
  const uint64_t b = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= nbins) return;
  double s = 0.0;
  for (unsigned c = 0; c < chunks; ++c) s += partial[(uint64_t)c * nbins + b];
  out[b] = s;
}

ProbGeo make_geo(int n, int m, const int* qubits, unsigned* chunks_out, uint64_t* qhi_blocks_out) {
  ProbGeo g{};
  g.L = n < 8 ? n : 8;
  g.m = m;
  uint64_t qmask = 0;
  for (int r = 0; r < m; ++r) {
    g.qpos[r] = qubits[r];
    qmask |= 1ull << qubits[r];
  }
  const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
  const uint64_t low = (1ull << g.L) - 1ull;
  g.qhi_mask = qmask & ~low;
  g.rest_mask = all & ~qmask & ~low;
  g.restlo_mask = low & ~qmask;
  const int mh = __builtin_popcountll(g.qhi_mask);
  const int nr = __builtin_popcountll(g.rest_mask);
  uint64_t chunks = 1;
  // aim for ~4096 blocks in total, bounded by the rest values and the partial buffer
  while ((chunks << mh) < 4096 && chunks < (1ull << nr) && ((chunks * 2) << m) <= kMaxPartialDoubles) chunks *= 2;
  g.chunk = (1ull << nr) / chunks;
  g.qhi_blocks = 1ull << mh;
  *chunks_out = (unsigned)chunks;
  *qhi_blocks_out = 1ull << mh;
  return g;
}

// Reduction partials of sv_measure_probs_noalloc: one array per GPU, held
// until the process ends.  The block and chunk geometry above never needs
// more than 4096 blocks' worth of 256 bins (2^20 doubles), so every marginal
// fits; calls that overlap on one GPU share it (and race).
constexpr size_t kStaticScratchDoubles = 1ull << 20;  // 8 MiB
__device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t static_scratch_bytes() { return kStaticScratchDoubles * sizeof(double); }

// The device address of `scratch` on `device`, resolved once per device with
// that device current (in host code the array's name is only a stand-in).
hipError_t static_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

size_t probs_scratch_bytes(int n, int m, const int* qubits) {
  unsigned chunks;
  uint64_t qb;
  make_geo(n, m, qubits, &chunks, &qb);
  if (chunks == 1) return 0;  // a single chunk writes the output directly
  return (size_t)chunks * ((size_t)1 << m) * sizeof(double);
}

hipError_t launch_probs(sv_dtype dt, const void* psi, int n, const int* qubits, int m, double* out, void* scratch,
                        hipStream_t s) {
  unsigned chunks;
  uint64_t qb;
  ProbGeo g = make_geo(n, m, qubits, &chunks, &qb);
  double* partial = chunks == 1 ? out : (double*)scratch;
  dim3 grid((unsigned)capped_grid(qb), chunks);
  if (dt == SV_C128)
    hipLaunchKernelGGL(k_probs_partial<dbl2>, grid, dim3(kBlock), 0, s, (const dbl2*)psi, g, partial);
  else
    hipLaunchKernelGGL(k_probs_partial<flt2>, grid, dim3(kBlock), 0, s, (const flt2*)psi, g, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || chunks == 1) return e;
  const uint64_t nbins = 1ull << m;
  const uint64_t blocks = (nbins + kBlock - 1) / kBlock;  // chunks > 1 only when 2^m partials fit 64 MiB
  hipLaunchKernelGGL(k_probs_final, dim3((unsigned)blocks), dim3(kBlock), 0, s, (const double*)partial, nbins,
                     chunks, out);
  return hipGetLastError();
}

}  // namespace sv
