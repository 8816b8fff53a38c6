// Host-visible launchers of the gate-sweep, readout and utility kernels.
// Every launcher validates nothing (the C ABI layer has done that), enqueues
// on `stream`, and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <complex>
#include <mutex>

#include "sv.h"

namespace sv {

typedef std::complex<double> cd;

// --- gate sweeps -----------------------------------------------------------
// One sweep over the state; each work item owns one group of amplitudes
// (Eq. 2 pairs, Eq. 3 quads, or a touched subset of them).  Geometry is given
// in amplitude-index space:
//   groups = all indices with zeros at positions z[0..nz-1] (ascending), OR'd
//   with `set`; the members of a group sit at base + off[0..nv-1].
struct GroupSpec {
  int nz = 0;
  unsigned z[3] = {0, 0, 0};
  uint64_t set = 0;
  int nv = 1;
  uint64_t off[4] = {0, 0, 0, 0};
};

enum SweepOp {
  SWEEP_DENSE1 = 0,  // nv=2: (a0,a1) <- M (a0,a1), M 2x2 (m[0..3] row-major)
  SWEEP_DENSE2 = 1,  // nv=4: 4x4 matrix m[0..15]
  SWEEP_SWAP = 2,    // nv=2: exchange a0 and a1 (X, CNOT, SWAP)
  SWEEP_PHASE = 3,   // nv=1: a0 <- m[0] * a0 (phase on a fixed-bit subset)
  SWEEP_DIAG = 4,    // nv=1: a <- d[local(bits)] * a, local index from bits
                     //       b0 (MSB) [, b1]; m[0..3] = d
  SWEEP_SCALE = 5,   // nv=1: a <- m[0].real() * a
  SWEEP_SCALE_NORM = 7,  // nv=1: a <- a / sqrt(*norm2_dev) (FP64 factor)
  SWEEP_LOW = 6      // 1-/2-qubit matrix m (4^low_k entries) on qubits low_q
                     // (low_q[0] = MSB), at least one of them inside a
                     // 128-byte run; rows are exchanged between lanes.  Only
                     // indices with all low_fixed bits set are visited.
};

struct SweepArgs {
  SweepOp op;
  GroupSpec g;
  cd m[16];
  int diag_nbits = 0;
  unsigned diag_b0 = 0, diag_b1 = 0;
  const double* norm2_dev = nullptr;  // SWEEP_SCALE_NORM
  int low_k = 0;
  unsigned low_q[2] = {0, 0};
  uint64_t low_fixed = 0;
  // filled by plan_low(): the lane-exchange layout in element space
  int low_kind[2] = {-1, -1};      // LOW_INTRA / LOW_LANE / LOW_REG per matrix qubit
  unsigned low_lanebit[2] = {0, 0};
  int low_nz = 0;                  // zero-inserted element positions (REG target or fixed control)
  unsigned low_z[2] = {0, 0};
  uint64_t low_set = 0;            // element bits fixed to 1
  uint64_t low_off1 = 0;           // element offset of the REG register
};

enum { LOW_INTRA = 0, LOW_LANE = 1, LOW_REG = 2 };
constexpr unsigned kLaneBits = 6;  // element bits held across the 64 lanes of a wave

// Element-space layout of a SWEEP_LOW op for dtype dt: qubit kinds, lane bits,
// inserted positions.  Returns false if the op does not fit the kernel (at
// most one REG target or one fixed control).
bool plan_low(sv_dtype dt, SweepArgs* a);

hipError_t launch_sweep(sv_dtype dt, void* psi, int n, const SweepArgs& a, hipStream_t s);

// --- readout ----------------------------------------------------------------
// Scratch bytes the marginal-probability reduction needs.
size_t probs_scratch_bytes(int n, int m, const int* qubits);
hipError_t launch_probs(sv_dtype dt, const void* psi, int n, const int* qubits, int m, double* out,
                        void* scratch, hipStream_t s);
// The library's static reduction scratch on `device` (a file-scope device
// array; no allocation): its bytes, and its device address.
size_t static_scratch_bytes();
hipError_t static_scratch(int device, void** out);

// --- launch state -----------------------------------------------------------
// Per-device launch state of one kernel: the dynamic LDS limit raised with
// hipFuncSetAttribute and the number of blocks resident on the device per
// dynamic LDS size.  Launches may come from several host threads and several
// devices; the cache is guarded and kept per device.
struct KernelLaunchCache {
  static constexpr int kMaxDevices = 64;
  static constexpr int kSizes = 19;  // dynamic LDS sizes 2^0 .. 2^18 bytes
  std::mutex mu;
  size_t lds_attr[kMaxDevices] = {};
  uint64_t resident[kMaxDevices][kSizes] = {};
};

// Make `fn` launchable with `lds` bytes of dynamic LDS on the current device;
// *resident (if non-null) receives the blocks of `block` threads that fit on
// the device at once with that LDS (the persistent grid of a tile loop).
inline hipError_t prepare_launch(KernelLaunchCache& c, const void* fn, int block, size_t lds, uint64_t* resident) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= KernelLaunchCache::kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(c.mu);
  if (lds > c.lds_attr[dev]) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    c.lds_attr[dev] = lds;
  }
  if (!resident) return hipSuccess;
  int lg = 0;
  while (lg + 1 < KernelLaunchCache::kSizes && ((size_t)1 << lg) < lds) ++lg;
  uint64_t& r = c.resident[dev][lg];
  if (!r) {
    int nb = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fn, block, lds) != hipSuccess || nb < 1) nb = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    r = (uint64_t)nb * (uint64_t)cus;
  }
  *resident = r;
  return hipSuccess;
}

// --- utilities --------------------------------------------------------------
hipError_t launch_init_basis(sv_dtype dt, void* psi, int n, uint64_t index, hipStream_t s);
hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace sv
