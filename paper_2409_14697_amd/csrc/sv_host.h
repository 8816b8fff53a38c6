// Internal host-side declarations of the state-vector core (not part of the
// C ABI).  The planner parts (gate ops, fusion, pass planning) use no HIP
// call, so they run on machines without a GPU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <complex>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "sv.h"
#include "sv_kernels.h"
#include "sv_tile_kernels.h"

namespace sv {

// ------------------------------------------------------------------ errors
sv_status fail(sv_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define SV_HIP_TRY(expr)                                                               \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) return ::sv::fail(SV_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// Debug mode (environment SV_DEBUG_SYNC=1, read once): every kernel launch is
// followed by a synchronisation of its stream, so that a device fault is
// reported by the call that enqueued the faulting kernel, with the launch
// named in the message, instead of by a later call.
bool debug_sync_enabled();
#define SV_LAUNCH(expr, stream)                                                        \
  do {                                                                                 \
    SV_HIP_TRY(expr);                                                                  \
    if (::sv::debug_sync_enabled()) {                                                  \
      hipError_t _d = hipStreamSynchronize(stream);                                    \
      if (_d == hipSuccess) _d = hipGetLastError();                                    \
      if (_d != hipSuccess)                                                            \
        return ::sv::fail(SV_ERR_DEVICE, "%s (debug sync): %s", #expr, hipGetErrorString(_d)); \
    }                                                                                  \
  } while (0)

// ------------------------------------------------------------------ ops
// One operation in logical qubits: a 2^nq x 2^nq matrix on q[0..nq-1]
// (q[0] = most significant bit of the local index, as in Eq. 3).  `kind`
// keeps the named kind of an unfused gate so that special kernels (swaps,
// phases) can be used; fused or explicit matrices have kind SV_G_MATRIX.
struct Op {
  int kind = SV_G_MATRIX;
  int nq = 0;
  int q[SV_MAX_GATE_QUBITS] = {0, 0, 0, 0, 0, 0};
  double theta = 0.0;
  std::vector<cd> m;  // 4^nq entries, row-major
  int n_gates = 1;    // gates merged into this op
};

// Validate one gate against an n-qubit state (host only).
sv_status validate_gate(const sv_gate& g, int n);
// Build the op (with its FP64 matrix) of a validated gate.
Op op_from_gate(const sv_gate& g);
// Named-gate matrices (textbook definitions, FP64).
std::vector<cd> named_matrix(int kind, double theta);
int gate_arity(int kind);

// Structural class of an op, used by the kernels and the cost model.
enum OpClass { CLS_DENSE = 0, CLS_DIAG = 1, CLS_PERM = 2 };
OpClass classify(const Op& op);

// Sweep kernel arguments for an op with nq <= 2 (returns false for nq >= 3).
bool sweep_args_for(const Op& op, SweepArgs* out);
// Lane-exchange kernel arguments when one of the op's qubits lies inside one
// wave's row of 64 16-byte elements (returns false otherwise).
bool low_args_for(const Op& op, sv_dtype dt, SweepArgs* out);

// Fraction of amplitudes a single-op sweep reads and writes (touched subset).
double touched_fraction(const Op& op);

// ------------------------------------------------------------------ plan
enum PassKind { PASS_SWEEP = 0, PASS_TILE = 1, PASS_DENSE = 2, PASS_PERMUTE = 3, PASS_MATRIX = 4 };

struct StageHost {
  uint32_t q[kPassRegBitsMax] = {0, 0, 0, 0, 0};  // local bit of each register bit
  uint32_t form = PFORM_NONE;               // PassForm of the 2x2 part
  uint32_t slot_mask = 0;                   // register bits with a 2x2 (the others hold identities)
  uint32_t nsub = 0;                        // earlier layers (entries of `mats`; dr kPassNoTable: none)
  PassSubDev sub[kPassSubMax] = {};
  uint32_t flags = 0;                       // PassStageFlags
  uint32_t slots = 0, u2 = 0, dr = 0;       // entries of `mats`
  std::vector<PassItemDev> items;           // lane items (.mat indexes `mats`)
  std::vector<PassItemDev> px;              // permutation terms (PIT_PX)
  uint32_t colimg[kPassLocalMax] = {};     // store map: column images (local masks)
  uint32_t pconst = 0;
  std::vector<cd> mats;
  std::vector<uint8_t> raw;                 // per entry: 1 = two raw words (write_pool)
  uint32_t rows = 0, row_count = 0;         // fixed-point row table (PassStageDev)
  int n_ops = 0;                            // kernel ops (sv_plan_pass_ops)
  int n_fixed = 0;                          // fixed-point phase items among them
};

// Write `count` pool entries in the state precision (complex64: f32 = true).
// An entry with raw[e] set holds two words in the bit patterns of its real
// and imaginary parts (uint64 each); they are stored as two uint32 (complex64)
// or two uint64 (complex128) instead of being converted.  raw may be null.
void write_pool(unsigned char* dst, const cd* m, const uint8_t* raw, size_t count, bool f32);

struct Pass {
  int kind = PASS_SWEEP;
  int first_op = 0, n_ops = 0;  // ops (execution order) this pass implements
  int n_local = 0;
  // PASS_SWEEP / PASS_DENSE: the op in physical qubits
  Op phys;
  // PASS_TILE / PASS_PERMUTE / PASS_MATRIX
  uint32_t lpos[16] = {0};
  uint32_t wpos[16] = {0};
  std::vector<StageHost> stages;
  // PASS_MATRIX: stage width k (every stage a dense 2^k x 2^k op: q[0..k-1]
  // and a 2^k x 2^k matrix at mats entry 0)
  int mx_k = 0;
};

// Fill a pass descriptor's local-bit maps and store flags (lmask, lpos, wpos,
// winv, flags); false if the write positions are not a permutation of the
// load positions.
bool fill_pass_maps(const Pass& ps, sv_dtype dt, PassDescDev* d);

// The pass's stages hold fixed-point phase items (PIT_LP, PIT_QG).
inline bool pass_has_ladders(const Pass& ps) {
  for (const StageHost& sh : ps.stages)
    if (sh.n_fixed) return true;
  return false;
}

}  // namespace sv

struct sv_plan {
  int n = 0;
  sv_dtype dt = SV_C128;
  sv_opts opts{};
  std::vector<sv::Op> ops;        // logical qubits, execution order
  std::vector<int> op_pass;       // pass of each op
  std::vector<sv::Pass> passes;
  size_t n_gates_in = 0;
  double est_cost = 0.0;          // planner's estimate, in full-state sweeps
  // algorithmic flops per amplitude of every pass, filled by the first query
  struct FlopsCache {
    std::once_flag once;
    std::vector<double> per_pass;
  };
  std::unique_ptr<FlopsCache> flops = std::make_unique<FlopsCache>();
};

struct sv_state {
  int n = 0;
  sv_dtype dt = SV_C128;
  void* ptr = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  int device = 0;
  // device scratch (reduction partials)
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  // matrix uploads: pinned host staging + device buffer
  void* up_host = nullptr;
  void* up_dev = nullptr;
  size_t up_bytes = 0;
  hipEvent_t up_done = nullptr;
  bool up_pending = false;
};

namespace sv {
size_t elem_bytes(sv_dtype dt);
sv_status ensure_scratch(sv_state* s, size_t bytes);
// Validate a marginal's qubit list (sv_measure_probs rules); copies it to qs.
sv_status probs_args(int n, const int32_t* qubits, int m, const double* out_dev, int* qs);
// Copy `bytes` from host memory to the state's upload buffer (stream-ordered);
// returns the device address.  The previous upload's device contents stay
// valid for work enqueued before this call.
sv_status upload(sv_state* s, const void* host, size_t bytes, void** dev);
// Run one op as a full-state sweep (sweep kernels for nq <= 2, dense kernel
// for nq >= 3 with the matrix at m_dev in the state's precision; mfma selects
// the FP32 MFMA kernel for complex64 states and nq >= 4).
sv_status run_op_sweep(sv_state* s, const Op& op, const void* m_dev, bool mfma = true);
// Rescale the state to unit norm with an FP64 norm computed on the device
// (stream-ordered; no host synchronisation).
sv_status renormalize(sv_state* s);
// Plan building (host only).
sv_status build_plan(int n, sv_dtype dt, const sv_gate* g, size_t n_gates, const sv_opts& o, sv_plan* p);
// Greedy fusion of an op list (ops no wider than kmax qubits; kmax <= 1
// merges only one-qubit ops on the same qubit).
std::vector<Op> fuse_ops(std::vector<Op> in, int n, sv_dtype dt, int kmax, bool mfma);
// In-cache pass planning of an op list (logical qubits) into p->passes/ops.
// progress: every pass's write-back also moves data toward the position the
// remaining relabelings give it (fewer permutation passes at the end, at
// times more locality to pay in later passes; build_plan tries both).
// reserve: local bits each pass keeps free of its gates, for data moving
// toward its final position (smaller gate blocks, fewer permutation passes).
sv_status plan_tile_passes(const std::vector<Op>& ops, int n, sv_dtype dt, const sv_opts& o, sv_plan* p,
                           bool progress, int reserve = 0);
// Matrix passes over a fused op list (logical = physical qubits): runs of
// ops whose qubits, with the pinned low bits, fit one tile become one pass
// of matrix-core stages; ops that do not pay off grouped run as sweeps.
void plan_matrix_passes(const std::vector<Op>& fused, int n, sv_dtype dt, const sv_opts& o, sv_plan* p);
// Cost of one op run as its own sweep, in full read+write sweeps of the state.
double op_sweep_cost(const Op& op, sv_dtype dt, bool mfma);
// Tile size defaults.
int default_lds_qubits(sv_dtype dt);
int default_pinned_bits(sv_dtype dt);
sv_status execute_plan(sv_state* s, const sv_plan* p);

// Device image of a plan: dense matrices (state precision) and the tile-pass
// program [descriptors][stages][items][pool], every part 256-byte aligned.
// The single packer of both sv_apply_plan and sv_program_create.
struct PackedPlan {
  std::vector<unsigned char> host;
  std::vector<size_t> dense_off;   // per pass: offset of its dense matrix (PASS_DENSE)
  std::vector<int> desc_index;     // per pass: descriptor index (PASS_TILE / PASS_PERMUTE / PASS_MATRIX) or -1
  std::vector<char> pass_lp;       // per pass: holds fixed-point phase items
  size_t off_desc = 0, off_stage = 0, off_items = 0, off_pool = 0;
  int n_desc = 0, max_m = 0;
};
sv_status pack_plan(const sv_plan* p, PackedPlan* out);
}  // namespace sv
