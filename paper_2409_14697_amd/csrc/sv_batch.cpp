// Serving support: device-resident programs and the batcher that runs one
// pass of many states per step (continuous batching): the tile and
// permutation passes of all states in one launch, matrix, dense and sweep
// passes as launches of their own.
#include <algorithm>
#include <cstring>
#include <new>

#include "sv_host.h"

struct sv_program {
  int n = 0;
  sv_dtype dt = SV_C128;
  int n_passes = 0;
  int max_m = 0;
  bool mfma = true;           // complex64 dense passes on the FP32 matrix cores
  std::vector<int> pass_m;    // local qubits of each pass
  std::vector<int> pass_kind;  // PassKind of each pass
  std::vector<int> pass_mx_k;  // PASS_MATRIX: stage width
  std::vector<int> pass_stages;  // PASS_MATRIX: stages
  std::vector<sv::Op> pass_op;   // PASS_SWEEP / PASS_DENSE: the op in physical qubits
  sv::PackedPlan packed;      // device image, kept for the async upload
  void* dev = nullptr;
  bool owned = false;
  hipEvent_t uploaded = nullptr;  // after the upload: the host copy may be freed
  hipStream_t stream = nullptr;
};

struct sv_batcher {
  hipStream_t stream = nullptr;
  static constexpr int kSlots = 4;  // descriptor buffers in flight
  void* host[kSlots] = {nullptr, nullptr, nullptr, nullptr};
  void* dev[kSlots] = {nullptr, nullptr, nullptr, nullptr};
  size_t cap[kSlots] = {0, 0, 0, 0};
  hipEvent_t done[kSlots] = {nullptr, nullptr, nullptr, nullptr};
  bool used[kSlots] = {false, false, false, false};
  int next = 0;
  void* scratch = nullptr;  // reduction partials of sv_batcher_probs
  size_t scratch_bytes = 0;
};

namespace sv {
namespace {

// Pack the plan's passes into the program's device image.
sv_status pack_program(const sv_plan* p, sv_program* prog) {
  if (sv_status st = pack_plan(p, &prog->packed)) return st;
  prog->n = p->n;
  prog->dt = p->dt;
  prog->n_passes = (int)p->passes.size();
  prog->max_m = prog->packed.max_m;
  prog->mfma = p->opts.fp32_mfma != 0;
  prog->pass_m.clear();
  prog->pass_kind.clear();
  prog->pass_mx_k.clear();
  prog->pass_stages.clear();
  prog->pass_op.clear();
  for (const Pass& ps : p->passes) {
    prog->pass_m.push_back(ps.n_local);
    prog->pass_kind.push_back(ps.kind);
    prog->pass_mx_k.push_back(ps.mx_k);
    prog->pass_stages.push_back((int)ps.stages.size());
    prog->pass_op.push_back(ps.kind == PASS_SWEEP || ps.kind == PASS_DENSE ? ps.phys : Op());
  }
  return SV_OK;
}

// One pass of one state as its own launch on `stream`: matrix, dense and
// sweep passes (the batched kernel runs tile and permutation passes).
sv_status run_single_pass(const sv_program* p, int pass, sv_state* s, hipStream_t stream) {
  unsigned char* pd = (unsigned char*)p->dev;
  const int kind = p->pass_kind[pass];
  if (kind == PASS_MATRIX) {
    SV_LAUNCH(launch_matrix_pass(s->dt, p->pass_mx_k[pass], s->ptr, s->n, p->pass_m[pass],
                                 (const PassDescDev*)(pd + p->packed.off_desc), p->packed.desc_index[pass],
                                 p->pass_stages[pass], (const PassStageDev*)(pd + p->packed.off_stage),
                                 pd + p->packed.off_pool, stream),
              stream);
    return SV_OK;
  }
  const Op& op = p->pass_op[pass];
  if (kind == PASS_DENSE) {
    SV_LAUNCH(launch_dense_kq(s->dt, s->ptr, s->n, op.nq, op.q, pd + p->packed.dense_off[pass], p->mfma, stream),
              stream);
    return SV_OK;
  }
  SweepArgs a;
  if (!low_args_for(op, s->dt, &a) && !sweep_args_for(op, &a))
    return fail(SV_ERR_UNSUPPORTED, "internal: sweep pass of a %d-qubit op", op.nq);
  SV_LAUNCH(launch_sweep(s->dt, s->ptr, s->n, a, stream), stream);
  return SV_OK;
}

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_program_bytes(const sv_plan* p, size_t* bytes) {
  clear_error();
  if (!p || !bytes) return fail(SV_ERR_ARG, "null argument");
  sv_program tmp;
  if (sv_status st = pack_program(p, &tmp)) return st;
  *bytes = tmp.packed.host.size();
  return SV_OK;
}

sv_status sv_program_create(const sv_plan* p, void* dev_buf, size_t buf_bytes, void* stream, sv_program** out) {
  clear_error();
  if (!p || !out) return fail(SV_ERR_ARG, "null argument");
  *out = nullptr;
  if (dev_buf && ((uintptr_t)dev_buf & 255u)) return fail(SV_ERR_ARG, "program buffer not 256-byte aligned");
  sv_program* prog = new (std::nothrow) sv_program();
  if (!prog) return fail(SV_ERR_NOMEM, "host allocation failed");
  prog->stream = (hipStream_t)stream;
  sv_status st = pack_program(p, prog);
  if (st == SV_OK) {
    const size_t bytes = prog->packed.host.size();
    if (dev_buf) {
      if (buf_bytes < bytes) st = fail(SV_ERR_ARG, "program buffer of %zu bytes, %zu needed", buf_bytes, bytes);
      prog->dev = dev_buf;
    } else if (hipMalloc(&prog->dev, std::max<size_t>(bytes, 256)) != hipSuccess) {  // sweep-only programs hold 0 bytes
      prog->dev = nullptr;
      st = fail(SV_ERR_NOMEM, "cannot allocate %zu bytes for the program", bytes);
    } else {
      prog->owned = true;
    }
  }
  if (st == SV_OK && hipEventCreateWithFlags(&prog->uploaded, hipEventDisableTiming) != hipSuccess) {
    prog->uploaded = nullptr;
    st = fail(SV_ERR_DEVICE, "hipEventCreate failed");
  }
  if (st == SV_OK && (hipMemcpyAsync(prog->dev, prog->packed.host.data(), prog->packed.host.size(), hipMemcpyHostToDevice,
                                     prog->stream) != hipSuccess ||
                      hipEventRecord(prog->uploaded, prog->stream) != hipSuccess))
    st = fail(SV_ERR_DEVICE, "program upload failed");
  if (st != SV_OK) {
    (void)hipStreamSynchronize(prog->stream);
    if (prog->owned) (void)hipFree(prog->dev);
    if (prog->uploaded) (void)hipEventDestroy(prog->uploaded);
    delete prog;
    return st;
  }
  *out = prog;
  return SV_OK;
}

sv_status sv_program_info(const sv_program* prog, int32_t* n, sv_dtype* dt, int32_t* n_passes) {
  clear_error();
  if (!prog) return fail(SV_ERR_ARG, "null program");
  if (n) *n = prog->n;
  if (dt) *dt = prog->dt;
  if (n_passes) *n_passes = prog->n_passes;
  return SV_OK;
}

sv_status sv_program_destroy(sv_program* prog) {
  clear_error();
  if (!prog) return SV_OK;
  sv_status st = SV_OK;
  if (prog->owned) {
    if (hipStreamSynchronize(prog->stream) != hipSuccess) st = fail(SV_ERR_DEVICE, "stream sync failed");
    (void)hipFree(prog->dev);
  } else if (hipEventSynchronize(prog->uploaded) != hipSuccess) {  // the upload may still read the host copy
    st = fail(SV_ERR_DEVICE, "event sync failed");
  }
  (void)hipEventDestroy(prog->uploaded);
  delete prog;
  return st;
}

sv_status sv_batcher_create(void* stream, sv_batcher** out) {
  clear_error();
  if (!out) return fail(SV_ERR_ARG, "null output");
  sv_batcher* b = new (std::nothrow) sv_batcher();
  if (!b) return fail(SV_ERR_NOMEM, "host allocation failed");
  b->stream = (hipStream_t)stream;
  for (int i = 0; i < sv_batcher::kSlots; ++i)
    if (hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming) != hipSuccess) {
      sv_batcher_destroy(b);
      return fail(SV_ERR_DEVICE, "hipEventCreate failed");
    }
  *out = b;
  return SV_OK;
}

sv_status sv_batcher_run(sv_batcher* b, int count, sv_state* const* states, const sv_program* const* programs,
                         const int32_t* pass_index) {
  clear_error();
  if (!b) return fail(SV_ERR_ARG, "null batcher");
  if (count <= 0) return count == 0 ? SV_OK : fail(SV_ERR_ARG, "negative count");
  if (!states || !programs || !pass_index) return fail(SV_ERR_ARG, "null array");
  std::vector<BatchItemDev> items;
  items.reserve((size_t)count);
  std::vector<int> single;  // items whose pass runs as a launch of its own
  uint64_t tiles = 0;
  int max_m = 0;
  bool ladders = false;
  sv_dtype dt = SV_C128;
  for (int i = 0; i < count; ++i) {
    const sv_state* s = states[i];
    const sv_program* p = programs[i];
    if (!s || !p) return fail(SV_ERR_ARG, "null state or program at %d", i);
    if (i == 0) dt = s->dt;
    if (s->dt != dt || p->dt != dt) return fail(SV_ERR_ARG, "item %d: mixed dtypes in one batch", i);
    if (p->n != s->n) return fail(SV_ERR_ARG, "item %d: program for %d qubits, state has %d", i, p->n, s->n);
    if (pass_index[i] < 0 || pass_index[i] >= p->n_passes)
      return fail(SV_ERR_ARG, "item %d: pass %d out of range (%d passes)", i, pass_index[i], p->n_passes);
    for (int j = 0; j < i; ++j)
      if (states[j] == s) return fail(SV_ERR_ARG, "state %d appears twice in one batch", i);
    const int kind = p->pass_kind[pass_index[i]];
    if (kind != PASS_TILE && kind != PASS_PERMUTE) {
      single.push_back(i);
      continue;
    }
    const int m = p->pass_m[pass_index[i]];
    items.emplace_back();
    BatchItemDev& it = items.back();
    unsigned char* pd = (unsigned char*)p->dev;
    it.psi = s->ptr;
    it.passes = (const PassDescDev*)(pd + p->packed.off_desc);
    it.stages = (const PassStageDev*)(pd + p->packed.off_stage);
    it.items = (const PassItemDev*)(pd + p->packed.off_items);
    it.mats = pd + p->packed.off_pool;
    it.tile_begin = tiles;
    it.n = s->n;
    it.pass = p->packed.desc_index[pass_index[i]];
    tiles += 1ull << (s->n - m);
    max_m = std::max(max_m, m);
    ladders = ladders || p->packed.pass_lp[pass_index[i]];
  }
  for (int i : single)
    if (sv_status st = run_single_pass(programs[i], pass_index[i], states[i], b->stream)) return st;
  if (items.empty()) return SV_OK;
  const size_t bytes = items.size() * sizeof(BatchItemDev);
  const int k = b->next;
  b->next = (b->next + 1) % sv_batcher::kSlots;
  if (b->used[k]) SV_HIP_TRY(hipEventSynchronize(b->done[k]));  // slot's last launch has read it
  if (bytes > b->cap[k]) {
    // the slot's last launch has finished (waited above): its buffers can go
    if (b->dev[k]) (void)hipFree(b->dev[k]);
    if (b->host[k]) (void)hipHostFree(b->host[k]);
    b->dev[k] = b->host[k] = nullptr;
    b->cap[k] = 0;
    size_t cap = 4096;
    while (cap < bytes) cap <<= 1;
    if (hipMalloc(&b->dev[k], cap) != hipSuccess) {
      b->dev[k] = nullptr;
      return fail(SV_ERR_NOMEM, "batch descriptor buffer");
    }
    if (hipHostMalloc(&b->host[k], cap, hipHostMallocDefault) != hipSuccess) {
      b->host[k] = nullptr;
      (void)hipFree(b->dev[k]);
      b->dev[k] = nullptr;
      return fail(SV_ERR_NOMEM, "pinned batch descriptor buffer");
    }
    b->cap[k] = cap;
  }
  std::memcpy(b->host[k], items.data(), bytes);
  SV_HIP_TRY(hipMemcpyAsync(b->dev[k], b->host[k], bytes, hipMemcpyHostToDevice, b->stream));
  SV_LAUNCH(launch_pass_batch(dt, (const BatchItemDev*)b->dev[k], (int)items.size(), tiles, max_m, ladders, b->stream),
            b->stream);
  SV_HIP_TRY(hipEventRecord(b->done[k], b->stream));
  b->used[k] = true;
  return SV_OK;
}

sv_status sv_batcher_probs(sv_batcher* b, const sv_state* s, const int32_t* qubits, int m, double* out_dev) {
  clear_error();
  if (!b || !s) return fail(SV_ERR_ARG, "null batcher or state");
  int qs[SV_MAX_QUBITS];
  if (sv_status st = probs_args(s->n, qubits, m, out_dev, qs)) return st;
  const size_t need = std::max<size_t>(probs_scratch_bytes(s->n, m, qs), 256);
  if (need > b->scratch_bytes) {
    if (b->scratch) {
      SV_HIP_TRY(hipStreamSynchronize(b->stream));  // earlier reductions may still use it
      SV_HIP_TRY(hipFree(b->scratch));
      b->scratch = nullptr;
      b->scratch_bytes = 0;
    }
    if (hipMalloc(&b->scratch, need) != hipSuccess) {
      b->scratch = nullptr;
      return fail(SV_ERR_NOMEM, "cannot allocate %zu bytes of reduction scratch", need);
    }
    b->scratch_bytes = need;
  }
  SV_LAUNCH(launch_probs(s->dt, s->ptr, s->n, qs, m, out_dev, b->scratch, b->stream), b->stream);
  return SV_OK;
}

sv_status sv_batcher_destroy(sv_batcher* b) {
  clear_error();
  if (!b) return SV_OK;
  sv_status st = SV_OK;
  if (hipStreamSynchronize(b->stream) != hipSuccess) st = fail(SV_ERR_DEVICE, "stream sync failed");
  for (int i = 0; i < sv_batcher::kSlots; ++i) {
    if (b->dev[i]) (void)hipFree(b->dev[i]);
    if (b->host[i]) (void)hipHostFree(b->host[i]);
    if (b->done[i]) (void)hipEventDestroy(b->done[i]);
  }
  if (b->scratch) (void)hipFree(b->scratch);
  delete b;
  return st;
}

}  // extern "C"
