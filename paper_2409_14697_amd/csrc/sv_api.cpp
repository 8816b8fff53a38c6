// C ABI of the state-vector core (declared in include/sv.h).
#include <algorithm>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>

#include "sv_host.h"

namespace sv {

static thread_local std::string g_error;

sv_status fail(sv_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return st;
}

void clear_error() { g_error.clear(); }

bool debug_sync_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("SV_DEBUG_SYNC");
    return v && v[0] && v[0] != '0';
  }();
  return on;
}

size_t elem_bytes(sv_dtype dt) { return dt == SV_C128 ? 16 : 8; }

sv_status ensure_scratch(sv_state* s, size_t bytes) {
  if (bytes <= s->scratch_bytes) return SV_OK;
  if (s->scratch) {
    SV_HIP_TRY(hipStreamSynchronize(s->stream));  // in-flight work may still read it
    SV_HIP_TRY(hipFree(s->scratch));
    s->scratch = nullptr;
    s->scratch_bytes = 0;
  }
  if (hipMalloc(&s->scratch, bytes) != hipSuccess) {
    s->scratch = nullptr;
    return fail(SV_ERR_NOMEM, "cannot allocate %zu bytes of device scratch", bytes);
  }
  s->scratch_bytes = bytes;
  return SV_OK;
}

sv_status upload(sv_state* s, const void* host, size_t bytes, void** dev) {
  if (s->up_pending) {
    // the staging buffer is rewritten below: wait until the last copy read it
    SV_HIP_TRY(hipEventSynchronize(s->up_done));
    s->up_pending = false;
  }
  if (bytes > s->up_bytes) {
    if (s->up_dev) {
      SV_HIP_TRY(hipStreamSynchronize(s->stream));
      SV_HIP_TRY(hipFree(s->up_dev));
      SV_HIP_TRY(hipHostFree(s->up_host));
      s->up_dev = s->up_host = nullptr;
      s->up_bytes = 0;
    }
    size_t cap = 1 << 16;
    while (cap < bytes) cap <<= 1;
    if (hipMalloc(&s->up_dev, cap) != hipSuccess) return fail(SV_ERR_NOMEM, "cannot allocate upload buffer");
    if (hipHostMalloc(&s->up_host, cap, hipHostMallocDefault) != hipSuccess) {
      (void)hipFree(s->up_dev);
      s->up_dev = nullptr;
      return fail(SV_ERR_NOMEM, "cannot allocate pinned staging buffer");
    }
    s->up_bytes = cap;
  }
  std::memcpy(s->up_host, host, bytes);
  SV_HIP_TRY(hipMemcpyAsync(s->up_dev, s->up_host, bytes, hipMemcpyHostToDevice, s->stream));
  SV_HIP_TRY(hipEventRecord(s->up_done, s->stream));
  s->up_pending = true;
  *dev = s->up_dev;
  return SV_OK;
}

sv_status run_op_sweep(sv_state* s, const Op& op, const void* m_dev, bool mfma) {
  if (op.nq <= 2) {
    SweepArgs a;
    if (!low_args_for(op, s->dt, &a)) sweep_args_for(op, &a);
    SV_LAUNCH(launch_sweep(s->dt, s->ptr, s->n, a, s->stream), s->stream);
    return SV_OK;
  }
  if (op.nq > s->n) return fail(SV_ERR_QUBIT, "op on %d qubits exceeds the state's %d", op.nq, s->n);
  SV_LAUNCH(launch_dense_kq(s->dt, s->ptr, s->n, op.nq, op.q, m_dev, mfma, s->stream), s->stream);
  return SV_OK;
}

sv_status renormalize(sv_state* s) {
  // scratch: [squared norm][reduction partials]
  const size_t part = probs_scratch_bytes(s->n, 0, nullptr);
  if (sv_status st = ensure_scratch(s, 256 + part)) return st;
  double* norm2 = (double*)s->scratch;
  SV_LAUNCH(launch_probs(s->dt, s->ptr, s->n, nullptr, 0, norm2, (unsigned char*)s->scratch + 256, s->stream), s->stream);
  SweepArgs a{};
  a.op = SWEEP_SCALE_NORM;
  a.g.nz = 0;
  a.g.nv = 1;
  a.norm2_dev = norm2;
  SV_LAUNCH(launch_sweep(s->dt, s->ptr, s->n, a, s->stream), s->stream);
  return SV_OK;
}

sv_status probs_args(int n, const int32_t* qubits, int m, const double* out_dev, int* qs) {
  if (m < 0 || m > n) return fail(SV_ERR_ARG, "m=%d outside 0..%d", m, n);
  if (m > 0 && !qubits) return fail(SV_ERR_ARG, "null qubit list");
  if (!out_dev) return fail(SV_ERR_ARG, "null output");
  for (int r = 0; r < m; ++r) {
    if (qubits[r] < 0 || qubits[r] >= n) return fail(SV_ERR_QUBIT, "qubit %d out of range", qubits[r]);
    for (int j = 0; j < r; ++j)
      if (qubits[j] == qubits[r]) return fail(SV_ERR_QUBIT, "qubit %d repeated", qubits[r]);
    qs[r] = qubits[r];
  }
  return SV_OK;
}

static sv_status check_state(const sv_state* s) {
  if (!s) return fail(SV_ERR_ARG, "null state");
  return SV_OK;
}

static sv_status validate_opts(const sv_opts& o) {
  if (o.max_fuse_qubits < 0 || o.max_fuse_qubits > SV_MAX_GATE_QUBITS)
    return fail(SV_ERR_ARG, "max_fuse_qubits %d outside 0..%d", o.max_fuse_qubits, SV_MAX_GATE_QUBITS);
  if (o.lds_qubits < 0 || o.lds_qubits > 16) return fail(SV_ERR_ARG, "lds_qubits %d outside 0..16", o.lds_qubits);
  if (o.pinned_low_bits < 0 || o.pinned_low_bits > 8)
    return fail(SV_ERR_ARG, "pinned_low_bits %d outside 0..8", o.pinned_low_bits);
  if (o.renorm_interval < 0) return fail(SV_ERR_ARG, "negative renorm_interval");
  if (o.mode < SV_MODE_AUTO || o.mode > SV_MODE_MATRIX) return fail(SV_ERR_ARG, "bad mode %d", o.mode);
  if (o.max_pass_ops < 0) return fail(SV_ERR_ARG, "negative max_pass_ops");
  return SV_OK;
}

}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_default_opts(sv_opts* o) {
  if (!o) return fail(SV_ERR_ARG, "null opts");
  o->max_fuse_qubits = 5;
  o->lds_qubits = 0;
  o->pinned_low_bits = 0;
  o->reorder = 1;
  o->fp32_mfma = 1;
  o->renorm_interval = 0;
  o->mode = SV_MODE_AUTO;
  o->max_pass_ops = 0;
  return SV_OK;
}

sv_status sv_create(int n, sv_dtype dt, void* dev_ptr, void* stream, unsigned flags, sv_state** out) {
  clear_error();
  if (!out) return fail(SV_ERR_ARG, "null output handle");
  *out = nullptr;
  if (n < 1 || n > SV_MAX_QUBITS) return fail(SV_ERR_ARG, "n_qubits %d outside 1..%d", n, SV_MAX_QUBITS);
  if (dt != SV_C64 && dt != SV_C128) return fail(SV_ERR_ARG, "bad dtype %d", (int)dt);
  if (flags & ~SV_NO_INIT) return fail(SV_ERR_ARG, "unknown flags 0x%x", flags);
  if (dev_ptr && ((uintptr_t)dev_ptr & 255u)) return fail(SV_ERR_ARG, "device buffer not 256-byte aligned");
  sv_state* s = new (std::nothrow) sv_state();
  if (!s) return fail(SV_ERR_NOMEM, "host allocation failed");
  s->n = n;
  s->dt = dt;
  s->stream = (hipStream_t)stream;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(SV_ERR_DEVICE, "no HIP device");
  }
  if (hipEventCreateWithFlags(&s->up_done, hipEventDisableTiming) != hipSuccess) {
    delete s;
    return fail(SV_ERR_DEVICE, "hipEventCreate failed");
  }
  const size_t bytes = ((size_t)1 << n) * elem_bytes(dt);
  if (dev_ptr) {
    s->ptr = dev_ptr;
  } else {
    if (hipMalloc(&s->ptr, bytes) != hipSuccess) {
      (void)hipEventDestroy(s->up_done);
      delete s;
      return fail(SV_ERR_NOMEM, "cannot allocate %zu bytes for the state", bytes);
    }
    s->owned = true;
  }
  if (!(flags & SV_NO_INIT)) {
    hipError_t e = launch_init_basis(dt, s->ptr, n, 0, s->stream);
    if (e != hipSuccess) {
      sv_destroy(s);
      return fail(SV_ERR_DEVICE, "init: %s", hipGetErrorString(e));
    }
  }
  *out = s;
  return SV_OK;
}

sv_status sv_destroy(sv_state* s) {
  clear_error();
  if (!s) return SV_OK;
  sv_status st = SV_OK;
  const bool frees = (s->owned && s->ptr) || s->scratch || s->up_dev || s->up_host;
  if (frees && hipStreamSynchronize(s->stream) != hipSuccess) st = fail(SV_ERR_DEVICE, "stream sync failed in destroy");
  if (s->owned && s->ptr) (void)hipFree(s->ptr);
  if (s->scratch) (void)hipFree(s->scratch);
  if (s->up_dev) (void)hipFree(s->up_dev);
  if (s->up_host) (void)hipHostFree(s->up_host);
  if (s->up_done) (void)hipEventDestroy(s->up_done);
  delete s;
  return st;
}

sv_status sv_state_info(const sv_state* s, int* n, sv_dtype* dt, void** ptr) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  if (n) *n = s->n;
  if (dt) *dt = s->dt;
  if (ptr) *ptr = s->ptr;
  return SV_OK;
}

sv_status sv_set_stream(sv_state* s, void* stream) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  s->stream = (hipStream_t)stream;
  return SV_OK;
}

sv_status sv_init_basis(sv_state* s, uint64_t index) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  if (index >= (1ull << s->n)) return fail(SV_ERR_ARG, "basis index out of range");
  SV_LAUNCH(launch_init_basis(s->dt, s->ptr, s->n, index, s->stream), s->stream);
  return SV_OK;
}

sv_status sv_apply_gate(sv_state* s, const sv_gate* g) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  if (!g) return fail(SV_ERR_ARG, "null gate");
  if (sv_status st = validate_gate(*g, s->n)) return st;
  Op op = op_from_gate(*g);
  if (op.nq <= 2) return run_op_sweep(s, op, nullptr);
  const bool f32 = s->dt == SV_C64;
  std::vector<unsigned char> host(op.m.size() * 2 * (f32 ? 4 : 8));
  for (size_t e = 0; e < op.m.size(); ++e) {
    if (f32) {
      ((float*)host.data())[2 * e] = (float)op.m[e].real();
      ((float*)host.data())[2 * e + 1] = (float)op.m[e].imag();
    } else {
      ((double*)host.data())[2 * e] = op.m[e].real();
      ((double*)host.data())[2 * e + 1] = op.m[e].imag();
    }
  }
  void* dev = nullptr;
  if (sv_status st = upload(s, host.data(), host.size(), &dev)) return st;
  return run_op_sweep(s, op, dev);
}

sv_status sv_fuse(int n, sv_dtype dt, const sv_gate* g, size_t n_gates, const sv_opts* o, sv_plan** out) {
  clear_error();
  if (!out) return fail(SV_ERR_ARG, "null output plan");
  *out = nullptr;
  if (n < 1 || n > SV_MAX_QUBITS) return fail(SV_ERR_ARG, "n_qubits %d outside 1..%d", n, SV_MAX_QUBITS);
  if (dt != SV_C64 && dt != SV_C128) return fail(SV_ERR_ARG, "bad dtype %d", (int)dt);
  if (n_gates && !g) return fail(SV_ERR_ARG, "null gate list");
  sv_opts opts;
  if (o) opts = *o;
  else sv_default_opts(&opts);
  if (sv_status st = validate_opts(opts)) return st;
  for (size_t i = 0; i < n_gates; ++i) {
    if (sv_status st = validate_gate(g[i], n)) {
      std::string msg = sv_last_error();
      return fail(st, "gate %zu: %s", i, msg.c_str());
    }
  }
  sv_plan* p = new (std::nothrow) sv_plan();
  if (!p) return fail(SV_ERR_NOMEM, "host allocation failed");
  sv_status st = build_plan(n, dt, g, n_gates, opts, p);
  if (st != SV_OK) {
    delete p;
    return st;
  }
  *out = p;
  return SV_OK;
}

sv_status sv_plan_info(const sv_plan* p, size_t* n_ops, size_t* n_passes) {
  clear_error();
  if (!p) return fail(SV_ERR_ARG, "null plan");
  if (n_ops) *n_ops = p->ops.size();
  if (n_passes) *n_passes = p->passes.size();
  return SV_OK;
}

sv_status sv_plan_export(const sv_plan* p, size_t op, int32_t* nq, int32_t q[SV_MAX_GATE_QUBITS], double* m,
                         int32_t* pass) {
  clear_error();
  if (!p) return fail(SV_ERR_ARG, "null plan");
  if (op >= p->ops.size()) return fail(SV_ERR_ARG, "op %zu out of range (%zu ops)", op, p->ops.size());
  const Op& o = p->ops[op];
  if (nq) *nq = o.nq;
  if (q)
    for (int i = 0; i < SV_MAX_GATE_QUBITS; ++i) q[i] = i < o.nq ? o.q[i] : -1;
  if (m)
    for (size_t e = 0; e < o.m.size(); ++e) {
      m[2 * e] = o.m[e].real();
      m[2 * e + 1] = o.m[e].imag();
    }
  if (pass) *pass = op < p->op_pass.size() ? (int32_t)p->op_pass[op] : -1;
  return SV_OK;
}

sv_status sv_plan_pass_info(const sv_plan* p, size_t pass, int32_t* kind, int32_t* n_ops, int32_t* n_local,
                            int32_t* n_stages) {
  clear_error();
  if (!p) return fail(SV_ERR_ARG, "null plan");
  if (pass >= p->passes.size()) return fail(SV_ERR_ARG, "pass %zu out of range", pass);
  const Pass& ps = p->passes[pass];
  if (kind) *kind = ps.kind;
  if (n_ops) *n_ops = ps.n_ops;
  if (n_local) *n_local = ps.n_local;
  if (n_stages) *n_stages = (int32_t)ps.stages.size();
  return SV_OK;
}

namespace {
// Flops per amplitude of every pass, filled once per plan by one sweep over
// its ops (later queries are O(1) per pass).
const std::vector<double>& plan_flops(const sv_plan* p) {
  sv_plan::FlopsCache& fc = *p->flops;
  std::call_once(fc.once, [p, &fc]() {
    fc.per_pass.assign(p->passes.size(), 0.0);
    for (size_t i = 0; i < p->ops.size(); ++i) {
      const OpClass c = classify(p->ops[i]);
      fc.per_pass[(size_t)p->op_pass[i]] += c == CLS_PERM ? 0.0 : c == CLS_DIAG ? 6.0 : 8.0 * (double)(1 << p->ops[i].nq);
    }
  });
  return fc.per_pass;
}
}  // namespace

sv_status sv_plan_pass_flops(const sv_plan* p, size_t pass, double* flops_per_amp) {
  clear_error();
  if (!p || !flops_per_amp) return fail(SV_ERR_ARG, "null argument");
  if (pass >= p->passes.size()) return fail(SV_ERR_ARG, "pass %zu out of range", pass);
  *flops_per_amp = plan_flops(p)[pass];
  return SV_OK;
}

sv_status sv_plan_flops(const sv_plan* p, double* flops_per_amp, size_t count) {
  clear_error();
  if (!p || !flops_per_amp) return fail(SV_ERR_ARG, "null argument");
  if (count < p->passes.size()) return fail(SV_ERR_ARG, "room for %zu passes, plan has %zu", count, p->passes.size());
  const std::vector<double>& f = plan_flops(p);
  std::copy(f.begin(), f.end(), flops_per_amp);
  return SV_OK;
}

sv_status sv_plan_pass_ops(const sv_plan* p, size_t pass, int32_t* n_ops, int32_t* n_ladders) {
  clear_error();
  if (!p) return fail(SV_ERR_ARG, "null plan");
  if (pass >= p->passes.size()) return fail(SV_ERR_ARG, "pass %zu out of range", pass);
  int32_t ops = 0, ladders = 0;
  for (const StageHost& sh : p->passes[pass].stages) {
    ops += sh.n_ops;
    ladders += sh.n_fixed;
  }
  if (n_ops) *n_ops = ops;
  if (n_ladders) *n_ladders = ladders;
  return SV_OK;
}

sv_status sv_plan_destroy(sv_plan* p) {
  clear_error();
  delete p;
  return SV_OK;
}

sv_status sv_apply_plan(sv_state* s, const sv_plan* p) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  if (!p) return fail(SV_ERR_ARG, "null plan");
  if (p->n != s->n || p->dt != s->dt)
    return fail(SV_ERR_ARG, "plan built for n=%d dtype=%d, state has n=%d dtype=%d", p->n, (int)p->dt, s->n,
                (int)s->dt);
  return execute_plan(s, p);
}

sv_status sv_apply_circuit(sv_state* s, const sv_gate* g, size_t n_gates, const sv_opts* o) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  sv_plan* p = nullptr;
  if (sv_status st = sv_fuse(s->n, s->dt, g, n_gates, o, &p)) return st;
  sv_status st = execute_plan(s, p);
  delete p;
  return st;
}

sv_status sv_permute_qubits(sv_state* s, const int32_t* dest) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  if (!dest) return fail(SV_ERR_ARG, "null permutation");
  const int n = s->n;
  std::vector<int> target(n, -1);  // target[p]: the old qubit whose bit ends at position p
  for (int q = 0; q < n; ++q) {
    if (dest[q] < 0 || dest[q] >= n) return fail(SV_ERR_QUBIT, "dest[%d] = %d out of range", q, dest[q]);
    if (target[dest[q]] >= 0) return fail(SV_ERR_QUBIT, "dest is not a permutation (%d repeated)", dest[q]);
    target[dest[q]] = q;
  }
  // The permutation as transpositions of index bits (selection order, at most
  // n-1 SWAPs).  Planned in tile-pass mode, each SWAP only relabels qubits and
  // the data moves once, in the permutation passes that restore the labels.
  std::vector<int> cur(n);
  for (int p = 0; p < n; ++p) cur[p] = p;
  std::vector<sv_gate> swaps;
  for (int p = 0; p < n; ++p) {
    if (cur[p] == target[p]) continue;
    int j = p + 1;
    while (cur[j] != target[p]) ++j;
    sv_gate g{};
    g.kind = SV_G_SWAP;
    g.nq = 2;
    g.q[0] = p;
    g.q[1] = j;
    for (int r = 2; r < SV_MAX_GATE_QUBITS; ++r) g.q[r] = -1;
    swaps.push_back(g);
    std::swap(cur[p], cur[j]);
  }
  if (swaps.empty()) return SV_OK;
  sv_opts o;
  sv_default_opts(&o);
  o.max_fuse_qubits = 0;
  o.reorder = 1;
  // tiles need more local bits than one stage's registers; tiny states use SWAP sweeps
  o.mode = n > pass_reg_bits(s->dt) ? SV_MODE_PASS : SV_MODE_SWEEP;
  return sv_apply_circuit(s, swaps.data(), swaps.size(), &o);
}

sv_status sv_measure_probs(sv_state* s, const int32_t* qubits, int m, double* out_dev) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  int qs[SV_MAX_QUBITS];
  if (sv_status st = probs_args(s->n, qubits, m, out_dev, qs)) return st;
  const size_t need = probs_scratch_bytes(s->n, m, qs);
  if (sv_status st = ensure_scratch(s, 256 + need)) return st;
  SV_LAUNCH(launch_probs(s->dt, s->ptr, s->n, qs, m, out_dev, (unsigned char*)s->scratch + 256, s->stream), s->stream);
  return SV_OK;
}

sv_status sv_measure_probs_noalloc(sv_state* s, const int32_t* qubits, int m, double* out_dev) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  int qs[SV_MAX_QUBITS];
  if (sv_status st = probs_args(s->n, qubits, m, out_dev, qs)) return st;
  const size_t need = probs_scratch_bytes(s->n, m, qs);
  if (need > static_scratch_bytes())
    return fail(SV_ERR_UNSUPPORTED, "reduction needs %zu bytes of scratch, the static array holds %zu", need,
                static_scratch_bytes());
  void* scratch = nullptr;
  SV_HIP_TRY(static_scratch(s->device, &scratch));
  SV_LAUNCH(launch_probs(s->dt, s->ptr, s->n, qs, m, out_dev, scratch, s->stream), s->stream);
  return SV_OK;
}

sv_status sv_scale(sv_state* s, double scale) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  SweepArgs a{};
  a.op = SWEEP_SCALE;
  a.g.nz = 0;
  a.g.nv = 1;
  a.m[0] = scale;
  SV_LAUNCH(launch_sweep(s->dt, s->ptr, s->n, a, s->stream), s->stream);
  return SV_OK;
}

sv_status sv_sync(sv_state* s) {
  clear_error();
  if (sv_status st = check_state(s)) return st;
  SV_HIP_TRY(hipStreamSynchronize(s->stream));
  SV_HIP_TRY(hipGetLastError());
  return SV_OK;
}

sv_status sv_gate_kernel(int n, sv_dtype dt, const sv_gate* g, char* buf, size_t len) {
  clear_error();
  if (!g || !buf || len == 0) return fail(SV_ERR_ARG, "null argument");
  if (n < 1 || n > SV_MAX_QUBITS) return fail(SV_ERR_ARG, "n_qubits %d outside 1..%d", n, SV_MAX_QUBITS);
  if (dt != SV_C64 && dt != SV_C128) return fail(SV_ERR_ARG, "bad dtype %d", (int)dt);
  if (sv_status st = validate_gate(*g, n)) return st;
  const Op op = op_from_gate(*g);
  const char* dts = dt == SV_C128 ? "c128" : "c64";
  std::string name;
  SweepArgs a;
  if (op.nq >= 3) {
    name = std::string("dense/") + dts + "/k" + std::to_string(op.nq);
  } else if (low_args_for(op, dt, &a)) {
    static const char* kn[] = {"INTRA", "LANE", "REG"};
    name = std::string("lane/") + dts + "/K" + std::to_string(a.low_k) + "/" + kn[a.low_kind[0]];
    if (a.low_k == 2) name += std::string("-") + kn[a.low_kind[1]];
    name += "/z" + std::to_string(a.low_nz);
  } else {
    sweep_args_for(op, &a);
    static const char* on[] = {"DENSE1", "DENSE2", "SWAP", "PHASE", "DIAG", "SCALE", "LOW"};
    uint64_t used = a.g.set;
    for (int i = 0; i < a.g.nz; ++i) used |= 1ull << a.g.z[i];
    for (int i = 0; i < a.g.nv; ++i) used |= a.g.off[i];
    const char* el = dt == SV_C128 ? "c128" : ((used & 1ull) ? "c64x1" : "c64x2");
    name = std::string("group/") + el + "/" + on[a.op] + "/z" + std::to_string(a.g.nz) + "v" + std::to_string(a.g.nv);
  }
  if (name.size() + 1 > len) return fail(SV_ERR_ARG, "buffer of %zu bytes too small", len);
  std::memcpy(buf, name.c_str(), name.size() + 1);
  return SV_OK;
}

const char* sv_last_error(void) { return g_error.c_str(); }

const char* sv_version(void) { return "sv-mi355x 0.1 (gfx950)"; }

}  // extern "C"

#include "sv_util.h"

extern "C" sv_status sv_util_copy(void* dst, const void* src, size_t bytes, void* stream) {
  clear_error();
  if (!dst || !src) return fail(SV_ERR_ARG, "null buffer");
  if (bytes % 16) return fail(SV_ERR_ARG, "size %zu is not a multiple of 16", bytes);
  SV_LAUNCH(launch_copy_bytes(dst, src, bytes, (hipStream_t)stream), (hipStream_t)stream);
  return SV_OK;
}
