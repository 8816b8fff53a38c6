// Planner: general gate fusion (QueenV2 Sec. II-B "Gate Fusion", Sec. III-A
// tier 5) and the grouping of ops into state sweeps.  Host only: no HIP call
// is made here, so plans can be built and inspected without a GPU.
#include <algorithm>
#include <cstring>

#include "sv_host.h"

namespace sv {
namespace {

// Relative cost of one op executed as its own sweep, in units of one full
// read+write sweep of the state.  Memory time scales with the touched
// fraction; arithmetic time with the dense flops per amplitude (8 * 2^k for a
// complex 2^k x 2^k product) over the flop/byte ridge of the precision.
double sweep_cost(const Op& op, sv_dtype dt, bool mfma) {
  const double bytes_per_amp = 2.0 * (double)elem_bytes(dt);
  double ridge;  // flops per byte at which compute time equals memory time
  if (dt == SV_C128) ridge = 78.6 / 8.0;
  else ridge = (mfma && op.nq >= 4 ? 157.3 : 78.6) / 8.0;
  const OpClass cls = classify(op);
  double flops_per_amp;
  if (cls == CLS_PERM) flops_per_amp = 0.0;
  else if (cls == CLS_DIAG) flops_per_amp = 6.0;
  else flops_per_amp = 8.0 * (double)(1 << op.nq);
  const double mem = op.kind == SV_G_MATRIX ? 1.0 : touched_fraction(op);
  const double alu = flops_per_amp / (bytes_per_amp * ridge);
  return std::max(mem, alu);
}

// Left-multiply the d x d matrix `m` (k qubits, local order `uq`) by gate
// `g`: every column is treated as a k-qubit vector and g is applied to the
// groups of its positions (Eq. 2/3 on the fused space).
void apply_left(std::vector<cd>& m, int k, const int* uq, const Op& g) {
  const int d = 1 << k;
  const int dg = 1 << g.nq;
  int pos[SV_MAX_GATE_QUBITS];  // bit position (within the k-bit local index) of g's qubits
  for (int j = 0; j < g.nq; ++j) {
    int p = -1;
    for (int i = 0; i < k; ++i)
      if (uq[i] == g.q[j]) p = k - 1 - i;
    pos[j] = p;
  }
  int gmask = 0;
  for (int j = 0; j < g.nq; ++j) gmask |= 1 << pos[j];
  std::vector<cd> in(dg), out(dg);
  std::vector<int> idx(dg);
  for (int c = 0; c < d; ++c) {
    for (int base = 0; base < d; ++base) {
      if (base & gmask) continue;
      for (int r = 0; r < dg; ++r) {
        int i = base;
        for (int j = 0; j < g.nq; ++j)
          if ((r >> (g.nq - 1 - j)) & 1) i |= 1 << pos[j];
        idx[r] = i;
        in[r] = m[(size_t)i * d + c];
      }
      for (int r = 0; r < dg; ++r) {
        cd y = 0.0;
        for (int s = 0; s < dg; ++s) y += g.m[(size_t)r * dg + s] * in[s];
        out[r] = y;
      }
      for (int r = 0; r < dg; ++r) m[(size_t)idx[r] * d + c] = out[r];
    }
  }
}

// Fuse gate g into op o (g acts after o).  New qubits are appended as the
// least significant local bits, so o's matrix embeds as o (x) I.
Op merged(const Op& o, const Op& g) {
  Op r;
  r.kind = SV_G_MATRIX;
  r.nq = o.nq;
  for (int i = 0; i < o.nq; ++i) r.q[i] = o.q[i];
  for (int j = 0; j < g.nq; ++j) {
    bool have = false;
    for (int i = 0; i < r.nq; ++i) have |= r.q[i] == g.q[j];
    if (!have) r.q[r.nq++] = g.q[j];
  }
  const int k = r.nq, e = r.nq - o.nq;
  const int d = 1 << k, emask = (1 << e) - 1, dold = 1 << o.nq;
  r.m.assign((size_t)d * d, cd(0.0, 0.0));
  for (int row = 0; row < d; ++row)
    for (int col = 0; col < d; ++col)
      if ((row & emask) == (col & emask)) r.m[(size_t)row * d + col] = o.m[(size_t)(row >> e) * dold + (col >> e)];
  apply_left(r.m, k, r.q, g);
  r.n_gates = o.n_gates + g.n_gates;
  return r;
}

int union_size(const Op& a, const Op& b) {
  int u = a.nq;
  for (int j = 0; j < b.nq; ++j) {
    bool have = false;
    for (int i = 0; i < a.nq; ++i) have |= a.q[i] == b.q[j];
    if (!have) ++u;
  }
  return u;
}

}  // namespace

sv_status build_plan(int n, sv_dtype dt, const sv_gate* g, size_t n_gates, const sv_opts& o, sv_plan* p) {
  p->n = n;
  p->dt = dt;
  p->opts = o;
  p->n_gates_in = n_gates;
  p->ops.clear();
  p->passes.clear();
  const int kmax = o.max_fuse_qubits;
  const bool mfma = dt == SV_C64 && o.fp32_mfma;
  std::vector<int> last(n, -1);  // index of the last op touching each qubit
  for (size_t i = 0; i < n_gates; ++i) {
    Op op = op_from_gate(g[i]);
    int cand = -1;
    for (int j = 0; j < op.nq; ++j) cand = std::max(cand, last[op.q[j]]);
    // Every op after `cand` shares no qubit with this gate, so the gate may be
    // moved up to just after `cand` and fused into it.
    if (kmax >= 2 && cand >= 0 && union_size(p->ops[cand], op) <= kmax) {
      Op& prev = p->ops[cand];
      Op m = merged(prev, op);
      if (sweep_cost(m, dt, mfma) <= sweep_cost(prev, dt, mfma) + sweep_cost(op, dt, mfma) + 1e-12) {
        prev = std::move(m);
        // only the gate's qubits move to `cand`; the other qubits of the fused
        // op may already have later users
        for (int j = 0; j < op.nq; ++j) last[op.q[j]] = cand;
        continue;
      }
    }
    p->ops.push_back(std::move(op));
    const int idx = (int)p->ops.size() - 1;
    for (int j = 0; j < p->ops.back().nq; ++j) last[p->ops.back().q[j]] = idx;
  }
  // One sweep per op.
  for (size_t i = 0; i < p->ops.size(); ++i) {
    Pass ps;
    ps.kind = p->ops[i].nq >= 3 ? 2 : 0;
    ps.first_op = (int)i;
    ps.n_ops = 1;
    p->passes.push_back(ps);
  }
  return SV_OK;
}

sv_status execute_plan(sv_state* s, const sv_plan* p) {
  // Upload every matrix a dense kernel reads, in the state's precision, in one copy.
  std::vector<size_t> offs(p->ops.size(), 0);
  size_t total = 0;
  const bool f32 = s->dt == SV_C64;
  const size_t scal = f32 ? sizeof(float) : sizeof(double);
  for (size_t i = 0; i < p->ops.size(); ++i) {
    if (p->ops[i].nq >= 3) {
      offs[i] = total;
      total += p->ops[i].m.size() * 2 * scal;
      total = (total + 255) & ~(size_t)255;
    }
  }
  void* dev = nullptr;
  if (total) {
    std::vector<unsigned char> host(total);
    for (size_t i = 0; i < p->ops.size(); ++i) {
      if (p->ops[i].nq < 3) continue;
      const std::vector<cd>& m = p->ops[i].m;
      if (f32) {
        float* dst = (float*)(host.data() + offs[i]);
        for (size_t e = 0; e < m.size(); ++e) {
          dst[2 * e] = (float)m[e].real();
          dst[2 * e + 1] = (float)m[e].imag();
        }
      } else {
        double* dst = (double*)(host.data() + offs[i]);
        for (size_t e = 0; e < m.size(); ++e) {
          dst[2 * e] = m[e].real();
          dst[2 * e + 1] = m[e].imag();
        }
      }
    }
    sv_status st = upload(s, host.data(), total, &dev);
    if (st != SV_OK) return st;
  }
  for (size_t i = 0; i < p->ops.size(); ++i) {
    const void* mdev = p->ops[i].nq >= 3 ? (const void*)((const unsigned char*)dev + offs[i]) : nullptr;
    sv_status st = run_op_sweep(s, p->ops[i], mdev);
    if (st != SV_OK) return st;
  }
  return SV_OK;
}

}  // namespace sv
