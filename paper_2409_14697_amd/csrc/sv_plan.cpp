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
  if (op.nq >= 3) {
    // dense k-qubit kernels, in sweeps of the state (measured on MI355X at
    // N=30): HBM-bound up to k = 5, matrix-core bound at k = 6
    static const double c64_mfma[7] = {0, 0, 0, 1.15, 1.26, 1.26, 1.87};
    static const double c64_valu[7] = {0, 0, 0, 1.15, 1.4, 2.1, 4.2};
    static const double c128[7] = {0, 0, 0, 1.27, 1.27, 1.3, 3.2};
    const int k = op.nq > 6 ? 6 : op.nq;
    return dt == SV_C128 ? c128[k] : (mfma ? c64_mfma[k] : c64_valu[k]);
  }
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
  cd in[1 << SV_MAX_GATE_QUBITS], out[1 << SV_MAX_GATE_QUBITS];
  int idx[1 << SV_MAX_GATE_QUBITS];
  if (g.nq == 1) {
    // the common case: two rows mix.  The products and sums are those of the
    // general loop below, written on real parts (same roundings), so that the
    // column loop has no branches
    const double g0r = g.m[0].real(), g0i = g.m[0].imag(), g1r = g.m[1].real(), g1i = g.m[1].imag();
    const double g2r = g.m[2].real(), g2i = g.m[2].imag(), g3r = g.m[3].real(), g3i = g.m[3].imag();
    const int b0 = 1 << pos[0];
    for (int base = 0; base < d; ++base) {
      if (base & b0) continue;
      double* r0 = reinterpret_cast<double*>(m.data() + (size_t)base * d);
      double* r1 = reinterpret_cast<double*>(m.data() + (size_t)(base | b0) * d);
      for (int c = 0; c < d; ++c) {
        const double ar = r0[2 * c], ai = r0[2 * c + 1], br = r1[2 * c], bi = r1[2 * c + 1];
        r0[2 * c] = (0.0 + (g0r * ar - g0i * ai)) + (g1r * br - g1i * bi);
        r0[2 * c + 1] = (0.0 + (g0r * ai + g0i * ar)) + (g1r * bi + g1i * br);
        r1[2 * c] = (0.0 + (g2r * ar - g2i * ai)) + (g3r * br - g3i * bi);
        r1[2 * c + 1] = (0.0 + (g2r * ai + g2i * ar)) + (g3r * bi + g3i * br);
      }
    }
    return;
  }
  if (g.nq == 2) {  // four rows mix; the same sums as the general loop
    double gr[16], gi[16];
    for (int e = 0; e < 16; ++e) {
      gr[e] = g.m[e].real();
      gi[e] = g.m[e].imag();
    }
    const int bh = 1 << pos[0], bl = 1 << pos[1];  // r = 2 (bit of q[0]) + (bit of q[1])
    for (int base = 0; base < d; ++base) {
      if (base & gmask) continue;
      double* row[4] = {reinterpret_cast<double*>(m.data() + (size_t)base * d),
                        reinterpret_cast<double*>(m.data() + (size_t)(base | bl) * d),
                        reinterpret_cast<double*>(m.data() + (size_t)(base | bh) * d),
                        reinterpret_cast<double*>(m.data() + (size_t)(base | bh | bl) * d)};
      for (int c = 0; c < d; ++c) {
        double xr[4], xi[4];
        for (int s = 0; s < 4; ++s) {
          xr[s] = row[s][2 * c];
          xi[s] = row[s][2 * c + 1];
        }
        for (int r = 0; r < 4; ++r) {
          double yr = 0.0, yi = 0.0;
          for (int s = 0; s < 4; ++s) {
            const double ur = gr[4 * r + s], ui = gi[4 * r + s];
            yr = yr + (ur * xr[s] - ui * xi[s]);
            yi = yi + (ur * xi[s] + ui * xr[s]);
          }
          row[r][2 * c] = yr;
          row[r][2 * c + 1] = yi;
        }
      }
    }
    return;
  }
  // rows of one group (base: the rows with g's bits clear) mix; the group's
  // row indices are found once and every column is updated in turn
  for (int base = 0; base < d; ++base) {
    if (base & gmask) continue;
    for (int r = 0; r < dg; ++r) {
      int i = base;
      for (int j = 0; j < g.nq; ++j)
        if ((r >> (g.nq - 1 - j)) & 1) i |= 1 << pos[j];
      idx[r] = i;
    }
    for (int c = 0; c < d; ++c) {
      for (int r = 0; r < dg; ++r) in[r] = m[(size_t)idx[r] * d + c];
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

std::vector<Op> fuse_ops(std::vector<Op> in, int n, sv_dtype dt, int kmax, bool mfma) {
  std::vector<Op> out;
  out.reserve(in.size());
  std::vector<int> last(n, -1);  // index of the last op touching each qubit
  const int width = kmax < 1 ? 0 : kmax;
  for (Op& op : in) {
    int cand = -1;
    for (int j = 0; j < op.nq; ++j) cand = std::max(cand, last[op.q[j]]);
    // Every op after `cand` shares no qubit with this one, so it may be moved
    // up to just after `cand` and fused into it.
    if (width >= 1 && cand >= 0 && union_size(out[cand], op) <= width &&
        !(op.kind == SV_G_SWAP && width < 2)) {
      Op& prev = out[cand];
      if (prev.nq >= 3 && union_size(prev, op) == prev.nq) {
        // no new qubit: a dense op keeps its width and cost, so the merge
        // always pays; the product is formed in place (as `merged` would)
        prev.kind = SV_G_MATRIX;
        prev.theta = 0.0;
        apply_left(prev.m, prev.nq, prev.q, op);
        prev.n_gates += op.n_gates;
        for (int j = 0; j < op.nq; ++j) last[op.q[j]] = cand;
        continue;
      }
      Op m = merged(prev, op);
      if (sweep_cost(m, dt, mfma) <= sweep_cost(prev, dt, mfma) + sweep_cost(op, dt, mfma) + 1e-12) {
        prev = std::move(m);
        // only this op's qubits move to `cand`; the other qubits of the fused
        // op may already have later users
        for (int j = 0; j < op.nq; ++j) last[op.q[j]] = cand;
        continue;
      }
    }
    out.push_back(std::move(op));
    const int idx = (int)out.size() - 1;
    for (int j = 0; j < out.back().nq; ++j) last[out.back().q[j]] = idx;
  }
  if (width < 2) return out;
  // Forward pass: an op whose qubits all belong to the next op that touches
  // any of them commutes with everything in between and joins that op (the
  // greedy pass above only merges into the previous op).  Reverse order lets
  // merges chain.
  std::vector<char> gone(out.size(), 0);
  for (int i = (int)out.size() - 2; i >= 0; --i) {
    int j = i + 1;
    while (j < (int)out.size() && (gone[j] || union_size(out[j], out[i]) == out[j].nq + out[i].nq)) ++j;
    if (j == (int)out.size() || union_size(out[j], out[i]) != out[j].nq) continue;
    Op m = merged(out[i], out[j]);
    if (sweep_cost(m, dt, mfma) <= sweep_cost(out[i], dt, mfma) + sweep_cost(out[j], dt, mfma) + 1e-12) {
      out[j] = std::move(m);
      gone[i] = 1;
    }
  }
  std::vector<Op> kept;
  kept.reserve(out.size());
  for (size_t i = 0; i < out.size(); ++i)
    if (!gone[i]) kept.push_back(std::move(out[i]));
  return kept;
}

double op_sweep_cost(const Op& op, sv_dtype dt, bool mfma) { return sweep_cost(op, dt, mfma); }

namespace {

// The op times the identity on `e` further qubits (appended as the least
// significant bits of the local index).
Op widened(const Op& o, const int* extra, int e) {
  Op r;
  r.kind = SV_G_MATRIX;
  r.nq = o.nq + e;
  for (int i = 0; i < o.nq; ++i) r.q[i] = o.q[i];
  for (int i = 0; i < e; ++i) r.q[o.nq + i] = extra[i];
  r.n_gates = o.n_gates;
  const int d = 1 << r.nq, dold = 1 << o.nq, emask = (1 << e) - 1;
  r.m.assign((size_t)d * d, cd(0.0, 0.0));
  for (int row = 0; row < d; ++row)
    for (int col = 0; col < d; ++col)
      if ((row & emask) == (col & emask)) r.m[(size_t)row * d + col] = o.m[(size_t)(row >> e) * dold + (col >> e)];
  return r;
}

// Cost of a matrix pass in full-state sweeps, measured on MI355X at N = 30
// (both precisions): a fixed part (the tile traffic the stages do not hide)
// plus 0.84 sweeps per stage of 32 members (the matrix cores at about 0.65
// of their dense peak), half that for 16 members.
double matrix_pass_cost(int k, int stages) { return 0.65 + 0.84 * stages * (double)(1 << k) / 32.0; }

// Column orders and barriers of a matrix pass's stages: runs of consecutive
// stages share three wave bits that are a member of none of them (so each
// wave keeps its elements through the run and no barrier separates the
// run's stages); a run ends where no three such bits remain.
void assign_matrix_columns(Pass& ps, sv_dtype dt) {
  const int m = ps.n_local, kw = ps.mx_k;
  const int lane_bits = dt == SV_C64 ? 5 : 4;  // log2 of the instruction's columns
  const int nwb = std::min(3, m - kw - lane_bits);  // wave bits: kMatrixWaves = 2^3
  const uint32_t all = (1u << m) - 1u;
  auto targets = [&](const StageHost& sh) {
    uint32_t t = 0;
    for (int b = 0; b < kw; ++b) t |= 1u << sh.q[b];
    return t;
  };
  size_t s0 = 0;
  while (s0 < ps.stages.size()) {
    uint32_t free = all & ~targets(ps.stages[s0]);
    size_t s1 = s0 + 1;
    while (s1 < ps.stages.size() && __builtin_popcount(free & ~targets(ps.stages[s1])) >= nwb) {
      free &= ~targets(ps.stages[s1]);
      ++s1;
    }
    uint32_t wave = 0;  // the highest nwb free bits
    for (int b = m - 1, left = nwb; b >= 0 && left > 0; --b)
      if ((free >> b) & 1u) {
        wave |= 1u << b;
        --left;
      }
    for (size_t si = s0; si < s1; ++si) {
      StageHost& sh = ps.stages[si];
      const uint32_t rest = all & ~targets(sh) & ~wave;
      int j = 0, taken = 0;
      for (int b = 0; b < m && taken < lane_bits; ++b)
        if ((rest >> b) & 1u) {
          sh.colimg[j++] = (uint32_t)b;
          ++taken;
        }
      for (int b = 0; b < m; ++b)
        if ((wave >> b) & 1u) sh.colimg[j++] = (uint32_t)b;
      for (int b = 0, skip = lane_bits; b < m; ++b)
        if ((rest >> b) & 1u) {
          if (skip > 0) {
            --skip;
            continue;
          }
          sh.colimg[j++] = (uint32_t)b;
        }
      sh.flags = (si == s0 && si > 0) ? kMatrixStageSync : 0u;
    }
    s0 = s1;
  }
}

// Stage width of a matrix pass for ops of up to k qubits: FP32 products need
// 32 members, FP64 products 16.
int matrix_width(sv_dtype dt, int k) { return dt == SV_C64 ? 5 : std::max(4, k); }

}  // namespace

void plan_matrix_passes(const std::vector<Op>& fused, int n, sv_dtype dt, const sv_opts& o, sv_plan* p) {
  const bool mfma = dt == SV_C64 && o.fp32_mfma;
  const int m = std::min(n, dt == SV_C64 ? 13 : 12);  // 64 KiB tiles
  const int pin = std::min(default_pinned_bits(dt), m);
  // four column blocks of the instruction per stage (one per wave)
  const int min_cols = dt == SV_C64 ? 7 : 6;
  p->ops.clear();
  p->op_pass.clear();
  p->passes.clear();
  p->est_cost = 0.0;
  std::vector<char> done(fused.size(), 0);
  size_t first = 0;
  auto emit_sweep = [&](const Op& op) {
    Pass ps;
    ps.kind = op.nq >= 3 ? PASS_DENSE : PASS_SWEEP;
    ps.first_op = (int)p->ops.size();
    ps.n_ops = 1;
    ps.phys = op;
    p->op_pass.push_back((int)p->passes.size());
    p->ops.push_back(op);
    p->est_cost += sweep_cost(op, dt, mfma);
    p->passes.push_back(std::move(ps));
  };
  while (true) {
    while (first < fused.size() && done[first]) ++first;
    if (first == fused.size()) break;
    // the longest run of ops (each free of the qubits of the ops skipped
    // before it, so that it may move ahead of them) whose qubits fit a tile
    std::vector<char> in_l(n, 0), blocked(n, 0);
    int count = 0;
    for (int b = 0; b < pin; ++b) {
      in_l[b] = 1;
      ++count;
    }
    std::vector<size_t> members;
    int kw = 0;
    for (size_t j = first; j < fused.size(); ++j) {
      if (done[j]) continue;
      const Op& op = fused[j];
      bool blk = op.nq > 5;
      for (int i = 0; i < op.nq; ++i) blk = blk || blocked[op.q[i]];
      if (!blk) {
        int extra = 0;
        for (int i = 0; i < op.nq; ++i) extra += in_l[op.q[i]] ? 0 : 1;
        const int k2 = matrix_width(dt, std::max(kw, op.nq));
        if (count + extra <= m && m - k2 >= min_cols &&
            (int)members.size() < matrix_pass_max_stages(dt, k2, m)) {
          for (int i = 0; i < op.nq; ++i)
            if (!in_l[op.q[i]]) {
              in_l[op.q[i]] = 1;
              ++count;
            }
          members.push_back(j);
          kw = k2;
          continue;
        }
      }
      for (int i = 0; i < op.nq; ++i) blocked[op.q[i]] = 1;
    }
    double as_sweeps = 0.0;
    for (size_t j : members) as_sweeps += sweep_cost(fused[j], dt, mfma);
    const double cost = members.empty() ? 0.0 : matrix_pass_cost(kw, (int)members.size());
    if (members.empty() || cost >= as_sweeps) {
      emit_sweep(fused[first]);
      done[first] = 1;
      continue;
    }
    // the tile: the group's qubits, the pinned bits, then the lowest others
    for (int b = 0; b < n && count < m; ++b)
      if (!in_l[b]) {
        in_l[b] = 1;
        ++count;
      }
    Pass ps;
    ps.kind = PASS_MATRIX;
    ps.first_op = (int)p->ops.size();
    ps.n_ops = (int)members.size();
    ps.n_local = m;
    ps.mx_k = kw;
    int loc[64];
    for (int b = 0; b < 64; ++b) loc[b] = -1;
    int jl = 0;
    for (int b = 0; b < n; ++b)
      if (in_l[b]) {
        ps.lpos[jl] = ps.wpos[jl] = (uint32_t)b;
        loc[b] = jl++;
      }
    const int pass_id = (int)p->passes.size();
    for (size_t j : members) {
      const Op& op = fused[j];
      // widen to kw qubits with the lowest tile qubits the op does not use
      int extra[6], e = 0;
      for (int jj = 0; jj < m && op.nq + e < kw; ++jj) {
        const int x = (int)ps.lpos[jj];
        bool used = false;
        for (int i = 0; i < op.nq; ++i) used = used || op.q[i] == x;
        if (!used) extra[e++] = x;
      }
      const Op w = e ? widened(op, extra, e) : op;
      StageHost sh;
      // member bit b is op qubit q[kw - 1 - b] (q[0] is the most significant)
      for (int b = 0; b < kw; ++b) sh.q[b] = (uint32_t)loc[w.q[kw - 1 - b]];
      sh.u2 = 0;
      sh.mats = w.m;
      sh.raw.assign(sh.mats.size(), 0);
      sh.n_ops = 1;
      ps.stages.push_back(std::move(sh));
      p->ops.push_back(op);
      p->op_pass.push_back(pass_id);
      done[j] = 1;
    }
    assign_matrix_columns(ps, dt);
    p->est_cost += matrix_pass_cost(kw, (int)members.size());
    p->passes.push_back(std::move(ps));
  }
}

sv_status build_plan(int n, sv_dtype dt, const sv_gate* g, size_t n_gates, const sv_opts& o, sv_plan* p) {
  p->n = n;
  p->dt = dt;
  p->opts = o;
  p->n_gates_in = n_gates;
  p->ops.clear();
  p->op_pass.clear();
  p->passes.clear();
  const bool mfma = dt == SV_C64 && o.fp32_mfma;
  std::vector<Op> raw;
  raw.reserve(n_gates);
  for (size_t i = 0; i < n_gates; ++i) raw.push_back(op_from_gate(g[i]));

  if (o.mode == SV_MODE_MATRIX) {
    plan_matrix_passes(fuse_ops(raw, n, dt, o.max_fuse_qubits, mfma), n, dt, o, p);
    return SV_OK;
  }
  // in-cache passes need a tile of at least 2^(register bits + 1) amplitudes
  const bool tiles_ok = n > pass_reg_bits(dt);
  if (o.mode != SV_MODE_SWEEP && tiles_ok) {
    sv_plan tp;
    tp.n = n;
    tp.dt = dt;
    tp.opts = o;
    std::vector<Op> light = fuse_ops(raw, n, dt, std::min(o.max_fuse_qubits, 1), mfma);
    sv_status st = plan_tile_passes(light, n, dt, o, &tp, false);
    if (st != SV_OK) return st;
    // the same with data moved toward its final position in every pass's
    // write-back; the cheaper of the two is kept
    sv_plan tq;
    tq.n = n;
    tq.dt = dt;
    tq.opts = o;
    if (plan_tile_passes(light, n, dt, o, &tq, true) == SV_OK && tq.est_cost < tp.est_cost) tp = std::move(tq);
    // with relabelings (SWAPs) ahead, gate blocks that leave a few local bits
    // to moving data can save permutation passes at the end
    bool relabels = false;
    for (const Op& op : light) relabels = relabels || (o.reorder && op.kind == SV_G_SWAP);
    for (int reserve = 1; relabels && reserve <= 3; ++reserve) {
      sv_plan tr;
      tr.n = n;
      tr.dt = dt;
      tr.opts = o;
      if (plan_tile_passes(light, n, dt, o, &tr, true, reserve) == SV_OK && tr.est_cost < tp.est_cost)
        tp = std::move(tr);
    }
    if (o.mode == SV_MODE_PASS) {
      p->ops = std::move(tp.ops);
      p->op_pass = std::move(tp.op_pass);
      p->passes = std::move(tp.passes);
      p->est_cost = tp.est_cost;
      return SV_OK;
    }
    // SV_MODE_AUTO: the cheapest of the tile plan, the matrix-pass plan and
    // one sweep per fused op
    std::vector<Op> fused = fuse_ops(raw, n, dt, o.max_fuse_qubits, mfma);
    double sweep_total = 0.0;
    for (const Op& op : fused) sweep_total += sweep_cost(op, dt, mfma);
    sv_plan mq;
    mq.n = n;
    mq.dt = dt;
    mq.opts = o;
    plan_matrix_passes(fused, n, dt, o, &mq);
    sv_plan* best = tp.est_cost <= mq.est_cost ? &tp : &mq;
    if (best->est_cost <= sweep_total) {
      p->ops = std::move(best->ops);
      p->op_pass = std::move(best->op_pass);
      p->passes = std::move(best->passes);
      p->est_cost = best->est_cost;
      return SV_OK;
    }
    p->ops = std::move(fused);
  } else {
    p->ops = fuse_ops(raw, n, dt, o.max_fuse_qubits, mfma);
  }
  // one sweep per op
  p->est_cost = 0.0;
  for (size_t i = 0; i < p->ops.size(); ++i) {
    Pass ps;
    ps.kind = p->ops[i].nq >= 3 ? PASS_DENSE : PASS_SWEEP;
    ps.first_op = (int)i;
    ps.n_ops = 1;
    ps.phys = p->ops[i];
    p->passes.push_back(std::move(ps));
    p->op_pass.push_back((int)i);
    p->est_cost += sweep_cost(p->ops[i], dt, mfma);
  }
  return SV_OK;
}

sv_status pack_plan(const sv_plan* p, PackedPlan* out) {
  if (!p || (p->dt != SV_C64 && p->dt != SV_C128)) return fail(SV_ERR_ARG, "bad plan");
  const bool f32 = p->dt == SV_C64;
  const size_t scal = f32 ? sizeof(float) : sizeof(double);
  const int rb = pass_reg_bits(p->dt);
  std::vector<unsigned char>& host = out->host;
  host.clear();
  auto align = [&]() { host.resize((host.size() + 255) / 256 * 256); };
  auto put_cd = [&](const cd* m, size_t count, const uint8_t* raw) {
    align();
    const size_t at = host.size();
    host.resize(at + count * 2 * scal);
    write_pool(host.data() + at, m, raw, count, f32);
    return at;
  };
  auto put = [&](const void* src, size_t bytes) {
    align();
    const size_t at = host.size();
    host.resize(at + bytes);
    if (bytes) std::memcpy(host.data() + at, src, bytes);
    return at;
  };
  out->dense_off.assign(p->passes.size(), 0);
  out->desc_index.assign(p->passes.size(), -1);
  out->pass_lp.assign(p->passes.size(), 0);
  out->max_m = 0;
  std::vector<PassDescDev> descs;
  std::vector<PassStageDev> stages;
  std::vector<PassItemDev> items;
  std::vector<cd> pool;
  std::vector<uint8_t> pool_raw;
  for (size_t i = 0; i < p->passes.size(); ++i) {
    const Pass& ps = p->passes[i];
    if (ps.kind == PASS_DENSE || ps.kind == PASS_SWEEP) {
      if (ps.kind == PASS_DENSE) out->dense_off[i] = put_cd(ps.phys.m.data(), ps.phys.m.size(), nullptr);
      continue;
    }
    PassDescDev d{};
    d.m = (uint32_t)ps.n_local;
    d.stage_first = (uint32_t)stages.size();
    d.stage_count = (uint32_t)ps.stages.size();
    if (!fill_pass_maps(ps, p->dt, &d)) return fail(SV_ERR_UNSUPPORTED, "internal: pass write map is not a permutation");
    if (ps.kind == PASS_MATRIX)  // the matrix-pass kernel stores where it loaded
      for (int j = 0; j < ps.n_local; ++j)
        if (ps.wpos[j] != ps.lpos[j]) return fail(SV_ERR_UNSUPPORTED, "internal: matrix pass with a write map");
    for (const StageHost& sh : ps.stages) {
      PassStageDev sd{};
      // register bits of a tile stage, members of a matrix stage
      const int nq = ps.kind == PASS_MATRIX ? ps.mx_k : rb;
      uint32_t srt[kPassRegBitsMax];
      for (int r = 0; r < nq; ++r) sd.q[r] = srt[r] = sh.q[r];
      std::sort(srt, srt + nq);
      for (int r = 0; r < nq; ++r) sd.qsort[r] = srt[r];
      const uint32_t mbase = (uint32_t)pool.size();
      sd.form = sh.form;
      sd.slot_mask = sh.slot_mask;
      sd.nsub = sh.nsub;
      for (uint32_t k = 0; k < sh.nsub; ++k) {
        sd.sub[k] = sh.sub[k];
        sd.sub[k].slots += mbase;
        if (sd.sub[k].dr != kPassNoTable) sd.sub[k].dr += mbase;
      }
      sd.flags = sh.flags;
      sd.slots = mbase + sh.slots;
      sd.u2 = mbase + sh.u2;
      sd.dr = mbase + sh.dr;
      sd.mat_base = mbase;
      sd.rows = sh.rows;
      sd.row_count = sh.row_count;
      for (int l = 0; l < kPassLocalMax; ++l) sd.colimg[l] = sh.colimg[l];
      sd.pconst = sh.pconst;
      sd.item_first = (uint32_t)items.size();
      sd.item_count = (uint32_t)sh.items.size();
      for (PassItemDev it : sh.items) {
        it.mat += mbase;
        items.push_back(it);
      }
      sd.px_first = (uint32_t)items.size();
      sd.px_count = (uint32_t)sh.px.size();
      items.insert(items.end(), sh.px.begin(), sh.px.end());
      pool.insert(pool.end(), sh.mats.begin(), sh.mats.end());
      pool_raw.insert(pool_raw.end(), sh.raw.begin(), sh.raw.end());
      stages.push_back(sd);
    }
    out->desc_index[i] = (int)descs.size();
    out->pass_lp[i] = pass_has_ladders(ps) ? 1 : 0;
    out->max_m = std::max(out->max_m, ps.n_local);
    descs.push_back(d);
  }
  out->n_desc = (int)descs.size();
  if (!descs.empty()) {
    out->off_desc = put(descs.data(), descs.size() * sizeof(PassDescDev));
    out->off_stage = put(stages.data(), stages.size() * sizeof(PassStageDev));
    out->off_items = put(items.data(), items.size() * sizeof(PassItemDev));
    out->off_pool = put_cd(pool.data(), pool.size(), pool_raw.data());
  }
  align();
  return SV_OK;
}

sv_status execute_plan(sv_state* s, const sv_plan* p) {
  PackedPlan pk;
  if (sv_status st = pack_plan(p, &pk)) return st;
  void* dev = nullptr;
  if (!pk.host.empty()) {
    sv_status st = upload(s, pk.host.data(), pk.host.size(), &dev);
    if (st != SV_OK) return st;
  }
  unsigned char* db = (unsigned char*)dev;
  // complex64 states: FP64 renormalisation after every `renorm` dense ops
  const int renorm = s->dt == SV_C64 ? p->opts.renorm_interval : 0;
  int since = 0;
  for (size_t i = 0; i < p->passes.size(); ++i) {
    const Pass& ps = p->passes[i];
    if (ps.kind == PASS_SWEEP) {
      sv_status st = run_op_sweep(s, ps.phys, nullptr);
      if (st != SV_OK) return st;
    } else if (ps.kind == PASS_DENSE) {
      sv_status st = run_op_sweep(s, ps.phys, db + pk.dense_off[i], p->opts.fp32_mfma != 0);
      if (st != SV_OK) return st;
      if (renorm > 0 && ++since >= renorm) {
        if (sv_status r = renormalize(s)) return r;
        since = 0;
      }
    } else if (ps.kind == PASS_MATRIX) {
      SV_LAUNCH(launch_matrix_pass(s->dt, ps.mx_k, s->ptr, s->n, ps.n_local, (const PassDescDev*)(db + pk.off_desc),
                                   pk.desc_index[i], (int)ps.stages.size(), (const PassStageDev*)(db + pk.off_stage),
                                   db + pk.off_pool, s->stream),
                s->stream);
      if (renorm > 0 && (since += ps.n_ops) >= renorm) {
        if (sv_status r = renormalize(s)) return r;
        since = 0;
      }
    } else {
      SV_LAUNCH(launch_pass(s->dt, s->ptr, s->n, ps.n_local, (const PassDescDev*)(db + pk.off_desc),
                            pk.desc_index[i], (const PassStageDev*)(db + pk.off_stage),
                            (const PassItemDev*)(db + pk.off_items), db + pk.off_pool, pk.pass_lp[i] != 0,
                            s->stream),
                s->stream);
    }
  }
  if (renorm > 0 && since > 0) return renormalize(s);
  return SV_OK;
}

}  // namespace sv
