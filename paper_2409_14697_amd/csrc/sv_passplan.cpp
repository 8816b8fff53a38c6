// In-cache pass planner: groups ops into tile passes whose local qubits fit
// one LDS tile (QueenV2 Sec. III-A tier 4 "in-rank gate blocks", found
// greedily like Queen's findGB while considering control qubits), splits each
// pass into register stages, and keeps the bidirectional logical<->physical
// qubit map of Sec. III-A (qubit reordering, Sec. II-B): SWAP gates become
// relabelings, and the map is brought back to the identity by permutations
// fused into tile write-backs.  Host only.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sv_host.h"

namespace sv {

void write_pool(unsigned char* dst, const cd* m, const uint8_t* raw, size_t count, bool f32) {
  for (size_t e = 0; e < count; ++e) {
    if (raw && raw[e]) {
      uint64_t w[2];
      const double re = m[e].real(), im = m[e].imag();
      std::memcpy(&w[0], &re, sizeof re);
      std::memcpy(&w[1], &im, sizeof im);
      if (f32) {
        const uint32_t v[2] = {(uint32_t)w[0], (uint32_t)w[1]};
        std::memcpy(dst + 8 * e, v, 8);
      } else {
        std::memcpy(dst + 16 * e, w, 16);
      }
    } else if (f32) {
      const float v[2] = {(float)m[e].real(), (float)m[e].imag()};
      std::memcpy(dst + 8 * e, v, 8);
    } else {
      const double v[2] = {m[e].real(), m[e].imag()};
      std::memcpy(dst + 16 * e, v, 16);
    }
  }
}

bool fill_pass_maps(const Pass& ps, sv_dtype dt, PassDescDev* d) {
  d->lmask = 0;
  d->flags = kPassStoreLaneOrder;
  // local bits inside the lowest three 16-byte element bits (complex64
  // elements hold local bit 0 as well)
  const int low = dt == SV_C64 ? 4 : 3;
  for (int j = 0; j < ps.n_local; ++j) {
    d->lpos[j] = ps.lpos[j];
    d->wpos[j] = ps.wpos[j];
    d->lmask |= 1ull << ps.lpos[j];
    if (j < low && ps.wpos[j] != ps.lpos[j]) d->flags &= ~kPassStoreLaneOrder;
  }
  for (int k = 0; k < ps.n_local; ++k) {
    int found = -1, count = 0;
    for (int j = 0; j < ps.n_local; ++j)
      if (ps.wpos[j] == ps.lpos[k]) {
        found = j;
        ++count;
      }
    if (count != 1) return false;
    d->winv[k] = (uint32_t)found;
  }
  return true;
}

int default_lds_qubits(sv_dtype dt) { return dt == SV_C128 ? 12 : 13; }  // 64 KiB tiles
int default_pinned_bits(sv_dtype dt) { return dt == SV_C128 ? 3 : 4; }   // 128-byte runs

namespace {

bool is_diag(const Op& op) { return classify(op) == CLS_DIAG; }

// Qubits that must be local when the op runs inside a tile pass: none for a
// diagonal op (its phase depends only on bit values, which every amplitude
// knows from its index), the target for a CNOT (the control only selects),
// all of them otherwise.
int locality(const Op& op, int* q) {
  if (is_diag(op)) return 0;
  if (op.kind == SV_G_CNOT) {
    q[0] = op.q[1];
    return 1;
  }
  for (int i = 0; i < op.nq; ++i) q[i] = op.q[i];
  return op.nq;
}

Op to_physical(const Op& op, const std::vector<int>& phys) {
  Op r = op;
  for (int i = 0; i < op.nq; ++i) r.q[i] = phys[op.q[i]];
  return r;
}

// Arithmetic per amplitude of one op inside a pass (real flops).
double op_flops(const PassOpDev& od) {
  switch (od.type) {
    case POP_U1: return 16.0;
    case POP_U2: return 32.0;
    case POP_UR: case POP_UI: return 8.0;
    case POP_D1: case POP_D2: case POP_DG: return 6.0;
    case POP_P1: return od.lmask ? 8.0 : 3.0;  // a per-lane predicate costs register copies
    case POP_P2: return 1.5;
    case POP_X: return od.lmask ? 6.0 : 1.0;
    case POP_LP: return 14.0;
    case POP_DR: return 8.0;
    case POP_QG: return 12.0;
    default: return 1.0;
  }
}

bool all_real(const cd* m, int count) {
  for (int i = 0; i < count; ++i)
    if (m[i].imag() != 0.0) return false;
  return true;
}

// Real diagonal and imaginary off-diagonal (RX, Y).
bool real_diag_imag_offdiag(const cd* m) {
  return m[0].imag() == 0.0 && m[3].imag() == 0.0 && m[1].real() == 0.0 && m[2].real() == 0.0;
}

static_assert(kPassLPTileBits >= SV_MAX_QUBITS, "every physical qubit has a ladder word");

// Fewest two-qubit phase gates in a run worth fusing it into one phase
// function (its fixed cost is a few single phases).
constexpr int kPhaseRunMin = 3;

struct StageBuilder {
  const int* loc;  // physical bit -> local bit, or -1
  int m;
  int rb;          // register bits per stage
  std::vector<int> qs;   // register bits (local indices), in register order
  std::vector<Op> ops;   // physical qubits

  int reg(int physq) const {
    const int l = loc[physq];
    if (l < 0) return -1;
    for (size_t r = 0; r < qs.size(); ++r)
      if (qs[r] == l) return (int)r;
    return -1;
  }
  uint32_t src(int physq) const {
    const int l = loc[physq];
    return l >= 0 ? (uint32_t)l : kPassTileSel + (uint32_t)physq;
  }
  void predicate(PassOpDev* od, int physq) const {
    const int l = loc[physq];
    if (l >= 0) od->lmask |= 1u << l;
    else od->tmask |= 1ull << physq;
  }

  // A diagonal op on one or two qubits whose entries are unit phases: its
  // phase is c + h_a x_a (+ h_b x_b + J_ab x_a x_b) over the bits x of its
  // qubits, exact in fixed-point turns.
  bool phase_op(const Op& op) const {
    if (!is_diag(op) || op.nq > 2) return false;
    const int d = 1 << op.nq;
    for (int i = 0; i < d; ++i)
      if (std::abs(std::abs(op.m[(size_t)i * d + i]) - 1.0) >= 1e-14) return false;
    return true;
  }

  // Angle of a unit phase as a W-bit fixed-point turn (W = 32 for
  // complex64, 64 for complex128), held in the low W bits.
  uint64_t turns(const cd& e) const {
    double t = std::arg(e) / (2.0 * M_PI);
    t -= std::floor(t);
    if (rb == pass_reg_bits(SV_C64)) return (uint64_t)(uint32_t)(uint64_t)std::llround(std::ldexp(t, 32));
    return (uint64_t)std::ldexp(t, 63) * 2u;
  }

  // The unit phase of a W-bit fixed-point turn.
  cd phase_of(uint64_t w) const {
    const bool f32 = rb == pass_reg_bits(SV_C64);
    const double t = f32 ? (double)(int32_t)(uint32_t)w * 0x1p-32 : (double)(int64_t)w * 0x1p-64;
    return std::polar(1.0, 2.0 * M_PI * t);
  }

  // A diagonal op whose qubits are all register bits (a factor per register
  // index).
  bool reg_diag(const Op& op) const {
    if (!is_diag(op)) return false;
    for (int i = 0; i < op.nq; ++i)
      if (reg(op.q[i]) < 0) return false;
    return true;
  }

  // One POP_DR op: the product of the register-diagonal ops `run`.
  void encode_reg_diag(StageHost* sh, const std::vector<const Op*>& run) {
    const int nr = 1 << rb;
    std::vector<cd> d(nr, cd(1.0, 0.0));
    for (const Op* op : run) {
      const int dim = 1 << op->nq;
      for (int r = 0; r < nr; ++r) {
        int idx = 0;  // the op's local index: q[0] is its most significant bit
        for (int i = 0; i < op->nq; ++i) idx = (idx << 1) | ((r >> reg(op->q[i])) & 1);
        d[r] *= op->m[(size_t)idx * dim + idx];
      }
    }
    PassOpDev od{};
    od.type = POP_DR;
    od.sa = od.sb = kPassNoSel;
    od.mat = (uint32_t)sh->mats.size();
    sh->mats.insert(sh->mats.end(), d.begin(), d.end());
    sh->raw.insert(sh->raw.end(), d.size(), 0);
    sh->ops.push_back(od);
  }

  // Append `words` (kPassLPWords per row) to the pool, two per entry.
  static void put_words(StageHost* sh, const std::vector<uint64_t>& words) {
    for (size_t w = 0; w < words.size(); w += 2) {
      double re, im;
      std::memcpy(&re, &words[w], sizeof re);
      std::memcpy(&im, &words[w + 1], sizeof im);
      sh->mats.push_back(cd(re, im));
      sh->raw.push_back(1);
    }
  }

  // Ops [first, last): a run of phase ops (they commute), fused into one
  // quadratic phase over the bits of their qubits,
  //   theta(x) = c + sum_a h_a x_a + sum_{a<b} J_ab x_a x_b   (turns mod 1),
  // summed exactly in W-bit fixed point (the words of every gate's entries
  // are rounded once).  It is applied as at most three kinds of op:
  //   * a POP_LP ladder per register bit a with pair terms to bits outside
  //     the registers (its constant is h_a);
  //   * one POP_DR factor per register index for the terms over register
  //     bits only (and the constant when no POP_QG follows);
  //   * one POP_QG for the terms over the other bits (the lane's group bits
  //     and the tile bits).
  void encode_phase_run(StageHost* sh, size_t first, size_t last) {
    const bool f32 = rb == pass_reg_bits(SV_C64);
    const uint64_t wmask = f32 ? 0xffffffffull : ~0ull;
    constexpr int NQ = SV_MAX_QUBITS;
    uint64_t c = 0;
    std::vector<uint64_t> h(NQ, 0), J((size_t)NQ * NQ, 0);  // J[a * NQ + b], a < b
    std::vector<char> used(NQ, 0);
    for (size_t i = first; i < last; ++i) {
      const Op& op = ops[i];
      const int a = op.q[0];
      used[a] = 1;
      if (op.nq == 1) {
        const uint64_t t0 = turns(op.m[0]), t1 = turns(op.m[3]);
        c += t0;
        h[a] += t1 - t0;
        continue;
      }
      const int b = op.q[1];  // entry index (bit a) * 2 + (bit b)
      used[b] = 1;
      const uint64_t t00 = turns(op.m[0]), t01 = turns(op.m[5]), t10 = turns(op.m[10]), t11 = turns(op.m[15]);
      c += t00;
      h[a] += t10 - t00;
      h[b] += t01 - t00;
      J[(size_t)std::min(a, b) * NQ + std::max(a, b)] += t11 - t10 - t01 + t00;
    }
    c &= wmask;
    for (auto& w : h) w &= wmask;
    for (auto& w : J) w &= wmask;
    auto pair = [&](int a, int b) { return J[(size_t)std::min(a, b) * NQ + std::max(a, b)]; };
    // word index of a source bit outside the registers (ladder layout)
    auto word_of = [&](int q) { return loc[q] >= 0 ? loc[q] : kPassLPLocalBits + q; };
    std::vector<int> regq, other;  // qubits in / outside the registers
    for (int q = 0; q < NQ; ++q)
      if (used[q]) (reg(q) >= 0 ? regq : other).push_back(q);
    // order of the bits outside the registers: local (ascending local bit),
    // then tile (ascending physical bit); a pair term lives in the row of
    // the earlier bit
    std::sort(other.begin(), other.end(), [&](int x, int y) {
      const bool lx = loc[x] >= 0, ly = loc[y] >= 0;
      if (lx != ly) return lx;
      return lx ? loc[x] < loc[y] : x < y;
    });

    // ladders
    std::vector<char> in_ladder(NQ, 0);
    for (int a : regq) {
      std::vector<uint64_t> words(kPassLPWords, 0);
      PassOpDev od{};
      od.type = POP_LP;
      od.b0 = (uint32_t)reg(a);
      od.sa = od.sb = kPassNoSel;
      for (int b : other) {
        const uint64_t w = pair(a, b);
        if (!w) continue;
        words[word_of(b)] = w;
        if (loc[b] >= 0) od.lmask |= 1u << loc[b];
        else od.tmask |= 1ull << b;
      }
      if (!od.lmask && !od.tmask) continue;
      words[kPassLPConst] = h[a];
      in_ladder[a] = 1;
      od.mat = (uint32_t)sh->mats.size();
      put_words(sh, words);
      sh->ops.push_back(od);
    }

    // quadratic phase outside the registers
    std::vector<uint64_t> qw(kPassLPWords, 0);
    PassOpDev qg{};
    qg.type = POP_QG;
    qg.sa = qg.sb = kPassNoSel;
    bool any = false;
    auto mark = [&](PassOpDev& od, int q) {
      if (loc[q] >= 0) od.lmask |= 1u << loc[q];
      else od.tmask |= 1ull << q;
    };
    for (int a : other)
      if (h[a]) {
        qw[word_of(a)] = h[a];
        mark(qg, a);
        any = true;
      }
    uint64_t tile_targets = 0;
    for (size_t i = 0; i < other.size(); ++i) {
      const int a = other[i];
      std::vector<uint64_t> row(kPassLPWords, 0);
      bool nz = false;
      for (size_t k = i + 1; k < other.size(); ++k) {
        const int b = other[k];
        const uint64_t w = pair(a, b);
        if (!w) continue;
        row[word_of(b)] = w;
        mark(qg, b);
        nz = true;
      }
      if (!nz) continue;
      mark(qg, a);
      if (loc[a] >= 0) qg.b0 |= 1u << loc[a];
      else tile_targets |= 1ull << a;
      qw.insert(qw.end(), row.begin(), row.end());
      any = true;
    }
    qg.b1 = (uint32_t)tile_targets;
    qg.pad = (uint32_t)(tile_targets >> 32);
    if (any) {
      qw[kPassLPConst] = c;
      c = 0;
    }

    // register factors (and the constant when there is no POP_QG)
    const int nr = 1 << rb;
    std::vector<uint64_t> dw(nr, c);
    bool diag = c != 0;
    for (size_t i = 0; i < regq.size(); ++i) {
      const int a = regq[i], ra = reg(a);
      if (!in_ladder[a] && h[a]) {
        diag = true;
        for (int r = 0; r < nr; ++r)
          if ((r >> ra) & 1) dw[r] += h[a];
      }
      for (size_t k = i + 1; k < regq.size(); ++k) {
        const int b = regq[k], rbit = reg(b);
        const uint64_t w = pair(a, b);
        if (!w) continue;
        diag = true;
        for (int r = 0; r < nr; ++r)
          if (((r >> ra) & 1) && ((r >> rbit) & 1)) dw[r] += w;
      }
    }
    if (diag) {
      PassOpDev od{};
      od.type = POP_DR;
      od.sa = od.sb = kPassNoSel;
      od.mat = (uint32_t)sh->mats.size();
      for (int r = 0; r < nr; ++r) sh->mats.push_back(phase_of(dw[r] & wmask));
      sh->raw.insert(sh->raw.end(), nr, 0);
      sh->ops.push_back(od);
    }
    if (any) {
      qg.mat = (uint32_t)sh->mats.size();
      put_words(sh, qw);
      sh->ops.push_back(qg);
    }
  }

  static uint64_t qubit_mask(const Op& op) {
    uint64_t mk = 0;
    for (int i = 0; i < op.nq; ++i) mk |= 1ull << op.q[i];
    return mk;
  }

  // Gate reordering for diagonal visibility (Sec. III-A): every phase op
  // joins the phase ops before it when it commutes with the ops it moves
  // past, i.e. shares no qubit with any of them that is not a phase op
  // (phase ops commute with each other).  Program order is kept otherwise.
  void gather_phases() {
    std::vector<Op> out;
    out.reserve(ops.size());
    std::vector<char> taken(ops.size(), 0);
    for (size_t i = 0; i < ops.size(); ++i) {
      if (taken[i]) continue;
      out.push_back(ops[i]);
      taken[i] = 1;
      if (!phase_op(ops[i])) continue;
      uint64_t blocked = 0;  // qubits of the non-phase ops left in place so far
      for (size_t j = i + 1; j < ops.size(); ++j) {
        if (taken[j]) continue;
        const uint64_t mk = qubit_mask(ops[j]);
        if (!phase_op(ops[j])) {
          blocked |= mk;
        } else if (!(mk & blocked)) {
          out.push_back(ops[j]);
          taken[j] = 1;
        }
      }
    }
    ops.swap(out);
  }

  void encode(StageHost* sh) {
    // pad the register bits with the lowest unused local bits
    for (int l = 0; (int)qs.size() < rb && l < m; ++l)
      if (std::find(qs.begin(), qs.end(), l) == qs.end()) qs.push_back(l);
    for (int r = 0; r < rb; ++r) sh->q[r] = (uint32_t)qs[r];
    gather_phases();
    for (size_t i = 0; i < ops.size();) {
      // a run of phase gates with pair terms becomes one fixed-point
      // quadratic phase (single-qubit phases alone stay per-op: their own
      // ops are cheaper than a per-lane phase function)
      size_t e = i, pairs = 0;
      while (e < ops.size() && phase_op(ops[e])) pairs += ops[e++].nq == 2;
      if (pairs >= (size_t)kPhaseRunMin) {
        const size_t n_ops = sh->ops.size(), n_mats = sh->mats.size();
        encode_phase_run(sh, i, e);
        if (stage_rows(*sh) > (uint32_t)kPassStageRowsMax) {  // over the stage's row table: gate by gate
          sh->ops.resize(n_ops);
          sh->mats.resize(n_mats);
          sh->raw.resize(n_mats);
          for (size_t x = i; x < e; ++x) encode_op(sh, ops[x]);
        }
        i = e;
        continue;
      }
      // a run of diagonal gates on register bits becomes one factor per
      // register index
      size_t f = i;
      while (f < ops.size() && reg_diag(ops[f])) ++f;
      if (f - i >= 2) {
        std::vector<const Op*> run;
        for (size_t x = i; x < f; ++x) run.push_back(&ops[x]);
        encode_reg_diag(sh, run);
        i = f;
        continue;
      }
      encode_op(sh, ops[i]);
      ++i;
    }
    encode_rows(sh);
  }

  // Tile-summed rows of a phase op (the row table of PassStageDev).
  static uint32_t op_rows(const PassOpDev& od) {
    if (od.type == POP_LP) return 1;
    if (od.type == POP_QG)
      return 1u + (uint32_t)__builtin_popcount(od.b0) + (uint32_t)__builtin_popcountll(qg_tile_targets(od));
    return 0;
  }
  static uint64_t qg_tile_targets(const PassOpDev& od) { return ((uint64_t)od.pad << 32) | od.b1; }
  static uint32_t stage_rows(const StageHost& sh) {
    uint32_t r = 0;
    for (const PassOpDev& od : sh.ops) r += op_rows(od);
    return r;
  }

  // Four uint32 in pool words (two entries for complex64, one for complex128).
  void put_u32x4(StageHost* sh, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    auto entry = [&](uint64_t w0, uint64_t w1) {
      double re, im;
      std::memcpy(&re, &w0, sizeof re);
      std::memcpy(&im, &w1, sizeof im);
      sh->mats.push_back(cd(re, im));
      sh->raw.push_back(1);
    };
    if (rb == pass_reg_bits(SV_C64)) {
      entry(a, b);
      entry(c, d);
    } else {
      entry(a | (uint64_t)b << 32, c | (uint64_t)d << 32);
    }
  }

  // The stage's row table: per row, the word index of its tile words, the
  // tile bit that gates it (tile-target rows) and the tile mask.
  void encode_rows(StageHost* sh) {
    sh->rows = (uint32_t)sh->mats.size();
    sh->row_count = 0;
    const std::vector<PassOpDev> ops_now = sh->ops;
    for (const PassOpDev& od : ops_now) {
      const uint32_t nr = op_rows(od);
      const uint32_t nl = od.type == POP_QG ? (uint32_t)__builtin_popcount(od.b0) : 0u;
      uint64_t tt = od.type == POP_QG ? qg_tile_targets(od) : 0;
      for (uint32_t k = 0; k < nr; ++k) {
        uint32_t pred = kPassNoSel;
        if (k > nl) {
          pred = (uint32_t)__builtin_ctzll(tt);
          tt &= tt - 1;
        }
        put_u32x4(sh, 2u * od.mat + k * (uint32_t)kPassLPWords + (uint32_t)kPassLPLocalBits, pred,
                  (uint32_t)od.tmask, (uint32_t)(od.tmask >> 32));
        ++sh->row_count;
      }
    }
    if (!sh->row_count) sh->rows = 0;
  }

  void encode_op(StageHost* sh, const Op& op) {
    {
      PassOpDev od{};
      od.sa = od.sb = kPassNoSel;
      od.mat = (uint32_t)sh->mats.size();
      std::vector<cd> mv;
      const bool diag = is_diag(op);
      if (op.nq == 1) {
        const int q = op.q[0], b = reg(q);
        if (diag) {
          const cd d0 = op.m[0], d1 = op.m[3];
          if (b >= 0 && d0 == cd(1.0, 0.0)) {
            od.type = POP_P1;
            od.b0 = (uint32_t)b;
            mv = {d1};
          } else if (b >= 0) {
            od.type = POP_D1;
            od.b0 = (uint32_t)b;
            mv = {d0, d1};
          } else if (d0 == cd(1.0, 0.0)) {
            od.type = POP_DG;
            predicate(&od, q);
            mv = {d1};
          } else {
            od.type = POP_DG;
            od.sa = src(q);
            mv = {d0, d1};
          }
        } else if (op.kind == SV_G_X) {
          od.type = POP_X;
          od.b0 = (uint32_t)b;
        } else {
          od.type = all_real(op.m.data(), 4) ? POP_UR : real_diag_imag_offdiag(op.m.data()) ? POP_UI : POP_U1;
          od.b0 = (uint32_t)b;
          mv.assign(op.m.begin(), op.m.begin() + 4);
        }
      } else if (op.kind == SV_G_CNOT) {
        const int c = op.q[0], t = op.q[1];
        const int bt = reg(t), bc = reg(c);
        if (bc >= 0) {
          od.type = POP_CX;
          od.b0 = (uint32_t)bc;
          od.b1 = (uint32_t)bt;
        } else {
          od.type = POP_X;
          od.b0 = (uint32_t)bt;
          predicate(&od, c);
        }
      } else if (diag) {
        const cd d[4] = {op.m[0], op.m[5], op.m[10], op.m[15]};
        const int q0 = op.q[0], q1 = op.q[1];
        const int r0 = reg(q0), r1 = reg(q1);
        const cd one(1.0, 0.0);
        const bool cz_like = d[0] == one && d[1] == one && d[2] == one;
        if (r0 >= 0 && r1 >= 0 && cz_like) {
          od.type = POP_P2;
          od.b0 = (uint32_t)r0;
          od.b1 = (uint32_t)r1;
          mv = {d[3]};
        } else if (r0 >= 0 && r1 >= 0) {
          od.type = POP_D2;
          od.b0 = (uint32_t)r0;
          od.b1 = (uint32_t)r1;
          mv = {d[0], d[1], d[2], d[3]};
        } else if (r0 >= 0 || r1 >= 0) {
          // one qubit in registers (bit b of the register index), the other
          // (o) selects: entries by (bit of o, bit b)
          const bool first = r0 >= 0;
          const int b = first ? r0 : r1, o = first ? q1 : q0;
          const cd e00 = first ? d[0] : d[0], e01 = first ? d[2] : d[1];  // o = 0: b = 0, 1
          const cd e10 = first ? d[1] : d[2], e11 = first ? d[3] : d[3];  // o = 1: b = 0, 1
          od.b0 = (uint32_t)b;
          if (cz_like) {
            od.type = POP_P1;
            predicate(&od, o);
            mv = {d[3]};
          } else if (e00 == one && e10 == one) {
            od.type = POP_P1;  // only the b = 1 half changes
            od.sa = src(o);
            mv = {e01, e11};
          } else {
            od.type = POP_D1;
            od.sa = src(o);
            mv = {e00, e01, e10, e11};
          }
        } else {
          od.type = POP_DG;
          if (cz_like) {
            predicate(&od, q0);
            predicate(&od, q1);
            mv = {d[3]};
          } else {
            od.sa = src(q0);
            od.sb = src(q1);
            mv = {d[0], d[1], d[2], d[3]};
          }
        }
      } else {
        od.type = POP_U2;
        od.b0 = (uint32_t)reg(op.q[0]);
        od.b1 = (uint32_t)reg(op.q[1]);
        mv.assign(op.m.begin(), op.m.begin() + 16);
      }
      sh->mats.insert(sh->mats.end(), mv.begin(), mv.end());
      sh->raw.insert(sh->raw.end(), mv.size(), 0);
      sh->ops.push_back(od);
    }
  }
};

// Split the ops of one pass (physical qubits, program order) into stages of at
// most rb register bits.
std::vector<StageHost> build_stages(const std::vector<Op>& ops, const int* loc, int m, int rb) {
  std::vector<StageHost> out;
  StageBuilder sb{loc, m, rb, {}, {}};
  for (const Op& op : ops) {
    int q[SV_MAX_GATE_QUBITS];
    const int k = locality(op, q);
    std::vector<int> need;
    for (int i = 0; i < k; ++i) {
      const int l = loc[q[i]];
      if (std::find(sb.qs.begin(), sb.qs.end(), l) == sb.qs.end() &&
          std::find(need.begin(), need.end(), l) == need.end())
        need.push_back(l);
    }
    if (sb.qs.size() + need.size() > (size_t)rb) {
      StageHost sh;
      sb.encode(&sh);
      out.push_back(std::move(sh));
      sb.qs.clear();
      sb.ops.clear();
      need.clear();
      for (int i = 0; i < k; ++i)
        if (std::find(need.begin(), need.end(), loc[q[i]]) == need.end()) need.push_back(loc[q[i]]);
    }
    sb.qs.insert(sb.qs.end(), need.begin(), need.end());
    sb.ops.push_back(op);
  }
  if (!sb.ops.empty()) {
    StageHost sh;
    sb.encode(&sh);
    out.push_back(std::move(sh));
  }
  return out;
}

struct QubitMap {
  std::vector<int> phys, logi;  // logical -> physical, physical -> logical
  explicit QubitMap(int n) : phys(n), logi(n) {
    for (int i = 0; i < n; ++i) phys[i] = logi[i] = i;
  }
  void relabel_swap(int a, int b) {
    std::swap(phys[a], phys[b]);
    logi[phys[a]] = a;
    logi[phys[b]] = b;
  }
  bool identity() const {
    for (size_t i = 0; i < phys.size(); ++i)
      if (phys[i] != (int)i) return false;
    return true;
  }
};

// Fill a tile's local set up to m bits, lowest unused positions first (longest
// contiguous runs), after the bits in `prefer`.
void fill_local(std::vector<char>& in, int& count, int m, int n, const std::vector<int>& prefer) {
  for (int b : prefer)
    if (count < m && !in[b]) {
      in[b] = 1;
      ++count;
    }
  for (int b = 0; b < n && count < m; ++b)
    if (!in[b]) {
      in[b] = 1;
      ++count;
    }
}

// Cycles of the misplaced physical positions: data at x belongs at logi[x].
std::vector<std::vector<int>> cycles_of(const QubitMap& mp) {
  const int n = (int)mp.logi.size();
  std::vector<char> seen(n, 0);
  std::vector<std::vector<int>> cyc;
  for (int x = 0; x < n; ++x) {
    if (seen[x] || mp.logi[x] == x) continue;
    std::vector<int> c;
    for (int y = x; !seen[y]; y = mp.logi[y]) {
      seen[y] = 1;
      c.push_back(y);
    }
    cyc.push_back(c);
  }
  return cyc;
}

}  // namespace

sv_status plan_tile_passes(const std::vector<Op>& ops, int n, sv_dtype dt, const sv_opts& o, sv_plan* p) {
  int m = o.lds_qubits ? o.lds_qubits : default_lds_qubits(dt);
  // 64 KiB tiles: two blocks per CU, and 16 elements of 16 bytes per lane
  const int m_max = dt == SV_C128 ? 12 : 13;
  if (m > m_max) return fail(SV_ERR_ARG, "lds_qubits %d exceeds %d for this dtype", m, m_max);
  if (m > n) m = n;
  const int rb = pass_reg_bits(dt);
  if (m < rb) return fail(SV_ERR_ARG, "tile of %d qubits is too small for %d register bits", m, rb);
  int pin = o.pinned_low_bits ? o.pinned_low_bits : default_pinned_bits(dt);
  pin = std::min(pin, m - 2);
  const bool reorder = o.reorder != 0;
  // Cost of a tile pass in full-state sweeps (measured on MI355X at N=30):
  // the data movement alone takes ~1.2 sweeps and hides ~0.3 sweeps of
  // arithmetic; beyond that the stages and ops add up.  flop_scale: op flops
  // per amplitude that take one sweep's time; stage_cost: one LDS round trip.
  const double flop_scale = dt == SV_C128 ? 180.0 : 100.0;
  const double stage_cost = 0.08;
  const double pass_base = 1.2, hidden = 0.3;

  p->ops.clear();
  p->op_pass.clear();
  p->passes.clear();
  p->est_cost = 0.0;
  QubitMap mp(n);
  std::vector<char> done(ops.size(), 0);
  size_t first = 0;
  auto emit_op = [&](const Op& op, int pass) {
    p->ops.push_back(op);
    p->op_pass.push_back(pass);
  };

  while (true) {
    while (first < ops.size() && done[first]) ++first;
    if (first == ops.size()) break;
    const Op& head = ops[first];
    if (reorder && head.kind == SV_G_SWAP) {  // relabel: no data moves
      mp.relabel_swap(head.q[0], head.q[1]);
      emit_op(head, -1);
      done[first] = 1;
      continue;
    }
    if (head.nq >= 3) {  // dense op: its own sweep
      Pass ps;
      ps.kind = PASS_DENSE;
      ps.first_op = (int)p->ops.size();
      ps.n_ops = 1;
      ps.phys = to_physical(head, mp.phys);
      emit_op(head, (int)p->passes.size());
      p->est_cost += op_sweep_cost(head, dt, dt == SV_C64 && o.fp32_mfma);
      p->passes.push_back(std::move(ps));
      done[first] = 1;
      continue;
    }
    // ---- one tile pass: gate-block search over the remaining ops
    std::vector<char> in_l(n, 0), blocked(n, 0);
    int count = 0;
    for (int b = 0; b < pin; ++b) {
      in_l[b] = 1;
      ++count;
    }
    int n_blocked = 0;
    std::vector<Op> members;  // physical qubits
    const int pass_id = (int)p->passes.size();
    const int first_op = (int)p->ops.size();
    const size_t cap = o.max_pass_ops > 0 ? (size_t)o.max_pass_ops : ops.size();
    for (size_t j = first; j < ops.size() && n_blocked < n && members.size() < cap; ++j) {
      if (done[j]) continue;
      const Op& op = ops[j];
      bool blk = op.nq >= 3;
      for (int i = 0; i < op.nq; ++i) blk = blk || blocked[op.q[i]];
      if (!blk && reorder && op.kind == SV_G_SWAP) {
        mp.relabel_swap(op.q[0], op.q[1]);
        emit_op(op, -1);
        done[j] = 1;
        continue;
      }
      if (!blk) {
        int q[SV_MAX_GATE_QUBITS];
        const int k = locality(op, q);
        int extra = 0;
        for (int i = 0; i < k; ++i) extra += in_l[mp.phys[q[i]]] ? 0 : 1;
        if (count + extra <= m) {
          for (int i = 0; i < k; ++i)
            if (!in_l[mp.phys[q[i]]]) {
              in_l[mp.phys[q[i]]] = 1;
              ++count;
            }
          members.push_back(to_physical(op, mp.phys));
          emit_op(op, pass_id);
          done[j] = 1;
          continue;
        }
      }
      // deferred: every later op on these qubits must wait too
      for (int i = 0; i < op.nq; ++i)
        if (!blocked[op.q[i]]) {
          blocked[op.q[i]] = 1;
          ++n_blocked;
        }
    }
    bool last = true;
    for (size_t j = first; j < ops.size(); ++j) last = last && done[j];
    // the last pass also takes the bits whose data must move back home
    std::vector<int> prefer;
    if (last && !mp.identity()) {
      int room = m - count;
      for (const auto& c : cycles_of(mp)) {
        int extra = 0;
        for (int x : c) extra += in_l[x] ? 0 : 1;
        if (extra > room) continue;
        room -= extra;
        prefer.insert(prefer.end(), c.begin(), c.end());
      }
    }
    fill_local(in_l, count, m, n, prefer);
    Pass ps;
    ps.kind = PASS_TILE;
    ps.first_op = first_op;
    ps.n_ops = (int)members.size();
    ps.n_local = m;
    int loc[64];
    for (int b = 0; b < 64; ++b) loc[b] = -1;
    int j = 0;
    for (int b = 0; b < n; ++b)
      if (in_l[b]) {
        ps.lpos[j] = ps.wpos[j] = (uint32_t)b;
        loc[b] = j++;
      }
    ps.stages = build_stages(members, loc, m, rb);
    // write-back: complete cycles of the map that lie inside the tile go home
    if (last && !mp.identity()) {
      for (const auto& c : cycles_of(mp)) {
        bool inside = true;
        for (int x : c) inside = inside && in_l[x];
        if (!inside) continue;
        for (int x : c) ps.wpos[loc[x]] = (uint32_t)mp.logi[x];
      }
      QubitMap nm = mp;
      for (int jj = 0; jj < m; ++jj) {
        const int l = mp.logi[ps.lpos[jj]];
        nm.phys[l] = (int)ps.wpos[jj];
        nm.logi[ps.wpos[jj]] = l;
      }
      mp = nm;
    }
    double alu = stage_cost * (double)ps.stages.size();
    for (const StageHost& sh : ps.stages)
      for (const PassOpDev& od : sh.ops) alu += op_flops(od) / flop_scale;
    p->est_cost += pass_base + std::max(0.0, alu - hidden);
    p->passes.push_back(std::move(ps));
  }

  // ---- restore the logical order: permutation-only passes
  while (!mp.identity()) {
    std::vector<char> in_l(n, 0);
    int count = 0;
    for (int b = 0; b < pin; ++b) {
      in_l[b] = 1;
      ++count;
    }
    Pass ps;
    ps.kind = PASS_PERMUTE;
    ps.first_op = (int)p->ops.size();
    ps.n_ops = 0;
    ps.n_local = m;
    // choose cycles (or a segment of one) that fit
    std::vector<std::pair<int, int>> moves;  // (from, to)
    for (const auto& c : cycles_of(mp)) {
      int extra = 0;
      for (int x : c) extra += in_l[x] ? 0 : 1;
      if (count + extra <= m) {
        for (int x : c) {
          if (!in_l[x]) {
            in_l[x] = 1;
            ++count;
          }
          moves.push_back({x, mp.logi[x]});
        }
      } else if (moves.empty()) {
        // segment x1..xc of a long cycle: x_i -> x_{i+1}, x_c -> x1
        std::vector<int> seg;
        for (int x : c) {
          const int add = in_l[x] ? 0 : 1;
          if (count + add > m) break;
          if (add) {
            in_l[x] = 1;
            ++count;
          }
          seg.push_back(x);
        }
        if (seg.size() < 2) return fail(SV_ERR_UNSUPPORTED, "tile too small to restore the qubit order");
        for (size_t i = 0; i + 1 < seg.size(); ++i) moves.push_back({seg[i], seg[i + 1]});
        moves.push_back({seg.back(), seg[0]});
        break;
      }
    }
    fill_local(in_l, count, m, n, {});
    int loc[64];
    for (int b = 0; b < 64; ++b) loc[b] = -1;
    int j = 0;
    for (int b = 0; b < n; ++b)
      if (in_l[b]) {
        ps.lpos[j] = ps.wpos[j] = (uint32_t)b;
        loc[b] = j++;
      }
    for (const auto& mv : moves) ps.wpos[loc[mv.first]] = (uint32_t)mv.second;
    QubitMap nm = mp;
    for (int jj = 0; jj < m; ++jj) {
      const int l = mp.logi[ps.lpos[jj]];
      nm.phys[l] = (int)ps.wpos[jj];
      nm.logi[ps.wpos[jj]] = l;
    }
    mp = nm;
    p->est_cost += pass_base;
    p->passes.push_back(std::move(ps));
  }
  // the pass kernels move complex64 amplitudes in pairs on physical bit 0,
  // which the pinned low bits keep local as local bit 0
  for (const Pass& ps : p->passes)
    if ((ps.kind == PASS_TILE || ps.kind == PASS_PERMUTE) && ps.lpos[0] != 0)
      return fail(SV_ERR_UNSUPPORTED, "internal: a tile pass without physical bit 0 local");
  return SV_OK;
}

}  // namespace sv
