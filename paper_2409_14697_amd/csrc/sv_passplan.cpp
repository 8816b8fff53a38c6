// In-cache pass planner: groups ops into tile passes whose local qubits fit
// one LDS tile (QueenV2 Sec. III-A tier 4 "in-rank gate blocks", found
// greedily like Queen's findGB while considering control qubits), splits each
// pass into register stages, and keeps the bidirectional logical<->physical
// qubit map of Sec. III-A (qubit reordering, Sec. II-B): SWAP gates become
// relabelings, and the map is brought back to the identity by permutations
// fused into tile write-backs.  Host only.
#include <algorithm>
#include <array>
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

typedef std::array<cd, 4> M2;

const M2 kIdentity2 = {cd(1.0, 0.0), cd(0.0, 0.0), cd(0.0, 0.0), cd(1.0, 0.0)};

// a * b (2x2, row-major)
M2 mul2(const M2& a, const M2& b) {
  return {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3], a[2] * b[0] + a[3] * b[2],
          a[2] * b[1] + a[3] * b[3]};
}

// The cheapest 2x2 form that holds m exactly.
uint32_t form_of(const M2& m) {
  const bool real_diag = m[0].imag() == 0.0 && m[3].imag() == 0.0;
  if (real_diag && m[1].imag() == 0.0 && m[2].imag() == 0.0) return PFORM_UR;
  if (real_diag && m[1].real() == 0.0 && m[2].real() == 0.0) return PFORM_UI;
  if (real_diag) return PFORM_RC;
  return PFORM_U;
}

// VALU instructions per amplitude of a 2x2 in each form (the kernel applies
// one 2x2 per register bit).
double form_ops(uint32_t f) {
  switch (f) {
    case PFORM_UR: case PFORM_UI: return 4.0;
    case PFORM_RC: return 6.0;
    case PFORM_U: return 8.0;
    default: return 0.0;
  }
}

static_assert(kPassLPTileBits >= SV_MAX_QUBITS, "every physical qubit has a ladder word");

// Fewest two-qubit phase gates among a stage's diagonal gates worth fusing
// them into one fixed-point phase function (its fixed cost is a few
// per-lane factors).
constexpr int kPhaseRunMin = 3;

uint64_t qubit_mask(const Op& op) {
  uint64_t mk = 0;
  for (int i = 0; i < op.nq; ++i) mk |= 1ull << op.q[i];
  return mk;
}

// Builds the register stages of one tile pass from its ops (program order,
// physical qubits).  A stage applies, in this order, an optional 4x4 on
// register bits (1, 0), one 2x2 per register bit, a diagonal and a register
// permutation (see PassStageDev).  Each gate joins the current stage when it
// may move to its part of that order: a single-qubit gate when no diagonal
// or permutation gate of the stage involves its qubit, a diagonal gate when
// the permutation leaves its register bits unchanged, a permutation gate
// always (it is the latest); otherwise the stage is closed and a new one
// starts.  A stage is also closed when its register bits are all taken.
struct LayerBuilder {
  const int* loc;  // physical bit -> local bit, or -1
  int m;
  int rb;          // register bits per stage
  sv_dtype dt;
  std::vector<StageHost>* out;

  // the stage being built
  std::vector<int> qs;  // local bit of each register bit, in register order
  bool has_u2 = false;
  std::vector<cd> u2m;
  M2 slot[kPassRegBitsMax];
  bool slot_on[kPassRegBitsMax] = {};
  std::vector<Op> diag;  // diagonal gates (physical qubits), program order
  uint64_t diag_q = 0;   // physical qubits of the diagonal gates
  // the stage's store map of the local index, x -> M x ^ cl ^ (tile terms)
  // over GF(2): the X, CNOT and SWAP gates of the stage
  uint32_t Mc[kPassLocalMax];  // column images (local masks)
  uint32_t cl = 0;
  std::vector<std::pair<uint32_t, uint32_t>> tterms;  // (tile selector code, local mask)
  int n_perm = 0;          // permutation gates composed
  int n_members = 0;
  // earlier layers of the stage: their 2x2s and the diagonal gates (all on
  // register bits) that follow them
  struct SubLayer {
    M2 slot[kPassRegBitsMax];
    bool on[kPassRegBitsMax];
    std::vector<Op> diag;
  };
  std::vector<SubLayer> subs;

  bool f32() const { return dt == SV_C64; }

  void reset() {
    qs.clear();
    has_u2 = false;
    u2m.clear();
    for (int r = 0; r < kPassRegBitsMax; ++r) {
      slot[r] = kIdentity2;
      slot_on[r] = false;
    }
    for (int l = 0; l < kPassLocalMax; ++l) Mc[l] = 1u << l;
    diag.clear();
    diag_q = 0;
    cl = 0;
    tterms.clear();
    n_perm = 0;
    n_members = 0;
    subs.clear();
  }

  int reg(int physq) const {
    const int l = loc[physq];
    if (l < 0) return -1;
    for (size_t r = 0; r < qs.size(); ++r)
      if (qs[r] == l) return (int)r;
    return -1;
  }
  // selector code of a bit outside the registers
  uint32_t src(int physq) const {
    const int l = loc[physq];
    return l >= 0 ? (uint32_t)l : kPassTileSel + (uint32_t)physq;
  }

  // local bits whose value the store map may change
  uint32_t unstable() const {
    uint32_t un = cl;
    for (const auto& t : tterms) un |= t.second;
    for (int l = 0; l < m; ++l) un |= Mc[l] & ~(1u << l);  // bits that receive another bit
    for (int l = 0; l < m; ++l)
      if (!((Mc[l] >> l) & 1u)) un |= 1u << l;
    return un;
  }
  // local bits the store map involves (their value changes or is read)
  uint32_t moved() const {
    uint32_t mv = unstable();
    for (int l = 0; l < m; ++l)
      if (Mc[l] != (1u << l)) mv |= 1u << l;
    return mv;
  }
  bool local_moved(int physq) const {
    const int l = loc[physq];
    return l >= 0 && ((moved() >> l) & 1u);
  }

  // The register bit of local qubit `physq`, taking a free one if needed;
  // -1 if none is free or the qubit selects a permutation term.
  int want_reg(int physq) {
    const int j = reg(physq);
    if (j >= 0) return j;
    const int l = loc[physq];
    if (l < 0 || (int)qs.size() >= rb) return -1;
    qs.push_back(l);
    return (int)qs.size() - 1;
  }

  // Compose the store map with a row operation on the local index: bit t
  // flips when bit c is set (a CNOT on local bits), or with a swap of two
  // local bits.
  void compose_cx(int c, int t) {
    auto f = [&](uint32_t x) { return ((x >> c) & 1u) ? x ^ (1u << t) : x; };
    for (int l = 0; l < m; ++l) Mc[l] = f(Mc[l]);
    cl = f(cl);
    for (auto& p : tterms) p.second = f(p.second);
  }
  void compose_swap(int a, int b) {
    auto f = [&](uint32_t x) {
      const uint32_t xa = (x >> a) & 1u, xb = (x >> b) & 1u;
      return (x & ~((1u << a) | (1u << b))) | (xa << b) | (xb << a);
    };
    for (int l = 0; l < m; ++l) Mc[l] = f(Mc[l]);
    cl = f(cl);
    for (auto& p : tterms) p.second = f(p.second);
  }

  bool perm_pending() const {
    if (cl != 0 || !tterms.empty()) return true;
    for (int l = 0; l < m; ++l)
      if (Mc[l] != (1u << l)) return true;
    return false;
  }

  // A single-qubit gate on q that must follow diagonal gates of the stage on
  // q: when q and every qubit of those gates can be register bits (and no
  // permutation is pending), the layer so far and the diagonal gates on
  // register bits close an earlier layer of the stage (its 2x2s, then their
  // register factors) and the gate opens the next; false: close the stage.
  bool start_sub_layer(int q) {
    if ((int)subs.size() >= kPassSubMax || perm_pending()) return false;
    // register bits for q and for the qubits the gates on q share with it
    std::vector<int> need = {q};
    for (const Op& d : diag) {
      bool on_q = false;
      for (int i = 0; i < d.nq; ++i) on_q = on_q || d.q[i] == q;
      if (!on_q) continue;
      for (int i = 0; i < d.nq; ++i) need.push_back(d.q[i]);
    }
    int missing = 0;
    for (size_t i = 0; i < need.size(); ++i) {
      bool dup = false;
      for (size_t k = 0; k < i; ++k) dup = dup || need[k] == need[i];
      if (dup || reg(need[i]) >= 0) continue;
      if (loc[need[i]] < 0) return false;
      ++missing;
    }
    if ((int)qs.size() + missing > rb) return false;
    for (int x : need)
      if (reg(x) < 0) want_reg(x);
    SubLayer sl;
    for (int r = 0; r < kPassRegBitsMax; ++r) {
      sl.slot[r] = slot[r];
      sl.on[r] = slot_on[r];
      slot[r] = kIdentity2;
      slot_on[r] = false;
    }
    // the diagonal gates on register bits move into the earlier layer; the
    // others stay pending (they commute with the gate on q)
    std::vector<Op> rest;
    diag_q = 0;
    for (Op& d : diag) {
      bool all_reg = true;
      for (int i = 0; i < d.nq; ++i) all_reg = all_reg && reg(d.q[i]) >= 0;
      if (all_reg) {
        sl.diag.push_back(std::move(d));
      } else {
        diag_q |= qubit_mask(d);
        rest.push_back(std::move(d));
      }
    }
    diag = std::move(rest);
    subs.push_back(std::move(sl));
    return true;
  }

  bool is_perm_gate(const Op& op) const {
    return op.kind == SV_G_X || op.kind == SV_G_CNOT || op.kind == SV_G_SWAP;
  }

  // Add a permutation gate to the current stage's store map (its targets
  // are local bits of the pass; a CNOT's control may be a tile bit, which
  // makes a term of the map selected per tile).  Always possible: the map
  // needs no register bits.
  void add_perm(const Op& op) {
    if (op.kind == SV_G_X) {
      cl ^= 1u << loc[op.q[0]];
      return;
    }
    if (op.kind == SV_G_SWAP) {
      compose_swap(loc[op.q[0]], loc[op.q[1]]);
      return;
    }
    const int c = op.q[0], lt = loc[op.q[1]];  // CNOT: control q[0], target q[1]
    if (loc[c] >= 0) compose_cx(loc[c], lt);
    else tterms.push_back({src(c), 1u << lt});
  }

  void add(const Op& op) {
    const OpClass cls = classify(op);
    if (cls == CLS_DIAG) {
      uint32_t lbits = 0;
      for (int i = 0; i < op.nq; ++i)
        if (loc[op.q[i]] >= 0) lbits |= 1u << loc[op.q[i]];
      if (lbits & unstable()) close();
      diag.push_back(op);
      diag_q |= qubit_mask(op);
      ++n_members;
      return;
    }
    if (is_perm_gate(op)) {
      add_perm(op);
      ++n_perm;
      ++n_members;
      return;
    }
    if (op.nq == 2) {  // dense 4x4: first in a fresh stage, on register bits (1, 0)
      close();
      qs = {loc[op.q[1]], loc[op.q[0]]};
      has_u2 = true;
      u2m = op.m;
      ++n_members;
      return;
    }
    // single-qubit, not diagonal: the 2x2 of its register bit
    const int q = op.q[0];
    int j = reg(q);
    const bool moved_q = local_moved(q);
    bool conflict = ((diag_q >> q) & 1ull) || moved_q;
    if (conflict && !moved_q && start_sub_layer(q)) {
      conflict = false;
      j = reg(q);
    }
    if (!conflict && j < 0) {
      j = want_reg(q);
      conflict = j < 0;
    }
    if (conflict) {
      close();
      j = want_reg(q);
    }
    slot[j] = mul2({op.m[0], op.m[1], op.m[2], op.m[3]}, slot[j]);
    slot_on[j] = true;
    ++n_members;
  }

  // ---- encoding of the stage ----------------------------------------------
  // A unit-phase diagonal gate on one or two qubits: its phase is
  // c + h_a x_a (+ h_b x_b + J_ab x_a x_b) over the bits x of its qubits,
  // exact in fixed-point turns.
  bool phase_op(const Op& op) const {
    if (op.nq > 2) return false;
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
    if (f32()) return (uint64_t)(uint32_t)(uint64_t)std::llround(std::ldexp(t, 32));
    return (uint64_t)std::ldexp(t, 63) * 2u;
  }

  // The unit phase of a W-bit fixed-point turn.
  cd phase_of(uint64_t w) const {
    const double t = f32() ? (double)(int32_t)(uint32_t)w * 0x1p-32 : (double)(int64_t)w * 0x1p-64;
    return std::polar(1.0, 2.0 * M_PI * t);
  }

  static uint32_t push_entries(StageHost* sh, const cd* e, size_t count) {
    const uint32_t at = (uint32_t)sh->mats.size();
    sh->mats.insert(sh->mats.end(), e, e + count);
    sh->raw.insert(sh->raw.end(), count, 0);
    return at;
  }

  // Append `words` (kPassLPWords per row) to the pool, two per entry.
  static uint32_t put_words(StageHost* sh, const std::vector<uint64_t>& words) {
    const uint32_t at = (uint32_t)sh->mats.size();
    for (size_t w = 0; w < words.size(); w += 2) {
      double re, im;
      std::memcpy(&re, &words[w], sizeof re);
      std::memcpy(&im, &words[w + 1], sizeof im);
      sh->mats.push_back(cd(re, im));
      sh->raw.push_back(1);
    }
    return at;
  }

  static PassItemDev item(uint32_t type) {
    PassItemDev it{};
    it.type = type;
    it.sel = kPassNoSel | (kPassNoSel << 8);
    return it;
  }

  // The phase gates `run` (they commute) as one quadratic phase over the bits
  // of their qubits,
  //   theta(x) = c + sum_a h_a x_a + sum_{a<b} J_ab x_a x_b   (turns mod 1),
  // summed exactly in W-bit fixed point (the words of every gate's entries
  // are rounded once).  Terms over register bits only (and the constant when
  // no quadratic item follows) multiply the register factors `dr`; every
  // register bit with pair terms to bits outside the registers gets a phase
  // ladder; the terms over the other bits (the lane's group bits and the tile
  // bits) form one quadratic-phase item.
  void encode_phase_run(StageHost* sh, const std::vector<const Op*>& run, std::vector<cd>* dr) {
    const uint64_t wmask = f32() ? 0xffffffffull : ~0ull;
    constexpr int NQ = SV_MAX_QUBITS;
    uint64_t c = 0;
    std::vector<uint64_t> h(NQ, 0), J((size_t)NQ * NQ, 0);  // J[a * NQ + b], a < b
    std::vector<char> used(NQ, 0);
    for (const Op* op : run) {
      const int a = op->q[0];
      used[a] = 1;
      if (op->nq == 1) {
        const uint64_t t0 = turns(op->m[0]), t1 = turns(op->m[3]);
        c += t0;
        h[a] += t1 - t0;
        continue;
      }
      const int b = op->q[1];  // entry index (bit a) * 2 + (bit b)
      used[b] = 1;
      const uint64_t t00 = turns(op->m[0]), t01 = turns(op->m[5]), t10 = turns(op->m[10]), t11 = turns(op->m[15]);
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
      PassItemDev it = item(PIT_LP);
      it.a = (uint32_t)reg(a);
      for (int b : other) {
        const uint64_t w = pair(a, b);
        if (!w) continue;
        words[word_of(b)] = w;
        if (loc[b] >= 0) it.lmask |= 1u << loc[b];
        else it.tmask |= 1ull << b;
      }
      if (!it.lmask && !it.tmask) continue;
      words[kPassLPConst] = h[a];
      in_ladder[a] = 1;
      it.mat = put_words(sh, words);
      sh->items.push_back(it);
      ++sh->n_fixed;
    }

    // quadratic phase outside the registers
    std::vector<uint64_t> qw(kPassLPWords, 0);
    PassItemDev qg = item(PIT_QG);
    bool any = false;
    auto mark = [&](PassItemDev& it, int q) {
      if (loc[q] >= 0) it.lmask |= 1u << loc[q];
      else it.tmask |= 1ull << q;
    };
    for (int a : other)
      if (h[a]) {
        qw[word_of(a)] = h[a];
        mark(qg, a);
        any = true;
      }
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
      if (loc[a] >= 0) qg.a |= 1u << loc[a];
      else qg.tt |= 1ull << a;
      qw.insert(qw.end(), row.begin(), row.end());
      any = true;
    }
    if (any) {
      qw[kPassLPConst] = c;
      c = 0;
    }

    // register factors (and the constant when there is no quadratic item)
    const int nr = 1 << rb;
    std::vector<uint64_t> dw(nr, c);
    for (size_t i = 0; i < regq.size(); ++i) {
      const int a = regq[i], ra = reg(a);
      if (!in_ladder[a] && h[a])
        for (int r = 0; r < nr; ++r)
          if ((r >> ra) & 1) dw[r] += h[a];
      for (size_t k = i + 1; k < regq.size(); ++k) {
        const int b = regq[k], rbit = reg(b);
        const uint64_t w = pair(a, b);
        if (!w) continue;
        for (int r = 0; r < nr; ++r)
          if (((r >> ra) & 1) && ((r >> rbit) & 1)) dw[r] += w;
      }
    }
    for (int r = 0; r < nr; ++r) (*dr)[r] *= phase_of(dw[r] & wmask);
    if (any) {
      qg.mat = put_words(sh, qw);
      sh->items.push_back(qg);
      ++sh->n_fixed;
    }
  }

  // A diagonal gate applied exactly: a factor per register index when all
  // its qubits are register bits, else a lane item.
  void encode_exact(StageHost* sh, const Op& op, std::vector<cd>* dr, bool* any_dr) {
    const int dim = 1 << op.nq;
    int regs[2] = {-1, -1};
    int nreg = 0;
    for (int i = 0; i < op.nq; ++i) {
      regs[i] = reg(op.q[i]);
      nreg += regs[i] >= 0;
    }
    if (nreg == op.nq) {
      const int nr = 1 << rb;
      for (int r = 0; r < nr; ++r) {
        int idx = 0;  // the gate's local index: q[0] is its most significant bit
        for (int i = 0; i < op.nq; ++i) idx = (idx << 1) | ((r >> regs[i]) & 1);
        (*dr)[r] *= op.m[(size_t)idx * dim + idx];
      }
      *any_dr = true;
      return;
    }
    auto d = [&](int idx) { return op.m[(size_t)idx * dim + idx]; };
    if (nreg == 0) {  // every qubit outside the registers: one factor per lane
      PassItemDev it = item(PIT_DG);
      cd tab[4];
      if (op.nq == 1) {
        it.sel = src(op.q[0]) | (kPassNoSel << 8);
        tab[0] = d(0);
        tab[1] = d(1);
      } else {
        it.sel = src(op.q[0]) | (src(op.q[1]) << 8);
        for (int i = 0; i < 4; ++i) tab[i] = d(i);
      }
      it.mat = push_entries(sh, tab, (size_t)dim);
      sh->items.push_back(it);
      return;
    }
    // two qubits, one in the registers (bit a), the other (o) selects
    const bool first = regs[0] >= 0;
    const int a = first ? regs[0] : regs[1], o = first ? op.q[1] : op.q[0];
    PassItemDev it = item(PIT_D1);
    it.a = (uint32_t)a;
    it.sel = src(o) | (kPassNoSel << 8);
    cd tab[4];
    for (int var = 0; var < 2; ++var)
      for (int bit = 0; bit < 2; ++bit) tab[2 * var + bit] = d(first ? 2 * bit + var : 2 * var + bit);
    it.mat = push_entries(sh, tab, 4);
    if (tab[0] != cd(1.0, 0.0) || tab[2] != cd(1.0, 0.0)) sh->flags |= PSF_F0;
    sh->items.push_back(it);
  }

  void encode_diag(StageHost* sh) {
    if (diag.empty()) return;
    const int nr = 1 << rb;
    std::vector<cd> dr(nr, cd(1.0, 0.0));
    bool any_dr = false;
    size_t pairs = 0;
    for (const Op& op : diag) pairs += op.nq == 2 && phase_op(op);
    std::vector<const Op*> exact;
    if (pairs >= (size_t)kPhaseRunMin) {
      std::vector<const Op*> run;
      for (const Op& op : diag) (phase_op(op) ? run : exact).push_back(&op);
      const size_t n_items = sh->items.size(), n_mats = sh->mats.size();
      encode_phase_run(sh, run, &dr);
      any_dr = true;
      if (stage_rows(*sh) > (uint32_t)kPassStageRowsMax) {  // over the row table: gate by gate
        sh->items.resize(n_items);
        sh->mats.resize(n_mats);
        sh->raw.resize(n_mats);
        sh->n_fixed = 0;
        std::fill(dr.begin(), dr.end(), cd(1.0, 0.0));
        any_dr = false;
        exact.clear();
        for (const Op& op : diag) exact.push_back(&op);
      }
    } else {
      for (const Op& op : diag) exact.push_back(&op);
    }
    for (const Op* op : exact) encode_exact(sh, *op, &dr, &any_dr);
    if (!sh->items.empty()) {
      sh->flags |= PSF_LANE;
      any_dr = true;  // the lane path multiplies by the register factors too
    }
    if (any_dr) {
      sh->flags |= PSF_DR;
      sh->dr = push_entries(sh, dr.data(), dr.size());
    }
  }

  // Tile-summed rows of a fixed-point item (the row table of PassStageDev).
  static uint32_t item_rows(const PassItemDev& it) {
    if (it.type == PIT_LP) return 1;
    if (it.type == PIT_QG) return 1u + (uint32_t)__builtin_popcount(it.a) + (uint32_t)__builtin_popcountll(it.tt);
    return 0;
  }
  static uint32_t stage_rows(const StageHost& sh) {
    uint32_t r = 0;
    for (const PassItemDev& it : sh.items) r += item_rows(it);
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
    if (f32()) {
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
    const std::vector<PassItemDev> items_now = sh->items;
    for (const PassItemDev& it : items_now) {
      const uint32_t nr = item_rows(it);
      const uint32_t nl = it.type == PIT_QG ? (uint32_t)__builtin_popcount(it.a) : 0u;
      uint64_t tt = it.type == PIT_QG ? it.tt : 0;
      for (uint32_t k = 0; k < nr; ++k) {
        uint32_t pred = kPassRowAlways;
        if (k > nl) {
          pred = (uint32_t)__builtin_ctzll(tt);
          tt &= tt - 1;
        }
        put_u32x4(sh, 2u * it.mat + k * (uint32_t)kPassLPWords + (uint32_t)kPassLPLocalBits, pred,
                  (uint32_t)it.tmask, (uint32_t)(it.tmask >> 32));
        ++sh->row_count;
      }
    }
    if (!sh->row_count) sh->rows = 0;
  }

  void encode(StageHost* sh) {
    // pad the register bits with the lowest local bits that are neither
    // register bits nor permutation selectors
    for (int l = 0; (int)qs.size() < rb && l < m; ++l)
      if (std::find(qs.begin(), qs.end(), l) == qs.end()) qs.push_back(l);
    for (int r = 0; r < rb; ++r) sh->q[r] = (uint32_t)qs[r];
    int n_slots = 0;
    uint32_t form = 0;  // one PassForm per register bit
    for (int r = 0; r < rb; ++r)
      if (slot_on[r]) {
        form |= form_of(slot[r]) << (kPassFormBits * r);
        sh->slot_mask |= 1u << r;
        ++n_slots;
      }
    // earlier layers: 2x2s, then the factors of their diagonal gates
    int n_sub_ops = 0;
    sh->nsub = (uint32_t)subs.size();
    for (size_t k = 0; k < subs.size(); ++k) {
      const SubLayer& sl = subs[k];
      PassSubDev sd{0, 0, 0, kPassNoTable};
      std::vector<cd> e;
      for (int r = 0; r < rb; ++r) {
        if (sl.on[r]) {
          sd.form |= form_of(sl.slot[r]) << (kPassFormBits * r);
          sd.slot_mask |= 1u << r;
          ++n_sub_ops;
        }
        e.insert(e.end(), sl.slot[r].begin(), sl.slot[r].end());
      }
      sd.slots = push_entries(sh, e.data(), e.size());
      if (!sl.diag.empty()) {
        std::vector<cd> dr(1u << rb, cd(1.0, 0.0));
        bool any = false;
        for (const Op& d : sl.diag) encode_exact(sh, d, &dr, &any);
        sd.dr = push_entries(sh, dr.data(), dr.size());
        ++n_sub_ops;
      }
      sh->sub[k] = sd;
    }
    if (n_slots) {
      // absent 2x2s are identities (the kernel skips their bits)
      sh->form = form;
      std::vector<cd> e;
      for (int r = 0; r < rb; ++r) e.insert(e.end(), slot[r].begin(), slot[r].end());
      sh->slots = push_entries(sh, e.data(), e.size());
    }
    if (has_u2) {
      sh->flags |= PSF_U2;
      sh->u2 = push_entries(sh, u2m.data(), 16);
    }
    encode_diag(sh);
    bool perm = cl != 0 || !tterms.empty();
    uint32_t regmask = 0;
    for (int r = 0; r < rb; ++r) regmask |= 1u << qs[r];
    bool cross = false;  // the map moves amplitudes between groups
    for (int l = 0; l < kPassLocalMax; ++l) {
      sh->colimg[l] = l < m ? Mc[l] : 1u << l;
      if (l < m && Mc[l] != (1u << l)) {
        perm = true;
        cross = cross || ((Mc[l] | (1u << l)) & ~regmask);
      }
    }
    sh->pconst = cl;
    cross = cross || (cl & ~regmask);
    for (const auto& t : tterms) {
      PassItemDev it = item(PIT_PX);
      it.sel = t.first | (kPassNoSel << 8);
      it.a = t.second;
      sh->px.push_back(it);
      cross = cross || (t.second & ~regmask);
    }
    if (cross) sh->flags |= PSF_XPERM;
    if (perm) sh->flags |= PSF_PERM;
    encode_rows(sh);
    sh->n_ops = n_sub_ops + n_slots + (has_u2 ? 1 : 0) + ((sh->flags & PSF_DR) ? 1 : 0) + (int)sh->items.size() +
                n_perm;
  }

  void close() {
    if (n_members == 0) {
      reset();
      return;
    }
    StageHost sh;
    encode(&sh);
    out->push_back(std::move(sh));
    reset();
  }
};

// Split the ops of one pass (physical qubits, program order) into register
// stages of rb register bits.
std::vector<StageHost> build_stages(const std::vector<Op>& ops, const int* loc, int m, sv_dtype dt) {
  std::vector<StageHost> out;
  LayerBuilder lb;
  lb.loc = loc;
  lb.m = m;
  lb.rb = pass_reg_bits(dt);
  lb.dt = dt;
  lb.out = &out;
  lb.reset();
  for (const Op& op : ops) lb.add(op);
  lb.close();
  return out;
}

// Cost of a stage in VALU instructions per amplitude (the 2x2 part, the
// diagonal part) plus its LDS round trip.
double stage_ops(const StageHost& sh, sv_dtype dt) {
  const int rb = pass_reg_bits(dt);
  double ops = (dt == SV_C64 ? 8.0 : 16.0);  // LDS read + write of every amplitude, barrier
  for (int r = 0; r < rb; ++r) ops += form_ops(pass_form_of(sh.form, r));
  if (sh.flags & PSF_U2) ops += 32.0;
  for (uint32_t k = 0; k < sh.nsub; ++k) {
    for (int r = 0; r < rb; ++r) ops += form_ops(pass_form_of(sh.sub[k].form, r));
    if (sh.sub[k].dr != kPassNoTable) ops += 4.0;
  }
  if (sh.flags & PSF_LANE) ops += 12.0 + 4.0 * (double)sh.items.size();
  else if (sh.flags & PSF_DR) ops += 4.0;
  return ops;
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

// Final position of the data at every physical position.  SWAP gates still
// ahead in the op list will be relabelings (they rename data, no data
// moves), and the plan must leave label l at position l: the data now
// labelled l ends labelled f(l), so it belongs at position f(l).
std::vector<int> destinations(const QubitMap& mp, const std::vector<Op>& ops, const std::vector<char>& done,
                              size_t first, bool reorder) {
  const int n = (int)mp.logi.size();
  std::vector<int> f(n);
  for (int l = 0; l < n; ++l) f[l] = l;
  if (reorder)
    for (size_t j = first; j < ops.size(); ++j) {
      if (done[j] || ops[j].kind != SV_G_SWAP) continue;
      const int a = ops[j].q[0], b = ops[j].q[1];
      for (int l = 0; l < n; ++l) f[l] = f[l] == a ? b : f[l] == b ? a : f[l];
    }
  std::vector<int> d(n);
  for (int x = 0; x < n; ++x) d[x] = f[mp.logi[x]];
  return d;
}

// Cycles of the position permutation x -> d[x] (fixed points left out).
std::vector<std::vector<int>> dest_cycles(const std::vector<int>& d) {
  const int n = (int)d.size();
  std::vector<char> seen(n, 0);
  std::vector<std::vector<int>> cyc;
  for (int x = 0; x < n; ++x) {
    if (seen[x] || d[x] == x) continue;
    std::vector<int> c;
    for (int y = x; !seen[y]; y = d[y]) {
      seen[y] = 1;
      c.push_back(y);
    }
    cyc.push_back(c);
  }
  return cyc;
}

}  // namespace

sv_status plan_tile_passes(const std::vector<Op>& ops, int n, sv_dtype dt, const sv_opts& o, sv_plan* p,
                           bool progress, int reserve) {
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
  // Cost of a tile pass in full-state sweeps: the data movement alone takes
  // pass_base sweeps and hides `hidden` sweeps of arithmetic; beyond that the
  // stages add up.  ops_per_sweep: VALU instructions per amplitude that take
  // one sweep's time (MI355X: 2.4 GHz x 64 lanes per CU against 8 TB/s, at
  // about 70 % of the issue rate).
  const double ops_per_sweep = dt == SV_C128 ? 110.0 : 55.0;
  const double pass_base = 1.15, hidden = 0.5;

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
        // the reserve never keeps a pass from taking its first op
        if (count + extra <= (members.empty() ? m : m - reserve)) {
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
    // Data moves of the write-back: the last pass brings data home; with
    // `progress`, every pass moves the data whose final position (after the
    // relabelings still ahead) lies in its tile, and fills its free tile
    // bits with whole cycles of those moves, fewest new bits first.
    const bool moves = last || progress;
    std::vector<int> dest;
    std::vector<int> prefer;
    if (moves) {
      dest = destinations(mp, ops, done, first, reorder);
      std::vector<std::vector<int>> cyc = dest_cycles(dest);
      std::vector<std::pair<int, size_t>> order;  // (new bits, cycle)
      for (size_t c = 0; c < cyc.size(); ++c) {
        int extra = 0;
        for (int x : cyc[c]) extra += in_l[x] ? 0 : 1;
        order.push_back({extra, c});
      }
      std::stable_sort(order.begin(), order.end());
      int room = m - count;
      for (const auto& oc : order) {
        if (oc.first > room) continue;
        room -= oc.first;
        prefer.insert(prefer.end(), cyc[oc.second].begin(), cyc[oc.second].end());
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
    ps.stages = build_stages(members, loc, m, dt);
    if (moves) {
      // data whose destination is local goes there; the rest take the local
      // positions nobody moves into (their own when free)
      std::vector<char> taken(n, 0), placed(m, 0);
      for (int jj = 0; jj < m; ++jj) {
        const int x = (int)ps.lpos[jj], dx = dest[x];
        if (in_l[dx]) {
          ps.wpos[jj] = (uint32_t)dx;
          taken[dx] = 1;
          placed[jj] = 1;
        }
      }
      for (int jj = 0; jj < m; ++jj)
        if (!placed[jj] && !taken[ps.lpos[jj]]) {
          ps.wpos[jj] = ps.lpos[jj];
          taken[ps.lpos[jj]] = 1;
          placed[jj] = 1;
        }
      int free_at = 0;
      for (int jj = 0; jj < m; ++jj) {
        if (placed[jj]) continue;
        while (taken[ps.lpos[free_at]]) ++free_at;
        ps.wpos[jj] = ps.lpos[free_at];
        taken[ps.lpos[free_at]] = 1;
      }
      QubitMap nm = mp;
      for (int jj = 0; jj < m; ++jj) {
        const int l = mp.logi[ps.lpos[jj]];
        nm.phys[l] = (int)ps.wpos[jj];
        nm.logi[ps.wpos[jj]] = l;
      }
      mp = nm;
    }
    double alu = 0.0;
    for (const StageHost& sh : ps.stages) alu += stage_ops(sh, dt) / ops_per_sweep;
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
