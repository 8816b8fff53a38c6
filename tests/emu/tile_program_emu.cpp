// Host model of the in-cache tile-pass kernel (test infrastructure).
//
// Reads a circuit on stdin ("n dtype mode lds_qubits", then one gate per
// line: kind nq q... theta [2 * 4^nq matrix doubles for SV_G_MATRIX]) and
// an initial state from the file named by SV_EMU_INIT (2^n lines "re im").
// It plans the circuit with the library's planner (build_plan), packs the
// device image with the library's packer (pack_plan), and executes every
// pass on the CPU the way the pass kernel does: tiles gathered at the pass's
// local bit positions, register stages (4x4 on register bits (1, 0), one 2x2
// per register bit, register factors and lane items, the register
// permutation applied at the stage's store), the write-back to wpos.  Every
// read of a descriptor, stage, item, pool entry, fixed-point word and row is
// bounds-checked; a violation or an inconsistency (a form that does not hold
// its entries, a permutation that is not a bijection of the registers, a
// selector that is a register bit, a row count that does not match) exits
// with status 3.  Sweep and dense passes are applied by definition.  Prints
// the final state, one "re im" line per amplitude.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iostream>
#include <string>
#include <vector>

#include "sv_host.h"

using namespace sv;

// ---- stubs for the device-side functions the planner objects reference
namespace sv {
sv_status upload(sv_state*, const void*, size_t, void**) { return SV_ERR_DEVICE; }
sv_status run_op_sweep(sv_state*, const Op&, const void*, bool) { return SV_ERR_DEVICE; }
sv_status renormalize(sv_state*) { return SV_ERR_DEVICE; }
hipError_t launch_pass(sv_dtype, void*, int, int, const PassDescDev*, int, const PassStageDev*, const PassItemDev*,
                       const void*, bool, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_matrix_pass(sv_dtype, int, void*, int, int, const PassDescDev*, int, int, const PassStageDev*,
                              const void*, hipStream_t) { return hipErrorInvalidValue; }
static std::string g_err;
sv_status fail(sv_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}
void clear_error() { g_err.clear(); }
size_t elem_bytes(sv_dtype dt) { return dt == SV_C128 ? 16 : 8; }
bool debug_sync_enabled() { return false; }
}  // namespace sv

extern "C" const char* hipGetErrorString(hipError_t) { return "stub"; }
extern "C" hipError_t hipStreamSynchronize(hipStream_t) { return hipErrorInvalidValue; }
extern "C" hipError_t hipGetLastError(void) { return hipErrorInvalidValue; }

static void die(const char* msg) {
  fprintf(stderr, "EMU ERROR: %s\n", msg);
  exit(3);
}

struct Prog {
  const std::vector<unsigned char>* host;
  const PackedPlan* pk;
  bool f32;
  size_t pool_entries;
  size_t n_stages, n_items;
  const PassDescDev* desc(int i) const { return (const PassDescDev*)(host->data() + pk->off_desc) + i; }
  const PassStageDev* stage(uint32_t i) const {
    if (i >= n_stages) die("stage index out of range");
    return (const PassStageDev*)(host->data() + pk->off_stage) + i;
  }
  const PassItemDev* item(uint32_t i) const {
    if (i >= n_items) die("item index out of range");
    return (const PassItemDev*)(host->data() + pk->off_items) + i;
  }
  cd entry(uint32_t e) const {
    if (e >= pool_entries) die("pool entry out of range");
    const unsigned char* p = host->data() + pk->off_pool + (size_t)e * (f32 ? 8 : 16);
    if (f32) {
      float v[2];
      memcpy(v, p, 8);
      return cd(v[0], v[1]);
    }
    double v[2];
    memcpy(v, p, 16);
    return cd(v[0], v[1]);
  }
  // fixed-point word w (two per entry), counted from entry `base`
  uint64_t word(uint32_t base, uint32_t w) const {
    const uint32_t e = base + w / 2;
    if (e >= pool_entries) die("word out of range");
    const unsigned char* p = host->data() + pk->off_pool + (size_t)e * (f32 ? 8 : 16);
    if (f32) {
      uint32_t v[2];
      memcpy(v, p, 8);
      return v[w & 1];
    }
    uint64_t v[2];
    memcpy(v, p, 16);
    return v[w & 1];
  }
  uint32_t u32(uint32_t base, uint32_t i) const {  // uint32 i of the words from entry base
    const size_t byte = (size_t)base * (f32 ? 8 : 16) + (size_t)i * 4;
    if (byte + 4 > pool_entries * (f32 ? 8 : 16)) die("row table out of range");
    uint32_t v;
    memcpy(&v, host->data() + pk->off_pool + byte, 4);
    return v;
  }
};

static uint64_t deposit(uint64_t x, uint64_t mask) {
  uint64_t r = 0;
  while (mask) {
    const uint64_t low = mask & (~mask + 1ull);
    if (x & 1ull) r |= low;
    x >>= 1;
    mask &= mask - 1ull;
  }
  return r;
}

static cd phase_of_word(uint64_t t, bool f32) {
  const double turns = f32 ? (double)(int32_t)(uint32_t)t * 0x1p-32 : (double)(int64_t)t * 0x1p-64;
  return std::polar(1.0, 2.0 * M_PI * turns);
}

static uint32_t sel_bit(uint32_t c, uint32_t xg, uint64_t base) {
  if (c == kPassNoSel) die("selector none used");
  return c < kPassTileSel ? (xg >> c) & 1u : (uint32_t)(base >> (c - kPassTileSel)) & 1u;
}
static uint32_t item_var(uint32_t sel, uint32_t xg, uint64_t base) {
  const uint32_t a = sel & 0xffu, b = (sel >> 8) & 0xffu;
  uint32_t var = a == kPassNoSel ? 0u : sel_bit(a, xg, base);
  if (b != kPassNoSel) var = (var << 1) | sel_bit(b, xg, base);
  return var;
}

int main() {
  int n;
  std::string dts, mode;
  int lds;
  std::cin >> n >> dts >> mode >> lds;
  const sv_dtype dt = dts == "c64" ? SV_C64 : SV_C128;
  std::vector<sv_gate> gates;
  std::vector<std::vector<double>> mats;
  std::string kind;
  while (std::cin >> kind) {
    sv_gate g{};
    int nq;
    std::cin >> nq;
    g.nq = nq;
    for (int i = 0; i < nq; ++i) std::cin >> g.q[i];
    std::cin >> g.theta;
    g.kind = std::stoi(kind);
    if (g.kind == SV_G_MATRIX) {
      mats.emplace_back((size_t)2 << (2 * nq));
      for (double& x : mats.back()) std::cin >> x;
    }
    gates.push_back(g);
  }
  size_t mi = 0;
  for (auto& g : gates)
    if (g.kind == SV_G_MATRIX) g.m = mats[mi++].data();
  sv_opts o{};
  o.max_fuse_qubits = 5;
  o.reorder = 1;
  o.fp32_mfma = 1;
  o.mode = mode == "pass" ? SV_MODE_PASS : mode == "sweep" ? SV_MODE_SWEEP : mode == "matrix" ? SV_MODE_MATRIX : SV_MODE_AUTO;
  o.lds_qubits = lds;
  sv_plan p;
  if (build_plan(n, dt, gates.data(), gates.size(), o, &p) != SV_OK) die(g_err.c_str());
  PackedPlan pk;
  if (pack_plan(&p, &pk) != SV_OK) die(g_err.c_str());
  Prog pr{&pk.host, &pk, dt == SV_C64, 0, 0, 0};
  const size_t esz = dt == SV_C64 ? 8 : 16;
  pr.pool_entries = pk.n_desc ? (pk.host.size() - pk.off_pool) / esz : 0;
  pr.n_stages = pk.n_desc ? (pk.off_items - pk.off_stage) / sizeof(PassStageDev) : 0;
  pr.n_items = pk.n_desc ? (pk.off_pool - pk.off_items) / sizeof(PassItemDev) : 0;
  const int RB = pass_reg_bits(dt), NR = 1 << RB;
  const uint64_t N = 1ull << n;
  std::vector<cd> psi(N);
  // initial state from env: SV_EMU_INIT file of 2^n complex (re im)
  if (const char* f = getenv("SV_EMU_INIT")) {
    FILE* fp = fopen(f, "r");
    for (uint64_t i = 0; i < N; ++i) {
      double re, im;
      if (fscanf(fp, "%lf %lf", &re, &im) != 2) die("init read");
      psi[i] = cd(re, im);
    }
    fclose(fp);
  } else {
    psi[0] = 1.0;
  }
  for (size_t pi = 0; pi < p.passes.size(); ++pi) {
    const Pass& ps = p.passes[pi];
    if (ps.kind == PASS_SWEEP || ps.kind == PASS_DENSE) {
      const Op& op = ps.phys;
      const int k = op.nq, d = 1 << k;
      uint64_t mk = 0;
      for (int i = 0; i < k; ++i) mk |= 1ull << op.q[i];
      std::vector<cd> x(d), y(d);
      for (uint64_t b = 0; b < N; ++b) {
        if (b & mk) continue;
        std::vector<uint64_t> idx(d);
        for (int r = 0; r < d; ++r) {
          uint64_t i = b;
          for (int j = 0; j < k; ++j)
            if ((r >> (k - 1 - j)) & 1) i |= 1ull << op.q[j];
          idx[r] = i;
          x[r] = psi[i];
        }
        for (int r = 0; r < d; ++r) {
          cd s = 0;
          for (int c = 0; c < d; ++c) s += op.m[(size_t)r * d + c] * x[c];
          y[r] = s;
        }
        for (int r = 0; r < d; ++r) psi[idx[r]] = y[r];
      }
      continue;
    }
    const PassDescDev* D = pr.desc(pk.desc_index[pi]);
    const uint32_t m = D->m;
    uint64_t lmask = 0;
    for (uint32_t j = 0; j < m; ++j) lmask |= 1ull << D->lpos[j];
    if (lmask != D->lmask) die("lmask mismatch");
    const uint64_t rest = (N - 1) & ~lmask;
    const uint64_t tiles = N >> m;
    std::vector<cd> tile(1u << m);
    for (uint64_t t = 0; t < tiles; ++t) {
      const uint64_t base = deposit(t, rest);
      for (uint32_t x = 0; x < (1u << m); ++x) {
        uint64_t a = base;
        for (uint32_t j = 0; j < m; ++j)
          if ((x >> j) & 1) a |= 1ull << D->lpos[j];
        tile[x] = psi[a];
      }
      if (ps.kind == PASS_MATRIX) {
        // Matrix stages: a dense 2^K x 2^K op on the member bits q[]; the
        // column order puts lane bits, then wave bits first; a stage without
        // the barrier flag must leave every element with the wave that held it.
        const int K = ps.mx_k, D2 = 1 << K;
        const int lane_bits = dt == SV_C64 ? 5 : 4;
        const int nc = (int)m - K, nwb = std::min(3, nc - lane_bits);
        if (nc < lane_bits + 2) die("matrix stage: too few column bits");
        for (uint32_t j = 0; j < m; ++j)
          if (D->wpos[j] != D->lpos[j]) die("matrix pass with a write map");
        std::vector<int> owner(1u << m, -1);
        for (uint32_t si = 0; si < D->stage_count; ++si) {
          const PassStageDev& S = *pr.stage(D->stage_first + si);
          uint32_t tmask = 0;
          for (int b = 0; b < K; ++b) {
            if (S.q[b] >= m || ((tmask >> S.q[b]) & 1u)) die("matrix stage: bad member bits");
            tmask |= 1u << S.q[b];
          }
          uint32_t cmask = 0;
          for (int j = 0; j < nc; ++j) {
            if (S.colimg[j] >= m || ((cmask >> S.colimg[j]) & 1u) || ((tmask >> S.colimg[j]) & 1u))
              die("matrix stage: column order is not the other local bits");
            cmask |= 1u << S.colimg[j];
          }
          std::vector<int> own(1u << m);
          for (uint32_t x = 0; x < (1u << m); ++x) {
            int w = 0;
            for (int j = 0; j < nwb; ++j) w |= (int)((x >> S.colimg[lane_bits + j]) & 1u) << j;
            own[x] = w;
            if (si > 0 && !(S.flags & kMatrixStageSync) && owner[x] != w)
              die("matrix stage without a barrier moves an element to another wave");
          }
          owner.swap(own);
          std::vector<cd> xin(D2), yout(D2);
          for (uint32_t b0 = 0; b0 < (1u << m); ++b0) {
            if (b0 & tmask) continue;
            for (int r = 0; r < D2; ++r) {
              uint32_t x = b0;
              for (int b = 0; b < K; ++b)
                if ((r >> b) & 1) x |= 1u << S.q[b];
              xin[r] = tile[x];
            }
            for (int r = 0; r < D2; ++r) {
              cd acc = 0;
              for (int c = 0; c < D2; ++c) acc += pr.entry(S.u2 + (uint32_t)(r * D2 + c)) * xin[c];
              yout[r] = acc;
            }
            for (int r = 0; r < D2; ++r) {
              uint32_t x = b0;
              for (int b = 0; b < K; ++b)
                if ((r >> b) & 1) x |= 1u << S.q[b];
              tile[x] = yout[r];
            }
          }
        }
        for (uint32_t x = 0; x < (1u << m); ++x) {
          uint64_t a = base;
          for (uint32_t j = 0; j < m; ++j)
            if ((x >> j) & 1) a |= 1ull << D->lpos[j];
          psi[a] = tile[x];
        }
        continue;
      }
      for (uint32_t si = 0; si < D->stage_count; ++si) {
        const PassStageDev S = *pr.stage(D->stage_first + si);
        if (t == 0 && getenv("SV_EMU_DUMP")) {  // plan structure, for inspection
          int ni[5] = {0, 0, 0, 0, 0};
          for (uint32_t k = 0; k < S.item_count; ++k) ++ni[pr.item(S.item_first + k)->type % 5];
          fprintf(stderr, "pass %zu stage %u: q=%u,%u,%u,%u,%u form %u mask %x flags %x items DG%d D1%d LP%d QG%d px %u rows %u\n",
                  pi, si, S.q[0], S.q[1], S.q[2], S.q[3], RB > 4 ? S.q[4] : 0, S.form, S.slot_mask, S.flags, ni[0], ni[1],
                  ni[2], ni[3], S.px_count, S.row_count);
        }
        // tile sums of rows
        std::vector<uint64_t> ts(S.row_count);
        for (uint32_t j = 0; j < S.row_count; ++j) {
          const uint32_t rb = S.mat_base + S.rows;
          const uint32_t word = pr.u32(rb, 4 * j), pred = pr.u32(rb, 4 * j + 1);
          const uint64_t sel = base & (pr.u32(rb, 4 * j + 2) | ((uint64_t)pr.u32(rb, 4 * j + 3) << 32));
          uint64_t acc = 0;
          for (int i = 0; i < kPassLPTileBits; ++i)
            if ((sel >> i) & 1) acc += pr.word(S.mat_base, word + i);
          ts[j] = (pred == kPassRowAlways || ((base >> pred) & 1)) ? acc : 0;
        }
        uint32_t regmask = 0;
        for (int b = 0; b < RB; ++b) {
          if (S.q[b] >= m) die("register bit beyond the tile");
          regmask |= 1u << S.q[b];
        }
        if (__builtin_popcount(regmask) != RB) die("register bits not distinct");
        const uint32_t groups = (1u << m) >> RB;
        const uint32_t gmask = ((1u << m) - 1) & ~regmask;
        std::vector<cd> nt(1u << m);
        std::vector<char> written(1u << m, 0);
        for (uint32_t gi = 0; gi < groups; ++gi) {
          const uint32_t xg = (uint32_t)deposit(gi, gmask);
          auto addr = [&](uint32_t r) {
            uint32_t o = xg;
            for (int b = 0; b < RB; ++b)
              if ((r >> b) & 1) o |= 1u << S.q[b];
            return o;
          };
          std::vector<cd> v(NR);
          for (int r = 0; r < NR; ++r) v[r] = tile[addr(r)];
          if (S.flags & PSF_U2) {
            for (int r = 0; r < NR; r += 4) {
              cd x[4] = {v[r], v[r | 1], v[r | 2], v[r | 3]};
              for (int oo = 0; oo < 4; ++oo) {
                cd y = 0;
                for (int c = 0; c < 4; ++c) y += pr.entry(S.u2 + 4 * oo + c) * x[c];
                v[r | oo] = y;
              }
            }
          }
          // one layer: a 2x2 per register bit of the mask, in the layer's form
          auto apply_layer = [&](uint32_t forms, uint32_t slots, uint32_t mask) {
            if (forms == 0) return;
            if (forms >> (kPassFormBits * RB)) die("form word beyond the register bits");
            for (int b = 0; b < RB; ++b) {
              const uint32_t form = pass_form_of(forms, b);
              if (form > PFORM_U) die("unknown 2x2 form");
              if ((form != PFORM_NONE) != (((mask >> b) & 1u) != 0)) die("slot mask and forms disagree");
              if (form == PFORM_NONE) {
                // the kernel skips the bit: its entries must be the identity
                if (pr.entry(slots + 4 * b) != cd(1.0) || pr.entry(slots + 4 * b + 1) != cd(0.0) ||
                    pr.entry(slots + 4 * b + 2) != cd(0.0) || pr.entry(slots + 4 * b + 3) != cd(1.0))
                  die("2x2 without a form is not the identity");
                continue;
              }
              cd mm[4];
              for (int e = 0; e < 4; ++e) mm[e] = pr.entry(slots + 4 * b + e);
              // the form must hold the entries
              for (int e = 0; e < 4; ++e) {
                const bool diag = e == 0 || e == 3;
                if (form == PFORM_UR && mm[e].imag() != 0) die("UR form with imaginary entry");
                if (form == PFORM_UI && ((diag && mm[e].imag() != 0) || (!diag && mm[e].real() != 0))) die("UI form mismatch");
                if (form == PFORM_RC && diag && mm[e].imag() != 0) die("RC form mismatch");
              }
              for (int r = 0; r < NR; ++r)
                if (!((r >> b) & 1)) {
                  const cd a0 = v[r], a1 = v[r | (1 << b)];
                  v[r] = mm[0] * a0 + mm[1] * a1;
                  v[r | (1 << b)] = mm[2] * a0 + mm[3] * a1;
                }
            }
          };
          if (S.nsub > (uint32_t)kPassSubMax) die("too many earlier layers");
          for (uint32_t li = 0; li <= S.nsub; ++li) {
            const bool last = li == S.nsub;
            const PassSubDev L = last ? PassSubDev{S.form, S.slot_mask, S.slots, kPassNoTable} : S.sub[li];
            if (!last && L.form == 0 && L.dr == kPassNoTable) die("empty earlier layer");
            if (L.form == 0 && L.slot_mask) die("slot mask without a form");
            apply_layer(L.form, L.slots, L.slot_mask);
            if (L.dr != kPassNoTable) {
              if (last) die("last layer with its own table");
              for (int r = 0; r < NR; ++r) v[r] *= pr.entry(L.dr + r);
            }
          }
          if (S.flags & PSF_LANE) {
            cd G = 1.0, f0[5] = {1, 1, 1, 1, 1}, f1[5] = {1, 1, 1, 1, 1};
            uint32_t row = 0;
            for (uint32_t i = 0; i < S.item_count; ++i) {
              const PassItemDev it = *pr.item(S.item_first + i);
              if (it.type == PIT_DG) {
                const uint32_t var = item_var(it.sel, xg, base);
                G *= pr.entry(it.mat + var);
              } else if (it.type == PIT_D1) {
                if (it.a >= (uint32_t)RB) die("D1 bit");
                const uint32_t var = item_var(it.sel, xg, base);
                f0[it.a] *= pr.entry(it.mat + 2 * var);
                f1[it.a] *= pr.entry(it.mat + 2 * var + 1);
              } else if (it.type == PIT_LP || it.type == PIT_QG) {
                const uint32_t lsel = xg & it.lmask;
                auto local = [&](uint32_t wbase) {
                  uint64_t t2 = 0;
                  for (int b = 0; b < kPassLPLocalBits; ++b)
                    if ((lsel >> b) & 1) t2 += pr.word(it.mat, wbase + b);
                  return t2;
                };
                uint64_t tt = pr.word(it.mat, kPassLPConst) + ts.at(row) + local(0);
                if (it.type == PIT_LP) {
                  if (it.a >= (uint32_t)RB) die("LP bit");
                  f1[it.a] *= phase_of_word(dt == SV_C64 ? (uint32_t)tt : tt, dt == SV_C64);
                  row += 1;
                } else {
                  uint32_t k = 1;
                  for (uint32_t lt = it.a; lt; lt &= lt - 1u, ++k) {
                    const uint64_t h = ts.at(row + k) + local(k * kPassLPWords);
                    if ((xg >> __builtin_ctz(lt)) & 1u) tt += h;
                  }
                  const uint32_t end = 1u + __builtin_popcount(it.a) + __builtin_popcountll(it.tt);
                  for (; k < end; ++k) tt += ts.at(row + k);
                  G *= phase_of_word(dt == SV_C64 ? (uint32_t)tt : tt, dt == SV_C64);
                  row += end;
                }
              } else {
                die("bad item type");
              }
            }
            if (row != S.row_count) die("row count mismatch");
            if (!(S.flags & PSF_F0))
              for (int b = 0; b < RB; ++b)
                if (f0[b] != cd(1.0, 0.0)) die("f0 factor without PSF_F0");
            for (int r = 0; r < NR; ++r) {
              cd f = G * pr.entry(S.dr + r);
              for (int b = 0; b < RB; ++b) f *= ((r >> b) & 1) ? f1[b] : f0[b];
              v[r] *= f;
            }
          } else if (S.flags & PSF_DR) {
            for (int r = 0; r < NR; ++r) v[r] *= pr.entry(S.dr + r);
          }
          // the store map x -> M x ^ c ^ c(tile), into the stage's output
          uint32_t c = S.pconst;
          for (uint32_t k = 0; k < S.px_count; ++k) {
            const PassItemDev it = *pr.item(S.px_first + k);
            if (it.type != PIT_PX) die("px item type");
            const uint32_t sc = it.sel & 0xffu;
            if (sc < kPassTileSel) die("store-map term not selected by a tile bit");
            if (sel_bit(sc, xg, base)) c ^= it.a;
          }
          for (int r = 0; r < NR; ++r) {
            const uint32_t x = addr(r);
            uint32_t y = c;
            for (uint32_t l = 0; l < m; ++l)
              if ((x >> l) & 1u) y ^= S.colimg[l];
            if (y >= (1u << m)) die("store map leaves the tile");
            if (!(S.flags & PSF_PERM) && y != x) die("store map without PSF_PERM");
            if (!(S.flags & PSF_XPERM) && (y & ~regmask) != xg) die("map between groups without PSF_XPERM");
            if (written[y]++) die("store map not a bijection");
            nt[y] = v[r];
          }
        }
        tile.swap(nt);
      }
      for (uint32_t x = 0; x < (1u << m); ++x) {
        uint64_t a = base;
        for (uint32_t j = 0; j < m; ++j)
          if ((x >> j) & 1) a |= 1ull << D->wpos[j];
        psi[a] = tile[x];
      }
    }
  }
  for (uint64_t i = 0; i < N; ++i) printf("%.17g %.17g\n", psi[i].real(), psi[i].imag());
  return 0;
}
