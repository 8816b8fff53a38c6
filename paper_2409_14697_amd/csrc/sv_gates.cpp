// Gate intermediate representation: validation, named-gate matrices (host,
// FP64), structural classification, and the mapping of one- and two-qubit
// ops onto the sweep kernels.
#include <cmath>
#include <cstring>

#include "sv_host.h"

namespace sv {

int gate_arity(int kind) {
  switch (kind) {
    case SV_G_H: case SV_G_X: case SV_G_Y: case SV_G_Z: case SV_G_S: case SV_G_T:
    case SV_G_RX: case SV_G_RY: case SV_G_RZ: case SV_G_P:
      return 1;
    case SV_G_CNOT: case SV_G_CZ: case SV_G_SWAP: case SV_G_CPHASE: case SV_G_RZZ:
      return 2;
    default:
      return -1;
  }
}

sv_status validate_gate(const sv_gate& g, int n) {
  if (g.kind < SV_G_MATRIX || g.kind > SV_G_RZZ) return fail(SV_ERR_ARG, "unknown gate kind %d", g.kind);
  if (g.kind == SV_G_MATRIX) {
    if (g.nq < 1 || g.nq > SV_MAX_GATE_QUBITS)
      return fail(SV_ERR_ARG, "matrix gate with %d qubits (1..%d allowed)", g.nq, SV_MAX_GATE_QUBITS);
    if (!g.m) return fail(SV_ERR_ARG, "matrix gate without a matrix");
  } else if (g.nq != gate_arity(g.kind)) {
    return fail(SV_ERR_ARG, "gate kind %d takes %d qubits, got nq=%d", g.kind, gate_arity(g.kind), g.nq);
  }
  for (int i = 0; i < g.nq; ++i) {
    if (g.q[i] < 0 || g.q[i] >= n) return fail(SV_ERR_QUBIT, "qubit %d out of range [0,%d)", g.q[i], n);
    for (int j = 0; j < i; ++j)
      if (g.q[i] == g.q[j]) return fail(SV_ERR_QUBIT, "qubit %d repeated in one gate", g.q[i]);
  }
  if (g.kind != SV_G_MATRIX && !std::isfinite(g.theta)) return fail(SV_ERR_ARG, "non-finite angle");
  return SV_OK;
}

// Textbook definitions; row order as in Eq. 3 (first qubit most significant).
std::vector<cd> named_matrix(int kind, double th) {
  const double r2 = 1.0 / std::sqrt(2.0);
  const double c = std::cos(0.5 * th), s = std::sin(0.5 * th);
  const cd I(0.0, 1.0);
  auto ph = [](double a) { return cd(std::cos(a), std::sin(a)); };
  switch (kind) {
    case SV_G_H: return {r2, r2, r2, -r2};
    case SV_G_X: return {0.0, 1.0, 1.0, 0.0};
    case SV_G_Y: return {0.0, -I, I, 0.0};
    case SV_G_Z: return {1.0, 0.0, 0.0, -1.0};
    case SV_G_S: return {1.0, 0.0, 0.0, I};
    case SV_G_T: return {1.0, 0.0, 0.0, ph(M_PI / 4.0)};
    case SV_G_RX: return {c, -I * s, -I * s, c};
    case SV_G_RY: return {c, -s, s, c};
    case SV_G_RZ: return {ph(-0.5 * th), 0.0, 0.0, ph(0.5 * th)};
    case SV_G_P: return {1.0, 0.0, 0.0, ph(th)};
    case SV_G_CNOT: return {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0};
    case SV_G_CZ: return {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, -1};
    case SV_G_SWAP: return {1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1};
    case SV_G_CPHASE: {
      std::vector<cd> m(16, 0.0);
      m[0] = m[5] = m[10] = 1.0;
      m[15] = ph(th);
      return m;
    }
    case SV_G_RZZ: {
      std::vector<cd> m(16, 0.0);
      m[0] = m[15] = ph(-0.5 * th);
      m[5] = m[10] = ph(0.5 * th);
      return m;
    }
  }
  return {};
}

Op op_from_gate(const sv_gate& g) {
  Op op;
  op.kind = g.kind;
  op.nq = g.nq;
  for (int i = 0; i < g.nq; ++i) op.q[i] = g.q[i];
  op.theta = g.theta;
  if (g.kind == SV_G_MATRIX) {
    const size_t d = (size_t)1 << g.nq;
    op.m.resize(d * d);
    for (size_t i = 0; i < d * d; ++i) op.m[i] = cd(g.m[2 * i], g.m[2 * i + 1]);
  } else {
    op.m = named_matrix(g.kind, g.theta);
  }
  return op;
}

OpClass classify(const Op& op) {
  const size_t d = (size_t)1 << op.nq;
  bool diag = true, perm = true;
  for (size_t r = 0; r < d; ++r) {
    int nz = 0;
    for (size_t c = 0; c < d; ++c) {
      const cd v = op.m[r * d + c];
      if (v != cd(0.0, 0.0)) {
        ++nz;
        if (r != c) diag = false;
        if (v != cd(1.0, 0.0)) perm = false;
      }
    }
    if (nz != 1) perm = false;
  }
  if (diag && !perm) return CLS_DIAG;
  if (perm) return CLS_PERM;
  return CLS_DENSE;
}

namespace {
void sort2(unsigned a, unsigned b, unsigned* z) {
  z[0] = a < b ? a : b;
  z[1] = a < b ? b : a;
}
}  // namespace

bool sweep_args_for(const Op& op, SweepArgs* out) {
  SweepArgs a{};
  if (op.nq == 1) {
    const unsigned t = (unsigned)op.q[0];
    a.g.nz = 1;
    a.g.z[0] = t;
    switch (op.kind) {
      case SV_G_X:
        a.op = SWEEP_SWAP;
        a.g.nv = 2;
        a.g.off[0] = 0;
        a.g.off[1] = 1ull << t;
        break;
      case SV_G_Z: case SV_G_S: case SV_G_T: case SV_G_P:
        a.op = SWEEP_PHASE;  // diag(1, d1): only the bit-t = 1 half changes
        a.g.set = 1ull << t;
        a.g.nv = 1;
        a.m[0] = op.m[3];
        break;
      case SV_G_RZ:
        a.op = SWEEP_DIAG;
        a.g.nz = 0;
        a.g.nv = 1;
        a.diag_nbits = 1;
        a.diag_b0 = t;
        a.m[0] = op.m[0];
        a.m[1] = op.m[3];
        break;
      default:
        a.op = SWEEP_DENSE1;
        a.g.nv = 2;
        a.g.off[0] = 0;
        a.g.off[1] = 1ull << t;
        for (int i = 0; i < 4; ++i) a.m[i] = op.m[i];
        break;
    }
    *out = a;
    return true;
  }
  if (op.nq == 2) {
    const unsigned q0 = (unsigned)op.q[0], q1 = (unsigned)op.q[1];
    a.g.nz = 2;
    sort2(q0, q1, a.g.z);
    switch (op.kind) {
      case SV_G_CNOT:  // Eq. 3: where the control is 1, exchange target 0 and 1
        a.op = SWEEP_SWAP;
        a.g.set = 1ull << q0;
        a.g.nv = 2;
        a.g.off[0] = 0;
        a.g.off[1] = 1ull << q1;
        break;
      case SV_G_SWAP:
        a.op = SWEEP_SWAP;
        a.g.nv = 2;
        a.g.off[0] = 1ull << q1;
        a.g.off[1] = 1ull << q0;
        break;
      case SV_G_CZ: case SV_G_CPHASE:
        a.op = SWEEP_PHASE;
        a.g.set = (1ull << q0) | (1ull << q1);
        a.g.nv = 1;
        a.m[0] = op.m[15];
        break;
      case SV_G_RZZ:
        a.op = SWEEP_DIAG;
        a.g.nz = 0;
        a.g.nv = 1;
        a.diag_nbits = 2;
        a.diag_b0 = q0;
        a.diag_b1 = q1;
        for (int r = 0; r < 4; ++r) a.m[r] = op.m[5 * r];
        break;
      default:
        a.op = SWEEP_DENSE2;
        a.g.nv = 4;
        a.g.off[0] = 0;
        a.g.off[1] = 1ull << q1;
        a.g.off[2] = 1ull << q0;
        a.g.off[3] = (1ull << q0) | (1ull << q1);
        for (int i = 0; i < 16; ++i) a.m[i] = op.m[i];
        break;
    }
    *out = a;
    return true;
  }
  return false;
}

// Position classes of a qubit for the sweep kernels, in units of 16-byte
// elements (one complex128 amplitude, or a complex64 pair whose bit 0 is
// inside the element):
//   in_wave   -- the partner lies in the same row of 64 elements that one
//                wave loads per instruction (element bit < 6): a target there
//                is paired by lane exchange;
//   sub_burst -- the bit lies inside one 64-byte DRAM burst (element bit < 2):
//                a control or phase bit there cannot select a subset of
//                bursts, so the whole row is read and the bit is handled in
//                lanes; a higher control or phase bit restricts the sweep to
//                the touched subset.
static int elem_bit(int q, sv_dtype dt) { return dt == SV_C128 ? q : q - 1; }
static bool in_wave(int q, sv_dtype dt) { return dt == SV_C64 && q == 0 ? true : elem_bit(q, dt) < 6; }
static bool sub_burst(int q, sv_dtype dt) { return dt == SV_C64 && q == 0 ? true : elem_bit(q, dt) < 2; }
static bool low_args_for_layout(const Op& op, sv_dtype dt, SweepArgs* out);

bool plan_low(sv_dtype dt, SweepArgs* a) {
  const bool pair = dt == SV_C64;
  const unsigned shift = pair ? 1u : 0u;
  unsigned epos[2] = {0, 0};
  a->low_nz = 0;
  a->low_set = 0;
  a->low_off1 = 0;
  for (int m = 0; m < a->low_k; ++m) {
    const unsigned p = a->low_q[m];
    if (pair && p == 0) {
      a->low_kind[m] = LOW_INTRA;
    } else if (p - shift < kLaneBits) {
      a->low_kind[m] = LOW_LANE;
      epos[m] = p - shift;
    } else {
      if (a->low_nz == 2) return false;
      a->low_kind[m] = LOW_REG;
      a->low_z[a->low_nz++] = p - shift;
      a->low_off1 = 1ull << (p - shift);
    }
  }
  for (unsigned p = 0; p < 64; ++p)
    if ((a->low_fixed >> p) & 1ull) {
      if (a->low_nz == 2 || (pair && p == 0)) return false;
      a->low_z[a->low_nz++] = p - shift;
      a->low_set |= 1ull << (p - shift);
    }
  if (a->low_nz > 1) return false;
  // a lane holds element bits 0..5 minus the inserted positions below them
  for (int m = 0; m < a->low_k; ++m)
    if (a->low_kind[m] == LOW_LANE) {
      unsigned below = 0;
      for (int z = 0; z < a->low_nz; ++z) below += a->low_z[z] < epos[m] ? 1u : 0u;
      a->low_lanebit[m] = epos[m] - below;
    }
  return true;
}

bool low_args_for(const Op& op, sv_dtype dt, SweepArgs* out) {
  const bool ok = low_args_for_layout(op, dt, out);
  return ok && plan_low(dt, out);
}

static bool low_args_for_layout(const Op& op, sv_dtype dt, SweepArgs* out) {
  SweepArgs a{};
  a.op = SWEEP_LOW;
  if (op.nq == 1) {
    const int t = op.q[0];
    if (op.kind == SV_G_RZ) return false;  // elementwise sweep
    const bool phase = op.kind == SV_G_Z || op.kind == SV_G_S || op.kind == SV_G_T || op.kind == SV_G_P;
    if (phase ? !sub_burst(t, dt) : !in_wave(t, dt)) return false;
    a.low_k = 1;
    a.low_q[0] = (unsigned)t;
    for (int i = 0; i < 4; ++i) a.m[i] = op.m[i];
    *out = a;
    return true;
  }
  if (op.nq != 2 || op.kind == SV_G_RZZ) return false;
  const int q0 = op.q[0], q1 = op.q[1];
  if (op.kind == SV_G_CNOT) {
    const bool cfix = !sub_burst(q0, dt), tw = in_wave(q1, dt);
    if (cfix && !tw) return false;
    if (cfix) {  // control fixed to 1, X on the target
      a.low_k = 1;
      a.low_q[0] = (unsigned)q1;
      a.low_fixed = 1ull << q0;
      a.m[0] = 0.0; a.m[1] = 1.0; a.m[2] = 1.0; a.m[3] = 0.0;
    } else {
      a.low_k = 2;
      a.low_q[0] = (unsigned)q0;
      a.low_q[1] = (unsigned)q1;
      for (int i = 0; i < 16; ++i) a.m[i] = op.m[i];
    }
    *out = a;
    return true;
  }
  if (op.kind == SV_G_CZ || op.kind == SV_G_CPHASE) {
    const bool s0 = sub_burst(q0, dt), s1 = sub_burst(q1, dt);
    if (!s0 && !s1) return false;
    if (s0 && s1) {
      a.low_k = 2;
      a.low_q[0] = (unsigned)q0;
      a.low_q[1] = (unsigned)q1;
      for (int i = 0; i < 16; ++i) a.m[i] = op.m[i];
    } else {  // diag(1, phase) on the sub-burst qubit where the other is 1
      a.low_k = 1;
      a.low_q[0] = (unsigned)(s0 ? q0 : q1);
      a.low_fixed = 1ull << (s0 ? q1 : q0);
      a.m[0] = 1.0; a.m[1] = 0.0; a.m[2] = 0.0; a.m[3] = op.m[15];
    }
    *out = a;
    return true;
  }
  // SWAP changes only the (0,1) and (1,0) members: it keeps the touched
  // subset unless one qubit is inside a burst.  Dense two-qubit matrices
  // change every amplitude: lane exchange whenever a qubit is in the row.
  if (op.kind == SV_G_SWAP ? !(sub_burst(q0, dt) || sub_burst(q1, dt)) : !(in_wave(q0, dt) || in_wave(q1, dt)))
    return false;
  a.low_k = 2;
  a.low_q[0] = (unsigned)q0;
  a.low_q[1] = (unsigned)q1;
  for (int i = 0; i < 16; ++i) a.m[i] = op.m[i];
  *out = a;
  return true;
}

double touched_fraction(const Op& op) {
  switch (op.kind) {
    case SV_G_Z: case SV_G_S: case SV_G_T: case SV_G_P: case SV_G_CNOT: case SV_G_SWAP:
      return 0.5;
    case SV_G_CZ: case SV_G_CPHASE:
      return 0.25;
    default:
      return 1.0;
  }
}

}  // namespace sv
