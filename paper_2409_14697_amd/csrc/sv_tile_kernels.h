// Host-visible launchers of the in-cache tile-pass kernels and of the dense
// k-qubit kernels (same conventions as sv_kernels.h: no validation, enqueue
// on the given stream, return the launch status).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sv.h"

namespace sv {

// --- in-cache tile passes (LDS) --------------------------------------------
// A pass loads tiles of 2^m amplitudes (local bits = physical positions
// lpos[0..m-1], ascending), runs its stages on each tile in LDS and
// registers, and stores local bit j to physical position wpos[j] (a
// permutation of lpos: qubit reordering fused into the write-back).
// A stage holds 2^rb register amplitudes per group (rb = pass_reg_bits:
// 5 for complex64, 4 for complex128): register bit r is local bit q[r];
// groups enumerate the other local bits.
constexpr int kPassRegBitsMax = 5;
constexpr int kPassLocalMax = 16;  // local bits of a tile, at most
inline constexpr int pass_reg_bits(sv_dtype dt) { return dt == SV_C64 ? 5 : 4; }

// A register stage of a tile pass applies, in this order (each part a block
// of gates in program order that the planner proved may run in that order):
//   1. optionally a dense 4x4 on register bits (1, 0)          (PSF_U2)
//   2. nsub earlier layers (PassSubDev), each one 2x2 per register bit of
//      its mask followed by a factor per register index: single-qubit gates
//      separated by diagonal gates on register bits (the Hadamard and
//      controlled-phase ladder of a QFT block, say) stay in registers
//   3. one 2x2 on every register bit: the tensor product of a layer of
//      single-qubit gates (identity on bits without a gate); `form` holds
//      three bits per register bit (bit r at 3 r) saying which entries of its
//      2x2 are nonzero or real, so the kernel runs the cheapest code for
//      each (PFORM_NONE: the bit has no gate and is skipped)
//   4. a diagonal: a factor per register index (PSF_DR) times per-lane
//      factors of the lane items (PSF_LANE): phases and diagonal gates that
//      involve bits outside the registers
//   5. an affine map of the local index, x -> M x ^ c ^ c(tile) over GF(2)
//      (the stage's X, CNOT and SWAP gates on any local bits: PSF_PERM),
//      which costs no arithmetic: the stage's LDS store writes the amplitude
//      of local index x to the address of M x ^ c ^ c(tile).  When the map
//      moves amplitudes between the lanes' groups (PSF_XPERM) every lane
//      reads its group before any lane writes.
enum PassForm : uint32_t {
  PFORM_NONE = 0,  // no 2x2 part
  PFORM_UR = 1,    // every 2x2 real (H, RY)
  PFORM_UI = 2,    // real diagonal, imaginary off-diagonal (RX, Y)
  PFORM_RC = 3,    // real diagonal, complex off-diagonal (mixtures of the two)
  PFORM_U = 4      // general complex 2x2
};
enum PassStageFlags : uint32_t {
  PSF_U2 = 1,    // dense 4x4 on register bits (1 = MSB, 0) first
  PSF_DR = 2,    // factor table over the register index
  PSF_LANE = 4,  // lane items
  PSF_F0 = 8,    // some lane item multiplies the amplitudes whose register bit is 0
  PSF_PERM = 16,  // affine map of the local index at the store
  PSF_XPERM = 32  // ... which moves amplitudes between groups
};
enum PassItemType : uint32_t {
  PIT_DG = 0,  // factor on all the lane's amplitudes: table[var] (var from sel)
  PIT_D1 = 1,  // register bit a: amplitudes with bit a = 0 times table[2 var],
               // bit a = 1 times table[2 var + 1]
  PIT_LP = 2,  // phase ladder on register bit a (the terms of a fused run of
               // phase gates that pair that bit with bits outside the
               // registers): the amplitudes whose bit a is 1 are multiplied by
               // exp(2 pi i t / 2^W), t = the constant word plus the angle
               // words of the set source bits (W-bit fixed-point turns,
               // summed modulo one turn; W = 32 for complex64, 64 for
               // complex128).  Words at mat: kPassLPWords, two per entry:
               // local bits 0..15, tile physical bits 0..kPassLPTileBits-1,
               // the constant.  lmask / tmask name the source bits with a
               // nonzero word.
  PIT_QG = 3,  // quadratic phase over the bits outside the registers (one
               // phase per lane, on all its amplitudes): exp(2 pi i t / 2^W),
               // t = the sum of the row-0 words of the set bits plus the
               // constant word, plus, for every target bit that is set, the
               // sum of its row's words of the set bits (the pair terms).
               // Rows of kPassLPWords words in the ladder layout: row 0, then
               // one row per local target (ascending local bit; `a` is their
               // mask), then one per tile target (ascending physical bit; `tt`
               // is their mask).  lmask / tmask cover every bit with a nonzero
               // word or a row.
  PIT_PX = 4   // term of the store map: when the selector (a tile bit) is 1,
               // the local index is XORed with the mask `a` (a CNOT whose
               // control lies outside the tile)
};
constexpr int kPassLPLocalBits = 16;
constexpr int kPassLPTileBits = 34;
constexpr int kPassLPConst = kPassLPLocalBits + kPassLPTileBits;  // word of the constant angle
constexpr int kPassLPWords = kPassLPConst + 2;                    // (even: whole entries)
constexpr uint32_t kPassNoSel = 0xffu;
constexpr uint32_t kPassTileSel = 64;  // selector codes >= 64 name tile (non-local) physical bits

// Selector codes of an item: sel & 0xff (first) and (sel >> 8) & 0xff
// (second); a code < 64 is a local bit outside the registers, 64 + p the tile
// physical bit p; kPassNoSel = none.  var = bit(first) [* 2 + bit(second)].
struct alignas(16) PassItemDev {
  uint32_t type;    // PassItemType
  uint32_t a;       // register bit (D1, LP), register-index mask (PX), local targets (QG)
  uint32_t mat;     // first pool entry of the item's table or words
  uint32_t sel;     // variant selectors (DG, D1, PX)
  uint32_t lmask;   // LP / QG: local source bits
  uint32_t pad;
  uint64_t tmask;   // LP / QG: tile source bits
  uint64_t tt;      // QG: tile targets
};

// Rows of the stage's fixed-point phase items whose tile part is summed once
// per tile (before the stage's groups run): one per PIT_LP, and per PIT_QG
// row 0, its local-target rows and its tile-target rows, in item order.  A
// row descriptor is four uint32 pool words: the word index of the row's
// first tile word (counted from the stage's first pool entry, two words per
// entry), the tile bit that must be set for the row to count (kPassNoSel:
// always), and the tile mask (low, high).
constexpr int kPassStageRowsMax = 256;
constexpr uint32_t kPassRowAlways = 0xffffffffu;  // row descriptor: no gating tile bit

// An earlier layer of a stage: 2x2s (form, mask and pool entry as for the
// stage's last layer), then the register factors at pool entry `dr`
// (kPassNoTable: none).
constexpr int kPassSubMax = 4;
constexpr uint32_t kPassNoTable = 0xffffffffu;
struct PassSubDev {
  uint32_t form, slot_mask, slots, dr;  // form: three bits per register bit
};
constexpr int kPassFormBits = 3;  // bits of one register bit's PassForm in a form word
inline constexpr uint32_t pass_form_of(uint32_t word, int r) { return (word >> (kPassFormBits * r)) & 7u; }

struct alignas(16) PassStageDev {
  uint32_t q[kPassRegBitsMax];      // local bit of register bit r (r < rb)
  uint32_t qsort[kPassRegBitsMax];  // the same bits, ascending (group enumeration)
  uint32_t form;                    // PassForm of each register bit (kPassFormBits each, bit 0 lowest)
  uint32_t flags;                   // PassStageFlags
  uint32_t slots;                   // pool entry of the 2x2s: 4 per register bit, bit 0 first
  uint32_t u2;                      // pool entry of the 4x4 (16 entries, row-major)
  uint32_t dr;                      // pool entry of the register factors (2^rb entries)
  uint32_t item_first, item_count;  // lane items
  uint32_t px_first, px_count;      // permutation terms (PIT_PX items)
  uint32_t mat_base;                // the stage's first pool entry
  uint32_t rows;                    // row descriptors: pool entry, from mat_base
  uint32_t row_count;               // <= kPassStageRowsMax
  uint32_t colimg[kPassLocalMax];   // store map: image of local bit l (M e_l, a local mask)
  uint32_t pconst;                  // store map: constant XOR (local mask)
  uint32_t slot_mask;               // register bits whose 2x2 is not the identity
  uint32_t nsub;                    // earlier layers (<= kPassSubMax)
  PassSubDev sub[kPassSubMax];
};

// PassDescDev flag: the store can walk the tile in load order (the lowest
// three 16-byte element bits keep their positions, so every run of 8 lanes
// still writes 128 contiguous bytes); otherwise it walks destination order.
constexpr uint32_t kPassStoreLaneOrder = 1;

struct alignas(16) PassDescDev {
  uint32_t m;                    // local bits per tile
  uint32_t stage_first, stage_count;
  uint32_t flags;                // kPassStoreLaneOrder
  uint64_t lmask;                // physical mask of the local bits
  uint32_t lpos[16];             // physical position of local bit j on load (ascending)
  uint32_t wpos[16];             // physical position of local bit j on store (a permutation of lpos)
  uint32_t winv[16];             // local bit stored to position lpos[k] (wpos[winv[k]] = lpos[k])
};

// One state in a batched pass launch (device-resident array).
struct alignas(16) BatchItemDev {
  void* psi;                      // state amplitudes
  const PassDescDev* passes;      // the state's program
  const PassStageDev* stages;
  const PassItemDev* items;
  const void* mats;
  uint64_t tile_begin;            // first global tile of this item (ascending)
  int32_t n;                      // qubits
  int32_t pass;                   // pass of the program to run
};

// Run pass items[i].pass of every item in one launch (all items share dt).
// ladders: some item's pass holds PIT_LP or PIT_QG items (selects the kernel
// variant that decodes them; the other variant carries none of their code).
hipError_t launch_pass_batch(sv_dtype dt, const BatchItemDev* items, int count, uint64_t total_tiles, int max_m,
                             bool ladders, hipStream_t s);

// Launch pass `pass` of a program already resident in device memory
// (ladders: the pass holds PIT_LP or PIT_QG items).
hipError_t launch_pass(sv_dtype dt, void* psi, int n, int m, const PassDescDev* passes, int pass,
                       const PassStageDev* stages, const PassItemDev* items, const void* mats, bool ladders,
                       hipStream_t s);

// --- matrix passes -----------------------------------------------------------
// A matrix pass applies its stages, each a dense 2^k x 2^k op on k local bits
// of the tile, on the matrix cores (complex64: k = 5, FP32 MFMA; complex128:
// k = 4 or 5, FP64 MFMA).  Stage s (PassStageDev stage_first + s): q[b] = the
// local bit of member bit b (b = 0 least significant), u2 = pool entry of the
// matrix (row-major, rows and columns indexed by members), colimg and flags
// as below.  Every other PassStageDev field is unused.  The tile and the A
// fragments of all stages share one block's LDS, kMatrixPassLds bytes at
// most; 2^(m-k) must be at least four column blocks of the instruction
// (complex64 m >= 12; complex128 m >= k + 6).  The write-back stores every
// element where it was loaded from (the planner gives matrix passes
// wpos = lpos).
// Column order of a matrix stage: colimg[j] = the local bit of column bit j
// (the columns are the tile's other local bits: first the lane bits, log2 of
// the instruction's column count, then the wave bits, then the rest); wave w
// of kMatrixWaves owns the columns whose wave bits spell w.  Stage flag
// kMatrixStageSync: a barrier precedes the stage.  Consecutive stages without
// it have the same wave bits, none of them a member bit of either stage, so
// every wave keeps the same elements and runs those stages without waiting
// for the others.
constexpr uint32_t kMatrixStageSync = 1;
constexpr int kMatrixWaves = 8;
constexpr int kMatrixPassLds = 160 * 1024;
constexpr int kMatrixStageTable = 768;  // bytes of a stage's address table
// Stages of width k that fit beside a tile of 2^m amplitudes (A fragments:
// 2^k x 2^k complex entries per stage, and the stage's address table).
inline int matrix_pass_max_stages(sv_dtype dt, int k, int m) {
  const size_t eb = dt == SV_C64 ? 8 : 16;
  const size_t tile = ((size_t)1 << m) * eb, stage = ((size_t)1 << (2 * k)) * eb + kMatrixStageTable;
  return tile >= (size_t)kMatrixPassLds ? 0 : (int)(((size_t)kMatrixPassLds - tile) / stage);
}
hipError_t launch_matrix_pass(sv_dtype dt, int k, void* psi, int n, int m, const PassDescDev* passes, int pass,
                              int n_stages, const PassStageDev* stages, const void* mats, hipStream_t s);

// --- dense k-qubit fused gate (3 <= k <= 6) ---------------------------------
// m_dev: device copy of the 2^k x 2^k matrix, row-major interleaved, in the
// state's precision (double for SV_C128, float for SV_C64).  mfma: complex64
// states with k >= 4 use the FP32 MFMA kernel.
hipError_t launch_dense_kq(sv_dtype dt, void* psi, int n, int k, const int* q, const void* m_dev, bool mfma,
                           hipStream_t s);

}  // namespace sv
