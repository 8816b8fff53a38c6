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
inline constexpr int pass_reg_bits(sv_dtype dt) { return dt == SV_C64 ? 5 : 4; }

enum PassOpType : uint32_t {
  POP_U1 = 0,  // 2x2 on register bit b0                        (4 entries)
  POP_U2 = 1,  // 4x4 on register bits (b0 = MSB, b1)           (16 entries)
  POP_X = 2,   // exchange register pairs on bit b0              (0 entries)
  POP_CX = 3,  // exchange pairs on bit b1 where bit b0 is 1     (0 entries)
  POP_D1 = 4,  // diag(d0, d1) on register bit b0                (2 entries)
  POP_D2 = 5,  // diag(d0..d3) on register bits (b0 = MSB, b1)   (4 entries)
  POP_DG = 6,  // one phase for the whole group                  (1 entry)
  POP_UR = 7,  // real 2x2 on register bit b0 (H, RY)            (4 entries, real parts used)
  POP_UI = 8,  // 2x2 with real diagonal and imaginary off-diagonal
               // on register bit b0 (RX)                        (4 entries: re, im, im, re used)
  POP_P1 = 9,  // phase on the amplitudes whose bit b0 is 1     (1 entry)
  POP_P2 = 10, // phase on the amplitudes whose bits b0, b1 are 1 (1 entry)
  POP_LP = 11, // phase ladder on register bit b0 (the terms of a fused run of
               // phase gates that involve that bit): the amplitudes whose bit b0 is 1 are
               // multiplied by exp(2 pi i t / 2^W), t = the constant word plus
               // the angle words of the set source bits (W-bit fixed-point
               // turns, summed modulo one turn; W = 32 for complex64, 64 for
               // complex128).  Entries: kPassLPWords words, two per entry:
               // local bits 0..15, tile physical bits 0..kPassLPTileBits-1,
               // the constant.  lmask / tmask name the source bits with a
               // nonzero word (for this op they are not predicates).
  POP_DR = 12, // diagonal over the register index: amplitude r times d[r]
               // (NR entries; a run of diagonal gates on register bits)
  POP_QG = 13  // quadratic phase over the bits outside the registers (one
               // phase per lane, on all its amplitudes): exp(2 pi i t / 2^W),
               // t = the sum of the row-0 words of the set bits plus the
               // constant word, plus, for every target bit that is set, the
               // sum of its row's words of the set bits (the pair terms).
               // Rows of kPassLPWords words in the phase-ladder layout: row 0,
               // then one row per local target (ascending local bit: b0 is
               // their mask), then one per tile target (ascending physical
               // bit: b1 | pad << 32 is their mask).  lmask / tmask cover every
               // bit with a nonzero word or a row (not predicates).
};
constexpr int kPassLPLocalBits = 16;
constexpr int kPassLPTileBits = 34;
constexpr int kPassLPConst = kPassLPLocalBits + kPassLPTileBits;  // word of the constant angle
constexpr int kPassLPWords = kPassLPConst + 2;                    // (even: whole entries)
constexpr uint32_t kPassNoSel = 0xffffffffu;
constexpr uint32_t kPassTileSel = 64;  // select codes >= 64 name tile (non-local) physical bits

struct alignas(16) PassOpDev {
  uint32_t type;   // PassOpType
  uint32_t b0, b1; // register bits
  uint32_t mat;    // first complex entry in the matrix pool
  uint32_t lmask;  // local bits (outside the stage's register bits) that must all be 1
  uint32_t sa, sb; // matrix-variant selectors: local bit (< 64) or 64 + tile physical bit;
                   // variant = bit(sa) [*2 + bit(sb)]; entries of variant v at mat + v * size
  uint32_t pad;
  uint64_t tmask;  // tile (non-local) physical bits that must all be 1
};

// Rows of the stage's phase ops whose tile part is summed once per tile
// (before the stage's groups run): one per POP_LP, and per POP_QG row 0, its
// local-target rows and its tile-target rows, in op order.  A row
// descriptor is four uint32 pool words: the word index of the row's first
// tile word (counted from the stage's first pool entry, two words per entry),
// the tile bit that must be set for the row to count (kPassNoSel: always),
// and the tile mask (low, high).
constexpr int kPassStageRowsMax = 256;

struct PassStageDev {
  uint32_t q[kPassRegBitsMax];      // local bit of register bit r (r < rb)
  uint32_t qsort[kPassRegBitsMax];  // the same bits, ascending (group enumeration)
  uint32_t op_first, op_count;
  uint32_t mat_base;                // the stage's first pool entry
  uint32_t rows;                    // row descriptors: pool entry, from mat_base
  uint32_t row_count;               // <= kPassStageRowsMax
  uint32_t pad;
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
  const PassOpDev* ops;
  const void* mats;
  uint64_t tile_begin;            // first global tile of this item (ascending)
  int32_t n;                      // qubits
  int32_t pass;                   // pass of the program to run
};

// Run pass items[i].pass of every item in one launch (all items share dt).
// ladders: some item's pass holds POP_LP or POP_QG ops (selects the kernel
// variant that decodes them; the other variant carries none of their code).
hipError_t launch_pass_batch(sv_dtype dt, const BatchItemDev* items, int count, uint64_t total_tiles, int max_m,
                             bool ladders, hipStream_t s);

// Launch pass `pass` of a program already resident in device memory
// (ladders: the pass holds POP_LP or POP_QG ops).
hipError_t launch_pass(sv_dtype dt, void* psi, int n, int m, const PassDescDev* passes, int pass,
                       const PassStageDev* stages, const PassOpDev* ops, const void* mats, bool ladders,
                       hipStream_t s);

// --- dense k-qubit fused gate (3 <= k <= 6) ---------------------------------
// m_dev: device copy of the 2^k x 2^k matrix, row-major interleaved, in the
// state's precision (double for SV_C128, float for SV_C64).  mfma: complex64
// states with k >= 4 use the FP32 MFMA kernel.
hipError_t launch_dense_kq(sv_dtype dt, void* psi, int n, int k, const int* q, const void* m_dev, bool mfma,
                           hipStream_t s);

}  // namespace sv
