// Device-side encoding of a fused tile pass, shared by the host planner and the kernels.
//
// A tile pass covers the state in tiles of 2^m amplitudes.  The tile's qubits T (a
// 64-bit mask, always containing the lowest qubits so loads stay coalesced) are its
// "local" bits: tile-local index j has bit i <-> the i-th lowest qubit of T.  Every other
// bit of a global index x is fixed per tile (the tile's "base").  A workgroup loads one
// tile into LDS, runs the pass's op list on it, and writes it back.
#pragma once
#include <stdint.h>

namespace qsv {

enum OpType : int32_t {
  OP_DENSE1 = 0,  // 2x2 complex matrix on local bit a
  OP_DENSE2 = 1,  // 4x4 complex matrix on local bits a (row/col bit 0) and b (bit 1)
  OP_DIAG = 2,    // run of diagonal gates: DiagEntry[first .. first+count)
  OP_ZZ = 3,      // exp(-i theta/2 * sum_e Z_u Z_v) over EdgeTable[first .. first+count):
                  // amplitude x is multiplied by ctab[mat + c(x)], c(x) = #edges with
                  // x_u != x_v.  In register-blocked passes the edges are sorted by class
                  // (ZZEdge::tmask etc.): class i (the i-th register-bit mask with at most
                  // two bits) has byte i of (a, b, lmask) edges
  OP_REMAP = 4,   // register-blocked passes: move amplitudes through LDS into a new
                  // layout: register (slot) bit i holds local bit (b >> 8i) & 255, thread
                  // bit t holds local bit (omask >> 4t) & 15; `a` is the register mask
  OP_XSWAP = 5,   // register-blocked passes: one transposition, `mat` = slot bit (low 2
                  // bits) | lane bit (4 or 5) << 4, exchanging the local bit on a register
                  // slot bit with the one on lane bit 4 or 5 of the wave by cross-lane moves
                  // (no LDS); the layout after it is given as for OP_REMAP (count = 1)
  OP_BLOCK = 6,   // register-blocked forward passes: a dense 8x8 complex matrix on the local
                  // bits of lane bit 4 (block index bit 0), lane bit 5 (bit 1) and register
                  // slot bit `a` (bit 2), applied with matrix-core instructions (16x16x4):
                  // ctab[mat .. mat + 128) holds its real 16x16 form as each lane's four
                  // A-operand values, lane-major (see block_operands)
};
// In register-blocked passes each thread holds 2^RB amplitudes; DENSE1 then names a
// register-bit index (a in [0, RB)) instead of a local bit, and the other ops are
// elementwise.  A DENSE1 op with b = 1 first applies the sign-only diagonal run
// DiagEntry[first .. first+count) (the flush that the gate required).  The initial (load)
// layout is PassArgs::lr0.

// Matrices, phases and generator weights live in a per-batch-item table of complex
// numbers (ctab); ops refer to it by offset.
// Register-blocked passes: bit 31 of TileOp::lmask is set when omask is not 0, so ops
// without outside controls skip reading it.
constexpr uint32_t kHasOutsideControls = 0x80000000u;

struct TileOp {
  // Register-blocked passes: a run of sign flips alone has plain = kPlainSigns.  A one-qubit
  // gate on a register slot without controls, optionally after a run of sign flips
  // (kPlainSigns), has plain = 1 + slot (| kPlainSigns)
  // | the form of its matrix (kPlainForm bits): kPlainSplit, a phase on the slot's 1 half
  // then a real 2x2 matrix (ctab[mat] = (R00, R01), ctab[mat + 1] = (R10, R11), ctab[mat + 2]
  // = the phase); kPlainReal, a real matrix (RY, H, X); kPlainXlike, real diagonal and
  // imaginary off-diagonal entries (RX, Y); none: a general 2x2.  A fused block has plain =
  // kPlainBlock | (1 + slot) (| kPlainSigns).  The kernel reads the first eight fields at once
  // and decodes nothing else for these ops.  0 for every other op.
  int32_t  plain;
  int32_t  mat;        // ctab offset of the matrix (DENSE) or phase table (ZZ)
  int32_t  first;      // DIAG / ZZ / sign runs: first entry
  int32_t  count;      // DIAG / ZZ / sign runs: number of entries
  int32_t  gen;        // adjoint: ctab offset of the scaled generator (DENSE: 4/16 entries,
                       // ZZ: count+1 real weights in .x), -1 if no gradient here
  int32_t  pslot;      // adjoint: output column of the accumulated gradient (or -1)
  int32_t  flush;      // adjoint: reduce the accumulator into pslot after this op
  int32_t  gkind;      // adjoint DENSE1: the generator's form (GEN_*), for a cheaper
                       // gradient term than the general 2x2 product
  int32_t  type;
  int32_t  a, b;       // local target bits (DENSE1 / DENSE2)
  uint32_t lmask;      // controls on local bits, in j-space: apply where (j & lmask) == lmask
  uint64_t omask;      // controls on bits outside the tile: apply iff (base & omask) == omask
};
constexpr int32_t kPlainSigns = 8, kPlainBlock = 16;
constexpr int32_t kPlainSplit = 32, kPlainReal = 64, kPlainXlike = 96, kPlainForm = 96;
static_assert(offsetof(TileOp, plain) == 0 && offsetof(TileOp, gkind) == 28 && alignof(TileOp) == 8,
              "plain .. gkind form the record's first 32 bytes");
// Generator forms of DENSE1 ops (k = the chain-rule factor, read from the generator table):
// GEN_GENERAL: any 2x2; GEN_X: k X (ctab[gen + 1] = k); GEN_Y: k Y (ctab[gen + 2] = i k).
enum GenForm : int32_t { GEN_GENERAL = 0, GEN_X = 1, GEN_Y = 2 };

// One diagonal gate inside an OP_DIAG run.  The gate's qubits q0, q1 (q1 = -1 for one
// qubit) and control mask are global positions; the phase applied to amplitude x is
// ctab[mat + ((x>>q1 & 1) << 1 | (x>>q0 & 1))] when all control bits of x are set.
// kind SIGN: the phase is -1 when all bits of smask are set in x, 1 otherwise (Z, CZ,
// multi-controlled Z), and no table is read.
enum DiagKind : int32_t { DIAG_PHASE = 0, DIAG_SIGN = 1 };
struct DiagEntry {
  int32_t  kind;
  int32_t  q0, q1;
  int32_t  mat;
  uint64_t cmask;      // PHASE: controls; SIGN: all bits that must be 1
  int32_t  gen;        // adjoint: ctab offset of 4 real generator weights (.x), or -1
  // The same entry relative to its pass's tile (used by register-blocked passes, which
  // index amplitudes by tile-local position): l0 / l1 are the local bits of q0 / q1 (-1
  // when the qubit lies outside the tile, whose bit then comes from the tile's base);
  // lcmask / ocmask split cmask into local bits and outside (global) bits.
  int32_t  l0, l1;
  uint32_t lcmask;
  uint64_t ocmask;
  // Register-blocked passes, for the register layout in force when the entry runs:
  // tmask = the bits of lcmask that are thread-index bits; kmask bit k is set when
  // register slot k has every register bit of lcmask set.  The local condition
  // (j & lcmask) == lcmask then reads ((j_thread & tmask) == tmask) && (kmask >> k & 1).
  uint32_t tmask, kmask;
};

// One edge of an OP_ZZ run: global qubits (u, v) and their local bits in the pass's tile
// (lu, lv; -1 when outside the tile).  For register-blocked passes, in the register layout
// in force when the op runs: tmask = the endpoints that are thread-index bits (local bit
// positions), omask = the endpoints outside the tile (global bits); the endpoints that are
// register bits define the edge's class, the 3-bit mask with bit r set for each endpoint on
// register bit r.  The edge differs in register slot k iff
// popcount(j_thread & tmask) + popcount(base & omask) + popcount(k & class) is odd.
struct ZZEdge {
  int32_t  u, v, lu, lv;
  uint32_t tmask, pad;
  uint64_t omask;
};

// Planner tables per register-blocked pass (entries of 64 bits):
//   [0, 256)    where local index j is read: entry j & 127 ORed with entry 128 + (j >> 7)
//   [256, 512)  where local index j is written (the same tables unless the pass relayouts)
//   kRunsLogical, kRunsLoad, kRunsStore: a run count, then up to kMaxRuns runs
//               lo | len << 8 | shift << 16, each putting tile-index bits
//               [shift, shift + len) at bits [lo, lo + len) of the tile's base: the logical
//               base (qubit values, for controls and phases), and the bases read and written
constexpr int kRunsLogical = 512, kRunsLoad = 544, kRunsStore = 576, kMaxRuns = 31;
constexpr int kDepEntries = 608;

// Largest ctab window (complex entries) a register-blocked pass stages in LDS.
constexpr int kMaxWindow = 256;

struct PassArgs {
  void*        psi;           // state(s), batch item b at psi + b * bstride amplitudes
  void*        lam;           // adjoint: costate(s), same layout
  const void*  src;           // first forward pass: read from src (+ b * src_bstride)
  void*        dst;           // written instead of psi when not null (relayouting passes)
  int64_t      bstride;
  int64_t      src_bstride;
  const TileOp*    ops;
  const DiagEntry* diag;
  const ZZEdge*    edges;
  const uint64_t*  dep;       // register-blocked: kDepEntries per pass (deposits of local
                              // indices, 256 entries; runs of outside bits, from entry 256)
  const void*  ctab;          // per batch item: ctab + b * ctab_bstride complex entries
  int64_t      ctab_bstride;
  double*      partials;      // adjoint: [batch][n_pslots][n_tiles]
  uint64_t     tile_mask;
  int32_t      n_ops;
  int32_t      n_qubits;
  int32_t      m;             // tile qubits = popcount(tile_mask)
  int32_t      n_pslots;
  int32_t      lr0;           // register-blocked passes: local register mask at load time
  uint32_t     lay0_reg;      // register-blocked passes: load layout, packed as OP_REMAP's b
  uint64_t     lay0_thr;      //   and omask
  int32_t      win_n;         // register-blocked passes: ctab entries [win_lo, win_lo + win_n)
                              // copied to LDS for per-lane table lookups (0: read ctab)
  int64_t      n_tiles;       // tiles of this state (column length of partials)
  int64_t      win_lo;
  int32_t      pass_pslots;   // adjoint: gradient slots (pslot values) used by this pass
  int32_t      relayout;      // 1: stores use their own tables and base (see kDepEntries)
};

// Adjoint register-blocked passes keep each gradient slot's per-wave sums in LDS until the
// end of the pass when pass_pslots x waves fits in this many doubles (else each slot is
// reduced across the workgroup when it is complete).
constexpr int kMaxDeferredSums = 2048;

// One circuit's share of a multi-circuit Pauli-sum pass: lambda = H psi and the
// expectation partials of 2^n amplitudes, in chunks of one workgroup each.
struct PauliJob {
  const void*     psi;
  void*           lam;
  const uint64_t* xmasks;     // terms
  const uint64_t* zmasks;
  const double*   cre;        // coefficient * i^{popcount(x & z)}
  const double*   cim;
  double*         partials;   // two doubles (re, im) per chunk
  int32_t         n_terms;
  int32_t         n_qubits;
};

// Pauli-sum pass over one group of terms sharing an x-mask.
struct PauliGroupArgs {
  const void*  psi;
  void*        lam;           // output H psi (or NULL for expectation only)
  int64_t      bstride;
  const uint64_t* zmasks;     // terms of the group
  const double*   cre;        // coefficient * i^{popcount(x & z)} (real part)
  const double*   cim;        // (imaginary part)
  double*      partials;      // [batch][ncols][nblocks]; this group writes columns col, col+1
  uint64_t     xmask;
  int32_t      n_terms;
  int32_t      n_qubits;
  int32_t      accumulate;    // lam += (1) or lam = (0)
  int32_t      col;           // first partial column (real part; imaginary part at col + 1)
  int32_t      ncols;
  int32_t      real_coeffs;   // 1 when every cim is 0 (the imaginary part is not accumulated)
  // Diagonal groups over n >= 12 qubits (n_pats > 0): the terms sorted by their pattern on
  // the 12 low qubits; pats[p] = pattern | (index of its first term) << 12, and the patterns
  // whose bits 8-11 equal r are pats[rfirst[r] .. rfirst[r + 1]) (r = 0..15).  The pass
  // walks such a group by pattern when its coefficients are real (always, for the real
  // coefficients the ABI takes), with the term table in LDS up to 512 terms.
  const uint32_t* pats;
  const int32_t*  rfirst;
  int32_t      n_pats;
};
constexpr int kPauliMaxPatterns = 256;

}  // namespace qsv
