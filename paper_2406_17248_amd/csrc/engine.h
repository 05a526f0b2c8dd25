// Host side of the engine: gate lowering, tile-pass planning and parameter binding.
// Pure C++ (no HIP calls), so it runs and is tested on machines without a GPU.
#pragma once
#include <complex>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/qsv.h"
#include "qsv_ops.h"

namespace qsv {

using cplx = std::complex<double>;

// Thrown inside the library only; converted to a status code at the ABI boundary.
struct Error {
  int status;
  std::string msg;
};

// Generator G of a rotation exp(-i theta G / 2) (times the control projector): the
// adjoint-method gradient of an angle is Im<lambda|G|psi> at the point after the gate.
enum GenKind : int32_t {
  G_NONE = 0, G_X, G_Y, G_Z, G_XX, G_YY, G_ZZ,
  G_PS,      // diag(0, -2): PhaseShift(theta) = exp(-i theta diag(0,-2) / 2)
};

// How a primitive's numbers are formed at bind time.
enum MatRecipe : int32_t {
  M_GATE = 0,    // the gate's own matrix (all angles)
  M_RZ_ANGLE,    // RZ(angle[angle_slot]) - parts of a lowered U3
  M_RY_ANGLE,    // RY(angle[angle_slot])
  M_SIGN,        // no numbers (sign flip)
  M_H,           // Hadamard (basis change of a lowered RXX)
  M_RX_PLUS,     // RX(+pi/2) (basis change of a lowered RYY)
  M_RX_MINUS,    // RX(-pi/2)
  M_ZZ_ANGLE,    // diag(e^{-i a/2}, e^{i a/2}, e^{i a/2}, e^{-i a/2}), a = angle[0]
};

enum PrimType : int32_t { P_DENSE1 = 0, P_DENSE2, P_DIAG1, P_DIAG2, P_SIGN };

struct Prim {
  int32_t  type;
  int32_t  gate;        // source gate index
  int32_t  q0, q1;      // targets (q1 = -1 for one qubit)
  uint64_t cmask;       // controls (P_SIGN: every bit that must be 1)
  int32_t  recipe;
  int32_t  angle_slot;
  bool     dagger;
  int32_t  gen;         // GenKind
  int32_t  param;       // parameter index receiving the gradient (-1: none)
  double   coeff;       // chain-rule factor d angle / d param
  // planning masks
  uint64_t nondiag;     // qubits acted on non-diagonally (must be tile qubits)
  uint64_t touched;     // every qubit involved (targets and controls)
};

struct Pass {
  uint64_t tile_mask = 0;
  int32_t  m = 0;
  std::vector<int32_t> prims;  // primitive indices in execution order
};

// Where a ctab entry block comes from at bind time.
enum FillKind : int32_t {
  F_PRIM_MATRIX = 0,  // the primitive's matrix: 4 (dense1), 16 (dense2), 2 or 4 (diag) entries
  F_PRIM_GEN,         // coeff * generator of the primitive: same sizes (diag: real weights)
  F_ZZ_PHASES,        // exp(-+ i theta/2 (E - 2c)), c = 0..E (sign by dagger)
  F_ZZ_GEN,           // coeff * (E - 2c) as real weights
  F_BLOCK,            // the product of a fused block's primitives as matrix-core operands
                      // (Fill::prim indexes Plan::blocks; 128 entries)
  F_GATE_CHAIN,       // a one-qubit gate of a phase chain (Plan::split): its matrix times the
                      // phase its qubit carries from the previous gate of the chain; count = 1:
                      // split into (real matrix, phase), the left phase carried on, count = 0:
                      // the chain's last gate, dense (4 entries either way)
};
struct Fill {
  int32_t kind;
  int32_t prim;       // primitive (for ZZ runs: the first RZZ of the run)
  int32_t count;      // ZZ: number of edges
  int32_t offset;     // ctab offset (complex entries)
};

// Register-blocked layout of a pass's tile: slot bit i of a thread's register block holds
// local bit reg[i]; thread-index bit t holds local bit thr[t] (t < 6: a lane bit of the
// wave, so amplitudes on it can trade places with a slot by cross-lane moves; higher t:
// the wave within the workgroup, reachable only through LDS).
struct RbLayout {
  int32_t r = 0, nt = 0;
  int32_t reg[4] = {0, 0, 0, 0};
  int32_t thr[16] = {};
  uint32_t regmask() const {
    uint32_t m = 0;
    for (int i = 0; i < r; ++i) m |= 1u << reg[i];
    return m;
  }
  uint32_t regpack() const {
    uint32_t p = 0;
    for (int i = 0; i < r; ++i) p |= (uint32_t)reg[i] << (8 * i);
    return p;
  }
  uint64_t thrpack() const {
    uint64_t p = 0;
    for (int t = 0; t < nt; ++t) p |= (uint64_t)thr[t] << (4 * t);
    return p;
  }
  int slot_of(int bit) const {
    for (int i = 0; i < r; ++i)
      if (reg[i] == bit) return i;
    return -1;
  }
  int thread_pos_of(int bit) const {
    for (int t = 0; t < nt; ++t)
      if (thr[t] == bit) return t;
    return -1;
  }
  int lanes() const { return nt < 6 ? nt : 6; }
  // thread bits a cross-lane transposition can use: lane bits 4 and 5 (the row and
  // half-wave swaps); the others cost more VALU work than an LDS remap, which runs beside
  // other waves' arithmetic
  bool swappable(int t) const { return (t == 4 || t == 5) && t < nt; }
};
// Register bits = the set bits of lr (ascending), thread bits = the other local bits
// (ascending).
RbLayout canonical_layout(uint32_t lr, int m, int r);

struct DevPass {
  uint64_t tile_mask;
  int32_t  m;
  int32_t  maxm;       // LDS capacity instantiation
  int32_t  rb;         // register-blocked kernel: its register bits (3 or 4); 0: LDS sweep
  int32_t  lr0;        // register-blocked: local register mask at load time
  uint32_t lay0_reg;   // register-blocked: load layout (RbLayout::regpack / thrpack)
  uint64_t lay0_thr;
  int32_t  op_first, op_count;
  int32_t  pslot_first, pslot_count;
  int32_t  win_lo, win_n;  // register-blocked: ctab window of the pass's per-lane lookups
  int32_t  dep_first;      // register-blocked: first of the pass's kDepEntries Plan::deps entries
  int32_t  relayout;       // register-blocked: stores go to another layout (and buffer)
};

// A fully planned execution (forward or adjoint reverse sweep) of one circuit structure.
// A fused block of primitives applied as one dense 8x8 matrix: q[b] is the global qubit of
// block index bit b (b = 0, 1 on lane bits 4 and 5, b = 2 on a register slot bit).
struct BlockSpec {
  int32_t q[3];
  std::vector<int32_t> prims;  // in execution order
};

struct Plan {
  bool adjoint = false;
  int32_t dtype = 1;
  bool unfused = false;     // per-primitive streaming kernels
  int32_t n_qubits = 0;
  std::vector<Prim> prims;
  std::vector<DevPass> passes;
  // register-blocked passes, kDepEntries per pass (layout in qsv_ops.h): where each local
  // index is read and written, and runs forming a tile's logical, load and store bases
  std::vector<uint64_t> deps;
  // forward passes move the state between bit layouts (pass p stores in a layout whose low
  // bits are pass p+1's tile); the first pass reads and the last writes the natural layout
  bool relayout = false;
  std::vector<TileOp> ops;
  std::vector<DiagEntry> diag;
  std::vector<ZZEdge> edges;
  std::vector<Fill> fills;
  std::vector<BlockSpec> blocks;    // fused blocks (OP_BLOCK)
  int32_t ctab_size = 0;            // complex entries per batch item
  std::vector<int32_t> pslot_param; // adjoint: parameter of each gradient slot
  int32_t n_pslots = 0;
  // unfused: one streaming launch per primitive
  std::vector<int32_t> stream_mat;  // ctab offset per primitive
  std::vector<int32_t> stream_diag; // diag entry per primitive (diag types)
};

struct PlanOptions {
  int32_t tile_qubits = 12;   // 0: unfused
  int32_t low_qubits = 3;     // always in the tile (coalescing)
  bool    fuse_zz = true;     // fuse runs of equally-bound RZZ into one phase-table op
  int32_t dtype = 1;
  bool    use_rb = true;      // register-blocked kernel for tiles of rb_min..13 qubits
  int32_t rb_min = 9;         // smallest register-blocked tile (smaller ones idle threads)
  int32_t reg_bits = 3;       // register bits of register-blocked passes (3, or 4 forward)
  bool    relayout = false;   // forward register-blocked plans: relayout between passes
  bool    blocks = false;     // forward register-blocked plans: fuse the one-qubit gates of
                              // three-qubit rounds into 8x8 blocks on the matrix cores
  double  block_min_gates = 3.0;  // ... keeping a round's blocks when they average this many
                                  // one-qubit gates
  bool    split = false;      // forward register-blocked plans without blocks: uncontrolled
                              // one-qubit gates followed on their qubit by another such gate
                              // run as a phase and a real 2x2 matrix; the rest of the gate (a
                              // diagonal) is carried into the qubit's next gate
};

// Block index bit b of an 8x8 fused block and the real 16x16 matrix-core operands: the real
// row of (block index beta, real/imaginary part ri) is (beta & 3) + 4 ri + 8 (beta >> 2); lane
// l's A operand for k-chunk j (j = 0..3) is row l % 16, column 4 j + l / 16 of the matrix
// whose rows are permuted as the accumulator layout of the amplitude type requires
// (complex64: accumulator row 4q + v holds real row q + 4v; complex128: row r holds row r).
// out receives 256 reals, lane-major (lane l's four values at 4l).
void block_operands(const cplx* M8, int dtype, double* out);

// A unitary 2x2 M (row-major) as diag(left[0], left[1]) R diag(1, out[2]) with R real: out[0] =
// (R00, R01) and out[1] = (R10, R11) as complex pairs of reals.
void split_gate(const cplx* M, cplx* left, cplx* out);

// Default tile widths of forward and adjoint plans, measured on the 30-qubit brick circuit
// (forward) and the 24-qubit QAOA batch (adjoint): wider tiles save passes but need more
// REMAPs per pass.
int32_t default_tile_qubits(int32_t dtype);
int32_t default_adj_tile_qubits(int32_t dtype);
// Plan options of a state's forward or adjoint plan, from its dtype, qubit count and tile
// width options (the one place these rules live, used by the library and the host checks).
PlanOptions state_plan_options(int32_t dtype, int32_t n, int32_t tile, int32_t adj_tile, bool adjoint, bool fuse_zz,
                               bool relayout);

// Validate a circuit against n_params (and the state's n).  Throws Error.
void validate_circuit(const qsv_circuit* c, size_t n_params, int32_t n_state);
void validate_pauli_sum(const qsv_pauli_sum* h, int32_t n);

// Lower gates into primitives: forward order, or the adjoint reverse sweep (daggered,
// with generators).
std::vector<Prim> lower_forward(const qsv_circuit* c);
std::vector<Prim> lower_adjoint(const qsv_circuit* c);

// Group primitives into tile passes (greedy; each pass maximizes the dense primitives it
// can execute given the order constraints).
std::vector<Pass> plan_passes(const std::vector<Prim>& prims, int32_t n, int32_t m, int32_t low_qubits);

// Smallest LDS tile instantiation (in qubits) holding 2^m amplitudes of each staged state
// (one for forward passes, psi and lambda for the adjoint) within 128 KiB, or -1.
int tile_capacity_host(int dtype, bool adj, int m);

// Register-blocked passes: 3 register bits (4 for complex64 forward passes when asked
// for); used for tiles of 9..13 qubits within 128 KiB.
constexpr int kRegBits = 3;
int rb_capacity_host(int dtype, int m, int reg_bits = kRegBits);

// Register rounds of one register-blocked pass: groups of the pass's primitives whose
// one-qubit dense targets fit in r register qubits (drawn from `allowed`).
std::vector<Pass> plan_rounds(const std::vector<Prim>& prims, const std::vector<int32_t>& seq, uint64_t allowed,
                              int32_t r);

// Full plan (passes + device op lists + binding recipe).
Plan build_plan(const qsv_circuit* c, bool adjoint, const PlanOptions& opt);

// Structure key for plan caching.
std::string structure_key(const qsv_circuit* c, bool adjoint, const PlanOptions& opt);

// Fill one batch item's complex table (fp64) for the given parameter values; angle
// overrides (for parameter shift) replace the bound angle of (gate, slot).
struct AngleOverride { int32_t gate; int32_t slot; double angle; };
void bind_ctab(const Plan& p, const qsv_circuit* c, const double* params,
               const AngleOverride* ov, int n_ov, cplx* out);

// Bound angles of one gate.
void gate_angles(const qsv_gate& g, const double* params, double out[3]);

// Pauli sum grouped by x-mask.
struct PauliGroup {
  uint64_t xmask;
  std::vector<uint64_t> zmasks;
  std::vector<double> cre, cim;   // coeff * i^{popcount(xmask & zmask)}
};
std::vector<PauliGroup> group_pauli_sum(const qsv_pauli_sum* h);

}  // namespace qsv
