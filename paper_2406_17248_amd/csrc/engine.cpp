// Gate lowering, tile-pass planning and parameter binding (host, pure C++).
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <sstream>

namespace qsv {

namespace {

const int kNAngles[QSV_GATE_KIND_COUNT] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 3, 0, 0, 0};
const int kNTargets[QSV_GATE_KIND_COUNT] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 1, 2, 1, 2};

const cplx I1(0.0, 1.0);

[[noreturn]] void fail(int status, const std::string& msg) { throw Error{status, msg}; }

int popc(uint64_t v) { return __builtin_popcountll(v); }

bool mat_is_diagonal(const qsv_circuit* c, const qsv_gate& g) {
  const int d = g.kind == QSV_GATE_MAT1 ? 2 : 4;
  const double* m = c->matrices + 2 * g.matrix_offset;
  for (int r = 0; r < d; ++r)
    for (int k = 0; k < d; ++k)
      if (r != k && (m[2 * (r * d + k)] != 0.0 || m[2 * (r * d + k) + 1] != 0.0)) return false;
  return true;
}

// A MAT1 matrix that is unitary to rounding (the split of one-qubit gates into phases and a
// real matrix reproduces only unitary matrices).
bool mat1_is_unitary(const qsv_circuit* c, const qsv_gate& g) {
  const double* m = c->matrices + 2 * g.matrix_offset;
  const cplx u[4] = {cplx(m[0], m[1]), cplx(m[2], m[3]), cplx(m[4], m[5]), cplx(m[6], m[7])};
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 2; ++k) {
      const cplx e = u[2 * r] * std::conj(u[2 * k]) + u[2 * r + 1] * std::conj(u[2 * k + 1]);
      if (std::abs(e - (r == k ? 1.0 : 0.0)) > 4e-15) return false;
    }
  return true;
}

bool kind_is_diagonal(const qsv_circuit* c, const qsv_gate& g) {
  switch (g.kind) {
    case QSV_GATE_Z: case QSV_GATE_S: case QSV_GATE_SDG: case QSV_GATE_T: case QSV_GATE_TDG:
    case QSV_GATE_RZ: case QSV_GATE_PS: case QSV_GATE_RZZ:
      return true;
    case QSV_GATE_MAT1: case QSV_GATE_MAT2:
      return mat_is_diagonal(c, g);
    default:
      return false;
  }
}

uint64_t target_mask(const qsv_gate& g) {
  uint64_t m = 1ull << g.targets[0];
  if (kNTargets[g.kind] == 2) m |= 1ull << g.targets[1];
  return m;
}

void finish_masks(Prim& p) {
  uint64_t t = 1ull << p.q0;
  if (p.q1 >= 0) t |= 1ull << p.q1;
  if (p.type == P_SIGN) {
    p.nondiag = 0;
    p.touched = p.cmask;
  } else {
    p.nondiag = (p.type == P_DENSE1 || p.type == P_DENSE2) ? t : 0;
    p.touched = t | p.cmask;
  }
}

Prim forward_prim(const qsv_circuit* c, int i) {
  const qsv_gate& g = c->gates[i];
  Prim p{};
  p.gate = i;
  p.q0 = g.targets[0];
  p.q1 = kNTargets[g.kind] == 2 ? g.targets[1] : -1;
  p.cmask = g.ctrl_mask;
  p.recipe = M_GATE;
  p.angle_slot = 0;
  p.dagger = false;
  p.gen = G_NONE;
  p.param = -1;
  p.coeff = 0.0;
  if (g.kind == QSV_GATE_Z) {
    p.type = P_SIGN;
    p.recipe = M_SIGN;
    p.cmask = g.ctrl_mask | (1ull << g.targets[0]);
  } else if (kind_is_diagonal(c, g)) {
    p.type = kNTargets[g.kind] == 2 ? P_DIAG2 : P_DIAG1;
  } else {
    p.type = kNTargets[g.kind] == 2 ? P_DENSE2 : P_DENSE1;
  }
  finish_masks(p);
  return p;
}

int32_t gen_of_kind(int kind) {
  switch (kind) {
    case QSV_GATE_RX: return G_X;
    case QSV_GATE_RY: return G_Y;
    case QSV_GATE_RZ: return G_Z;
    case QSV_GATE_PS: return G_PS;
    case QSV_GATE_RXX: return G_XX;
    case QSV_GATE_RYY: return G_YY;
    case QSV_GATE_RZZ: return G_ZZ;
    default: return G_NONE;
  }
}

// ---- matrices ----------------------------------------------------------------------------
// dense 2x2 / 4x4 row-major; diagonal kinds return the diagonal only.
int gate_numbers(const qsv_circuit* c, const qsv_gate& g, const double* ang, cplx* out) {
  const double h = 0.5 * ang[0];
  switch (g.kind) {
    case QSV_GATE_X: out[0] = 0; out[1] = 1; out[2] = 1; out[3] = 0; return 4;
    case QSV_GATE_Y: out[0] = 0; out[1] = -I1; out[2] = I1; out[3] = 0; return 4;
    case QSV_GATE_H: {
      const double r = std::sqrt(0.5);
      out[0] = r; out[1] = r; out[2] = r; out[3] = -r; return 4;
    }
    case QSV_GATE_S: out[0] = 1; out[1] = I1; return 2;
    case QSV_GATE_SDG: out[0] = 1; out[1] = -I1; return 2;
    case QSV_GATE_T: out[0] = 1; out[1] = std::polar(1.0, M_PI / 4); return 2;
    case QSV_GATE_TDG: out[0] = 1; out[1] = std::polar(1.0, -M_PI / 4); return 2;
    case QSV_GATE_RX: out[0] = std::cos(h); out[1] = -I1 * std::sin(h); out[2] = -I1 * std::sin(h); out[3] = std::cos(h); return 4;
    case QSV_GATE_RY: out[0] = std::cos(h); out[1] = -std::sin(h); out[2] = std::sin(h); out[3] = std::cos(h); return 4;
    case QSV_GATE_RZ: out[0] = std::polar(1.0, -h); out[1] = std::polar(1.0, h); return 2;
    case QSV_GATE_PS: out[0] = 1; out[1] = std::polar(1.0, ang[0]); return 2;
    case QSV_GATE_RXX: case QSV_GATE_RYY: {
      for (int k = 0; k < 16; ++k) out[k] = 0;
      for (int col = 0; col < 4; ++col) {
        out[col * 4 + col] = std::cos(h);
        // P(x)P maps |col> to s(col) |col ^ 3>
        double s = 1.0;
        if (g.kind == QSV_GATE_RYY) s = (popc(col) & 1) ? 1.0 : -1.0;
        out[(col ^ 3) * 4 + col] = -I1 * std::sin(h) * s;
      }
      return 16;
    }
    case QSV_GATE_RZZ:
      out[0] = std::polar(1.0, -h); out[1] = std::polar(1.0, h); out[2] = std::polar(1.0, h); out[3] = std::polar(1.0, -h);
      return 4;
    case QSV_GATE_U3: {
      // section 4.1: U3(theta, phi, lam) = RZ(phi) RY(theta) RZ(lam), global phase included
      const double th = ang[0], ph = ang[1], la = ang[2];
      const double c = std::cos(th / 2), s = std::sin(th / 2);
      out[0] = std::polar(c, -(ph + la) / 2);
      out[1] = std::polar(-s, -(ph - la) / 2);
      out[2] = std::polar(s, (ph - la) / 2);
      out[3] = std::polar(c, (ph + la) / 2);
      return 4;
    }
    case QSV_GATE_SWAP:
      for (int k = 0; k < 16; ++k) out[k] = 0;
      out[0] = 1; out[1 * 4 + 2] = 1; out[2 * 4 + 1] = 1; out[15] = 1;
      return 16;
    case QSV_GATE_MAT1: case QSV_GATE_MAT2: {
      const int d = g.kind == QSV_GATE_MAT1 ? 2 : 4;
      const double* m = c->matrices + 2 * g.matrix_offset;
      const bool diag = mat_is_diagonal(c, g);
      if (diag) {
        for (int r = 0; r < d; ++r) out[r] = cplx(m[2 * (r * d + r)], m[2 * (r * d + r) + 1]);
        return d;
      }
      for (int k = 0; k < d * d; ++k) out[k] = cplx(m[2 * k], m[2 * k + 1]);
      return d * d;
    }
    default:
      fail(QSV_EINVAL, "gate kind has no matrix");
  }
}

void dagger_numbers(int type, cplx* v, int count) {
  if (type == P_DENSE1 || type == P_DENSE2) {
    const int d = type == P_DENSE1 ? 2 : 4;
    cplx t[16];
    for (int r = 0; r < d; ++r)
      for (int k = 0; k < d; ++k) t[r * d + k] = std::conj(v[k * d + r]);
    for (int k = 0; k < d * d; ++k) v[k] = t[k];
  } else {
    for (int k = 0; k < count; ++k) v[k] = std::conj(v[k]);
  }
}

int prim_numbers(const Prim& p, const qsv_circuit* c, const double* ang, cplx* out) {
  int cnt = 0;
  const double a = ang[p.angle_slot];
  switch (p.recipe) {
    case M_GATE: cnt = gate_numbers(c, c->gates[p.gate], ang, out); break;
    case M_RZ_ANGLE: out[0] = std::polar(1.0, -a / 2); out[1] = std::polar(1.0, a / 2); cnt = 2; break;
    case M_RY_ANGLE:
      out[0] = std::cos(a / 2); out[1] = -std::sin(a / 2); out[2] = std::sin(a / 2); out[3] = std::cos(a / 2);
      cnt = 4;
      break;
    case M_H: {
      const double r = std::sqrt(0.5);
      out[0] = r; out[1] = r; out[2] = r; out[3] = -r; cnt = 4;
      break;
    }
    case M_RX_PLUS: case M_RX_MINUS: {
      const double r = std::sqrt(0.5);
      const double sg = p.recipe == M_RX_PLUS ? 1.0 : -1.0;
      out[0] = r; out[1] = -I1 * r * sg; out[2] = -I1 * r * sg; out[3] = r; cnt = 4;
      break;
    }
    case M_ZZ_ANGLE: {
      const double h = 0.5 * ang[0];
      out[0] = std::polar(1.0, -h); out[1] = std::polar(1.0, h); out[2] = std::polar(1.0, h); out[3] = std::polar(1.0, -h);
      cnt = 4;
      break;
    }
    default: return 0;
  }
  if (p.dagger) dagger_numbers(p.type, out, cnt);
  return cnt;
}

int prim_gen(const Prim& p, cplx* out) {
  const double k = p.coeff;
  switch (p.gen) {
    case G_X: out[0] = 0; out[1] = k; out[2] = k; out[3] = 0; return 4;
    case G_Y: out[0] = 0; out[1] = -I1 * k; out[2] = I1 * k; out[3] = 0; return 4;
    case G_Z: out[0] = k; out[1] = -k; return 2;
    case G_PS: out[0] = 0; out[1] = -2 * k; return 2;
    case G_ZZ: out[0] = k; out[1] = -k; out[2] = -k; out[3] = k; return 4;
    case G_XX: case G_YY:
      for (int i = 0; i < 16; ++i) out[i] = 0;
      for (int col = 0; col < 4; ++col) {
        double s = 1.0;
        if (p.gen == G_YY) s = (popc(col) & 1) ? 1.0 : -1.0;
        out[(col ^ 3) * 4 + col] = k * s;
      }
      return 16;
    default: return 0;
  }
}

// The structure of a one-qubit primitive's matrix (any angle, dagger or not): real (RY, H,
// X) or real diagonal with imaginary off-diagonal entries (RX, Y); 0 for general matrices.
int32_t matrix_form(const Prim& p, const qsv_circuit* c) {
  if (p.type != P_DENSE1) return 0;
  switch (p.recipe) {
    case M_RY_ANGLE: case M_H: return kPlainReal;
    case M_RX_PLUS: case M_RX_MINUS: return kPlainXlike;
    case M_GATE:
      switch (c->gates[p.gate].kind) {
        case QSV_GATE_RY: case QSV_GATE_H: case QSV_GATE_X: return kPlainReal;
        case QSV_GATE_RX: case QSV_GATE_Y: return kPlainXlike;
        default: return 0;
      }
    default: return 0;
  }
}

int prim_size(const Prim& p) {
  switch (p.type) {
    case P_DENSE1: return 4;
    case P_DENSE2: return 16;
    case P_DIAG1: return 2;
    case P_DIAG2: return 4;
    default: return 0;
  }
}

}  // namespace

// ---- options ----------------------------------------------------------------------------------
int32_t default_tile_qubits(int32_t dtype) { return dtype == QSV_C64 ? 12 : 11; }
int32_t default_adj_tile_qubits(int32_t dtype) { return dtype == QSV_C64 ? 10 : 11; }

PlanOptions state_plan_options(int32_t dtype, int32_t n, int32_t tile, int32_t adj_tile, bool adjoint, bool fuse_zz,
                               bool relayout) {
  PlanOptions o;
  o.relayout = relayout && !adjoint;
  o.tile_qubits = adjoint ? adj_tile : tile;
  if (adjoint && o.tile_qubits == 0) o.tile_qubits = default_adj_tile_qubits(dtype);
  // complex128 adjoint tiles above 12 qubits would spill registers at 1024 threads
  if (adjoint && dtype == QSV_C128) o.tile_qubits = std::min(o.tile_qubits, 12);
  // tiles below the register-blocked range use the LDS-sweep kernel, whose adjoint
  // variant stages psi and lambda together
  if (std::min<int>(o.tile_qubits, n) < o.rb_min || rb_capacity_host(dtype, std::min<int>(o.tile_qubits, n)) < 0)
    o.tile_qubits = std::min<int>(o.tile_qubits, adjoint ? (dtype == QSV_C64 ? 12 : 11) : 13);
  // qubits every tile keeps for dense global accesses: measured on the 30-qubit brick and
  // the 24-qubit QAOA batch (with XCD-ordered tiles, neighbouring tiles share cache lines
  // in one XCD's L2, so keeping only the lowest qubits costs less than the passes it saves;
  // complex64 forward passes keep two, below which partial-line writes grow by 40 %)
  o.low_qubits = adjoint ? (dtype == QSV_C128 ? 3 : 1) : (dtype == QSV_C64 ? 2 : 1);
  o.fuse_zz = fuse_zz;
  o.dtype = dtype;
  // complex64 forward passes keep 16 amplitudes per thread (registers still allow 4 waves
  // per SIMD): fewer REMAPs and half the per-op and per-tile work per amplitude
  if (!adjoint && dtype == QSV_C64) o.reg_bits = 4;
  // forward passes fuse three-qubit rounds of one-qubit gates into matrix-core blocks,
  // keeping a round's blocks when they average enough gates.  complex64: fp32 matrix cores
  // run at twice the rate of the (unpacked) fp32 vector ALU, so a block of 16x16x4 products
  // costs about two register gates plus its layout moves; 3 is the best threshold of
  // 2 / 2.5 / 3 / 3.5 on the brick and QAOA circuits.  complex128: fp64 matrix and vector
  // rates are equal, so a block costs about four gates, but the matrix cores run beside the
  // vector ALU's other work; 4.5 is the best of 3.5 / 4.5 / 5.5 / none (brick: -7 %).
  o.blocks = !adjoint && dtype == QSV_C64;
  o.block_min_gates = 3.0;
  // complex128 forward passes split one-qubit gates instead: a phase and a real 2x2 matrix
  // cost 12 vector instructions per amplitude pair instead of 16, more than a block saves
  o.split = !adjoint && dtype == QSV_C128;
  return o;
}

// ---- validation -----------------------------------------------------------------------------
void validate_circuit(const qsv_circuit* c, size_t n_params, int32_t n_state) {
  if (!c) fail(QSV_EINVAL, "circuit is NULL");
  const int n = c->n_qubits;
  if (n < 1 || n > 34) fail(QSV_ERANGE, "n_qubits must be in [1, 34]");
  if (n_state >= 0 && n != n_state) fail(QSV_EINVAL, "circuit n_qubits differs from the state's");
  if (c->n_gates && !c->gates) fail(QSV_EINVAL, "gates is NULL");
  const uint64_t full = (1ull << n) - 1;
  for (size_t i = 0; i < c->n_gates; ++i) {
    const qsv_gate& g = c->gates[i];
    std::ostringstream where;
    where << "gate " << i << ": ";
    if (g.kind < 0 || g.kind >= QSV_GATE_KIND_COUNT) fail(QSV_EINVAL, where.str() + "unknown kind");
    const int nt = kNTargets[g.kind];
    for (int t = 0; t < nt; ++t)
      if (g.targets[t] < 0 || g.targets[t] >= n) fail(QSV_EINVAL, where.str() + "target out of range");
    if (nt == 2 && g.targets[0] == g.targets[1]) fail(QSV_EINVAL, where.str() + "duplicate targets");
    if (g.ctrl_mask & ~full) fail(QSV_EINVAL, where.str() + "control out of range");
    if (g.ctrl_mask & target_mask(g)) fail(QSV_EINVAL, where.str() + "control on a target");
    for (int a = 0; a < 3; ++a) {
      if (a < kNAngles[g.kind]) {
        if (g.param_index[a] < -1 || (g.param_index[a] >= 0 && (size_t)g.param_index[a] >= n_params))
          fail(QSV_EINVAL, where.str() + "param_index out of range");
        if (!std::isfinite(g.angle_const[a]) || !std::isfinite(g.param_coeff[a]))
          fail(QSV_EINVAL, where.str() + "non-finite angle");
      } else if (g.param_index[a] != -1) {
        fail(QSV_EINVAL, where.str() + "unused angle slot must have param_index -1");
      }
    }
    if (g.kind == QSV_GATE_MAT1 || g.kind == QSV_GATE_MAT2) {
      const int64_t need = g.kind == QSV_GATE_MAT1 ? 4 : 16;
      if (!c->matrices || g.matrix_offset < 0 || (uint64_t)(2 * (g.matrix_offset + need)) > c->n_matrix_doubles)
        fail(QSV_EINVAL, where.str() + "matrix out of range");
      for (int k = 0; k < 2 * need; ++k)
        if (!std::isfinite(c->matrices[2 * g.matrix_offset + k])) fail(QSV_EINVAL, where.str() + "non-finite matrix");
    }
  }
}

void validate_pauli_sum(const qsv_pauli_sum* h, int32_t n) {
  if (!h) fail(QSV_EINVAL, "pauli sum is NULL");
  if (h->n_terms && (!h->coeffs || !h->x_masks || !h->z_masks)) fail(QSV_EINVAL, "pauli sum arrays are NULL");
  const uint64_t full = (1ull << n) - 1;
  for (size_t k = 0; k < h->n_terms; ++k) {
    if ((h->x_masks[k] | h->z_masks[k]) & ~full) fail(QSV_EINVAL, "pauli term acts on a qubit >= n");
    if (!std::isfinite(h->coeffs[k])) fail(QSV_EINVAL, "non-finite pauli coefficient");
  }
}

// ---- lowering -------------------------------------------------------------------------------
// RXX(t) = (H x H) RZZ(t) (H x H) and RYY(t) = RX(-pi/2)^2 RZZ(t) RX(pi/2)^2 (operator
// order), so both become one-qubit basis changes around a diagonal RZZ; with controls only
// the RZZ part is controlled.  Forward order of the parts.
static std::vector<Prim> lower_pauli_pair(const qsv_circuit* c, int i) {
  const qsv_gate& g = c->gates[i];
  const bool xx = g.kind == QSV_GATE_RXX;
  std::vector<Prim> parts;
  auto basis = [&](int q, int recipe) {
    Prim p{};
    p.type = P_DENSE1;
    p.gate = i;
    p.q0 = q;
    p.q1 = -1;
    p.cmask = 0;
    p.recipe = recipe;
    p.param = -1;
    p.gen = G_NONE;
    finish_masks(p);
    parts.push_back(p);
  };
  const int pre = xx ? M_H : M_RX_PLUS, post = xx ? M_H : M_RX_MINUS;
  basis(g.targets[0], pre);
  basis(g.targets[1], pre);
  Prim z{};
  z.type = P_DIAG2;
  z.gate = i;
  z.q0 = g.targets[0];
  z.q1 = g.targets[1];
  z.cmask = g.ctrl_mask;
  z.recipe = M_ZZ_ANGLE;
  z.param = -1;
  z.gen = G_NONE;
  finish_masks(z);
  parts.push_back(z);
  basis(g.targets[0], post);
  basis(g.targets[1], post);
  return parts;
}

std::vector<Prim> lower_forward(const qsv_circuit* c) {
  std::vector<Prim> out;
  out.reserve(c->n_gates);
  for (size_t i = 0; i < c->n_gates; ++i) {
    const int k = c->gates[i].kind;
    if (k == QSV_GATE_RXX || k == QSV_GATE_RYY) {
      for (const Prim& p : lower_pauli_pair(c, (int)i)) out.push_back(p);
    } else {
      out.push_back(forward_prim(c, (int)i));
    }
  }
  return out;
}

std::vector<Prim> lower_adjoint(const qsv_circuit* c) {
  std::vector<Prim> out;
  for (int i = (int)c->n_gates - 1; i >= 0; --i) {
    const qsv_gate& g = c->gates[i];
    const bool any_param = g.kind == QSV_GATE_U3 &&
                           (g.param_index[0] >= 0 || g.param_index[1] >= 0 || g.param_index[2] >= 0);
    if (any_param) {
      // U3 = RZ(phi) RY(theta) RZ(lam) (section 4.1), each part carrying the gate's
      // controls.  Forward order of the parts:
      struct Part { int type, recipe, slot, gen; };
      const Part parts[3] = {{P_DIAG1, M_RZ_ANGLE, 2, G_Z},
                             {P_DENSE1, M_RY_ANGLE, 0, G_Y},
                             {P_DIAG1, M_RZ_ANGLE, 1, G_Z}};
      for (int k = 2; k >= 0; --k) {
        Prim p{};
        p.type = parts[k].type;
        p.gate = i;
        p.q0 = g.targets[0];
        p.q1 = -1;
        p.cmask = g.ctrl_mask;
        p.recipe = parts[k].recipe;
        p.angle_slot = parts[k].slot;
        p.dagger = true;
        const int pi = g.param_index[parts[k].slot];
        p.param = pi;
        p.gen = pi >= 0 ? parts[k].gen : G_NONE;
        p.coeff = pi >= 0 ? g.param_coeff[parts[k].slot] : 0.0;
        finish_masks(p);
        out.push_back(p);
      }
      continue;
    }
    if (g.kind == QSV_GATE_RXX || g.kind == QSV_GATE_RYY) {
      std::vector<Prim> parts = lower_pauli_pair(c, i);
      for (int k = (int)parts.size() - 1; k >= 0; --k) {
        Prim p = parts[k];
        p.dagger = true;
        if (p.recipe == M_ZZ_ANGLE && g.param_index[0] >= 0) {
          p.gen = G_ZZ;
          p.param = g.param_index[0];
          p.coeff = g.param_coeff[0];
        }
        out.push_back(p);
      }
      continue;
    }
    Prim p = forward_prim(c, i);
    p.dagger = true;
    if (kNAngles[g.kind] == 1 && g.param_index[0] >= 0) {
      p.gen = gen_of_kind(g.kind);
      p.param = g.param_index[0];
      p.coeff = g.param_coeff[0];
    }
    out.push_back(p);
  }
  return out;
}

// ---- planning -------------------------------------------------------------------------------
namespace {

// Primitives of rem that can run in a pass over tile T (in order), given that a
// primitive may move ahead of an unscheduled earlier one only when every qubit they share
// is acted on diagonally by both.
void schedule(const std::vector<Prim>& prims, const std::vector<int32_t>& rem, uint64_t T,
              std::vector<int32_t>* sched, std::vector<int32_t>* left, int* n_dense) {
  uint64_t blocked_any = 0, blocked_nd = 0;
  int dense = 0;
  for (int32_t i : rem) {
    const Prim& p = prims[i];
    const bool ok = (p.nondiag & ~T) == 0 && (p.nondiag & blocked_any) == 0 &&
                    ((p.touched & ~p.nondiag) & blocked_nd) == 0;
    if (ok) {
      if (sched) sched->push_back(i);
      if (p.nondiag) ++dense;
    } else {
      if (left) left->push_back(i);
      blocked_any |= p.touched;
      blocked_nd |= p.nondiag;
    }
  }
  if (n_dense) *n_dense = dense;
}

}  // namespace

std::vector<Pass> plan_passes(const std::vector<Prim>& prims, int32_t n, int32_t m, int32_t low_qubits) {
  std::vector<Pass> passes;
  std::vector<int32_t> rem(prims.size());
  for (size_t i = 0; i < prims.size(); ++i) rem[i] = (int32_t)i;
  const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1);
  if (m >= n) {
    Pass p;
    p.tile_mask = full;
    p.m = n;
    p.prims = rem;
    passes.push_back(p);
    return passes;
  }
  // keep two free tile slots so any 2-qubit primitive can be scheduled
  const int low = std::max(0, std::min(low_qubits, m - 2));
  while (!rem.empty()) {
    uint64_t T = (low > 0) ? ((1ull << low) - 1) : 0;
    // earliest position at which each qubit is needed non-diagonally
    std::vector<int> first_need(n, 1 << 30);
    for (size_t k = 0; k < rem.size(); ++k) {
      uint64_t nd = prims[rem[k]].nondiag;
      while (nd) {
        const int q = __builtin_ctzll(nd);
        if (first_need[q] > (int)k) first_need[q] = (int)k;
        nd &= nd - 1;
      }
    }
    while (popc(T) < m) {
      int best_q = -1, best_dense = -1, best_first = 1 << 30;
      for (int q = 0; q < n; ++q) {
        if (T >> q & 1) continue;
        int dense = 0;
        schedule(prims, rem, T | (1ull << q), nullptr, nullptr, &dense);
        if (dense > best_dense || (dense == best_dense && first_need[q] < best_first)) {
          best_q = q;
          best_dense = dense;
          best_first = first_need[q];
        }
      }
      T |= 1ull << best_q;
    }
    // Also try the low qubits plus every contiguous window of the others (this suits
    // circuits with nearest-neighbour structure, where the greedy choice scatters) and keep
    // the tile that runs the most dense primitives.
    {
      int best = -1;
      schedule(prims, rem, T, nullptr, nullptr, &best);
      const int free = m - low;
      for (int start = low; start + free <= n; ++start) {
        const uint64_t W = ((1ull << low) - 1) | (((1ull << free) - 1) << start);
        int dense = 0;
        schedule(prims, rem, W, nullptr, nullptr, &dense);
        if (dense > best) {
          best = dense;
          T = W;
        }
      }
    }
    Pass ps;
    std::vector<int32_t> left;
    schedule(prims, rem, T, &ps.prims, &left, nullptr);
    if (ps.prims.empty()) {
      // cannot happen with the tie-break above; keep a safe fallback
      T = prims[rem[0]].nondiag;
      for (int q = 0; popc(T) < m && q < n; ++q) T |= 1ull << q;
      ps.prims.clear();
      left.clear();
      schedule(prims, rem, T, &ps.prims, &left, nullptr);
    }
    ps.tile_mask = T;
    ps.m = popc(T);
    passes.push_back(ps);
    rem.swap(left);
  }
  return passes;
}

int tile_capacity_host(int dtype, bool adj, int m) {
  static const int caps[] = {8, 10, 11, 12, 13, 14};
  const size_t amp = dtype == 0 ? 8 : 16;
  for (int c : caps) {
    if (c < m) continue;
    if (amp * ((size_t)1 << c) * (adj ? 2 : 1) > 131072) return -1;
    return c;
  }
  return -1;
}

static bool same_binding(const qsv_gate& a, const qsv_gate& b) {
  return a.param_index[0] == b.param_index[0] && a.param_coeff[0] == b.param_coeff[0] &&
         a.angle_const[0] == b.angle_const[0];
}

static bool zz_fusable(const Prim& p, const qsv_circuit* c) {
  return p.recipe == M_GATE && p.cmask == 0 && c->gates[p.gate].kind == QSV_GATE_RZZ;
}

int rb_capacity_host(int dtype, int m, int reg_bits) {
  if (m < reg_bits + 1 || m > 13) return -1;
  const size_t amp = dtype == 0 ? 8 : 16;
  return amp * ((size_t)1 << m) <= 131072 ? m : -1;
}

std::vector<Pass> plan_rounds(const std::vector<Prim>& prims, const std::vector<int32_t>& seq, uint64_t allowed,
                              int32_t r) {
  // Same greedy as plan_passes, but only one-qubit dense primitives need register
  // qubits (two-qubit dense ones run through LDS, diagonal ones are elementwise).
  std::vector<Pass> rounds;
  std::vector<int32_t> rem = seq;
  auto need = [&](const Prim& p) { return p.type == P_DENSE1 ? p.nondiag : 0ull; };
  auto sched = [&](uint64_t R, std::vector<int32_t>* out, std::vector<int32_t>* left, int* n_dense) {
    uint64_t blocked_any = 0, blocked_nd = 0;
    int dense = 0;
    for (int32_t i : rem) {
      const Prim& p = prims[i];
      const bool ok = (need(p) & ~R) == 0 && (p.nondiag & blocked_any) == 0 &&
                      ((p.touched & ~p.nondiag) & blocked_nd) == 0;
      if (ok) {
        if (out) out->push_back(i);
        if (need(p)) ++dense;
      } else {
        if (left) left->push_back(i);
        blocked_any |= p.touched;
        blocked_nd |= p.nondiag;
      }
    }
    if (n_dense) *n_dense = dense;
  };
  while (!rem.empty()) {
    std::vector<int> first_need(64, 1 << 30);
    for (size_t k = 0; k < rem.size(); ++k) {
      uint64_t nd = need(prims[rem[k]]);
      while (nd) {
        const int q = __builtin_ctzll(nd);
        if (first_need[q] > (int)k) first_need[q] = (int)k;
        nd &= nd - 1;
      }
    }
    uint64_t R = 0;
    while (popc(R) < r) {
      int best_q = -1, best_dense = -1, best_first = 1 << 30;
      for (int q = 0; q < 64; ++q) {
        if (!(allowed >> q & 1) || (R >> q & 1)) continue;
        int dense = 0;
        sched(R | (1ull << q), nullptr, nullptr, &dense);
        if (dense > best_dense || (dense == best_dense && first_need[q] < best_first)) {
          best_q = q;
          best_dense = dense;
          best_first = first_need[q];
        }
      }
      if (best_q < 0) break;
      R |= 1ull << best_q;
    }
    Pass rd;
    std::vector<int32_t> left;
    sched(R, &rd.prims, &left, nullptr);
    if (rd.prims.empty()) {
      R = need(prims[rem[0]]);
      for (int q = 0; popc(R) < r && q < 64; ++q)
        if (allowed >> q & 1) R |= 1ull << q;
      rd.prims.clear();
      left.clear();
      sched(R, &rd.prims, &left, nullptr);
    }
    rd.tile_mask = R;
    rd.m = popc(R);
    rounds.push_back(rd);
    rem.swap(left);
  }
  return rounds;
}

RbLayout canonical_layout(uint32_t lr, int m, int r) {
  RbLayout L;
  L.r = r;
  L.nt = m - r;
  int i = 0, t = 0;
  for (int bit = 0; bit < m; ++bit) {
    if (lr >> bit & 1) L.reg[i++] = bit;
    else L.thr[t++] = bit;
  }
  return L;
}

namespace {

struct PassEmitter {
  Plan& plan;
  const qsv_circuit* c;
  bool adjoint;
  const PlanOptions& opt;
  uint64_t T;
  int loc[64];
  std::vector<int32_t> op_param;  // gradient parameter of each op of the pass (-1 none)
  bool rb = false;                // register-blocked pass
  const std::vector<char>* chain = nullptr;  // per primitive: 0, 1 split, 2 last of a chain
  RbLayout lay;                   // register-blocked passes: the current register layout

  int alloc(int count) {
    const int off = plan.ctab_size;
    plan.ctab_size += count;
    return off;
  }
  uint32_t local_mask(uint64_t gm) const {
    uint32_t lm = 0;
    while (gm) {
      const int q = __builtin_ctzll(gm);
      lm |= 1u << loc[q];
      gm &= gm - 1;
    }
    return lm;
  }
  // Split a diagonal entry's local condition into its thread-index part and the set of
  // register slots that satisfy its register part, for the current register layout.
  void slot_masks(DiagEntry& d) const {
    if (!rb) {
      d.tmask = d.lcmask;
      d.kmask = 1;
      return;
    }
    const uint32_t lr = lay.regmask();
    d.tmask = d.lcmask & ~lr;
    const uint32_t rm = d.lcmask & lr;
    d.kmask = 0;
    for (int k = 0; k < (1 << lay.r); ++k) {
      uint32_t bits = 0;
      for (int i = 0; i < lay.r; ++i) bits |= (uint32_t)((k >> i) & 1) << lay.reg[i];
      if ((bits & rm) == rm) d.kmask |= 1u << k;
    }
  }
  // A ZZ edge with its thread-bit mask, outside-bit mask and (in pad, until the run is
  // sorted) its register class for the current register layout.
  ZZEdge edge_in_layout(int u, int v) const {
    ZZEdge ed{u, v, loc[u], loc[v], 0, 0, 0};
    for (int q : {u, v}) {
      const int l = loc[q];
      const int slot = (rb && l >= 0) ? lay.slot_of(l) : -1;
      if (l < 0) {
        ed.omask |= 1ull << q;
      } else if (slot >= 0) {
        ed.pad ^= 1u << slot;
      } else {
        ed.tmask |= 1u << l;
      }
    }
    return ed;
  }
  void push(const TileOp& op, int32_t param) {
    plan.ops.push_back(op);
    op_param.push_back(param);
  }
  // Move to layout L through LDS.
  void remap(const RbLayout& L) {
    TileOp op{};
    op.type = OP_REMAP;
    op.a = (int32_t)L.regmask();
    op.b = (int32_t)L.regpack();
    op.omask = L.thrpack();
    op.gen = -1;
    op.pslot = -1;
    push(op, -1);
    lay = L;
  }
  // Transpositions (slot bit, lane bit) applied in order by cross-lane moves, one per op.
  void xswap(const std::vector<std::pair<int, int>>& sw) {
    for (const auto& ts : sw) {
      TileOp op{};
      op.type = OP_XSWAP;
      op.count = 1;
      const int i = ts.first, t = ts.second;
      if (i < 0 || i >= lay.r || !lay.swappable(t)) fail(QSV_EINVAL, "internal: bad transposition");
      std::swap(lay.reg[i], lay.thr[t]);
      op.mat = (int32_t)(i | t << 4);
      op.a = (int32_t)lay.regmask();
      op.b = (int32_t)lay.regpack();
      op.omask = lay.thrpack();
      op.gen = -1;
      op.pslot = -1;
      push(op, -1);
    }
  }
  // Diagonal primitives are buffered and emitted as late as possible: a dense primitive
  // commutes with every buffered diagonal one that does not touch its non-diagonal
  // qubits, so the buffer is flushed (as few merged DIAG / ZZ ops) only when a dense
  // primitive needs it, or at the end of the pass.
  std::vector<int32_t> pending;
  uint64_t pending_touched = 0;

  // Fused blocks (block rounds of forward register-blocked passes): the round's one-qubit
  // gates, and the diagonal primitives between them that act only on the block's qubits,
  // are multiplied into one 8x8 matrix on (lane bit 4, lane bit 5, register slot bslot).
  bool bmode = false;
  uint64_t bq = 0;            // global qubits of the block
  int32_t bqs[3] = {0, 0, 0}; // global qubit of block index bits 0..2
  int32_t bslot = -1;
  int32_t open = -1;          // the open block (index in plan.blocks), -1 if none
  size_t merge_floor = 0;  // ops before this index belong to an earlier round (kept on rollback)
  void close_block() {
    if (open < 0) return;
    TileOp op{};
    op.type = OP_BLOCK;
    op.a = bslot;
    op.plain = kPlainBlock | (1 + bslot);
    // a sign-only diagonal run right before the block rides on it
    if (plan.ops.size() > merge_floor && plan.ops.back().type == OP_DIAG && plan.ops.back().b == 0 &&
        op_param.back() < 0) {
      op.first = plan.ops.back().first;
      op.count = plan.ops.back().count;
      op.plain |= kPlainSigns;
      plan.ops.pop_back();
      op_param.pop_back();
    }
    op.mat = alloc(128);
    op.gen = -1;
    op.pslot = -1;
    plan.fills.push_back({F_BLOCK, open, 0, op.mat});
    push(op, -1);
    open = -1;
  }
  bool absorbs(const Prim& p) const {
    if (p.type == P_DENSE1) return p.cmask == 0 && (bq >> p.q0 & 1);
    if (p.type == P_SIGN || p.type == P_DIAG1 || p.type == P_DIAG2) return open >= 0 && (p.touched & ~bq) == 0;
    return false;
  }

  // Emit ops for primitives seq (in order).  reg_index: for register-blocked passes the
  // register index of each local bit (-1 if not a register bit), else nullptr.
  void emit(const std::vector<int32_t>& seq, const int* reg_index) {
    for (int32_t pi : seq) {
      const Prim& p = plan.prims[pi];
      if (bmode && absorbs(p)) {
        if (pending_touched & p.nondiag) {
          // pending diagonal primitives act on the gate's qubit before it: the block so far
          // goes first, then they, then a new block
          close_block();
          flush();
        }
        if (open < 0) {
          plan.blocks.push_back({{bqs[0], bqs[1], bqs[2]}, {}});
          open = (int32_t)plan.blocks.size() - 1;
        }
        plan.blocks[open].prims.push_back(pi);
        continue;
      }
      if (!(p.type == P_DENSE1 || p.type == P_DENSE2)) {
        pending.push_back(pi);
        pending_touched |= p.touched;
        continue;
      }
      close_block();
      TileOp pre{};
      bool has_pre = false;
      if (pending_touched & p.nondiag) {
        flush();
        // a sign-only diagonal run right before an uncontrolled register gate rides on it
        // (one op instead of two); it is applied to every slot before the gate
        if (reg_index && p.type == P_DENSE1 && (p.cmask & ~T) == 0 && !plan.ops.empty() &&
            plan.ops.back().type == OP_DIAG && plan.ops.back().b == 0 && op_param.back() < 0) {
          pre = plan.ops.back();
          plan.ops.pop_back();
          op_param.pop_back();
          has_pre = true;
        }
      }
      TileOp op{};
      op.gen = -1;
      op.pslot = -1;
      op.flush = 0;
      if (has_pre) {
        op.b = 1;
        op.first = pre.first;
        op.count = pre.count;
      }
      op.type = p.type == P_DENSE1 ? OP_DENSE1 : OP_DENSE2;
      if (p.type == P_DENSE1 && reg_index) {
        op.a = reg_index[loc[p.q0]];
        if (op.a < 0) fail(QSV_EINVAL, "internal: dense target is not a register bit");
      } else {
        op.a = loc[p.q0];
        op.b = p.type == P_DENSE2 ? loc[p.q1] : 0;
      }
      op.lmask = local_mask(p.cmask & T);
      op.omask = p.cmask & ~T;
      if (reg_index && op.omask) op.lmask |= kHasOutsideControls;
      const int ch = (chain && reg_index && p.type == P_DENSE1) ? (*chain)[pi] : 0;
      op.mat = alloc(prim_size(p));
      if (ch) plan.fills.push_back({F_GATE_CHAIN, pi, ch == 1 ? 1 : 0, op.mat});
      else plan.fills.push_back({F_PRIM_MATRIX, pi, 0, op.mat});
      int32_t prm = -1;
      if (adjoint && p.gen != G_NONE) {
        if (reg_index && p.type == P_DENSE2) fail(QSV_EINVAL, "internal: gradient on an LDS two-qubit op");
        op.gen = alloc(prim_size(p));
        plan.fills.push_back({F_PRIM_GEN, pi, 0, op.gen});
        prm = p.param;
        if (p.type == P_DENSE1) op.gkind = p.gen == G_X ? GEN_X : p.gen == G_Y ? GEN_Y : GEN_GENERAL;
      }
      if (reg_index && op.type == OP_DENSE1 && op.lmask == 0)
        op.plain = (1 + op.a) | (op.b ? kPlainSigns : 0) | (ch == 1 ? kPlainSplit : ch ? 0 : matrix_form(p, c));
      if (ch && !op.plain) fail(QSV_EINVAL, "internal: phase chain through a decoded gate");
      push(op, prm);
    }
  }

  void flush() {
    close_block();
    const std::vector<int32_t> seq = pending;
    pending.clear();
    pending_touched = 0;
    size_t k = 0;
    while (k < seq.size()) {
      const Prim& p = plan.prims[seq[k]];
      TileOp op{};
      op.gen = -1;
      op.pslot = -1;
      op.flush = 0;
      if (opt.fuse_zz && zz_fusable(p, c)) {
        size_t e = k + 1;
        while (e < seq.size() && zz_fusable(plan.prims[seq[e]], c) &&
               same_binding(c->gates[plan.prims[seq[e]].gate], c->gates[p.gate]) &&
               plan.prims[seq[e]].param == p.param && plan.prims[seq[e]].coeff == p.coeff)
          ++e;
        if (e - k >= 2) {
          op.type = OP_ZZ;
          op.first = (int32_t)plan.edges.size();
          op.count = (int32_t)(e - k);
          std::vector<ZZEdge> run;
          for (size_t r = k; r < e; ++r) {
            const int u = plan.prims[seq[r]].q0, v = plan.prims[seq[r]].q1;
            run.push_back(edge_in_layout(u, v));
          }
          if (rb) {
            // register-blocked: edges grouped by class, class sizes packed in a and b
            std::stable_sort(run.begin(), run.end(),
                             [](const ZZEdge& x, const ZZEdge& y) { return x.pad < y.pad; });
            // class masks with at most two bits in increasing order; the count of the
            // i-th is byte i of (a, b, lmask)
            std::vector<uint32_t> classes;
            for (uint32_t c = 0; c < (1u << lay.r); ++c)
              if (__builtin_popcount(c) <= 2) classes.push_back(c);
            uint32_t words[3] = {0, 0, 0};
            for (size_t i = 0; i < classes.size(); ++i) {
              uint32_t n_c = 0;
              for (const ZZEdge& ed : run) n_c += ed.pad == classes[i];
              if (n_c > 255 || (i == 11 && n_c > 127)) fail(QSV_EINVAL, "internal: too many edges in one ZZ class");
              words[i >> 2] |= n_c << (8 * (i & 3));
            }
            op.a = (int32_t)words[0];
            op.b = (int32_t)words[1];
            op.lmask = words[2];
          }
          for (ZZEdge& ed : run) ed.pad = 0;
          plan.edges.insert(plan.edges.end(), run.begin(), run.end());
          op.mat = alloc(op.count + 1);
          plan.fills.push_back({F_ZZ_PHASES, seq[k], op.count, op.mat});
          if (adjoint && p.gen != G_NONE) {
            op.gen = alloc(op.count + 1);
            plan.fills.push_back({F_ZZ_GEN, seq[k], op.count, op.gen});
          }
          push(op, adjoint && p.gen != G_NONE ? p.param : -1);
          k = e;
          continue;
        }
      }
      op.type = OP_DIAG;
      op.first = (int32_t)plan.diag.size();
      op.b = 0;  // 1 when the run has a phase entry (else only sign flips)
      int32_t run_param = -1;
      size_t e = k;
      while (e < seq.size()) {
        const Prim& q = plan.prims[seq[e]];
        if (e > k && opt.fuse_zz && zz_fusable(q, c) && e + 1 < seq.size() &&
            zz_fusable(plan.prims[seq[e + 1]], c) &&
            same_binding(c->gates[plan.prims[seq[e + 1]].gate], c->gates[q.gate]))
          break;  // let the ZZ run start its own op
        const int32_t qp = (adjoint && q.gen != G_NONE) ? q.param : -1;
        if (qp >= 0) {
          if (run_param >= 0 && qp != run_param) break;
          run_param = qp;
        }
        DiagEntry d{};
        d.kind = q.type == P_SIGN ? DIAG_SIGN : DIAG_PHASE;
        d.q0 = q.q0;
        d.q1 = q.type == P_DIAG2 ? q.q1 : -1;
        d.cmask = q.cmask;
        d.l0 = loc[d.q0];
        d.l1 = d.q1 >= 0 ? loc[d.q1] : -1;
        d.lcmask = local_mask(q.cmask & T);
        d.ocmask = q.cmask & ~T;
        slot_masks(d);
        d.mat = -1;
        d.gen = -1;
        if (q.type != P_SIGN) {
          op.b = 1;
          d.mat = alloc(prim_size(q));
          plan.fills.push_back({F_PRIM_MATRIX, seq[e], 0, d.mat});
        }
        if (qp >= 0) {
          d.gen = alloc(prim_size(q));
          plan.fills.push_back({F_PRIM_GEN, seq[e], 0, d.gen});
        }
        plan.diag.push_back(d);
        ++e;
      }
      op.count = (int32_t)(plan.diag.size() - op.first);
      // register passes: sign-only runs take the kernel's short path
      if (rb && op.b == 0 && run_param < 0) op.plain = kPlainSigns;
      push(op, run_param);
      k = e;
    }
  }
};

// A local register mask of exactly r bits containing the round's register qubits,
// padded with the highest free local bits (away from the coalescing bits).
int32_t round_layout(const PassEmitter& em, uint64_t round_mask, int m, int r) {
  int32_t lr = (int32_t)em.local_mask(round_mask);
  for (int bit = m - 1; bit >= 0 && popc((uint64_t)lr) < r; --bit) lr |= 1 << bit;
  return lr;
}

}  // namespace

Plan build_plan(const qsv_circuit* c, bool adjoint, const PlanOptions& opt) {
  Plan plan;
  plan.adjoint = adjoint;
  plan.dtype = opt.dtype;
  plan.n_qubits = c->n_qubits;
  plan.prims = adjoint ? lower_adjoint(c) : lower_forward(c);
  const int n = c->n_qubits;
  auto alloc = [&](int count) {
    const int off = plan.ctab_size;
    plan.ctab_size += count;
    return off;
  };
  if (!adjoint && opt.tile_qubits == 0) {
    plan.unfused = true;
    for (size_t i = 0; i < plan.prims.size(); ++i) {
      const Prim& p = plan.prims[i];
      int mat = -1, de = -1;
      const int sz = prim_size(p);
      if (sz) {
        mat = alloc(sz);
        plan.fills.push_back({F_PRIM_MATRIX, (int32_t)i, 0, mat});
      }
      if (p.type == P_DIAG1 || p.type == P_DIAG2 || p.type == P_SIGN) {
        DiagEntry d{};
        d.kind = p.type == P_SIGN ? DIAG_SIGN : DIAG_PHASE;
        d.q0 = p.q0;
        d.q1 = p.type == P_DIAG2 ? p.q1 : -1;
        d.mat = mat;
        d.cmask = p.cmask;
        d.gen = -1;
        d.l0 = d.l1 = -1;
        d.lcmask = 0;
        d.ocmask = 0;
        de = (int)plan.diag.size();
        plan.diag.push_back(d);
      }
      plan.stream_mat.push_back(mat);
      plan.stream_diag.push_back(de);
    }
    return plan;
  }

  const int m = std::min<int>(std::max(opt.tile_qubits, 2), n);
  // four register bits only for forward passes whose workgroup still fills a wave
  const int reg_bits = (adjoint || std::min<int>(std::max(opt.tile_qubits, 2), n) < opt.reg_bits + 6) ? kRegBits : opt.reg_bits;
  const bool rb = opt.use_rb && m >= opt.rb_min && rb_capacity_host(opt.dtype, m, reg_bits) >= 0;
  const int maxm = rb ? std::max(m, reg_bits + 6) : tile_capacity_host(opt.dtype, adjoint, m);
  if (maxm < 0) fail(QSV_EINVAL, "tile width does not fit in LDS for this dtype");
  const std::vector<Pass> passes = plan_passes(plan.prims, n, m, opt.low_qubits);
  const int low_local = std::max(0, std::min(opt.low_qubits, m - 2));
  const int32_t low_mask = (1 << low_local) - 1;
  // Bit layouts between passes: lay[p][q] is the bit of qubit q in the layout pass p reads
  // (lay[P]: the layout the last pass writes).  Both ends use the natural layout.  With
  // relayout, pass p writes a layout with pass p+1's tile in its low bits (qubit order),
  // then the qubits of pass p's tile that pass p+1 lacks, then the rest: pass p+1 reads one
  // contiguous block per tile, and pass p writes each tile within 2^(m + |T_p - T_p+1|)
  // amplitudes.  A pass cannot read and write one buffer in two layouts, so passes alternate
  // between two buffers; with an odd pass count the first pass stays in place.
  const int P = (int)passes.size();
  const bool relay = rb && !adjoint && opt.relayout && P >= 2;
  std::vector<std::vector<int>> lay(P + 1, std::vector<int>(n));
  for (auto& L : lay)
    for (int q = 0; q < n; ++q) L[q] = q;
  if (relay) {
    for (int p = (P % 2 == 0) ? 1 : 2; p < P; ++p) {
      const uint64_t next = passes[p].tile_mask, prev = passes[p - 1].tile_mask;
      int pos = 0;
      for (int q = 0; q < n; ++q)
        if (next >> q & 1) lay[p][q] = pos++;
      for (int q = 0; q < n; ++q)
        if ((prev >> q & 1) && !(next >> q & 1)) lay[p][q] = pos++;
      for (int q = 0; q < n; ++q)
        if (!((prev | next) >> q & 1)) lay[p][q] = pos++;
    }
  }
  bool moved = false;
  for (int p = 0; p < P; ++p) moved |= lay[p] != lay[p + 1];
  plan.relayout = relay && moved;  // else every pass runs in place
  // register rounds of every pass (fused-block passes plan rounds of three qubits, the block
  // size)
  std::vector<std::vector<Pass>> pass_rounds(P);
  if (rb)
    for (int pi = 0; pi < P; ++pi) {
      const bool use_blocks = opt.blocks && !adjoint && passes[pi].m - reg_bits >= 6;
      pass_rounds[pi] = plan_rounds(plan.prims, passes[pi].prims, passes[pi].tile_mask, use_blocks ? 3 : reg_bits);
    }
  // Phase chains: an uncontrolled one-qubit gate whose qubit's next non-diagonal primitive
  // (in execution order, across passes) is again an uncontrolled one-qubit gate runs as
  // diag(1, e^{i phi}) then a real 2x2 matrix; the remaining left diagonal commutes with
  // everything up to that next gate, whose matrix absorbs it.  A chain's last gate stays
  // dense.
  std::vector<char> chain(plan.prims.size(), 0);
  if (rb && opt.split && !adjoint && !opt.blocks) {
    // (gates with real or X-like matrices cost 8 instructions per pair as they are, fewer
    // than a split gate's 12, so they neither join nor extend chains)
    auto splittable = [&](int32_t i) {
      const Prim& pr = plan.prims[i];
      if (pr.type != P_DENSE1 || pr.cmask != 0 || matrix_form(pr, c) != 0) return false;
      const qsv_gate& g = c->gates[pr.gate];
      return pr.recipe != M_GATE || g.kind != QSV_GATE_MAT1 || mat1_is_unitary(c, g);
    };
    std::vector<int32_t> last(n, -1);  // each qubit's previous non-diagonal primitive
    for (int pi = 0; pi < P; ++pi)
      for (const Pass& rd : pass_rounds[pi])
        for (int32_t i : rd.prims) {
          uint64_t nd = plan.prims[i].nondiag;
          while (nd) {
            const int q = __builtin_ctzll(nd);
            nd &= nd - 1;
            const int32_t prev = last[q];
            if (prev >= 0 && splittable(prev) && splittable(i)) {
              chain[prev] = 1;
              if (!chain[i]) chain[i] = 2;
            }
            last[q] = i;
          }
        }
  }
  for (int pi = 0; pi < P; ++pi) {
    const Pass& ps = passes[pi];
    DevPass dp{};
    dp.tile_mask = ps.tile_mask;
    dp.m = ps.m;
    dp.maxm = maxm;
    dp.rb = rb ? reg_bits : 0;
    dp.op_first = (int32_t)plan.ops.size();
    dp.pslot_first = plan.n_pslots;
    PassEmitter em{plan, c, adjoint, opt, ps.tile_mask, {}, {}};
    {
      int r = 0;
      for (int q = 0; q < 64; ++q) em.loc[q] = (ps.tile_mask >> q & 1) ? r++ : -1;
    }
    if (!rb) {
      em.emit(ps.prims, nullptr);
      em.flush();
    } else {
      const int r = reg_bits;
      // fused-block passes plan rounds of three qubits (the block size) and run each round
      // whose dense work is all uncontrolled one-qubit gates as blocks; other rounds stay
      // register rounds
      const bool use_blocks = opt.blocks && !adjoint && ps.m - r >= 6;
      const std::vector<Pass>& rounds = pass_rounds[pi];
      em.chain = &chain;
      const int32_t top = ((1 << r) - 1) << (ps.m - r);  // load/store layout
      const int R = (int)rounds.size();
      // local bits each round needs in registers (0: the round has no one-qubit dense gate)
      std::vector<uint32_t> need(R, 0);
      std::vector<char> blockable(R, 0);
      for (int ri = 0; ri < R; ++ri) {
        bool has_dense = false, simple = true;
        for (int32_t i : rounds[ri].prims) {
          const Prim& pr = plan.prims[i];
          has_dense |= pr.type == P_DENSE1;
          simple &= pr.type != P_DENSE2 && !(pr.type == P_DENSE1 && pr.cmask != 0);
        }
        if (has_dense) need[ri] = em.local_mask(rounds[ri].tile_mask);
        blockable[ri] = use_blocks && has_dense && simple;
      }
      auto next_use = [&](int bit, int from) {
        for (int k = from; k < R; ++k)
          if (need[k] >> bit & 1) return k;
        return R + ps.m - bit;  // never again: the higher local bits first
      };
      // A layout reached through LDS: register bits `regs` (slot order ascending, or `slot2`
      // first at slot `slot2_at`), the bits `l4` / `l5` (if >= 0) on lane bits 4 / 5, the bits
      // needed latest on the wave bits, the two needed soonest after them on lane bits 4 and 5
      // if still free, never a coalescing bit on a wave bit or lanes 4, 5; the rest ascending.
      auto lds_layout = [&](uint32_t regs, int l4, int l5, int slot2, int from) {
        RbLayout L;
        L.r = r;
        L.nt = ps.m - r;
        std::vector<int> cand;
        for (int bit = 0; bit < ps.m; ++bit)
          if (!(regs >> bit & 1) && bit != l4 && bit != l5 && bit >= low_local) cand.push_back(bit);
        std::stable_sort(cand.begin(), cand.end(),
                         [&](int x, int y) { return next_use(x, from) < next_use(y, from); });
        const int nl = L.lanes(), nw = L.nt - nl;
        std::vector<int> pos(ps.m, -1);
        std::vector<char> taken(L.nt, 0);
        uint32_t placed = regs;
        auto put = [&](int bit, int t) {
          pos[bit] = t;
          taken[t] = 1;
          placed |= 1u << bit;
        };
        if (l4 >= 0) put(l4, 4);
        if (l5 >= 0) put(l5, 5);
        for (int k = 0; k < nw && k < (int)cand.size(); ++k) put(cand[cand.size() - 1 - k], nl + k);
        for (int h = 4; h <= 5 && h < nl; ++h) {
          if (taken[h]) continue;
          for (int bit : cand)
            if (!(placed >> bit & 1)) { put(bit, h); break; }
        }
        for (int bit = 0, t = 0; bit < ps.m; ++bit) {
          if (placed >> bit & 1) continue;
          while (taken[t]) ++t;
          put(bit, t);
        }
        int i = 0;
        for (int bit = 0; bit < ps.m; ++bit) {
          if (regs >> bit & 1) L.reg[i++] = bit;
          else L.thr[pos[bit]] = bit;
        }
        if (slot2 >= 0) {  // put slot2's bit on slot slot2_at = 0
          const int at = L.slot_of(slot2);
          std::swap(L.reg[0], L.reg[at]);
        }
        return L;
      };
      // register bits for a round: its own and those needed soonest
      auto fill_regs = [&](uint32_t base_regs, int from, uint32_t exclude) {
        std::vector<int> cand;
        for (int bit = 0; bit < ps.m; ++bit)
          if (!(base_regs >> bit & 1) && !(exclude >> bit & 1)) cand.push_back(bit);
        std::stable_sort(cand.begin(), cand.end(),
                         [&](int x, int y) { return next_use(x, from) < next_use(y, from); });
        uint32_t regs = base_regs;
        for (size_t k = 0; k < cand.size() && popc(regs) < r; ++k) regs |= 1u << cand[k];
        return regs;
      };
      em.rb = true;
      bool started = false;
      for (int ri = 0; ri < R; ++ri) {
        if (!started) {
          // first round: load straight into its layout when the coalescing bits stay thread
          // bits in their places
          const int32_t lr =
              (need[ri] && !blockable[ri]) ? round_layout(em, rounds[ri].tile_mask, ps.m, r) : top;
          em.lay = canonical_layout((uint32_t)((lr & low_mask) == 0 ? lr : top), ps.m, r);
          dp.lr0 = (int32_t)em.lay.regmask();
          dp.lay0_reg = em.lay.regpack();
          dp.lay0_thr = em.lay.thrpack();
          started = true;
        }
        // A block round is kept only when its blocks carry enough gates to beat the
        // register path on the vector ALU; otherwise everything it emitted is undone and the
        // round runs as a register round.
        struct Saved {
          size_t ops, diag, edges, fills, blocks, op_param;
          int32_t ctab;
          std::vector<int32_t> pending;
          uint64_t pending_touched;
          RbLayout lay;
        };
        const Saved sv{plan.ops.size(), plan.diag.size(), plan.edges.size(), plan.fills.size(),
                       plan.blocks.size(), em.op_param.size(), plan.ctab_size, em.pending,
                       em.pending_touched, em.lay};
        em.merge_floor = sv.ops;
        if (blockable[ri]) {
          // block round: two of its qubits on lane bits 4 and 5, the third on a slot bit
          const uint32_t tb = need[ri];
          bool reachable = true;
          for (int bit = 0; bit < ps.m; ++bit)
            if (tb >> bit & 1) {
              const int t = em.lay.thread_pos_of(bit);
              reachable &= em.lay.slot_of(bit) >= 0 || t == 4 || t == 5;
            }
          if (reachable) {
            RbLayout L = em.lay;
            std::vector<std::pair<int, int>> sw;
            auto on_lane = [&](int bit) { return L.thr[4] == bit || L.thr[5] == bit; };
            int n_lane = 0, n_t = popc(tb);
            for (int bit = 0; bit < ps.m; ++bit) n_lane += (tb >> bit & 1) && on_lane(bit);
            // a slot's target moves onto a lane bit 4 / 5 whose bit is not a target
            while ((n_t == 3 && n_lane < 2) || (n_t == 2 && n_lane == 0)) {
              int from_slot = -1;
              for (int i = 0; i < r && from_slot < 0; ++i)
                if (tb >> L.reg[i] & 1) from_slot = i;
              int lane = -1, best = -1;
              for (int h = 4; h <= 5; ++h) {
                if (tb >> L.thr[h] & 1) continue;
                const int u = next_use(L.thr[h], ri + 1);
                if (u > best) { best = u; lane = h; }
              }
              sw.push_back({from_slot, lane});
              std::swap(L.reg[from_slot], L.thr[lane]);
              ++n_lane;
            }
            em.xswap(sw);
          } else {
            // through LDS: two targets on lanes 4 and 5, the third on slot 0
            std::vector<int> tbits;
            for (int bit = 0; bit < ps.m; ++bit)
              if (tb >> bit & 1) tbits.push_back(bit);
            const int l4 = tbits.size() > 0 ? tbits[0] : -1, l5 = tbits.size() > 1 ? tbits[1] : -1;
            const int s2 = tbits.size() > 2 ? tbits[2] : -1;
            uint32_t excl = 0;
            if (l4 >= 0) excl |= 1u << l4;
            if (l5 >= 0) excl |= 1u << l5;
            const uint32_t regs = fill_regs(s2 >= 0 ? 1u << s2 : 0u, ri + 1, excl);
            em.remap(lds_layout(regs, l4, l5, s2, ri + 1));
          }
          // the block: lane bits 4, 5 and the slot holding the round's third qubit (or slot 0)
          int slot = 0;
          for (int i = 0; i < r; ++i)
            if (tb >> em.lay.reg[i] & 1) slot = i;
          em.bslot = slot;
          const int lb[3] = {em.lay.thr[4], em.lay.thr[5], em.lay.reg[slot]};
          em.bq = 0;
          for (int t = 0; t < 3; ++t) {
            int gq = -1;
            for (int q = 0; q < 64; ++q)
              if (em.loc[q] == lb[t]) gq = q;
            em.bqs[t] = gq;
            em.bq |= 1ull << gq;
          }
          em.bmode = true;
          int reg_index[32];
          for (int bit = 0; bit < 32; ++bit) reg_index[bit] = -1;
          for (int i = 0; i < r; ++i) reg_index[em.lay.reg[i]] = i;
          em.emit(rounds[ri].prims, reg_index);
          em.close_block();
          em.bmode = false;
          int n_blocks = 0, n_gates = 0;
          for (size_t b = sv.blocks; b < plan.blocks.size(); ++b) {
            ++n_blocks;
            for (int32_t pi : plan.blocks[b].prims) n_gates += plan.prims[pi].type == P_DENSE1;
          }
          if (n_gates >= opt.block_min_gates * n_blocks) continue;
          plan.ops.resize(sv.ops);
          plan.diag.resize(sv.diag);
          plan.edges.resize(sv.edges);
          plan.fills.resize(sv.fills);
          plan.blocks.resize(sv.blocks);
          em.op_param.resize(sv.op_param);
          plan.ctab_size = sv.ctab;
          em.pending = sv.pending;
          em.pending_touched = sv.pending_touched;
          em.lay = sv.lay;
        }
        if (need[ri] & ~em.lay.regmask()) {
          const uint32_t miss = need[ri] & ~em.lay.regmask();
          bool on_lanes = true;
          for (int bit = 0; bit < ps.m; ++bit)
            if (miss >> bit & 1) {
              on_lanes &= em.lay.swappable(em.lay.thread_pos_of(bit));
            }
          if (on_lanes) {
            // trade each missing bit for the register bit needed latest, by cross-lane moves
            std::vector<std::pair<int, int>> sw;
            RbLayout L = em.lay;
            for (int bit = 0; bit < ps.m; ++bit) {
              if (!(miss >> bit & 1)) continue;
              int best = -1, best_use = -1;
              for (int i = 0; i < r; ++i) {
                if (need[ri] >> L.reg[i] & 1) continue;
                const int u = next_use(L.reg[i], ri + 1);
                if (u > best_use) { best_use = u; best = i; }
              }
              const int t = L.thread_pos_of(bit);
              sw.push_back({best, t});
              std::swap(L.reg[best], L.thr[t]);
            }
            em.xswap(sw);
          } else {
            // through LDS: the round's bits and those needed soonest in registers
            em.remap(lds_layout(fill_regs(need[ri], ri + 1, 0), -1, -1, -1, ri + 1));
          }
        }
        int reg_index[32];
        for (int bit = 0; bit < 32; ++bit) reg_index[bit] = -1;
        for (int i = 0; i < r; ++i) reg_index[em.lay.reg[i]] = i;
        em.emit(rounds[ri].prims, reg_index);
      }
      if (!started) {
        em.lay = canonical_layout((uint32_t)top, ps.m, r);
        dp.lr0 = top;
        dp.lay0_reg = em.lay.regpack();
        dp.lay0_thr = em.lay.thrpack();
      }
      em.flush();
      // stores: the coalescing local bits back on their own lanes
      bool fixed = true;
      for (int t = 0; t < low_local; ++t) fixed &= em.lay.thr[t] == t;
      if (!fixed) em.remap(canonical_layout((uint32_t)top, ps.m, r));
    }
    // gradient slots: consecutive ops of one parameter share an accumulator
    if (adjoint) {
      int32_t cur_p = -1, last_op = -1, local = -1;
      for (size_t i = 0; i < em.op_param.size(); ++i) {
        const int32_t prm = em.op_param[i];
        if (prm < 0) continue;
        TileOp& o = plan.ops[dp.op_first + i];
        if (prm != cur_p) {
          if (last_op >= 0) plan.ops[last_op].flush = 1;
          cur_p = prm;
          ++local;
          plan.pslot_param.push_back(prm);
        }
        o.pslot = local;
        last_op = dp.op_first + (int32_t)i;
      }
      if (last_op >= 0) plan.ops[last_op].flush = 1;
      dp.pslot_count = local + 1;
      plan.n_pslots += dp.pslot_count;
    }
    dp.op_count = (int32_t)plan.ops.size() - dp.op_first;
    if (rb) {
      dp.dep_first = (int32_t)plan.deps.size();
      const std::vector<int>& Lr = lay[pi];
      const std::vector<int>& Lw = lay[pi + 1];
      dp.relayout = Lr != Lw ? 1 : 0;
      // tile qubits in local-bit order, and the outside qubits in tile-index-bit order
      std::vector<int> tq, ord;
      for (int q = 0; q < n; ++q)
        if (ps.tile_mask >> q & 1) tq.push_back(q);
      // with relayout, consecutive tiles differ first in the qubits that are low bits of
      // the layout this pass writes, so their writes fill the same lines; a pass reading
      // the natural layout with a tile that is not the lowest qubits keeps qubit order
      const bool reads_natural = Lr == lay[P] && ps.tile_mask != (1ull << ps.m) - 1;
      const bool store_first = dp.relayout && !reads_natural;
      if (store_first) {
        const uint64_t next = passes[pi + 1 < P ? pi + 1 : pi].tile_mask;
        for (int q = 0; q < n; ++q)
          if (!(ps.tile_mask >> q & 1) && (next >> q & 1)) ord.push_back(q);
        for (int q = 0; q < n; ++q)
          if (!(ps.tile_mask >> q & 1) && !(next >> q & 1)) ord.push_back(q);
      } else {
        for (int q = 0; q < n; ++q)
          if (!(ps.tile_mask >> q & 1)) ord.push_back(q);
      }
      auto tables = [&](const std::vector<int>& L) {
        for (int h = 0; h < 2; ++h)
          for (int v = 0; v < 128; ++v) {
            uint64_t r = 0;
            for (int b = 0; b < 7; ++b)
              if ((v >> b & 1) && 7 * h + b < (int)tq.size()) r |= 1ull << L[tq[7 * h + b]];
            plan.deps.push_back(r);
          }
      };
      tables(Lr);
      tables(Lw);
      auto runs = [&](const std::vector<int>& L, int at) {
        std::vector<uint64_t> r;
        for (size_t i = 0; i < ord.size();) {
          size_t len = 1;
          while (i + len < ord.size() && L[ord[i + len]] == L[ord[i]] + (int)len) ++len;
          r.push_back((uint64_t)L[ord[i]] | (uint64_t)len << 8 | (uint64_t)i << 16);
          i += len;
        }
        if ((int)r.size() > kMaxRuns) fail(QSV_EINVAL, "internal: too many runs of outside bits");
        plan.deps.resize(dp.dep_first + at, 0);
        plan.deps.push_back(r.size());
        plan.deps.insert(plan.deps.end(), r.begin(), r.end());
      };
      runs(lay[P], kRunsLogical);  // the natural layout: bit q is qubit q
      runs(Lr, kRunsLoad);
      runs(Lw, kRunsStore);
      plan.deps.resize(dp.dep_first + kDepEntries, 0);
    }
    if (rb) {
      // ctab window of the per-lane lookups (ZZ phase / generator tables, phase entries)
      int64_t lo = INT64_MAX, hi = INT64_MIN;
      auto cover = [&](int64_t off, int64_t n) {
        if (off < 0) return;
        lo = std::min(lo, off);
        hi = std::max(hi, off + n);
      };
      for (int i = 0; i < dp.op_count; ++i) {
        const TileOp& o = plan.ops[dp.op_first + i];
        if (o.type == OP_ZZ) {
          cover(o.mat, o.count + 1);
          cover(o.gen, o.count + 1);
        } else if (o.type == OP_DIAG && o.b) {
          for (int e = 0; e < o.count; ++e) {
            const DiagEntry& d = plan.diag[o.first + e];
            if (d.kind != DIAG_PHASE) continue;
            const int n = d.q1 >= 0 ? 4 : 2;
            cover(d.mat, n);
            cover(d.gen, n);
          }
        }
      }
      if (hi > lo && hi - lo <= kMaxWindow) {
        dp.win_lo = (int32_t)lo;
        dp.win_n = (int32_t)(hi - lo);
      }
    }
    plan.passes.push_back(dp);
  }
  return plan;
}

std::string structure_key(const qsv_circuit* c, bool adjoint, const PlanOptions& opt) {
  std::string key;
  auto put = [&](const void* p, size_t n) { key.append(reinterpret_cast<const char*>(p), n); };
  const int32_t head[10] = {c->n_qubits, adjoint ? 1 : 0, opt.tile_qubits, opt.low_qubits, opt.fuse_zz ? 1 : 0,
                            opt.dtype, opt.use_rb ? 1 : 0, opt.rb_min, opt.reg_bits, opt.relayout ? 1 : 0};
  put(head, sizeof(head));
  for (size_t i = 0; i < c->n_gates; ++i) {
    const qsv_gate& g = c->gates[i];
    int32_t rec[8] = {g.kind, g.targets[0], kNTargets[g.kind] == 2 ? g.targets[1] : -1, -1, -1, -1, 0, 0};
    for (int a = 0; a < kNAngles[g.kind]; ++a) rec[3 + a] = g.param_index[a];
    if (g.kind == QSV_GATE_MAT1 || g.kind == QSV_GATE_MAT2) rec[6] = mat_is_diagonal(c, g) ? 1 : 0;
    if (g.kind == QSV_GATE_MAT1 && mat1_is_unitary(c, g)) rec[6] |= 2;
    if (g.kind == QSV_GATE_RZZ && i > 0 && c->gates[i - 1].kind == QSV_GATE_RZZ)
      rec[7] = same_binding(g, c->gates[i - 1]) ? 1 : 0;
    if (g.kind == QSV_GATE_RZZ || (kNAngles[g.kind] > 0 && g.param_index[0] >= 0)) {
      // the chain-rule factor decides ZZ fusion in the reverse sweep
      put(&g.param_coeff[0], sizeof(double));
    }
    put(rec, sizeof(rec));
    put(&g.ctrl_mask, sizeof(g.ctrl_mask));
  }
  return key;
}

void gate_angles(const qsv_gate& g, const double* params, double out[3]) {
  for (int a = 0; a < 3; ++a) {
    out[a] = 0.0;
    if (a >= kNAngles[g.kind]) continue;
    out[a] = g.angle_const[a];
    if (g.param_index[a] >= 0) out[a] += g.param_coeff[a] * params[g.param_index[a]];
  }
}

void block_operands(const cplx* M8, int dtype, double* out) {
  double mr[16][16] = {};
  auto row = [](int beta, int ri) { return (beta & 3) + 4 * ri + 8 * (beta >> 2); };
  for (int bo = 0; bo < 8; ++bo)
    for (int bi = 0; bi < 8; ++bi) {
      const double a = M8[bo * 8 + bi].real(), b = M8[bo * 8 + bi].imag();
      mr[row(bo, 0)][row(bi, 0)] = a;
      mr[row(bo, 0)][row(bi, 1)] = -b;
      mr[row(bo, 1)][row(bi, 0)] = b;
      mr[row(bo, 1)][row(bi, 1)] = a;
    }
  for (int l = 0; l < 64; ++l)
    for (int j = 0; j < 4; ++j) {
      const int m = l % 16, col = 4 * j + l / 16;
      const int src = dtype == QSV_C64 ? (m / 4) + 4 * (m % 4) : m;
      out[4 * l + j] = mr[src][col];
    }
}

// The 8x8 matrix of a fused block: its primitives multiplied in execution order.
static void block_matrix(const Plan& p, const qsv_circuit* c, const std::vector<double>& ang, const BlockSpec& b,
                         cplx* M) {
  for (int i = 0; i < 64; ++i) M[i] = (i % 9 == 0) ? 1.0 : 0.0;
  auto bit_of = [&](int q) {
    for (int t = 0; t < 3; ++t)
      if (b.q[t] == q) return t;
    return -1;
  };
  for (int32_t pi : b.prims) {
    const Prim& pr = p.prims[pi];
    cplx num[16];
    prim_numbers(pr, c, &ang[3 * pr.gate], num);
    if (pr.type == P_DENSE1) {
      const int t = bit_of(pr.q0);
      for (int col = 0; col < 8; ++col)
        for (int beta = 0; beta < 8; ++beta) {
          if (beta >> t & 1) continue;
          const int b1 = beta | 1 << t;
          const cplx x = M[beta * 8 + col], y = M[b1 * 8 + col];
          M[beta * 8 + col] = num[0] * x + num[1] * y;
          M[b1 * 8 + col] = num[2] * x + num[3] * y;
        }
      continue;
    }
    for (int beta = 0; beta < 8; ++beta) {
      bool ctrl = true;
      for (uint64_t cm = pr.cmask; cm; cm &= cm - 1) ctrl &= (beta >> bit_of(__builtin_ctzll(cm)) & 1) != 0;
      if (!ctrl) continue;
      cplx f;
      if (pr.type == P_SIGN) f = -1.0;
      else if (pr.type == P_DIAG1) f = num[beta >> bit_of(pr.q0) & 1];
      else f = num[(beta >> bit_of(pr.q0) & 1) | (beta >> bit_of(pr.q1) & 1) << 1];
      for (int col = 0; col < 8; ++col) M[beta * 8 + col] *= f;
    }
  }
}

void split_gate(const cplx* M, cplx* left, cplx* out) {
  // M = diag(l0, l1) [[c, -s], [s, c]] diag(1, e^{i phi}) for unitary M: c = |M00| = |M11|,
  // s = |M10| = |M01|; each phase comes from an entry of modulus at least 1/sqrt(2) where
  // one exists, so rounding stays at the level of M's own.
  const double a = std::abs(M[0]), b = std::abs(M[2]), nrm = std::hypot(a, b);
  const double cs = a / nrm, sn = b / nrm;
  cplx l0, l1, ph(1.0, 0.0);
  auto unit = [](cplx z) { return z / std::abs(z); };
  if (a >= b) {
    l0 = unit(M[0]);
    if (b > 0.0) {
      l1 = unit(M[2]);
      ph = unit(M[3] / l1);
    } else {
      l1 = unit(M[3]);
    }
  } else {
    l1 = unit(M[2]);
    if (a > 0.0) {
      l0 = unit(M[0]);
      ph = unit(-M[1] / l0);
    } else {
      l0 = unit(-M[1]);
    }
  }
  left[0] = l0;
  left[1] = l1;
  out[0] = cplx(cs, -sn);  // row 0 of the real matrix
  out[1] = cplx(sn, cs);   // row 1
  out[2] = ph;
}

void bind_ctab(const Plan& p, const qsv_circuit* c, const double* params, const AngleOverride* ov, int n_ov,
               cplx* out) {
  std::vector<double> ang(3 * c->n_gates);
  for (size_t i = 0; i < c->n_gates; ++i) gate_angles(c->gates[i], params, &ang[3 * i]);
  for (int k = 0; k < n_ov; ++k) ang[3 * ov[k].gate + ov[k].slot] = ov[k].angle;
  // phase chains: the left diagonal each qubit carries to its next gate
  std::vector<cplx> carry(2 * (size_t)c->n_qubits, cplx(1.0, 0.0));
  for (const Fill& f : p.fills) {
    cplx* dst = out + f.offset;
    switch (f.kind) {
      case F_GATE_CHAIN: {
        const Prim& pr = p.prims[f.prim];
        cplx M[4];
        prim_numbers(pr, c, &ang[3 * pr.gate], M);
        cplx* cq = &carry[2 * (size_t)pr.q0];
        for (int r = 0; r < 2; ++r) {
          M[2 * r] *= cq[0];
          M[2 * r + 1] *= cq[1];
        }
        if (f.count) {
          split_gate(M, cq, dst);
          dst[3] = 0.0;
        } else {
          for (int e = 0; e < 4; ++e) dst[e] = M[e];
          cq[0] = cq[1] = cplx(1.0, 0.0);
        }
        break;
      }
      case F_PRIM_MATRIX: {
        const Prim& pr = p.prims[f.prim];
        prim_numbers(pr, c, &ang[3 * pr.gate], dst);
        break;
      }
      case F_PRIM_GEN:
        prim_gen(p.prims[f.prim], dst);
        break;
      case F_ZZ_PHASES: {
        const Prim& pr = p.prims[f.prim];
        const double th = ang[3 * pr.gate];
        const double sgn = pr.dagger ? 1.0 : -1.0;
        for (int cc = 0; cc <= f.count; ++cc) dst[cc] = std::polar(1.0, sgn * 0.5 * th * (f.count - 2 * cc));
        break;
      }
      case F_ZZ_GEN: {
        const Prim& pr = p.prims[f.prim];
        for (int cc = 0; cc <= f.count; ++cc) dst[cc] = cplx(pr.coeff * (double)(f.count - 2 * cc), 0.0);
        break;
      }
      case F_BLOCK: {
        cplx M[64];
        block_matrix(p, c, ang, p.blocks[f.prim], M);
        double r[256];
        block_operands(M, p.dtype, r);
        for (int e = 0; e < 128; ++e) dst[e] = cplx(r[2 * e], r[2 * e + 1]);
        break;
      }
      default:
        break;
    }
  }
}

std::vector<PauliGroup> group_pauli_sum(const qsv_pauli_sum* h) {
  std::vector<PauliGroup> groups;
  std::map<uint64_t, size_t> index;
  for (size_t k = 0; k < h->n_terms; ++k) {
    const uint64_t xm = h->x_masks[k], zm = h->z_masks[k];
    auto it = index.find(xm);
    size_t gi;
    if (it == index.end()) {
      gi = groups.size();
      index[xm] = gi;
      groups.push_back(PauliGroup{xm, {}, {}, {}});
    } else {
      gi = it->second;
    }
    // i^{popcount(x & z)}
    const int r = popc(xm & zm) & 3;
    const double c = h->coeffs[k];
    const double re[4] = {c, 0.0, -c, 0.0};
    const double im[4] = {0.0, c, 0.0, -c};
    groups[gi].zmasks.push_back(zm);
    groups[gi].cre.push_back(re[r]);
    groups[gi].cim.push_back(im[r]);
  }
  return groups;
}

}  // namespace qsv
