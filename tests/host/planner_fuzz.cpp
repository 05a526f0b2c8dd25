// Host driver of the planner under AddressSanitizer / UndefinedBehaviorSanitizer (no GPU).
//
// Random circuits with every gate kind, up to two controls, shared and fixed angles and
// explicit matrices are validated, lowered, planned (forward and adjoint, both amplitude
// types, every tile width from per-gate streaming up to 13 qubits, with and without
// relayout) and bound; Pauli sums are validated and grouped; invalid circuits must be
// rejected with QSV_EINVAL / QSV_ERANGE.  The structural facts checked on every plan:
// each op's table offsets and entry runs (diagonal runs, sign runs riding on gates, ZZ
// edges) lie inside the bound table and the plan's arrays,
// each pass's deposit entries and ops lie inside the plan's arrays, and every
// register layout of a register-blocked pass (load layout, after each LDS remap or
// cross-lane transposition) is a bijection of the tile's local bits whose transpositions
// name valid slot and lane bits and lead to the layout the op states, and every fused block's
// matrix-core operands decode to the real form of a complex matrix, unitary when its gates
// are (every kind but the explicit matrices, which this fuzzer draws at random, a third of
// them unitary).  One-qubit gates split into a phase and a real matrix (complex128 forward
// plans, on the random circuits and on brick-like circuits of general one-qubit gates):
// split_gate reproduces random and edge-case unitaries, and along each qubit the product of
// what the kernel applies (split gates, then the chain's dense last gate) equals the product
// of the gates' own matrices.
// Exit status 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "engine.h"
#include "qsv_ops.h"
using namespace qsv;

static const int kAngles[QSV_GATE_KIND_COUNT] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 3, 0, 0, 0};
static const int kTargets[QSV_GATE_KIND_COUNT] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 1, 2, 1, 2};

struct Circ {
  std::vector<qsv_gate> gates;
  std::vector<double> mats;
  qsv_circuit c{};
};

// A random 2x2 unitary: Gram-Schmidt on two complex Gaussian columns, times a random phase.
static void random_unitary(std::mt19937& rng, cplx* m) {
  std::normal_distribution<double> g(0.0, 1.0);
  cplx a0(g(rng), g(rng)), a1(g(rng), g(rng)), b0(g(rng), g(rng)), b1(g(rng), g(rng));
  const double na = std::sqrt(std::norm(a0) + std::norm(a1));
  a0 /= na;
  a1 /= na;
  const cplx pr = std::conj(a0) * b0 + std::conj(a1) * b1;
  b0 -= pr * a0;
  b1 -= pr * a1;
  const double nb = std::sqrt(std::norm(b0) + std::norm(b1));
  b0 /= nb;
  b1 /= nb;
  m[0] = a0;
  m[1] = b0;
  m[2] = a1;
  m[3] = b1;
}

static void random_circuit(Circ& k, int n, int n_gates, int n_params, std::mt19937& rng) {
  std::uniform_int_distribution<int> kind_d(0, QSV_GATE_KIND_COUNT - 1), q_d(0, n - 1), pi_d(0, n_params - 1);
  std::uniform_real_distribution<double> u(-3.0, 3.0);
  for (int i = 0; i < n_gates; ++i) {
    qsv_gate g{};
    g.kind = kind_d(rng);
    if (kTargets[g.kind] > n) g.kind = QSV_GATE_H;
    g.targets[0] = q_d(rng);
    g.targets[1] = -1;
    if (kTargets[g.kind] == 2)
      do g.targets[1] = q_d(rng); while (g.targets[1] == g.targets[0]);
    uint64_t used = 1ull << g.targets[0];
    if (g.targets[1] >= 0) used |= 1ull << g.targets[1];
    const int nc = (int)(rng() % 3);
    for (int j = 0; j < nc && __builtin_popcountll(used) < n; ++j) {
      int c;
      do c = q_d(rng); while (used >> c & 1);
      used |= 1ull << c;
      g.ctrl_mask |= 1ull << c;
    }
    for (int a = 0; a < 3; ++a) {
      g.param_index[a] = -1;
      if (a < kAngles[g.kind]) {
        if (rng() % 4 != 0) g.param_index[a] = pi_d(rng);
        g.param_coeff[a] = (rng() % 2) ? 1.0 : -0.5;
        g.angle_const[a] = u(rng);
      }
    }
    g.matrix_offset = -1;
    if (g.kind == QSV_GATE_MAT1 || g.kind == QSV_GATE_MAT2) {
      const int d = g.kind == QSV_GATE_MAT1 ? 2 : 4;
      g.matrix_offset = (int64_t)(k.mats.size() / 2);
      const int form = (int)(rng() % 3);  // 0: diagonal (the diagonal path), 1: random, 2: unitary
      if (form == 2 && d == 2) {
        cplx h[4];
        random_unitary(rng, h);
        for (const cplx& z : h) {
          k.mats.push_back(z.real());
          k.mats.push_back(z.imag());
        }
      } else {
        for (int r = 0; r < d; ++r)
          for (int cc = 0; cc < d; ++cc) {
            k.mats.push_back(form == 0 && r != cc ? 0.0 : u(rng));
            k.mats.push_back(form == 0 && r != cc ? 0.0 : u(rng));
          }
      }
    }
    k.gates.push_back(g);
  }
  k.c = qsv_circuit{n, 0, k.gates.data(), k.gates.size(), k.mats.data(), k.mats.size()};
}

static int g_unitary_blocks = 0;  // fused blocks whose unitarity was checked
static int g_split_gates = 0;     // split gates whose chain products were checked

static void mul2(const cplx* a, const cplx* b, cplx* out) {  // out = a b
  cplx t[4];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 2; ++k) t[2 * r + k] = a[2 * r] * b[k] + a[2 * r + 1] * b[2 + k];
  for (int i = 0; i < 4; ++i) out[i] = t[i];
}

// M = diag(l) R diag(1, ph) for random unitaries and unitaries with a zero or tiny entry.
static int check_split_gate(std::mt19937& rng) {
  std::vector<std::vector<cplx>> cases;
  for (int t = 0; t < 2000; ++t) {
    cplx m[4];
    random_unitary(rng, m);
    cases.push_back({m[0], m[1], m[2], m[3]});
  }
  const cplx e1 = std::polar(1.0, 0.7), e2 = std::polar(1.0, -2.1);
  for (double eps : {0.0, 1e-300, 1e-12, 1e-6}) {
    const double c = std::sqrt(1.0 - eps * eps);
    cases.push_back({e1 * c, -e2 * eps, std::conj(e2) * eps * e1 * e2, std::conj(e1) * c * e1 * e2});
    cases.push_back({e1 * eps, -e2 * c, std::conj(e2) * c * e1 * e2, std::conj(e1) * eps * e1 * e2});
  }
  for (const auto& M : cases) {
    // the split reproduces M to rounding plus M's own distance from unitarity
    double un = 0.0;
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 2; ++k)
        un = std::max(un, std::abs(M[2 * r] * std::conj(M[2 * k]) + M[2 * r + 1] * std::conj(M[2 * k + 1]) -
                                   (r == k ? 1.0 : 0.0)));
    cplx left[2], out[3];
    split_gate(M.data(), left, out);
    const cplx E[4] = {left[0] * out[0].real(), left[0] * out[0].imag() * out[2], left[1] * out[1].real(),
                       left[1] * out[1].imag() * out[2]};
    for (int i = 0; i < 4; ++i)
      if (std::abs(E[i] - M[i]) > 1e-15 + 4 * un) return 1;
    if (std::abs(std::abs(left[0]) - 1) > 1e-15 || std::abs(std::abs(left[1]) - 1) > 1e-15 ||
        std::abs(std::abs(out[2]) - 1) > 1e-15)
      return 2;
  }
  return 0;
}

// Along each qubit, the matrices the kernel applies for a phase chain (split gates as R
// diag(1, ph), the last gate dense) multiply to the gates' own matrices, read from the
// same circuit planned without the split; no phase is left at the end of the plan.
static int check_chains(const Plan& p, const Plan& plain, const qsv_circuit& c, const std::vector<double>& params) {
  std::vector<cplx> t1((size_t)p.ctab_size), t0((size_t)plain.ctab_size);
  bind_ctab(p, &c, params.data(), nullptr, 0, t1.data());
  bind_ctab(plain, &c, params.data(), nullptr, 0, t0.data());
  std::vector<int> own(p.prims.size(), -1);
  for (const Fill& f : plain.fills)
    if (f.kind == F_PRIM_MATRIX) own[f.prim] = f.offset;
  std::vector<cplx> E(4 * (size_t)c.n_qubits), U(4 * (size_t)c.n_qubits);
  std::vector<char> open(c.n_qubits, 0);
  auto reset = [&](int q) {
    for (int i = 0; i < 4; ++i) E[4 * q + i] = U[4 * q + i] = (i == 0 || i == 3) ? 1.0 : 0.0;
    open[q] = 0;
  };
  for (int q = 0; q < c.n_qubits; ++q) reset(q);
  for (const Fill& f : p.fills) {
    if (f.kind != F_GATE_CHAIN) continue;
    const int q = p.prims[f.prim].q0;
    if (own[f.prim] < 0) return 1;
    const cplx* g = &t0[own[f.prim]];
    const cplx* m = &t1[f.offset];
    cplx k[4];
    if (f.count) {
      k[0] = m[0].real();
      k[1] = m[0].imag() * m[2];
      k[2] = m[1].real();
      k[3] = m[1].imag() * m[2];
      ++g_split_gates;
    } else {
      for (int i = 0; i < 4; ++i) k[i] = m[i];
    }
    mul2(k, &E[4 * q], &E[4 * q]);
    mul2(g, &U[4 * q], &U[4 * q]);
    open[q] = f.count ? 1 : 0;
    if (!f.count) {
      for (int i = 0; i < 4; ++i)
        if (std::abs(E[4 * q + i] - U[4 * q + i]) > 1e-12) return 2;
      reset(q);
    }
  }
  for (int q = 0; q < c.n_qubits; ++q)
    if (open[q]) return 3;
  return 0;
}

static int check_plan(const Plan& p, const qsv_circuit& c, const std::vector<double>& params, int& checks) {
  std::vector<int> seen(p.prims.size(), 0);
  if (!p.unfused) {
    for (const DevPass& dp : p.passes) {
      if (dp.op_first < 0 || dp.op_first + dp.op_count > (int)p.ops.size()) return 1;
      if (dp.rb && (dp.dep_first < 0 || dp.dep_first + kDepEntries > (int)p.deps.size())) return 2;
      if (dp.m < 1 || dp.m > c.n_qubits || __builtin_popcountll(dp.tile_mask) != dp.m) return 3;
    }
    // register layouts of register-blocked passes: every layout is a bijection of the tile's
    // local bits onto slot and thread bits; cross-lane transpositions name a slot bit and a
    // lane bit of a full wave's lanes and lead exactly to the layout the op states; gates
    // name register slots of the current layout
    for (const DevPass& dp : p.passes) {
      if (!dp.rb) continue;
      const int r = dp.rb, nt = dp.m - r, lanes = nt < 6 ? nt : 6;
      int reg[4], thr[16];
      auto unpack = [&](uint32_t rp, uint64_t tp) {
        uint32_t seen_bits = 0;
        for (int i = 0; i < r; ++i) { reg[i] = (int)((rp >> (8 * i)) & 255); seen_bits |= 1u << reg[i]; }
        for (int t = 0; t < nt; ++t) { thr[t] = (int)((tp >> (4 * t)) & 15); seen_bits |= 1u << thr[t]; }
        return seen_bits == (1u << dp.m) - 1;
      };
      if (!unpack(dp.lay0_reg, dp.lay0_thr)) return 9;
      for (int i = 0; i < dp.op_count; ++i) {
        const TileOp& op = p.ops[dp.op_first + i];
        if (op.type == OP_XSWAP) {
          if (op.count != 1) return 10;
          for (int s2 = 0; s2 < op.count; ++s2) {
            const int code = (int)(((uint32_t)op.mat >> (8 * s2)) & 255u), sl = code & 3, ln = code >> 4;
            if (sl >= r || ln >= lanes || (code & 12)) return 10;
            std::swap(reg[sl], thr[ln]);
          }
          int reg2[4], thr2[16];
          std::copy(reg, reg + 4, reg2);
          std::copy(thr, thr + 16, thr2);
          if (!unpack((uint32_t)op.b, op.omask)) return 11;
          if (!std::equal(reg, reg + r, reg2) || !std::equal(thr, thr + nt, thr2)) return 11;
        } else if (op.type == OP_REMAP) {
          if (!unpack((uint32_t)op.b, op.omask)) return 12;
          uint32_t rm = 0;
          for (int k = 0; k < r; ++k) rm |= 1u << reg[k];
          if ((uint32_t)op.a != rm) return 12;
        } else if (op.type == OP_DENSE1 && (op.a < 0 || op.a >= r)) {
          return 13;
        } else if (op.type == OP_BLOCK && (op.a < 0 || op.a >= r || nt < 6 || op.mat + 128 > p.ctab_size)) {
          return 14;
        }
      }
    }
    for (const TileOp& op : p.ops) {
      if (op.type != OP_XSWAP && (op.mat >= p.ctab_size || op.gen >= p.ctab_size)) return 4;
      if ((op.type == OP_DIAG && op.first + op.count > (int)p.diag.size()) ||
          (op.type == OP_ZZ && op.first + op.count > (int)p.edges.size()))
        return 5;
      if (((op.type == OP_DENSE1 && op.b) || (op.plain & kPlainSigns)) && op.first + op.count > (int)p.diag.size())
        return 5;
    }
    for (const DiagEntry& d : p.diag)
      if (d.mat >= p.ctab_size || d.gen >= p.ctab_size) return 6;
  } else {
    for (size_t i = 0; i < p.stream_mat.size(); ++i)
      if (p.stream_mat[i] >= p.ctab_size) return 7;
  }
  std::vector<cplx> tab((size_t)p.ctab_size + 1);
  bind_ctab(p, &c, params.data(), nullptr, 0, tab.data());
  for (const cplx& v : tab)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return 8;
  // fused blocks: the matrix-core operands decode to a unitary 8x8 matrix (read back through
  // the lane-major A-operand layout, the accumulator row order of the amplitude type and the
  // real embedding of complex numbers, each written out here independently of the planner)
  for (const Fill& f : p.fills) {
    if (f.kind != F_BLOCK) continue;
    const auto& bs = p.blocks[f.prim];
    if (bs.q[0] == bs.q[1] || bs.q[0] == bs.q[2] || bs.q[1] == bs.q[2]) return 15;
    bool unitary_gates = true;  // this fuzzer's explicit matrices are not unitary
    for (int32_t pi : bs.prims) {
      const int kind = c.gates[p.prims[pi].gate].kind;
      unitary_gates &= kind != QSV_GATE_MAT1 && kind != QSV_GATE_MAT2;
    }
    double mp[16][16], mr[16][16];
    for (int l = 0; l < 64; ++l)
      for (int j = 0; j < 4; ++j) {
        const cplx e = tab[f.offset + (4 * l + j) / 2];
        mp[l % 16][4 * j + l / 16] = ((4 * l + j) % 2) ? e.imag() : e.real();
      }
    for (int m = 0; m < 16; ++m)
      for (int k = 0; k < 16; ++k) mr[p.dtype == QSV_C64 ? (m / 4) + 4 * (m % 4) : m][k] = mp[m][k];
    auto row = [](int beta, int ri) { return (beta & 3) + 4 * ri + 8 * (beta >> 2); };
    cplx M[8][8];
    for (int bo = 0; bo < 8; ++bo)
      for (int bi = 0; bi < 8; ++bi) {
        const double a = mr[row(bo, 0)][row(bi, 0)], b = mr[row(bo, 1)][row(bi, 0)];
        if (mr[row(bo, 1)][row(bi, 1)] != a || mr[row(bo, 0)][row(bi, 1)] != -b) return 16;
        M[bo][bi] = cplx(a, b);
      }
    g_unitary_blocks += unitary_gates;
    for (int i = 0; i < 8 && unitary_gates; ++i)
      for (int j = 0; j < 8; ++j) {
        cplx d = 0.0;
        for (int k = 0; k < 8; ++k) d += std::conj(M[k][i]) * M[k][j];
        if (std::abs(d - (i == j ? 1.0 : 0.0)) > 1e-12) return 17;
      }
  }
  ++checks;
  return 0;
}

int main() {
  std::mt19937 rng(2406);
  int bad = 0, checks = 0;
  try {
    if (const int r = check_split_gate(rng)) {
      printf("split_gate check %d failed\n", r);
      bad = 1;
    }
    // brick-like circuits of general one-qubit gates (unitary matrices and U3) between CZ
    // layers: long phase chains, across rounds and passes
    for (int trial = 0; trial < 12; ++trial) {
      const int n = 9 + trial % 6;
      Circ k;
      std::uniform_real_distribution<double> ang(-3.0, 3.0);
      for (int layer = 0; layer < 6; ++layer) {
        for (int q = 0; q < n; ++q) {
          qsv_gate g{};
          for (int a = 0; a < 3; ++a) g.param_index[a] = -1;
          g.targets[0] = q;
          g.targets[1] = -1;
          g.matrix_offset = -1;
          if ((q + layer + trial) % 3 == 0) {
            g.kind = QSV_GATE_U3;
            for (int a = 0; a < 3; ++a) g.angle_const[a] = ang(rng);
          } else {
            g.kind = QSV_GATE_MAT1;
            g.matrix_offset = (int64_t)(k.mats.size() / 2);
            cplx h[4];
            random_unitary(rng, h);
            for (const cplx& z : h) {
              k.mats.push_back(z.real());
              k.mats.push_back(z.imag());
            }
          }
          k.gates.push_back(g);
        }
        for (int a = layer % 2; a + 1 < n; a += 2) {
          qsv_gate g{};
          for (int b = 0; b < 3; ++b) g.param_index[b] = -1;
          g.kind = QSV_GATE_Z;
          g.targets[0] = a + 1;
          g.targets[1] = -1;
          g.ctrl_mask = 1ull << a;
          g.matrix_offset = -1;
          k.gates.push_back(g);
        }
      }
      k.c = qsv_circuit{n, 0, k.gates.data(), k.gates.size(), k.mats.data(), k.mats.size()};
      validate_circuit(&k.c, 0, n);
      for (int tile : {9, 10, 11, 12})
        for (bool relayout : {false, true}) {
          PlanOptions o = state_plan_options(QSV_C128, n, tile, tile, false, true, relayout);
          const Plan p = build_plan(&k.c, false, o);
          PlanOptions o2 = o;
          o2.split = false;
          const std::vector<double> none;
          int r = check_plan(p, k.c, none, checks);
          if (!r) r = check_chains(p, build_plan(&k.c, false, o2), k.c, none);
          if (r) {
            printf("brick trial %d n=%d tile=%d relayout=%d: check %d failed\n", trial, n, tile, (int)relayout, r);
            bad = 1;
          }
        }
    }
    for (int trial = 0; trial < 60; ++trial) {
      const int n = 2 + trial % 15;
      Circ k;
      random_circuit(k, n, 40 + trial, 5, rng);
      std::vector<double> params(5);
      for (double& v : params) v = std::uniform_real_distribution<double>(-3, 3)(rng);
      validate_circuit(&k.c, params.size(), n);
      for (int dtype : {QSV_C64, QSV_C128})
        for (bool adjoint : {false, true})
          for (int tile : {0, 2, 3, 5, 8, 9, 10, 11, 12, 13}) {
            if (adjoint && tile == 0) continue;
            for (bool relayout : {false, true}) {
              PlanOptions o = state_plan_options(dtype, n, tile, tile, adjoint, true, relayout);
              const Plan p = build_plan(&k.c, adjoint, o);
              int r = check_plan(p, k.c, params, checks);
              if (!r && o.split) {
                PlanOptions o2 = o;
                o2.split = false;
                const int rc = check_chains(p, build_plan(&k.c, adjoint, o2), k.c, params);
                if (rc) r = 100 + rc;
              }
              if (r) {
                printf("trial %d n=%d dtype=%d adjoint=%d tile=%d relayout=%d: check %d failed\n", trial, n, dtype,
                       (int)adjoint, tile, (int)relayout, r);
                bad = 1;
              }
            }
          }
      // Pauli sums
      std::vector<double> co(12);
      std::vector<uint64_t> xm(12), zm(12);
      for (int t = 0; t < 12; ++t) {
        co[t] = std::uniform_real_distribution<double>(-1, 1)(rng);
        xm[t] = rng() & ((1ull << n) - 1);
        zm[t] = rng() & ((1ull << n) - 1);
      }
      const qsv_pauli_sum h{co.size(), co.data(), xm.data(), zm.data()};
      validate_pauli_sum(&h, n);
      size_t terms = 0;
      for (const PauliGroup& g : group_pauli_sum(&h)) terms += g.zmasks.size();
      if (terms != co.size()) {
        printf("pauli grouping lost terms\n");
        bad = 1;
      }
    }
    // invalid circuits are rejected before planning
    auto expect_reject = [&](qsv_gate g, int n, size_t n_params, int status, const char* what) {
      const double m[32] = {1, 0, 0, 0, 0, 0, 1, 0};
      const qsv_circuit c{n, 0, &g, 1, m, 8};
      try {
        validate_circuit(&c, n_params, n);
      } catch (const Error& e) {
        if (e.status == status) return;
      }
      printf("not rejected: %s\n", what);
      bad = 1;
    };
    qsv_gate g{};
    g.kind = QSV_GATE_RX;
    g.targets[0] = 0;
    for (int a = 0; a < 3; ++a) g.param_index[a] = -1;
    qsv_gate t = g;
    t.targets[0] = 7;
    expect_reject(t, 3, 0, QSV_EINVAL, "target out of range");
    t = g;
    t.ctrl_mask = 1;
    expect_reject(t, 3, 0, QSV_EINVAL, "control on target");
    t = g;
    t.param_index[0] = 4;
    expect_reject(t, 3, 2, QSV_EINVAL, "parameter index out of range");
    t = g;
    t.param_index[1] = 0;
    expect_reject(t, 3, 2, QSV_EINVAL, "unused angle slot");
    t = g;
    t.angle_const[0] = NAN;
    expect_reject(t, 3, 0, QSV_EINVAL, "non-finite angle");
    t = g;
    t.kind = QSV_GATE_MAT2;
    t.targets[1] = 1;
    t.matrix_offset = 1;
    expect_reject(t, 3, 0, QSV_EINVAL, "matrix out of range");
    expect_reject(g, 40, 0, QSV_ERANGE, "too many qubits");
  } catch (const Error& e) {
    printf("planner error %d: %s\n", e.status, e.msg.c_str());
    return 2;
  }
  printf("plans checked: %d\n", checks);
  printf("unitary fused blocks checked: %d\n", g_unitary_blocks);
  printf("split gates checked along their chains: %d\n", g_split_gates);
  return bad || checks < 1000 || g_unitary_blocks < 100 || g_split_gates < 1000;
}
