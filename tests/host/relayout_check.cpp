// Host-side check of the planner's relayouting forward plans (no GPU).
//
// 1. Random brick-like circuits with long-range CZs at several widths and both register-
//    block sizes, n = 14..18: every logical amplitude is followed through the planner's
//    address tables.  Each pass must read it where the previous pass wrote it and write a
//    permutation of the state, and the last pass must leave the natural layout.
// 2. The 30-qubit depth-20 brick circuit (the structure the benchmark runs; its matrices
//    are dense, which is all the planner looks at) with the library's own default options
//    for both amplitude types.  Following 2^30 amplitudes is too slow, so the check uses
//    linearity instead: a tile's base is a deposit of tile-index bits (runs) and a local
//    index's offset is an OR of two deposit tables, so once the tables are shown to be
//    linear with disjoint images, each pass's read and write maps are fixed by the images
//    of single logical bits.  Each must be a bit permutation, pass p+1 must read with the
//    permutation pass p wrote with, and the first read and last write must be the identity.
//
// Prints one line per plan; exit status 0 when every check holds.  Built with
// -fsanitize=address,undefined by the test that runs it.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "engine.h"
#include "qsv_ops.h"
using namespace qsv;

static uint64_t run_base(const uint64_t* d, int at, uint64_t tile) {
  uint64_t r = 0;
  const int nr = (int)d[at];
  for (int i = 0; i < nr; ++i) {
    const uint64_t e = d[at + 1 + i];
    const int lo = e & 255, len = (e >> 8) & 255, sh = (e >> 16) & 255;
    r |= ((tile >> sh) & ((1ull << len) - 1)) << lo;
  }
  return r;
}

static void append_gate(std::vector<qsv_gate>& gates, int kind, int target, uint64_t ctrls, int64_t moff) {
  qsv_gate g{};
  g.kind = kind;
  g.targets[0] = target;
  g.targets[1] = -1;
  g.ctrl_mask = ctrls;
  for (int a = 0; a < 3; ++a) g.param_index[a] = -1;
  g.matrix_offset = moff;
  gates.push_back(g);
}

// One dense 2x2 matrix (a real rotation), appended to mats; returns its offset in complex
// elements, as qsv_gate::matrix_offset counts.
static int64_t push_matrix(std::vector<double>& mats, double t) {
  const int64_t off = (int64_t)(mats.size() / 2);
  const double c = std::cos(t), s = std::sin(t);
  const double m[8] = {c, 0, -s, 0, s, 0, c, 0};
  mats.insert(mats.end(), m, m + 8);
  return off;
}

static Plan plan_for(const qsv_circuit& c, const PlanOptions& o) {
  validate_circuit(&c, 0, c.n_qubits);
  return build_plan(&c, false, o);
}

// ---- 1: every amplitude, small n ---------------------------------------------------------------
static int check_walk(const qsv_circuit& c, int tile, int dtype, int low, int* relayouted) {
  PlanOptions o;
  o.tile_qubits = tile;
  o.dtype = dtype;
  o.low_qubits = low;
  o.relayout = true;
  if (dtype == QSV_C64) o.reg_bits = 4;
  Plan p = plan_for(c, o);
  const int n = c.n_qubits;
  const uint64_t N = 1ull << n;
  std::vector<uint64_t> where(N);  // where[logical] = physical position holding it
  for (uint64_t i = 0; i < N; ++i) where[i] = i;
  for (size_t pi = 0; pi < p.passes.size(); ++pi) {
    const DevPass& dp = p.passes[pi];
    const uint64_t* d = p.deps.data() + dp.dep_first;
    std::vector<uint64_t> nw(N, ~0ull);
    std::vector<char> seen(N, 0);
    const uint64_t tiles = 1ull << (n - dp.m);
    for (uint64_t t = 0; t < tiles; ++t) {
      const uint64_t lb = run_base(d, kRunsLogical, t);
      const uint64_t ldb = dp.relayout ? run_base(d, kRunsLoad, t) : lb;
      const uint64_t stb = dp.relayout ? run_base(d, kRunsStore, t) : lb;
      for (uint64_t j = 0; j < (1ull << dp.m); ++j) {
        uint64_t lg = lb, mm = dp.tile_mask, jj = j;  // local bits deposited at the tile qubits
        for (; mm; mm &= mm - 1, jj >>= 1)
          if (jj & 1) lg |= mm & (~mm + 1);
        const uint64_t rd = ldb | d[j & 127] | d[128 + (j >> 7)];
        const uint64_t wr =
            stb | (dp.relayout ? (d[256 + (j & 127)] | d[384 + (j >> 7)]) : (d[j & 127] | d[128 + (j >> 7)]));
        if (rd != where[lg]) {
          printf("pass %zu tile %llu j %llu: reads %llx, data at %llx\n", pi, (unsigned long long)t,
                 (unsigned long long)j, (unsigned long long)rd, (unsigned long long)where[lg]);
          return 1;
        }
        if (wr >= N || seen[wr]) {
          printf("pass %zu: store collision/out of range at %llx\n", pi, (unsigned long long)wr);
          return 1;
        }
        seen[wr] = 1;
        nw[lg] = wr;
      }
    }
    where.swap(nw);
  }
  for (uint64_t i = 0; i < N; ++i)
    if (where[i] != i) {
      printf("final layout not natural at %llu\n", (unsigned long long)i);
      return 1;
    }
  int nrel = 0, ndense = 0;
  for (auto& dp : p.passes) nrel += dp.relayout;
  for (auto& op : p.ops) ndense += op.type == OP_DENSE1;
  *relayouted += p.relayout ? 1 : 0;
  printf("ok walk n=%d tile=%d dtype=%d passes=%zu relayout=%d relayout_passes=%d dense_ops=%d\n", n, tile, dtype,
         p.passes.size(), (int)p.relayout, nrel, ndense);
  return ndense > 0 ? 0 : 1;  // the dense gates must reach the plan
}

// ---- 2: single-bit images, any n ---------------------------------------------------------------
static bool single_bit(uint64_t v) { return v && !(v & (v - 1)); }

// Linear deposit table: entry j is the OR of the entries of j's bits, and those are disjoint
// single bits.  `used` entries are checked.
static bool table_linear(const uint64_t* t, int used) {
  if (t[0] != 0) return false;
  uint64_t seen = 0;
  for (int b = 0; (1 << b) < used; ++b) {
    const uint64_t v = t[1 << b];
    if (!single_bit(v) || (v & seen)) return false;
    seen |= v;
  }
  for (int j = 0; j < used; ++j) {
    uint64_t o = 0;
    for (int b = 0; (1 << b) <= j; ++b)
      if (j >> b & 1) o |= t[1 << b];
    if (t[j] != o) return false;
  }
  return true;
}

// Images of the n logical bits under a pass's read (store = false) or write map.
static bool pass_map(const DevPass& dp, const uint64_t* d, int n, bool store, std::vector<uint64_t>& img) {
  const int lo_used = dp.m >= 7 ? 128 : (1 << dp.m);
  const int hi_used = dp.m > 7 ? (1 << (dp.m - 7)) : 1;
  const uint64_t* tl = d + (store && dp.relayout ? 256 : 0);
  const uint64_t* th = tl + 128;
  if (!table_linear(tl, lo_used) || !table_linear(th, hi_used)) {
    printf("deposit table not linear\n");
    return false;
  }
  const int runs = dp.relayout ? (store ? kRunsStore : kRunsLoad) : kRunsLogical;
  img.assign(n, 0);
  int local = 0;
  for (int q = 0; q < n; ++q) {
    if (dp.tile_mask >> q & 1) {
      const uint64_t j = 1ull << local++;
      img[q] = tl[j & 127] | th[j >> 7];
      continue;
    }
    // the tile-index bit whose logical base is qubit q
    int tbit = -1;
    for (int t = 0; t < n - dp.m; ++t)
      if (run_base(d, kRunsLogical, 1ull << t) == (1ull << q)) tbit = t;
    if (tbit < 0) {
      printf("qubit %d is neither a tile qubit nor a tile-index bit\n", q);
      return false;
    }
    img[q] = run_base(d, runs, 1ull << tbit);
  }
  uint64_t all = 0;
  for (int q = 0; q < n; ++q) {
    if (!single_bit(img[q]) || (img[q] & all) || img[q] >> n) {
      printf("map is not a bit permutation at qubit %d\n", q);
      return false;
    }
    all |= img[q];
  }
  return true;
}

static int check_linear(const qsv_circuit& c, const PlanOptions& o, const char* name) {
  Plan p = plan_for(c, o);
  const int n = c.n_qubits;
  std::vector<uint64_t> prev(n), rd, wr;
  for (int q = 0; q < n; ++q) prev[q] = 1ull << q;
  int nrel = 0;
  for (size_t pi = 0; pi < p.passes.size(); ++pi) {
    const DevPass& dp = p.passes[pi];
    if (!dp.rb) {
      printf("%s: pass %zu is not register-blocked\n", name, pi);
      return 1;
    }
    const uint64_t* d = p.deps.data() + dp.dep_first;
    if (!pass_map(dp, d, n, false, rd) || !pass_map(dp, d, n, true, wr)) {
      printf("%s: pass %zu\n", name, pi);
      return 1;
    }
    if (rd != prev) {
      printf("%s: pass %zu does not read where pass %zu wrote\n", name, pi, pi - 1);
      return 1;
    }
    prev = wr;
    nrel += dp.relayout;
  }
  for (int q = 0; q < n; ++q)
    if (prev[q] != (1ull << q)) {
      printf("%s: final layout not natural\n", name);
      return 1;
    }
  printf("ok linear %s n=%d tile=%d passes=%zu relayout=%d relayout_passes=%d\n", name, n, o.tile_qubits,
         p.passes.size(), (int)p.relayout, nrel);
  return (p.relayout && nrel > 0) ? 0 : 1;
}

// The benchmark's brick structure: per layer a dense 2x2 gate on every qubit, then CZ on
// (2i, 2i+1) for even layers and (2i+1, 2i+2) for odd layers.
static void brick(int n, int depth, std::vector<qsv_gate>& gates, std::vector<double>& mats, std::mt19937& rng) {
  std::uniform_real_distribution<double> ang(0.1, 1.4);
  for (int l = 0; l < depth; ++l) {
    for (int q = 0; q < n; ++q) append_gate(gates, QSV_GATE_MAT1, q, 0, push_matrix(mats, ang(rng)));
    for (int a = l % 2; a + 1 < n; a += 2) append_gate(gates, QSV_GATE_Z, a + 1, 1ull << a, -1);
  }
}

int main() {
  int bad = 0;
  try {
    std::mt19937 rng(7);
    int relayouted = 0;
    for (int trial = 0; trial < 24; ++trial) {
      const int n = 14 + trial % 5;
      std::vector<qsv_gate> gates;
      std::vector<double> mats;
      brick(n, 8, gates, mats, rng);
      for (int k = 0; k < 8; ++k) {  // random long-range CZs
        int a = rng() % n, b = rng() % n;
        if (a == b) b = (a + 1) % n;
        append_gate(gates, QSV_GATE_Z, a, 1ull << b, -1);
      }
      const qsv_circuit c{n, 0, gates.data(), gates.size(), mats.data(), mats.size()};
      bad |= check_walk(c, 9 + trial % 3, trial % 2, 1 + trial % 2, &relayouted);
    }
    printf("relayouting plans: %d\n", relayouted);
    bad |= relayouted < 6;

    std::vector<qsv_gate> gates;
    std::vector<double> mats;
    brick(30, 20, gates, mats, rng);
    const qsv_circuit c{30, 0, gates.data(), gates.size(), mats.data(), mats.size()};
    for (int dtype : {QSV_C128, QSV_C64}) {
      const PlanOptions o = state_plan_options(dtype, 30, default_tile_qubits(dtype), default_adj_tile_qubits(dtype),
                                               false, true, true);
      bad |= check_linear(c, o, dtype == QSV_C64 ? "brick30 complex64" : "brick30 complex128");
    }
  } catch (const Error& e) {
    printf("planner error %d: %s\n", e.status, e.msg.c_str());
    return 2;
  }
  return bad;
}
