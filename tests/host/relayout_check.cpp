// Host-side check of the planner's relayouting forward plans (no GPU): following every
// logical amplitude through the planner's address tables, each pass must read it where the
// previous pass wrote it, write a permutation of the state, and the last pass must leave the
// natural layout.  Random brick-like circuits with long-range CZs, several widths and both
// register-block sizes.  Prints one line per plan; exit status 0 when all hold.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <random>
#include "engine.h"
#include "qsv_ops.h"
using namespace qsv;
static uint64_t run_base(const uint64_t* d, int at, uint64_t tile) {
  uint64_t r = 0; int nr = (int)d[at];
  for (int i = 0; i < nr; ++i) { uint64_t e = d[at + 1 + i]; int lo = e & 255, len = (e >> 8) & 255, sh = (e >> 16) & 255;
    r |= ((tile >> sh) & ((1ull << len) - 1)) << lo; }
  return r;
}
static int check(const qsv_circuit& c, int tile, int dtype, int low, int* relayouted) {
  PlanOptions o; o.tile_qubits = tile; o.dtype = dtype; o.low_qubits = low; o.relayout = true;
  if (dtype == 0) o.reg_bits = 4;
  Plan p = build_plan(&c, false, o);
  const int n = c.n_qubits;
  const uint64_t N = 1ull << n;
  // where[logical] = physical position currently holding it
  std::vector<uint64_t> where(N);
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
        // logical index: local bits deposited at the tile qubits
        uint64_t lg = lb, mm = dp.tile_mask, jj = j;
        for (; mm; mm &= mm - 1, jj >>= 1) if (jj & 1) lg |= mm & (~mm + 1);
        const uint64_t rd = ldb | d[j & 127] | d[128 + (j >> 7)];
        const uint64_t wr = stb | (dp.relayout ? (d[256 + (j & 127)] | d[384 + (j >> 7)]) : (d[j & 127] | d[128 + (j >> 7)]));
        if (rd != where[lg]) { printf("pass %zu tile %llu j %llu: reads %llx, data at %llx\n", pi, (unsigned long long)t, (unsigned long long)j, (unsigned long long)rd, (unsigned long long)where[lg]); return 1; }
        if (wr >= N || seen[wr]) { printf("pass %zu: store collision/out of range at %llx\n", pi, (unsigned long long)wr); return 1; }
        seen[wr] = 1;
        nw[lg] = wr;
      }
    }
    where.swap(nw);
  }
  for (uint64_t i = 0; i < N; ++i) if (where[i] != i) { printf("final layout not natural at %llu\n", (unsigned long long)i); return 1; }
  int nrel = 0;
  for (auto& dp : p.passes) nrel += dp.relayout;
  *relayouted += p.relayout ? 1 : 0;
  printf("ok n=%d tile=%d dtype=%d passes=%zu relayout=%d relayout_passes=%d\n", n, tile, dtype, p.passes.size(), (int)p.relayout, nrel);
  return 0;
}
int main() {
  std::mt19937 rng(7);
  int bad = 0;
  int relayouted = 0;
  for (int trial = 0; trial < 24; ++trial) {
    const int n = 14 + trial % 5;
    std::vector<qsv_gate> gates;
    std::vector<double> mats;
    for (int l = 0; l < 8; ++l) {
      for (int q = 0; q < n; ++q) {
        qsv_gate g{}; g.kind = QSV_GATE_MAT1; g.targets[0] = q; g.matrix_offset = (int64_t)mats.size();
        for (int k = 0; k < 8; ++k) mats.push_back(k == 0 || k == 6 ? 1.0 : 0.0);
        for (int a = 0; a < 3; ++a) g.param_index[a] = -1;
        gates.push_back(g);
      }
      for (int a = (l % 2); a + 1 < n; a += 2) {
        qsv_gate g{}; g.kind = QSV_GATE_Z; g.targets[0] = a + 1; g.ctrl_mask = 1ull << a;
        for (int k = 0; k < 3; ++k) g.param_index[k] = -1;
        gates.push_back(g);
      }
      // a random long-range CZ
      qsv_gate g{}; g.kind = QSV_GATE_Z; int a = rng() % n, b = rng() % n; if (a == b) b = (a + 1) % n;
      g.targets[0] = a; g.ctrl_mask = 1ull << b; for (int k = 0; k < 3; ++k) g.param_index[k] = -1;
      gates.push_back(g);
    }
    qsv_circuit c{n, 0, gates.data(), gates.size(), mats.data(), mats.size()};
    bad |= check(c, 9 + trial % 3, trial % 2, 1 + trial % 2, &relayouted);
  }
  printf("relayouting plans: %d\n", relayouted);
  return bad || relayouted < 6;
}
