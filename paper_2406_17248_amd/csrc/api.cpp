// C ABI of the engine: state management, uploads, pass orchestration, reductions.
#include <algorithm>
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/qsv.h"
#include "engine.h"
#include "hip_util.h"
#include "noalloc.h"
#include "qsv_kernels.h"

using namespace qsv;

namespace qsv {
std::string& last_error() {
  thread_local std::string msg;
  return msg;
}
}  // namespace qsv

namespace {

[[noreturn]] void fail(int status, const std::string& msg) { throw Error{status, msg}; }

}  // namespace

struct qsv_state {
  int32_t n = 0;
  int32_t dtype = 0;
  int device = 0;
  void* psi = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  int64_t opt[QSV_OPT_COUNT] = {0, 0, 0, 0, 0};
  // profiling: per kernel class, pending (start, stop) event pairs and bytes
  struct Rec { hipEvent_t a, b; int cls; double bytes; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> free_events;
  double prof_ms[QSV_K_COUNT] = {0, 0, 0, 0, 0};
  int64_t prof_n[QSV_K_COUNT] = {0, 0, 0, 0, 0};
  double prof_bytes[QSV_K_COUNT] = {0, 0, 0, 0, 0};
  DevBuf ws_psi, ws_lam, ws_aux1, ws_aux2, upload, partials, gpart, outbuf, pauli;
  DevBuf relay;               // second state buffer of relayouting forward passes
  bool relay_failed = false;  // its allocation failed once: run in place from then on
  // pinned staging for uploads and downloads, guarded by an event
  void* stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_ev = nullptr;
  bool stage_pending = false;
  // identity of the evolved states left in ws_psi by qsv_forward_batch ("" if none); it
  // includes `generation`, which every entry point that writes the amplitudes bumps
  std::string fwd_token;
  uint64_t generation = 0;
  std::unordered_map<std::string, std::unique_ptr<Plan>> plans;

  size_t amp_bytes() const { return dtype == QSV_C64 ? 8 : 16; }
  uint64_t namps() const { return 1ull << n; }
};

namespace {

void set_device(qsv_state* s) { hip_check(hipSetDevice(s->device), "hipSetDevice"); }

hipEvent_t take_event(qsv_state* s) {
  if (!s->free_events.empty()) {
    hipEvent_t e = s->free_events.back();
    s->free_events.pop_back();
    return e;
  }
  hipEvent_t e;
  hip_check(hipEventCreate(&e), "hipEventCreate");
  return e;
}

// Collect finished profiling records into the per-class totals.
void prof_collect(qsv_state* s) {
  for (auto& r : s->recs) {
    hip_check(hipEventSynchronize(r.b), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
    s->prof_ms[r.cls] += ms;
    s->prof_n[r.cls] += 1;
    s->prof_bytes[r.cls] += r.bytes;
    s->free_events.push_back(r.a);
    s->free_events.push_back(r.b);
  }
  s->recs.clear();
}

// Time one launch (when profiling is on).
template <typename F>
void timed(qsv_state* s, int cls, double bytes, F&& launch, const char* what) {
  if (!s->opt[QSV_OPT_PROFILE]) {
    hip_check(launch(), what);
    return;
  }
  if (s->recs.size() > 4096) prof_collect(s);
  hipEvent_t a = take_event(s), b = take_event(s);
  hip_check(hipEventRecord(a, s->stream), "hipEventRecord");
  hip_check(launch(), what);
  hip_check(hipEventRecord(b, s->stream), "hipEventRecord");
  s->recs.push_back({a, b, cls, bytes});
}

void* stage_acquire(qsv_state* s, size_t bytes) {
  if (s->stage_pending) {
    hip_check(hipEventSynchronize(s->stage_ev), "hipEventSynchronize");
    s->stage_pending = false;
  }
  if (bytes > s->stage_bytes) {
    if (s->stage) (void)hipHostFree(s->stage);
    s->stage = nullptr;
    s->stage_bytes = 0;
    const size_t nb = align_up(bytes, 1 << 20);
    hip_check(hipHostMalloc(&s->stage, nb, hipHostMallocDefault), "hipHostMalloc staging");
    s->stage_bytes = nb;
  }
  return s->stage;
}

void stage_release_after_queue(qsv_state* s) {
  hip_check(hipEventRecord(s->stage_ev, s->stream), "hipEventRecord");
  s->stage_pending = true;
}

// Default options per dtype.
void default_options(qsv_state* s) {
  s->opt[QSV_OPT_TILE_QUBITS] = default_tile_qubits(s->dtype);
  s->opt[QSV_OPT_ADJ_TILE_QUBITS] = default_adj_tile_qubits(s->dtype);
  s->opt[QSV_OPT_THREADS] = 512;
  s->opt[QSV_OPT_RELAYOUT] = 1;
}

PlanOptions plan_options(const qsv_state* s, bool adjoint, bool fuse_zz, bool relayout = false) {
  return state_plan_options(s->dtype, s->n, (int32_t)s->opt[QSV_OPT_TILE_QUBITS],
                            (int32_t)s->opt[QSV_OPT_ADJ_TILE_QUBITS], adjoint, fuse_zz, relayout);
}

const Plan& get_plan(qsv_state* s, const qsv_circuit* c, bool adjoint, bool fuse_zz, bool relayout = false) {
  const PlanOptions o = plan_options(s, adjoint, fuse_zz, relayout);
  std::string key = structure_key(c, adjoint, o);
  auto it = s->plans.find(key);
  if (it != s->plans.end()) return *it->second;
  if (s->plans.size() > 64) s->plans.clear();
  auto p = std::make_unique<Plan>(build_plan(c, adjoint, o));
  const Plan& ref = *p;
  s->plans.emplace(std::move(key), std::move(p));
  return ref;
}

// Device copies of a plan's op lists and of per-batch-item complex tables.
struct Uploaded {
  TileOp* ops = nullptr;
  DiagEntry* diag = nullptr;
  ZZEdge* edges = nullptr;
  uint64_t* deps = nullptr;
  void* ctab = nullptr;
  int64_t ctab_stride = 0;  // complex entries per batch item
};

// Pack one or two plans and their bound tables into one upload.
struct UploadReq {
  const Plan* plan;
  const std::vector<cplx>* ctab;  // batch * plan->ctab_size entries
  int batch;
};

void upload_plans(qsv_state* s, const UploadReq* reqs, int n_req, Uploaded* out) {
  const size_t cs = s->amp_bytes();
  size_t off = 0;
  std::vector<size_t> o_ops(n_req), o_diag(n_req), o_edges(n_req), o_deps(n_req), o_ctab(n_req);
  for (int r = 0; r < n_req; ++r) {
    const Plan& p = *reqs[r].plan;
    o_ops[r] = off; off = align_up(off + p.ops.size() * sizeof(TileOp), 256);
    o_diag[r] = off; off = align_up(off + p.diag.size() * sizeof(DiagEntry), 256);
    o_edges[r] = off; off = align_up(off + p.edges.size() * sizeof(ZZEdge), 256);
    o_deps[r] = off; off = align_up(off + p.deps.size() * sizeof(uint64_t), 256);
    o_ctab[r] = off; off = align_up(off + (size_t)reqs[r].batch * p.ctab_size * cs, 256);
  }
  const size_t total = off ? off : 256;
  char* st = static_cast<char*>(stage_acquire(s, total));
  for (int r = 0; r < n_req; ++r) {
    const Plan& p = *reqs[r].plan;
    if (!p.ops.empty()) std::memcpy(st + o_ops[r], p.ops.data(), p.ops.size() * sizeof(TileOp));
    if (!p.diag.empty()) std::memcpy(st + o_diag[r], p.diag.data(), p.diag.size() * sizeof(DiagEntry));
    if (!p.edges.empty()) std::memcpy(st + o_edges[r], p.edges.data(), p.edges.size() * sizeof(ZZEdge));
    if (!p.deps.empty()) std::memcpy(st + o_deps[r], p.deps.data(), p.deps.size() * sizeof(uint64_t));
    const std::vector<cplx>& ct = *reqs[r].ctab;
    const size_t ne = (size_t)reqs[r].batch * p.ctab_size;
    if (s->dtype == QSV_C64) {
      float* d = reinterpret_cast<float*>(st + o_ctab[r]);
      for (size_t k = 0; k < ne; ++k) { d[2 * k] = (float)ct[k].real(); d[2 * k + 1] = (float)ct[k].imag(); }
    } else {
      double* d = reinterpret_cast<double*>(st + o_ctab[r]);
      for (size_t k = 0; k < ne; ++k) { d[2 * k] = ct[k].real(); d[2 * k + 1] = ct[k].imag(); }
    }
  }
  s->upload.reserve(total);
  hip_check(hipMemcpyAsync(s->upload.p, st, total, hipMemcpyHostToDevice, s->stream), "upload");
  stage_release_after_queue(s);
  char* d = static_cast<char*>(s->upload.p);
  for (int r = 0; r < n_req; ++r) {
    out[r].ops = reinterpret_cast<TileOp*>(d + o_ops[r]);
    out[r].diag = reinterpret_cast<DiagEntry*>(d + o_diag[r]);
    out[r].edges = reinterpret_cast<ZZEdge*>(d + o_edges[r]);
    out[r].deps = reinterpret_cast<uint64_t*>(d + o_deps[r]);
    out[r].ctab = d + o_ctab[r];
    out[r].ctab_stride = reqs[r].plan->ctab_size;
  }
}

hipError_t launch_pass(const qsv_state* s, const DevPass& dp, PassArgs A, int batch, bool adj) {
  A.lr0 = dp.lr0;
  A.lay0_reg = dp.lay0_reg;
  A.lay0_thr = dp.lay0_thr;
  A.relayout = dp.rb ? dp.relayout : 0;
  A.win_lo = dp.win_lo;
  A.win_n = dp.rb ? dp.win_n : 0;
  A.pass_pslots = adj ? dp.pslot_count : 0;
  const uint64_t tiles = 1ull << (s->n - dp.m);
  A.n_tiles = (int64_t)tiles;
  if (dp.rb) return launch_tile_pass_rb(s->dtype, adj, dp.rb, dp.maxm, A, tiles, batch, s->stream);
  return launch_tile_pass(s->dtype, adj, dp.maxm, A, tiles, batch, s->stream);
}

// Run a forward plan on batch states.  src (may equal psi) is read by the first pass with
// stride src_bstride; all later work is in place on psi.
void run_forward(qsv_state* s, const Plan& p, const Uploaded& u, void* psi, int64_t bstride, const void* src,
                 int64_t src_bstride, int batch) {
  const int n = s->n;
  if (p.unfused) {
    if (src != psi) {
      hip_check(launch_broadcast_state(s->dtype, psi, bstride, batch, src, n, s->stream), "broadcast");
      if (src_bstride != 0) fail(QSV_EINVAL, "internal: unfused forward with strided source");
    }
    for (size_t i = 0; i < p.prims.size(); ++i) {
      const Prim& pr = p.prims[i];
      // algorithmic bytes: every amplitude the gate changes is read and written once
      const int nc = __builtin_popcountll(pr.cmask);
      double frac = 1.0 / (double)(1ull << nc);
      if (pr.type == P_SIGN) frac = 1.0 / (double)(1ull << (nc - 1));
      const double bytes = 2.0 * frac * (double)batch * (double)s->namps() * (double)s->amp_bytes();
      timed(s, QSV_K_GATE_STREAM, bytes, [&] {
        if (pr.type == P_DENSE1)
          return launch_gate1(s->dtype, psi, bstride, batch, n, pr.q0, pr.cmask, u.ctab, u.ctab_stride,
                              p.stream_mat[i], s->stream);
        if (pr.type == P_DENSE2)
          return launch_gate2(s->dtype, psi, bstride, batch, n, pr.q0, pr.q1, pr.cmask, u.ctab, u.ctab_stride,
                              p.stream_mat[i], s->stream);
        return launch_diag(s->dtype, psi, bstride, batch, n, u.diag, p.stream_diag[i], 1, u.ctab, u.ctab_stride,
                           s->stream);
      }, "gate kernel launch");
    }
    return;
  }
  // Relayouting plans alternate between psi and the scratch buffer so that the last pass
  // writes psi (with an odd pass count the planner keeps the first pass in place).
  const int np = (int)p.passes.size();
  if (p.relayout && (batch != 1 || s->relay.bytes < s->namps() * s->amp_bytes()))
    fail(QSV_EINVAL, "internal: relayout plan without its scratch buffer");
  bool first = true;
  for (int pi = 0; pi < np; ++pi) {
    const DevPass& dp = p.passes[pi];
    void* in = psi;
    void* out = nullptr;
    if (p.relayout) {
      void* other = s->relay.p;
      in = (pi == 0 || (np - pi) % 2 == 0) ? psi : other;
      out = ((np - 1 - pi) % 2 == 0) ? psi : other;
      if (out == in) out = nullptr;
    }
    PassArgs A{};
    A.psi = in;
    A.dst = out;
    A.lam = nullptr;
    A.src = (first && src != psi) ? src : nullptr;
    A.bstride = bstride;
    A.src_bstride = src_bstride;
    A.ops = u.ops + dp.op_first;
    A.diag = u.diag;
    A.edges = u.edges;
    A.dep = u.deps + dp.dep_first;
    A.ctab = u.ctab;
    A.ctab_bstride = u.ctab_stride;
    A.partials = nullptr;
    A.tile_mask = dp.tile_mask;
    A.n_ops = dp.op_count;
    A.n_qubits = n;
    A.m = dp.m;
    A.n_pslots = 0;
    const double bytes = 2.0 * (double)batch * (double)s->namps() * (double)s->amp_bytes();
    timed(s, QSV_K_TILE_FORWARD, bytes,
          [&] { return launch_pass(s, dp, A, batch, false); },
          "tile pass");
    first = false;
  }
  if (first && src != psi)  // empty circuit
    hip_check(launch_broadcast_state(s->dtype, psi, bstride, batch, src, n, s->stream), "broadcast");
}

// Pauli-sum groups uploaded once per call.
struct DevPauli {
  std::vector<PauliGroup> groups;
  std::vector<const uint64_t*> z;
  std::vector<const double*> cre, cim;
  std::vector<const uint32_t*> pats;   // diagonal groups over >= 12 qubits, else null
  std::vector<const int32_t*> rfirst;
  std::vector<int32_t> n_pats;
};

// A diagonal group's terms sorted by their pattern on the 12 low qubits, with the pattern
// table of PauliGroupArgs::pats / rfirst (empty when the group does not qualify).
void pattern_tables(PauliGroup& g, int n, std::vector<uint32_t>& pats, std::vector<int32_t>& rfirst) {
  pats.clear();
  rfirst.clear();
  if (g.xmask != 0 || n < 12 || g.zmasks.empty()) return;
  std::vector<size_t> ord(g.zmasks.size());
  for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
    return (g.zmasks[a] & 0xFFF) < (g.zmasks[b] & 0xFFF);
  });
  PauliGroup h = g;
  for (size_t k = 0; k < ord.size(); ++k) {
    h.zmasks[k] = g.zmasks[ord[k]];
    h.cre[k] = g.cre[ord[k]];
    h.cim[k] = g.cim[ord[k]];
  }
  for (size_t k = 0; k < h.zmasks.size(); ++k) {
    const uint32_t pat = (uint32_t)(h.zmasks[k] & 0xFFF);
    if (pats.empty() || (pats.back() & 0xFFF) != pat) pats.push_back(pat | (uint32_t)k << 12);
  }
  if (pats.size() > (size_t)kPauliMaxPatterns || h.zmasks.size() >= (1u << 20)) {
    pats.clear();
    return;
  }
  for (int r = 0, p = 0; r <= 16; ++r) {
    while (p < (int)pats.size() && (int)((pats[p] & 0xFFF) >> 8) < r) ++p;
    rfirst.push_back(p);
  }
  g = h;
}

// Bytes of the groups' term tables (z masks, coefficient real and imaginary parts, and for
// qualifying diagonal groups the pattern tables, each array `align`-byte aligned).  Sorts
// the terms of diagonal groups by pattern (pattern_tables).
size_t pauli_table_bytes(std::vector<PauliGroup>& groups, int n, size_t align = 256) {
  size_t total = 0;
  std::vector<uint32_t> pats;
  std::vector<int32_t> rfirst;
  for (auto& g : groups) {
    total += align_up(g.zmasks.size() * 8, align) * 3;
    pattern_tables(g, n, pats, rfirst);
    if (!pats.empty()) total += align_up(pats.size() * 4, align) + align_up(rfirst.size() * 4, align);
  }
  return total;
}

// Pack the tables into host bytes `host`; the returned pointers are where they sit once
// the bytes are copied to device address `dev`.  The groups must have passed through
// pauli_table_bytes (diagonal groups sorted).
DevPauli pack_pauli(std::vector<PauliGroup> groups, int n, char* host, char* dev, size_t align = 256) {
  DevPauli dp;
  dp.groups = std::move(groups);
  size_t off = 0;
  std::vector<uint32_t> pats;
  std::vector<int32_t> rfirst;
  for (auto& g : dp.groups) {
    const size_t sz = g.zmasks.size() * 8, al = align_up(sz, align);
    std::memcpy(host + off, g.zmasks.data(), sz);
    std::memcpy(host + off + al, g.cre.data(), sz);
    std::memcpy(host + off + 2 * al, g.cim.data(), sz);
    dp.z.push_back(reinterpret_cast<const uint64_t*>(dev + off));
    dp.cre.push_back(reinterpret_cast<const double*>(dev + off + al));
    dp.cim.push_back(reinterpret_cast<const double*>(dev + off + 2 * al));
    off += 3 * al;
    pattern_tables(g, n, pats, rfirst);  // already sorted: this only rebuilds the tables
    if (pats.empty()) {
      dp.pats.push_back(nullptr);
      dp.rfirst.push_back(nullptr);
      dp.n_pats.push_back(0);
      continue;
    }
    std::memcpy(host + off, pats.data(), pats.size() * 4);
    dp.pats.push_back(reinterpret_cast<const uint32_t*>(dev + off));
    off += align_up(pats.size() * 4, align);
    std::memcpy(host + off, rfirst.data(), rfirst.size() * 4);
    dp.rfirst.push_back(reinterpret_cast<const int32_t*>(dev + off));
    off += align_up(rfirst.size() * 4, align);
    dp.n_pats.push_back((int32_t)pats.size());
  }
  return dp;
}

DevPauli upload_pauli(qsv_state* s, const qsv_pauli_sum* h, DevBuf& buf) {
  std::vector<PauliGroup> groups = group_pauli_sum(h);
  const size_t bytes = pauli_table_bytes(groups, s->n);
  const size_t total = bytes ? bytes : 256;
  char* st = static_cast<char*>(stage_acquire(s, total));
  buf.reserve(total);
  DevPauli dp = pack_pauli(std::move(groups), s->n, st, static_cast<char*>(buf.p));
  hip_check(hipMemcpyAsync(buf.p, st, total, hipMemcpyHostToDevice, s->stream), "upload pauli");
  stage_release_after_queue(s);
  return dp;
}

// Expectation partials (and optionally lambda = H psi) for batch states; returns the device
// pointer of reduced columns [batch][2 * groups] in s->outbuf at byte offset out_off.
// partials: NULL for the state's workspace (all groups at once), or a caller's buffer of
// 2 * chunk * pauli_blocks(n) doubles that groups reuse `chunk` at a time, each chunk's
// columns reduced before the next chunk starts (batch 1 only; the same sums in the same
// order).  untimed: launch without profiling events.
void run_pauli(qsv_state* s, const DevPauli& dp, const void* psi, void* lam, int64_t bstride, int batch,
               double* out_cols, double* partials = nullptr, int chunk = 0, bool untimed = false) {
  const int G = (int)dp.groups.size();
  const unsigned nblk = pauli_blocks(s->n);
  if (!partials) {
    const size_t need = (size_t)batch * 2 * G * nblk * sizeof(double);
    s->partials.reserve(need ? need : 8);
    partials = static_cast<double*>(s->partials.p);
    chunk = G;
  } else if (chunk < 1 || (batch != 1 && chunk < G)) {
    fail(QSV_EINVAL, "internal: chunked Pauli partials need batch 1");
  }
  if (lam && G == 0)
    hip_check(launch_set_basis(s->dtype, lam, bstride, batch, s->n, ~0ull, s->stream), "zero lambda");
  for (int g0 = 0; g0 < G; g0 += chunk) {
  const int g1 = std::min(G, g0 + chunk), nc = 2 * (g1 - g0);
  for (int g = g0; g < g1; ++g) {
    PauliGroupArgs A{};
    A.psi = psi;
    A.lam = lam;
    A.bstride = bstride;
    A.zmasks = dp.z[g];
    A.cre = dp.cre[g];
    A.cim = dp.cim[g];
    A.partials = partials;
    A.xmask = dp.groups[g].xmask;
    A.n_terms = (int32_t)dp.groups[g].zmasks.size();
    A.n_qubits = s->n;
    A.accumulate = g > 0 ? 1 : 0;
    A.col = 2 * (g - g0);
    A.ncols = nc;
    A.real_coeffs = std::all_of(dp.groups[g].cim.begin(), dp.groups[g].cim.end(), [](double c) { return c == 0.0; });
    A.pats = dp.pats[g];
    A.rfirst = dp.rfirst[g];
    A.n_pats = dp.n_pats[g];
    // read psi; write lambda (and read it when accumulating)
    const double sb = (double)batch * (double)s->namps() * (double)s->amp_bytes();
    const double bytes = sb * (1.0 + (lam ? 1.0 : 0.0) + (lam && g > 0 ? 1.0 : 0.0));
    if (untimed) hip_check(launch_pauli_group(s->dtype, A, batch, s->stream), "pauli pass");
    else timed(s, QSV_K_PAULI, bytes, [&] { return launch_pauli_group(s->dtype, A, batch, s->stream); }, "pauli pass");
  }
  hip_check(launch_reduce_columns(partials, nblk, (int64_t)batch * nc, out_cols + 2 * g0, s->stream), "reduce");
  }
}

qsv_state* check_state(const qsv_state* s) {
  if (!s) fail(QSV_EINVAL, "state is NULL");
  return const_cast<qsv_state*>(s);
}

// Energies (and optionally gradients) of `batch` bound tables.  Shared by the batch entry
// points and the parameter-shift comparator.
// Adjoint reverse sweep of plan adj over (psi, lam) batch items; writes the reduced
// gradient columns [batch][n_pslots] to d_cols (device).
void run_adjoint(qsv_state* s, const Plan& adj, const Uploaded& u, void* psi, void* lam, int64_t bstride, int batch,
                 double* d_cols) {
  const int P = adj.n_pslots;
  if (P == 0 || adj.passes.empty()) return;
  const uint64_t tiles = 1ull << (s->n - adj.passes[0].m);
  s->gpart.reserve((size_t)batch * P * tiles * sizeof(double));
  for (const DevPass& ap : adj.passes) {
    PassArgs A{};
    A.psi = psi;
    A.lam = lam;
    A.src = nullptr;
    A.bstride = bstride;
    A.src_bstride = 0;
    A.ops = u.ops + ap.op_first;
    A.diag = u.diag;
    A.edges = u.edges;
    A.dep = u.deps + ap.dep_first;
    A.ctab = u.ctab;
    A.ctab_bstride = u.ctab_stride;
    A.partials = static_cast<double*>(s->gpart.p) + (size_t)ap.pslot_first * tiles;
    A.tile_mask = ap.tile_mask;
    A.n_ops = ap.op_count;
    A.n_qubits = s->n;
    A.m = ap.m;
    A.n_pslots = P;
    const double bytes = 4.0 * (double)batch * (double)s->namps() * (double)s->amp_bytes();
    timed(s, QSV_K_TILE_ADJOINT, bytes, [&] { return launch_pass(s, ap, A, batch, true); }, "adjoint tile pass");
  }
  hip_check(launch_reduce_columns(static_cast<double*>(s->gpart.p), (int64_t)tiles, (int64_t)batch * P, d_cols,
                                  s->stream),
            "reduce gradients");
}

// run_fwd = false: the evolved states of an earlier forward-only call are still in the
// workspace (qsv_backward_batch), so only lambda and the reverse sweep run.
void energies_and_grads(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h, const Plan& fwd,
                        const std::vector<cplx>& ctab_fwd, const Plan* adj, const std::vector<cplx>* ctab_adj,
                        int batch, double* out_E, std::vector<double>* gcols, bool run_fwd = true) {
  const uint64_t N = s->namps();
  const int64_t bstride = (int64_t)N;
  s->fwd_token.clear();
  s->ws_psi.reserve((size_t)batch * N * s->amp_bytes());
  if (adj) s->ws_lam.reserve((size_t)batch * N * s->amp_bytes());
  Uploaded up[2];
  if (run_fwd) {
    UploadReq req[2] = {{&fwd, &ctab_fwd, batch}, {adj, ctab_adj, batch}};
    upload_plans(s, req, adj ? 2 : 1, up);
  } else {
    UploadReq req = {adj, ctab_adj, batch};
    upload_plans(s, &req, 1, &up[1]);
  }
  DevPauli dp = upload_pauli(s, h, s->pauli);
  const int G = (int)dp.groups.size();
  if (run_fwd) run_forward(s, fwd, up[0], s->ws_psi.p, bstride, s->psi, 0, batch);
  // output columns: energies [batch][2G] then gradient slots [batch][P]
  const int P = adj ? adj->n_pslots : 0;
  const size_t ne = (size_t)batch * 2 * G, ng = (size_t)batch * P;
  s->outbuf.reserve((ne + ng + 1) * sizeof(double));
  double* d_out = static_cast<double*>(s->outbuf.p);
  run_pauli(s, dp, s->ws_psi.p, adj ? s->ws_lam.p : nullptr, bstride, batch, d_out);
  if (adj && P > 0) run_adjoint(s, *adj, up[1], s->ws_psi.p, s->ws_lam.p, bstride, batch, d_out + ne);
  double* host = static_cast<double*>(stage_acquire(s, (ne + ng + 1) * sizeof(double)));
  hip_check(hipMemcpyAsync(host, d_out, (ne + ng) * sizeof(double), hipMemcpyDeviceToHost, s->stream), "download");
  hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
  for (int b = 0; b < batch; ++b) {
    double e = 0.0;
    for (int g = 0; g < G; ++g) e += host[(size_t)b * 2 * G + 2 * g];
    out_E[b] = e;
  }
  if (gcols) gcols->assign(host + ne, host + ne + ng);
  (void)c;
}

}  // namespace

// =============================================================================================
extern "C" {

const char* qsv_status_string(int status) {
  switch (status) {
    case QSV_OK: return "ok";
    case QSV_EINVAL: return "invalid argument";
    case QSV_ENOMEM: return "out of memory";
    case QSV_EDTYPE: return "bad dtype";
    case QSV_EHIP: return "HIP runtime error";
    case QSV_ERANGE: return "size out of range";
    case QSV_ENOTSUP: return "not supported";
    default: return "unknown status";
  }
}

const char* qsv_last_error(void) { return last_error().c_str(); }

const char* qsv_version(void) { return "qsv 0.1 (gfx950)"; }

static int state_init(qsv_state* s, int32_t n, int32_t dtype) {
  s->n = n;
  s->dtype = dtype;
  default_options(s);
  hip_check(hipGetDevice(&s->device), "hipGetDevice");
  hip_check(hipEventCreateWithFlags(&s->stage_ev, hipEventDisableTiming), "hipEventCreate");
  return 0;
}

int qsv_state_create(int32_t n_qubits, int32_t dtype, qsv_state** out) {
  return guarded([&] {
    if (!out) fail(QSV_EINVAL, "out is NULL");
    *out = nullptr;
    if (dtype != QSV_C64 && dtype != QSV_C128) fail(QSV_EDTYPE, "dtype must be QSV_C64 or QSV_C128");
    if (n_qubits < 1 || n_qubits > 34) fail(QSV_ERANGE, "n_qubits must be in [1, 34]");
    auto s = std::make_unique<qsv_state>();
    state_init(s.get(), n_qubits, dtype);
    const size_t bytes = s->namps() * s->amp_bytes();
    hip_check(hipMalloc(&s->psi, bytes), "hipMalloc state");
    s->owned = true;
    hip_check(launch_set_basis(dtype, s->psi, 0, 1, n_qubits, 0, s->stream), "init state");
    *out = s.release();
  });
}

int qsv_state_wrap(void* device_ptr, int32_t n_qubits, int32_t dtype, qsv_state** out) {
  return guarded([&] {
    if (!out) fail(QSV_EINVAL, "out is NULL");
    *out = nullptr;
    if (!device_ptr) fail(QSV_EINVAL, "device_ptr is NULL");
    if (dtype != QSV_C64 && dtype != QSV_C128) fail(QSV_EDTYPE, "dtype must be QSV_C64 or QSV_C128");
    if (n_qubits < 1 || n_qubits > 34) fail(QSV_ERANGE, "n_qubits must be in [1, 34]");
    auto s = std::make_unique<qsv_state>();
    state_init(s.get(), n_qubits, dtype);
    s->psi = device_ptr;
    s->owned = false;
    *out = s.release();
  });
}

int qsv_state_destroy(qsv_state* s) {
  if (!s) return QSV_OK;
  return guarded([&] {
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    if (s->owned && s->psi) (void)hipFree(s->psi);
    s->ws_psi.release();
    s->ws_lam.release();
    s->ws_aux1.release();
    s->ws_aux2.release();
    s->upload.release();
    s->partials.release();
    s->gpart.release();
    s->outbuf.release();
    s->pauli.release();
    s->relay.release();
    if (s->stage) (void)hipHostFree(s->stage);
    if (s->stage_ev) (void)hipEventDestroy(s->stage_ev);
    for (auto& r : s->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : s->free_events) (void)hipEventDestroy(e);
    delete s;
  });
}

int qsv_state_release_workspace(qsv_state* s) {
  return guarded([&] {
    check_state(s);
    set_device(s);
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    s->fwd_token.clear();
    s->ws_psi.release();
    s->ws_lam.release();
    s->ws_aux1.release();
    s->ws_aux2.release();
    s->partials.release();
    s->gpart.release();
    s->relay.release();
    s->relay_failed = false;
  });
}

int qsv_state_set_stream(qsv_state* s, void* hip_stream) {
  return guarded([&] {
    check_state(s);
    s->stream = static_cast<hipStream_t>(hip_stream);
  });
}

int qsv_state_synchronize(qsv_state* s) {
  return guarded([&] {
    check_state(s);
    set_device(s);
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
  });
}

int qsv_state_info(const qsv_state* s, int32_t* n_qubits, int32_t* dtype, void** device_ptr) {
  return guarded([&] {
    check_state(s);
    if (n_qubits) *n_qubits = s->n;
    if (dtype) *dtype = s->dtype;
    if (device_ptr) *device_ptr = s->psi;
  });
}

int qsv_state_reset(qsv_state* s) {
  return guarded([&] {
    check_state(s);
    set_device(s);
    ++s->generation;
    timed(s, QSV_K_OTHER, (double)s->namps() * (double)s->amp_bytes(),
          [&] { return launch_set_basis(s->dtype, s->psi, 0, 1, s->n, 0, s->stream); }, "reset");
  });
}

int qsv_state_set(qsv_state* s, const void* host_amps, size_t n_amps) {
  return guarded([&] {
    check_state(s);
    if (!host_amps) fail(QSV_EINVAL, "host_amps is NULL");
    if (n_amps != s->namps()) fail(QSV_EINVAL, "n_amps must be 2^n_qubits");
    set_device(s);
    ++s->generation;
    hip_check(hipMemcpyAsync(s->psi, host_amps, n_amps * s->amp_bytes(), hipMemcpyHostToDevice, s->stream),
              "set state");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
  });
}

int qsv_state_get(qsv_state* s, void* host_amps, size_t n_amps) {
  return guarded([&] {
    check_state(s);
    if (!host_amps) fail(QSV_EINVAL, "host_amps is NULL");
    if (n_amps != s->namps()) fail(QSV_EINVAL, "n_amps must be 2^n_qubits");
    set_device(s);
    hip_check(hipMemcpyAsync(host_amps, s->psi, n_amps * s->amp_bytes(), hipMemcpyDeviceToHost, s->stream),
              "get state");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
  });
}

int qsv_state_copy(qsv_state* dst, const qsv_state* src) {
  return guarded([&] {
    check_state(dst);
    check_state(src);
    if (dst->dtype != src->dtype) fail(QSV_EDTYPE, "dtype mismatch");
    if (dst->n != src->n) fail(QSV_EINVAL, "n_qubits mismatch");
    if (dst == src) return;
    set_device(dst);
    ++dst->generation;
    timed(dst, QSV_K_OTHER, 2.0 * (double)dst->namps() * (double)dst->amp_bytes(),
          [&] { return launch_broadcast_state(dst->dtype, dst->psi, 0, 1, src->psi, dst->n, dst->stream); },
          "copy state");
  });
}

int qsv_state_set_option(qsv_state* s, int32_t option, int64_t value) {
  return guarded([&] {
    check_state(s);
    if (option < 0 || option >= QSV_OPT_COUNT) fail(QSV_EINVAL, "unknown option");
    if (option == QSV_OPT_TILE_QUBITS) {
      if (value != 0 && (value < 2 || value > 13))
        fail(QSV_EINVAL, "tile width must be 0 (per-gate kernels) or in [2, 13]");
    } else if (option == QSV_OPT_ADJ_TILE_QUBITS) {
      if (value < 2 || value > 13) fail(QSV_EINVAL, "adjoint tile width must be in [2, 13]");
    } else if (option == QSV_OPT_THREADS) {
      if (value != 256 && value != 512 && value != 1024) fail(QSV_EINVAL, "threads must be 256, 512 or 1024");
    } else if (option == QSV_OPT_PROFILE) {
      if (value != 0 && value != 1) fail(QSV_EINVAL, "profile must be 0 or 1");
    } else if (option == QSV_OPT_RELAYOUT) {
      if (value != 0 && value != 1) fail(QSV_EINVAL, "relayout must be 0 or 1");
    }
    s->opt[option] = value;
  });
}

int qsv_state_get_option(const qsv_state* s, int32_t option, int64_t* value) {
  return guarded([&] {
    check_state(s);
    if (option < 0 || option >= QSV_OPT_COUNT || !value) fail(QSV_EINVAL, "bad option query");
    *value = s->opt[option];
  });
}

int qsv_apply_circuit(qsv_state* s, const qsv_circuit* c, const double* params, size_t n_params) {
  return guarded([&] {
    check_state(s);
    validate_circuit(c, params ? n_params : 0, s->n);
    set_device(s);
    ++s->generation;
    bool relay = s->opt[QSV_OPT_RELAYOUT] != 0 && !s->relay_failed;
    if (relay) {
      // relayout only pays when the plan has several register-blocked passes
      const Plan& probe = get_plan(s, c, false, true, true);
      relay = probe.relayout;
      const size_t need = s->namps() * s->amp_bytes();
      if (relay && s->relay.bytes < need) {
        s->relay.release();
        // keep head room for the tables and partial sums of later calls: relayout is an
        // optimization, in-place passes give the same result
        size_t free_b = 0, total_b = 0;
        hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        const size_t headroom = need / 8 + ((size_t)256 << 20);
        void* ptr = nullptr;
        if (free_b >= need + headroom && hipMalloc(&ptr, need) == hipSuccess) {
          s->relay.p = ptr;
          s->relay.bytes = need;
        } else {
          (void)hipGetLastError();
          s->relay_failed = true;
          relay = false;
        }
      }
    }
    const Plan& p = get_plan(s, c, false, true, relay);
    std::vector<cplx> ctab(p.ctab_size);
    bind_ctab(p, c, params, nullptr, 0, ctab.data());
    Uploaded u;
    UploadReq req{&p, &ctab, 1};
    upload_plans(s, &req, 1, &u);
    run_forward(s, p, u, s->psi, 0, s->psi, 0, 1);
  });
}

int qsv_expectation(qsv_state* s, const qsv_pauli_sum* h, double* out_re, double* out_im) {
  return guarded([&] {
    check_state(s);
    validate_pauli_sum(h, s->n);
    set_device(s);
    DevPauli dp = upload_pauli(s, h, s->pauli);
    const int G = (int)dp.groups.size();
    s->outbuf.reserve((2 * G + 1) * sizeof(double));
    run_pauli(s, dp, s->psi, nullptr, 0, 1, static_cast<double*>(s->outbuf.p));
    double* host = static_cast<double*>(stage_acquire(s, (2 * G + 1) * sizeof(double)));
    if (G) hip_check(hipMemcpyAsync(host, s->outbuf.p, 2 * G * sizeof(double), hipMemcpyDeviceToHost, s->stream),
                     "download");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    double re = 0, im = 0;
    for (int g = 0; g < G; ++g) { re += host[2 * g]; im += host[2 * g + 1]; }
    if (out_re) *out_re = re;
    if (out_im) *out_im = im;
  });
}

int qsv_expectation_noalloc(qsv_state* s, const qsv_pauli_sum* h, double* out_re, double* out_im) {
  return guarded([&] {
    check_state(s);
    validate_pauli_sum(h, s->n);
    if (h->n_terms > kNoallocMaxTerms) fail(QSV_ERANGE, "more Pauli terms than the fixed scratch holds");
    set_device(s);
    char* scr = static_cast<char*>(noalloc_scratch());
    std::vector<PauliGroup> groups = group_pauli_sum(h);
    const int G = (int)groups.size();
    double re = 0, im = 0;
    if (G > 0) {
      // scratch layout: term tables | reduced columns | partials of kNoallocChunk groups
      const size_t tab = pauli_table_bytes(groups, s->n, 8);
      const size_t out_off = align_up(tab, 256);
      const size_t part_off = align_up(out_off + (size_t)2 * G * sizeof(double), 256);
      const size_t part_bytes = (size_t)2 * kNoallocChunk * pauli_blocks(s->n) * sizeof(double);
      if (part_off + part_bytes > kNoallocScratchBytes) fail(QSV_ERANGE, "Pauli sum too large for the fixed scratch");
      std::vector<char> host(tab);
      DevPauli dp = pack_pauli(std::move(groups), s->n, host.data(), scr, 8);
      hip_check(hipMemcpyAsync(scr, host.data(), tab, hipMemcpyHostToDevice, s->stream), "upload pauli");
      double* d_out = reinterpret_cast<double*>(scr + out_off);
      run_pauli(s, dp, s->psi, nullptr, 0, 1, d_out, reinterpret_cast<double*>(scr + part_off), kNoallocChunk, true);
      std::vector<double> cols((size_t)2 * G);
      hip_check(hipMemcpyAsync(cols.data(), d_out, (size_t)2 * G * sizeof(double), hipMemcpyDeviceToHost, s->stream),
                "download");
      hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
      for (int g = 0; g < G; ++g) { re += cols[2 * g]; im += cols[2 * g + 1]; }
    }
    if (out_re) *out_re = re;
    if (out_im) *out_im = im;
  });
}

int qsv_apply_pauli_sum(qsv_state* dst, const qsv_state* src, const qsv_pauli_sum* h) {
  return guarded([&] {
    check_state(dst);
    check_state(src);
    if (dst == src) fail(QSV_EINVAL, "dst must differ from src");
    if (dst->dtype != src->dtype) fail(QSV_EDTYPE, "dtype mismatch");
    if (dst->n != src->n) fail(QSV_EINVAL, "n_qubits mismatch");
    validate_pauli_sum(h, dst->n);
    set_device(dst);
    ++dst->generation;
    DevPauli dp = upload_pauli(dst, h, dst->pauli);
    const int G = (int)dp.groups.size();
    dst->outbuf.reserve((2 * G + 1) * sizeof(double));
    run_pauli(dst, dp, src->psi, dst->psi, 0, 1, static_cast<double*>(dst->outbuf.p));
    hip_check(hipStreamSynchronize(dst->stream), "hipStreamSynchronize");
  });
}

static void batch_common(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h, const double* params,
                         size_t batch, size_t n_params, double* out_E) {
  check_state(s);
  if (batch < 1 || batch > 65535) fail(QSV_ERANGE, "batch must be in [1, 65535]");
  if (!out_E) fail(QSV_EINVAL, "out_E is NULL");
  if (n_params && !params) fail(QSV_EINVAL, "params is NULL");
  validate_circuit(c, n_params, s->n);
  validate_pauli_sum(h, s->n);
  set_device(s);
}

int qsv_expectation_and_grad_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h,
                                   const double* params, size_t batch, size_t n_params, double* out_E,
                                   double* out_grad) {
  return guarded([&] {
    batch_common(s, c, h, params, batch, n_params, out_E);
    if (n_params && !out_grad) fail(QSV_EINVAL, "out_grad is NULL");
    const Plan& fwd = get_plan(s, c, false, true);
    const Plan& adj = get_plan(s, c, true, true);
    std::vector<cplx> cf((size_t)batch * fwd.ctab_size), ca((size_t)batch * adj.ctab_size);
    for (size_t b = 0; b < batch; ++b) {
      bind_ctab(fwd, c, params + b * n_params, nullptr, 0, cf.data() + b * fwd.ctab_size);
      bind_ctab(adj, c, params + b * n_params, nullptr, 0, ca.data() + b * adj.ctab_size);
    }
    std::vector<double> gcols;
    energies_and_grads(s, c, h, fwd, cf, &adj, &ca, (int)batch, out_E, &gcols);
    const int P = adj.n_pslots;
    for (size_t b = 0; b < batch; ++b) {
      double* g = out_grad + b * n_params;
      for (size_t k = 0; k < n_params; ++k) g[k] = 0.0;
      for (int k = 0; k < P; ++k) g[adj.pslot_param[k]] += gcols[b * P + k];
    }
  });
}

int qsv_expectation_and_grad(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h, const double* params,
                             size_t n_params, double* out_E, double* out_grad) {
  return qsv_expectation_and_grad_batch(s, c, h, params, 1, n_params, out_E, out_grad);
}

int qsv_expectation_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h, const double* params,
                          size_t batch, size_t n_params, double* out_E) {
  return guarded([&] {
    batch_common(s, c, h, params, batch, n_params, out_E);
    const Plan& fwd = get_plan(s, c, false, true);
    std::vector<cplx> cf((size_t)batch * fwd.ctab_size);
    for (size_t b = 0; b < batch; ++b)
      bind_ctab(fwd, c, params + b * n_params, nullptr, 0, cf.data() + b * fwd.ctab_size);
    energies_and_grads(s, c, h, fwd, cf, nullptr, nullptr, (int)batch, out_E, nullptr);
  });
}

static std::string forward_token(const qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h,
                                 const double* params, size_t batch, size_t n_params) {
  std::string t = structure_key(c, false, plan_options(s, false, true));
  auto put = [&](const void* p, size_t n) { if (n) t.append(reinterpret_cast<const char*>(p), n); };
  for (size_t i = 0; i < c->n_gates; ++i) {
    put(c->gates[i].param_coeff, sizeof(double) * 3);
    put(c->gates[i].angle_const, sizeof(double) * 3);
    put(&c->gates[i].matrix_offset, sizeof(int64_t));
  }
  if (c->matrices) put(c->matrices, c->n_matrix_doubles * sizeof(double));
  put(h->coeffs, h->n_terms * sizeof(double));
  put(h->x_masks, h->n_terms * sizeof(uint64_t));
  put(h->z_masks, h->n_terms * sizeof(uint64_t));
  put(params, batch * n_params * sizeof(double));
  put(&batch, sizeof(batch));
  put(&s->psi, sizeof(void*));
  put(&s->generation, sizeof(s->generation));
  return t;
}

int qsv_forward_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h, const double* params, size_t batch,
                      size_t n_params, double* out_E) {
  return guarded([&] {
    batch_common(s, c, h, params, batch, n_params, out_E);
    const Plan& fwd = get_plan(s, c, false, true);
    std::vector<cplx> cf((size_t)batch * fwd.ctab_size);
    for (size_t b = 0; b < batch; ++b)
      bind_ctab(fwd, c, params + b * n_params, nullptr, 0, cf.data() + b * fwd.ctab_size);
    energies_and_grads(s, c, h, fwd, cf, nullptr, nullptr, (int)batch, out_E, nullptr);
    s->fwd_token = forward_token(s, c, h, params, batch, n_params);
  });
}

int qsv_backward_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h, const double* params,
                       size_t batch, size_t n_params, const double* dE_weights, double* out_grad) {
  return guarded([&] {
    std::vector<double> E(batch > 0 && batch <= 65535 ? batch : 1);
    batch_common(s, c, h, params, batch, n_params, E.data());
    if (n_params && !out_grad) fail(QSV_EINVAL, "out_grad is NULL");
    if (!dE_weights) fail(QSV_EINVAL, "dE_weights is NULL");
    for (size_t b = 0; b < batch; ++b)
      if (!std::isfinite(dE_weights[b])) fail(QSV_EINVAL, "non-finite dE weight");
    const Plan& fwd = get_plan(s, c, false, true);
    const Plan& adj = get_plan(s, c, true, true);
    const bool kept = !s->fwd_token.empty() && s->fwd_token == forward_token(s, c, h, params, batch, n_params);
    std::vector<cplx> cf(kept ? 0 : (size_t)batch * fwd.ctab_size), ca((size_t)batch * adj.ctab_size);
    for (size_t b = 0; b < batch; ++b) {
      if (!kept) bind_ctab(fwd, c, params + b * n_params, nullptr, 0, cf.data() + b * fwd.ctab_size);
      bind_ctab(adj, c, params + b * n_params, nullptr, 0, ca.data() + b * adj.ctab_size);
    }
    std::vector<double> gcols;
    energies_and_grads(s, c, h, fwd, cf, &adj, &ca, (int)batch, E.data(), &gcols, !kept);
    const int P = adj.n_pslots;
    for (size_t b = 0; b < batch; ++b) {
      double* g = out_grad + b * n_params;
      for (size_t k = 0; k < n_params; ++k) g[k] = 0.0;
      for (int k = 0; k < P; ++k) g[adj.pslot_param[k]] += gcols[b * P + k];
      for (size_t k = 0; k < n_params; ++k) g[k] *= dE_weights[b];
    }
  });
}

int qsv_expectation_general(qsv_state* psi, const qsv_circuit* c_r, const double* params_r, size_t n_r,
                            const qsv_state* phi, const qsv_circuit* c_l, const double* params_l, size_t n_l,
                            const qsv_pauli_sum* h, double* out_E, double* grad_r, double* grad_l) {
  return guarded([&] {
    check_state(psi);
    check_state(phi);
    if (!out_E) fail(QSV_EINVAL, "out_E is NULL");
    if (psi->dtype != phi->dtype) fail(QSV_EDTYPE, "dtype mismatch");
    if (psi->n != phi->n) fail(QSV_EINVAL, "n_qubits mismatch");
    if (n_r && !params_r) fail(QSV_EINVAL, "params_r is NULL");
    if (n_l && !params_l) fail(QSV_EINVAL, "params_l is NULL");
    validate_circuit(c_r, n_r, psi->n);
    if (c_l) validate_circuit(c_l, n_l, psi->n);
    validate_pauli_sum(h, psi->n);
    qsv_state* s = psi;
    set_device(s);
    s->fwd_token.clear();
    const uint64_t N = s->namps();
    const int64_t bs = (int64_t)N;
    const size_t pair = 2 * N * s->amp_bytes();
    s->ws_psi.reserve(pair);
    s->ws_lam.reserve(pair);
    s->ws_aux1.reserve(pair);
    s->ws_aux2.reserve(pair);
    const Plan& fr = get_plan(s, c_r, false, true);
    const Plan* ar = grad_r ? &get_plan(s, c_r, true, true) : nullptr;
    const Plan* fl = c_l ? &get_plan(s, c_l, false, true) : nullptr;
    const Plan* al = (c_l && grad_l) ? &get_plan(s, c_l, true, true) : nullptr;
    auto bind2 = [&](const Plan* p, const qsv_circuit* c, const double* prm) {
      std::vector<cplx> t(p ? 2 * (size_t)p->ctab_size : 0);
      if (p) {
        bind_ctab(*p, c, prm, nullptr, 0, t.data());
        bind_ctab(*p, c, prm, nullptr, 0, t.data() + p->ctab_size);
      }
      return t;
    };
    const std::vector<cplx> t_fr = bind2(&fr, c_r, params_r), t_ar = bind2(ar, c_r, params_r),
                            t_fl = bind2(fl, c_l, params_l), t_al = bind2(al, c_l, params_l);
    const Plan* plans[4] = {&fr, ar, fl, al};
    const std::vector<cplx>* tabs[4] = {&t_fr, &t_ar, &t_fl, &t_al};
    UploadReq req[4];
    int map[4], nreq = 0;
    for (int k = 0; k < 4; ++k) {
      map[k] = -1;
      if (plans[k]) {
        map[k] = nreq;
        req[nreq++] = UploadReq{plans[k], tabs[k], 2};
      }
    }
    Uploaded up[4];
    upload_plans(s, req, nreq, up);
    char* P1 = static_cast<char*>(s->ws_psi.p);   // U_r psi (two copies)
    char* L1 = static_cast<char*>(s->ws_lam.p);   // H U_l phi, i H U_l phi
    char* P2 = static_cast<char*>(s->ws_aux1.p);  // U_l phi (two copies)
    char* L2 = static_cast<char*>(s->ws_aux2.p);  // H U_r psi, i H U_r psi
    const size_t one = N * s->amp_bytes();
    run_forward(s, fr, up[map[0]], P1, bs, psi->psi, 0, 2);
    if (fl) run_forward(s, *fl, up[map[2]], P2, bs, phi->psi, 0, 2);
    else hip_check(launch_broadcast_state(s->dtype, P2, bs, 2, phi->psi, s->n, s->stream), "copy phi");
    DevPauli dp = upload_pauli(s, h, s->pauli);
    const int G = (int)dp.groups.size();
    const int Pr = ar ? ar->n_pslots : 0, Pl = al ? al->n_pslots : 0;
    const size_t o_tmp = 0, o_E = 2 * (size_t)G, o_r = o_E + 2, o_l = o_r + 2 * (size_t)Pr, total = o_l + 2 * (size_t)Pl;
    s->outbuf.reserve((total + 1) * sizeof(double));
    double* d_out = static_cast<double*>(s->outbuf.p);
    run_pauli(s, dp, P1, L2, bs, 1, d_out + o_tmp);  // chi = H U_r psi
    run_pauli(s, dp, P2, L1, bs, 1, d_out + o_tmp);  // lambda_r = H U_l phi
    const unsigned ib = inner_blocks(s->n);
    s->partials.reserve(2 * ib * sizeof(double));
    hip_check(launch_inner_product(s->dtype, P2, L2, s->n, static_cast<double*>(s->partials.p), s->stream), "inner");
    hip_check(launch_reduce_columns(static_cast<double*>(s->partials.p), ib, 2, d_out + o_E, s->stream), "reduce");
    hip_check(launch_scale_copy(s->dtype, L1 + one, L1, s->n, 0.0, 1.0, s->stream), "i lambda");
    hip_check(launch_scale_copy(s->dtype, L2 + one, L2, s->n, 0.0, 1.0, s->stream), "i chi");
    if (ar) run_adjoint(s, *ar, up[map[1]], P1, L1, bs, 2, d_out + o_r);
    if (al) run_adjoint(s, *al, up[map[3]], P2, L2, bs, 2, d_out + o_l);
    double* host = static_cast<double*>(stage_acquire(s, (total + 1) * sizeof(double)));
    hip_check(hipMemcpyAsync(host, d_out, total * sizeof(double), hipMemcpyDeviceToHost, s->stream), "download");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    out_E[0] = host[o_E];
    out_E[1] = host[o_E + 1];
    // Im<lam|G|psi> with lam and with i lam give the two parts of the derivative:
    // right circuit dE = (I1 + i I2) / 2; left circuit dE = (I1 - i I2) / 2.
    if (grad_r) {
      for (size_t k = 0; k < 2 * n_r; ++k) grad_r[k] = 0.0;
      for (int k = 0; k < Pr; ++k) {
        const int prm = ar->pslot_param[k];
        grad_r[2 * prm] += 0.5 * host[o_r + k];
        grad_r[2 * prm + 1] += 0.5 * host[o_r + Pr + k];
      }
    }
    if (grad_l) {
      for (size_t k = 0; k < 2 * n_l; ++k) grad_l[k] = 0.0;
      for (int k = 0; k < Pl; ++k) {
        const int prm = al->pslot_param[k];
        grad_l[2 * prm] += 0.5 * host[o_l + k];
        grad_l[2 * prm + 1] -= 0.5 * host[o_l + Pl + k];
      }
    }
  });
}

int qsv_expectation_and_grad_multi(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* hams, size_t n_hams,
                                   const double* params, size_t n_params, double* out_E, double* out_grad) {
  return guarded([&] {
    check_state(s);
    if (n_hams < 1 || n_hams > 65535) fail(QSV_ERANGE, "n_hams must be in [1, 65535]");
    if (!hams || !out_E) fail(QSV_EINVAL, "NULL argument");
    if (n_params && (!params || !out_grad)) fail(QSV_EINVAL, "params / out_grad are NULL");
    validate_circuit(c, n_params, s->n);
    for (size_t k = 0; k < n_hams; ++k) validate_pauli_sum(&hams[k], s->n);
    set_device(s);
    s->fwd_token.clear();
    const uint64_t N = s->namps();
    const int64_t bs = (int64_t)N;
    const size_t one = N * s->amp_bytes();
    s->ws_psi.reserve(n_hams * one);
    s->ws_lam.reserve(n_hams * one);
    const Plan& fwd = get_plan(s, c, false, true);
    const Plan& adj = get_plan(s, c, true, true);
    std::vector<cplx> tf(fwd.ctab_size), ta((size_t)n_hams * adj.ctab_size);
    bind_ctab(fwd, c, params, nullptr, 0, tf.data());
    for (size_t k = 0; k < n_hams; ++k) bind_ctab(adj, c, params, nullptr, 0, ta.data() + k * adj.ctab_size);
    UploadReq req[2] = {{&fwd, &tf, 1}, {&adj, &ta, (int)n_hams}};
    Uploaded up[2];
    upload_plans(s, req, 2, up);
    char* P = static_cast<char*>(s->ws_psi.p);
    char* L = static_cast<char*>(s->ws_lam.p);
    run_forward(s, fwd, up[0], P, bs, s->psi, 0, 1);
    if (n_hams > 1)
      hip_check(launch_broadcast_state(s->dtype, P + one, bs, (int)n_hams - 1, P, s->n, s->stream), "copy psi");
    std::vector<int> ngroups(n_hams);
    size_t ecols = 0;
    for (size_t k = 0; k < n_hams; ++k) ecols += 2 * group_pauli_sum(&hams[k]).size();
    const int Pn = adj.n_pslots;
    s->outbuf.reserve((ecols + n_hams * (size_t)Pn + 1) * sizeof(double));
    double* d_out = static_cast<double*>(s->outbuf.p);
    size_t col = 0;
    for (size_t k = 0; k < n_hams; ++k) {
      DevPauli dp = upload_pauli(s, &hams[k], s->pauli);
      ngroups[k] = (int)dp.groups.size();
      run_pauli(s, dp, P + k * one, L + k * one, bs, 1, d_out + col);
      col += 2 * dp.groups.size();
    }
    run_adjoint(s, adj, up[1], P, L, bs, (int)n_hams, d_out + ecols);
    double* host = static_cast<double*>(stage_acquire(s, (ecols + n_hams * (size_t)Pn + 1) * sizeof(double)));
    hip_check(hipMemcpyAsync(host, d_out, (ecols + n_hams * (size_t)Pn) * sizeof(double), hipMemcpyDeviceToHost,
                             s->stream),
              "download");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    col = 0;
    for (size_t k = 0; k < n_hams; ++k) {
      double e = 0.0;
      for (int g = 0; g < ngroups[k]; ++g) e += host[col + 2 * g];
      col += 2 * ngroups[k];
      out_E[k] = e;
      if (!n_params) continue;
      double* gk = out_grad + k * n_params;
      for (size_t q = 0; q < n_params; ++q) gk[q] = 0.0;
      for (int q = 0; q < Pn; ++q) gk[adj.pslot_param[q]] += host[ecols + k * Pn + q];
    }
  });
}

int qsv_param_shift_grad_batch(qsv_state* s, const qsv_circuit* c, const qsv_pauli_sum* h,
                               const double* params, size_t batch, size_t n_params, double* out_E,
                               double* out_grad) {
  return guarded([&] {
    batch_common(s, c, h, params, batch, n_params, out_E);
    if (n_params && !out_grad) fail(QSV_EINVAL, "out_grad is NULL");
    // every parameterized angle occurrence, shifted by +-pi/2
    struct Occ { int gate, slot, param; double coeff; };
    std::vector<Occ> occ;
    for (size_t i = 0; i < c->n_gates; ++i) {
      const qsv_gate& g = c->gates[i];
      const int na = g.kind == QSV_GATE_U3 ? 3 : (g.kind >= QSV_GATE_RX && g.kind <= QSV_GATE_RZZ ? 1 : 0);
      for (int a = 0; a < na; ++a) {
        if (g.param_index[a] < 0) continue;
        if (g.ctrl_mask) fail(QSV_ENOTSUP, "two-term parameter shift does not hold for controlled rotations");
        occ.push_back({(int)i, a, g.param_index[a], g.param_coeff[a]});
      }
    }
    const Plan& fwd = get_plan(s, c, false, false);
    const size_t per = 1 + 2 * occ.size();  // unshifted + shifted variants
    const size_t state_bytes = s->namps() * s->amp_bytes();
    const size_t budget = std::max<size_t>((size_t)8 << 30, s->ws_psi.bytes);
    size_t chunk = std::max<size_t>(1, std::min<size_t>(budget / state_bytes, 4096));
    std::vector<double> energies(per);
    for (size_t b = 0; b < batch; ++b) {
      const double* pb = params + b * n_params;
      std::vector<double> ang(3 * c->n_gates);
      for (size_t i = 0; i < c->n_gates; ++i) gate_angles(c->gates[i], pb, &ang[3 * i]);
      for (size_t v0 = 0; v0 < per; v0 += chunk) {
        const size_t nv = std::min(chunk, per - v0);
        std::vector<cplx> cf(nv * fwd.ctab_size);
        for (size_t v = 0; v < nv; ++v) {
          const size_t id = v0 + v;
          AngleOverride ov{};
          int nov = 0;
          if (id > 0) {
            const Occ& o = occ[(id - 1) / 2];
            ov.gate = o.gate;
            ov.slot = o.slot;
            ov.angle = ang[3 * o.gate + o.slot] + (((id - 1) % 2 == 0) ? M_PI / 2 : -M_PI / 2);
            nov = 1;
          }
          bind_ctab(fwd, c, pb, &ov, nov, cf.data() + v * fwd.ctab_size);
        }
        energies_and_grads(s, c, h, fwd, cf, nullptr, nullptr, (int)nv, energies.data() + v0, nullptr);
      }
      out_E[b] = energies[0];
      double* g = out_grad + b * n_params;
      for (size_t k = 0; k < n_params; ++k) g[k] = 0.0;
      for (size_t k = 0; k < occ.size(); ++k)
        g[occ[k].param] += occ[k].coeff * 0.5 * (energies[1 + 2 * k] - energies[2 + 2 * k]);
    }
  });
}

int qsv_profile_read(qsv_state* s, int32_t kernel_class, double* total_ms, int64_t* launches,
                     double* algorithmic_bytes) {
  return guarded([&] {
    check_state(s);
    if (kernel_class < 0 || kernel_class >= QSV_K_COUNT) fail(QSV_EINVAL, "unknown kernel class");
    set_device(s);
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    prof_collect(s);
    if (total_ms) *total_ms = s->prof_ms[kernel_class];
    if (launches) *launches = s->prof_n[kernel_class];
    if (algorithmic_bytes) *algorithmic_bytes = s->prof_bytes[kernel_class];
    s->prof_ms[kernel_class] = 0;
    s->prof_n[kernel_class] = 0;
    s->prof_bytes[kernel_class] = 0;
  });
}

int qsv_plan_debug(const qsv_circuit* c, int32_t tile_qubits, int32_t* order, int32_t* pass_of,
                   int32_t max_entries, int32_t* n_entries, int32_t* n_passes, uint64_t* tile_masks,
                   int32_t max_passes) {
  return guarded([&] {
    validate_circuit(c, (size_t)1 << 30, -1);
    if (!order || !pass_of || !n_passes || !n_entries) fail(QSV_EINVAL, "output arrays are NULL");
    if (tile_qubits < 2 || tile_qubits > 34) fail(QSV_EINVAL, "tile_qubits must be in [2, 34]");
    const std::vector<Prim> prims = lower_forward(c);
    if ((int64_t)prims.size() > max_entries) fail(QSV_ERANGE, "order / pass_of arrays are too small");
    const std::vector<Pass> passes = plan_passes(prims, c->n_qubits, std::min(tile_qubits, c->n_qubits), 3);
    int32_t k = 0;
    for (size_t p = 0; p < passes.size(); ++p) {
      for (int32_t i : passes[p].prims) {
        order[k] = prims[i].gate;
        pass_of[k] = (int32_t)p;
        ++k;
      }
      if (tile_masks && (int32_t)p < max_passes) tile_masks[p] = passes[p].tile_mask;
    }
    *n_entries = k;
    *n_passes = (int32_t)passes.size();
  });
}

}  // extern "C"
