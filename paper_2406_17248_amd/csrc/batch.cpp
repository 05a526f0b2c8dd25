// Batched evaluation of many independent circuits of uneven size and depth.
//
// Every circuit keeps its own plans (forward and adjoint), state and costate buffers.  One
// evaluation is: fill the states with |0...0>, forward pass rounds (round r runs pass r of
// every circuit that has one, all circuits in one launch), one multi-circuit Pauli pass
// (lambda = H psi and the energies, gather form), adjoint rounds, one segmented reduction.
// The whole sequence is captured once into a HIP graph and replayed per evaluation; only
// the bound-matrix table (which depends on the parameters) is copied up before the replay.
// The tile width of the fused passes is picked by timing candidate widths (autotune).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "../../include/qsv.h"
#include "engine.h"
#include "hip_util.h"
#include "qsv_kernels.h"

using namespace qsv;

namespace {

struct CircuitCopy {
  int32_t n = 0;
  std::vector<qsv_gate> gates;
  std::vector<double> mats;
  qsv_circuit view() const {
    return qsv_circuit{n, 0, gates.data(), gates.size(), mats.empty() ? nullptr : mats.data(), mats.size()};
  }
};

struct HamCopy {
  std::vector<double> coeffs;
  std::vector<uint64_t> x, z;
};

struct Round {
  std::vector<PassArgs> items;
  std::vector<uint32_t> prefix;  // n_items + 1
  int maxm = 9;
  int max_win = 0;                       // largest ctab window of the items (LDS entries)
  int max_pslots = 0;                    // adjoint: largest per-pass gradient slot count
  size_t items_off = 0, prefix_off = 0;  // byte offsets in the static device table
};

}  // namespace

struct qsv_batch {
  int32_t dtype = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<CircuitCopy> circ;
  std::vector<HamCopy> ham;
  std::vector<int64_t> param_off;  // n + 1
  int32_t tile = 12;
  int32_t low = 0;  // qubits every tile keeps (0: 4 for complex64, 3 for complex128)
  double last_ms = 0.0;
  // built configuration
  bool built = false;
  std::vector<Plan> fwd, adj;
  std::vector<int64_t> ctab_fwd_off, ctab_adj_off;  // complex entries
  int64_t ctab_total = 0;
  std::vector<Round> frounds, arounds;
  std::vector<int64_t> slot_out_off;  // per circuit: first gradient column in the result vector
  int64_t n_out = 0;                  // results: n_circuits energies then all gradient slots
  DevBuf states, statics, ctab, partials, results;
  void* host = nullptr;               // pinned: bound tables up, results down
  size_t host_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  size_t amp() const { return dtype == QSV_C64 ? 8 : 16; }
};

namespace {

void drop_graph(qsv_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

void* host_buffer(qsv_batch* b, size_t bytes) {
  if (bytes > b->host_bytes) {
    if (b->host) (void)hipHostFree(b->host);
    b->host = nullptr;
    b->host_bytes = 0;
    hip_check(hipHostMalloc(&b->host, align_up(bytes, 1 << 20), hipHostMallocDefault), "hipHostMalloc");
    b->host_bytes = align_up(bytes, 1 << 20);
  }
  return b->host;
}

// Build plans, device tables and the graph for the current tile width.
void build(qsv_batch* b) {
  drop_graph(b);
  b->built = false;
  const size_t nc = b->circ.size();
  PlanOptions of, oa;
  of.tile_qubits = b->tile;
  oa.tile_qubits = std::min<int>(b->tile, b->dtype == QSV_C64 ? 13 : 12);
  of.low_qubits = oa.low_qubits = b->low > 0 ? b->low : (b->dtype == QSV_C64 ? 4 : 3);
  of.dtype = oa.dtype = b->dtype;
  of.rb_min = oa.rb_min = 4;  // every pass register-blocked, small tiles with idle threads
  b->fwd.clear();
  b->adj.clear();
  for (size_t i = 0; i < nc; ++i) {
    const qsv_circuit c = b->circ[i].view();
    b->fwd.push_back(build_plan(&c, false, of));
    b->adj.push_back(build_plan(&c, true, oa));
  }
  // state buffers: psi then lambda of every circuit
  std::vector<int64_t> st_off(nc);
  int64_t amps = 0;
  for (size_t i = 0; i < nc; ++i) {
    st_off[i] = amps;
    amps += 1ll << b->circ[i].n;
  }
  b->states.reserve(2 * (size_t)amps * b->amp());
  char* psi0 = static_cast<char*>(b->states.p);
  char* lam0 = psi0 + (size_t)amps * b->amp();
  // bound tables
  b->ctab_fwd_off.assign(nc, 0);
  b->ctab_adj_off.assign(nc, 0);
  int64_t ct = 0;
  for (size_t i = 0; i < nc; ++i) {
    b->ctab_fwd_off[i] = ct;
    ct += b->fwd[i].ctab_size;
    b->ctab_adj_off[i] = ct;
    ct += b->adj[i].ctab_size;
  }
  b->ctab_total = ct;
  b->ctab.reserve(std::max<int64_t>(ct, 1) * b->amp());
  // static tables: ops, diag, edges per plan; Pauli terms; rounds; segments
  std::vector<char> st;
  auto put = [&](const void* p, size_t bytes) {
    const size_t off = align_up(st.size(), 256);
    st.resize(off + bytes);
    if (bytes) std::memcpy(st.data() + off, p, bytes);
    return off;
  };
  struct PlanOffs { size_t ops, diag, edges, deps; };
  std::vector<PlanOffs> fo(nc), ao(nc);
  for (size_t i = 0; i < nc; ++i) {
    for (int k = 0; k < 2; ++k) {
      const Plan& p = k == 0 ? b->fwd[i] : b->adj[i];
      PlanOffs& o = k == 0 ? fo[i] : ao[i];
      o.ops = put(p.ops.data(), p.ops.size() * sizeof(TileOp));
      o.diag = put(p.diag.data(), p.diag.size() * sizeof(DiagEntry));
      o.edges = put(p.edges.data(), p.edges.size() * sizeof(ZZEdge));
      o.deps = put(p.deps.data(), p.deps.size() * sizeof(uint64_t));
    }
  }
  // Pauli terms and jobs
  std::vector<size_t> term_off(nc), tz_off(nc), tc_off(nc), ti_off(nc);
  for (size_t i = 0; i < nc; ++i) {
    const HamCopy& h = b->ham[i];
    const size_t nt = h.coeffs.size();
    std::vector<double> cre(nt), cim(nt);
    for (size_t k = 0; k < nt; ++k) {
      const int r = __builtin_popcountll(h.x[k] & h.z[k]) & 3;
      const double c = h.coeffs[k];
      const double re[4] = {c, 0.0, -c, 0.0}, im[4] = {0.0, c, 0.0, -c};
      cre[k] = re[r];
      cim[k] = im[r];
    }
    term_off[i] = put(h.x.data(), nt * 8);
    tz_off[i] = put(h.z.data(), nt * 8);
    tc_off[i] = put(cre.data(), nt * 8);
    ti_off[i] = put(cim.data(), nt * 8);
  }
  // partials: per circuit, Pauli chunk partials (2 doubles per chunk) then gradient
  // partials (pslots x tiles)
  std::vector<int64_t> e_off(nc), g_off(nc), chunks(nc), atiles(nc);
  int64_t pt = 0;
  for (size_t i = 0; i < nc; ++i) {
    chunks[i] = ((1ll << b->circ[i].n) + kPauliChunk - 1) / kPauliChunk;
    e_off[i] = pt;
    pt += 2 * chunks[i];
    atiles[i] = b->adj[i].passes.empty() ? 1 : (1ll << (b->circ[i].n - b->adj[i].passes[0].m));
    g_off[i] = pt;
    pt += (int64_t)b->adj[i].n_pslots * atiles[i];
  }
  b->partials.reserve(std::max<int64_t>(pt, 1) * sizeof(double));
  double* part = static_cast<double*>(b->partials.p);
  // results: energies, then gradient slots
  b->slot_out_off.assign(nc, 0);
  int64_t no = (int64_t)nc;
  for (size_t i = 0; i < nc; ++i) {
    b->slot_out_off[i] = no;
    no += b->adj[i].n_pslots;
  }
  b->n_out = no;
  b->results.reserve(std::max<int64_t>(no, 1) * sizeof(double));
  // segments
  std::vector<int64_t> soffs;
  std::vector<int32_t> slens, sstr;
  for (size_t i = 0; i < nc; ++i) {
    soffs.push_back(e_off[i]);
    slens.push_back((int32_t)chunks[i]);
    sstr.push_back(2);
  }
  for (size_t i = 0; i < nc; ++i)
    for (int g = 0; g < b->adj[i].n_pslots; ++g) {
      soffs.push_back(g_off[i] + g * atiles[i]);
      slens.push_back((int32_t)atiles[i]);
      sstr.push_back(1);
    }
  const size_t seg_offs = put(soffs.data(), soffs.size() * 8);
  const size_t seg_lens = put(slens.data(), slens.size() * 4);
  const size_t seg_str = put(sstr.data(), sstr.size() * 4);
  // zero-state jobs
  std::vector<int32_t> znq(nc);
  std::vector<uint32_t> zpre(nc + 1, 0);
  for (size_t i = 0; i < nc; ++i) {
    znq[i] = b->circ[i].n;
    zpre[i + 1] = zpre[i] + (uint32_t)(((1ll << b->circ[i].n) + 4095) / 4096);
  }
  const size_t z_ptrs = align_up(st.size(), 256);
  st.resize(z_ptrs + nc * sizeof(void*));  // filled after the device base is known
  const size_t z_nq = put(znq.data(), nc * 4);
  const size_t z_pre = put(zpre.data(), zpre.size() * 4);
  // Pauli jobs (pointers filled below) and prefix
  std::vector<uint32_t> ppre(nc + 1, 0);
  for (size_t i = 0; i < nc; ++i) ppre[i + 1] = ppre[i] + (uint32_t)chunks[i];
  const size_t p_jobs = align_up(st.size(), 256);
  st.resize(p_jobs + nc * sizeof(PauliJob));
  const size_t p_pre = put(ppre.data(), ppre.size() * 4);
  // rounds (PassArgs filled below with device pointers)
  auto make_rounds = [&](bool adjoint, std::vector<Round>& rounds) {
    rounds.clear();
    size_t R = 0;
    for (size_t i = 0; i < nc; ++i) R = std::max(R, (adjoint ? b->adj[i] : b->fwd[i]).passes.size());
    rounds.resize(R);
    for (size_t r = 0; r < R; ++r) {
      Round& rd = rounds[r];
      rd.prefix.push_back(0);
      for (size_t i = 0; i < nc; ++i) {
        const Plan& p = adjoint ? b->adj[i] : b->fwd[i];
        if (r >= p.passes.size()) continue;
        const DevPass& dp = p.passes[r];
        if (!dp.rb) raise(QSV_EINVAL, "internal: batched pass is not register-blocked");
        PassArgs A{};
        A.tile_mask = dp.tile_mask;
        A.n_ops = dp.op_count;
        A.n_qubits = b->circ[i].n;
        A.m = dp.m;
        A.lr0 = dp.lr0;
        A.lay0_reg = dp.lay0_reg;
        A.lay0_thr = dp.lay0_thr;
        A.win_lo = dp.win_lo;
        A.win_n = dp.win_n;
        A.pass_pslots = adjoint ? dp.pslot_count : 0;
        A.n_tiles = 1ll << (b->circ[i].n - dp.m);
        A.n_pslots = adjoint ? p.n_pslots : 0;
        // pointer fields hold offsets for now: fixed up once the device base is known
        A.psi = reinterpret_cast<void*>((uintptr_t)st_off[i]);
        A.ops = reinterpret_cast<const TileOp*>((uintptr_t)((adjoint ? ao[i] : fo[i]).ops + dp.op_first * sizeof(TileOp)));
        A.diag = reinterpret_cast<const DiagEntry*>((uintptr_t)(adjoint ? ao[i] : fo[i]).diag);
        A.edges = reinterpret_cast<const ZZEdge*>((uintptr_t)(adjoint ? ao[i] : fo[i]).edges);
        A.dep = reinterpret_cast<const uint64_t*>(
            (uintptr_t)((adjoint ? ao[i] : fo[i]).deps + (size_t)dp.dep_first * sizeof(uint64_t)));
        A.ctab = reinterpret_cast<const void*>((uintptr_t)(adjoint ? b->ctab_adj_off[i] : b->ctab_fwd_off[i]));
        A.partials = adjoint ? reinterpret_cast<double*>((uintptr_t)(g_off[i] + (int64_t)dp.pslot_first * atiles[i]))
                             : nullptr;
        rd.items.push_back(A);
        rd.prefix.push_back(rd.prefix.back() + (uint32_t)A.n_tiles);
        rd.maxm = std::max(rd.maxm, dp.maxm);
        rd.max_win = std::max(rd.max_win, dp.win_n);
        rd.max_pslots = std::max(rd.max_pslots, A.pass_pslots);
      }
      rd.items_off = align_up(st.size(), 256);
      st.resize(rd.items_off + rd.items.size() * sizeof(PassArgs));
      rd.prefix_off = put(rd.prefix.data(), rd.prefix.size() * 4);
    }
  };
  make_rounds(false, b->frounds);
  make_rounds(true, b->arounds);
  b->statics.reserve(std::max<size_t>(st.size(), 256));
  char* sbase = static_cast<char*>(b->statics.p);
  char* cbase = static_cast<char*>(b->ctab.p);
  // fix up device pointers
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<Round>& rounds = pass == 0 ? b->frounds : b->arounds;
    for (Round& rd : rounds) {
      for (PassArgs& A : rd.items) {
        const int64_t so = (int64_t)(uintptr_t)A.psi;
        A.psi = psi0 + so * b->amp();
        A.lam = pass == 1 ? lam0 + so * b->amp() : nullptr;
        A.src = nullptr;
        A.bstride = 0;
        A.src_bstride = 0;
        A.ops = reinterpret_cast<const TileOp*>(sbase + (uintptr_t)A.ops);
        A.diag = reinterpret_cast<const DiagEntry*>(sbase + (uintptr_t)A.diag);
        A.edges = reinterpret_cast<const ZZEdge*>(sbase + (uintptr_t)A.edges);
        A.dep = reinterpret_cast<const uint64_t*>(sbase + (uintptr_t)A.dep);
        A.ctab = cbase + (uintptr_t)A.ctab * b->amp();
        A.ctab_bstride = 0;
        if (pass == 1) A.partials = part + (uintptr_t)A.partials;
      }
      std::memcpy(st.data() + rd.items_off, rd.items.data(), rd.items.size() * sizeof(PassArgs));
    }
  }
  for (size_t i = 0; i < nc; ++i) {
    void* p = psi0 + st_off[i] * b->amp();
    std::memcpy(st.data() + z_ptrs + i * sizeof(void*), &p, sizeof(void*));
    const size_t nt = b->ham[i].coeffs.size();
    const size_t t = term_off[i];
    PauliJob J{};
    J.psi = psi0 + st_off[i] * b->amp();
    J.lam = lam0 + st_off[i] * b->amp();
    J.xmasks = reinterpret_cast<const uint64_t*>(sbase + t);
    J.zmasks = reinterpret_cast<const uint64_t*>(sbase + tz_off[i]);
    J.cre = reinterpret_cast<const double*>(sbase + tc_off[i]);
    J.cim = reinterpret_cast<const double*>(sbase + ti_off[i]);
    J.partials = part + e_off[i];
    J.n_terms = (int32_t)nt;
    J.n_qubits = b->circ[i].n;
    std::memcpy(st.data() + p_jobs + i * sizeof(PauliJob), &J, sizeof(J));
  }
  hip_check(hipMemcpy(b->statics.p, st.data(), st.size(), hipMemcpyHostToDevice), "upload batch tables");
  // capture the evaluation
  const int dt = b->dtype;
  const int ncols = (int)soffs.size();
  hip_check(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  hipError_t e = launch_set_zero_multi(dt, reinterpret_cast<void* const*>(sbase + z_ptrs),
                                       reinterpret_cast<const int32_t*>(sbase + z_nq),
                                       reinterpret_cast<const uint32_t*>(sbase + z_pre), (int)nc, zpre[nc], b->stream);
  for (const Round& rd : b->frounds) {
    if (e != hipSuccess) break;
    e = launch_tile_pass_rb_multi(dt, false, rd.maxm, reinterpret_cast<const PassArgs*>(sbase + rd.items_off),
                                  reinterpret_cast<const uint32_t*>(sbase + rd.prefix_off), (int)rd.items.size(),
                                  rd.prefix.back(), rd.max_win, rd.max_pslots, b->stream);
  }
  if (e == hipSuccess)
    e = launch_pauli_apply_multi(dt, reinterpret_cast<const PauliJob*>(sbase + p_jobs),
                                 reinterpret_cast<const uint32_t*>(sbase + p_pre), (int)nc, ppre[nc], b->stream);
  for (const Round& rd : b->arounds) {
    if (e != hipSuccess) break;
    e = launch_tile_pass_rb_multi(dt, true, rd.maxm, reinterpret_cast<const PassArgs*>(sbase + rd.items_off),
                                  reinterpret_cast<const uint32_t*>(sbase + rd.prefix_off), (int)rd.items.size(),
                                  rd.prefix.back(), rd.max_win, rd.max_pslots, b->stream);
  }
  if (e == hipSuccess)
    e = launch_reduce_segments(part, reinterpret_cast<const int64_t*>(sbase + seg_offs),
                               reinterpret_cast<const int32_t*>(sbase + seg_lens),
                               reinterpret_cast<const int32_t*>(sbase + seg_str), static_cast<double*>(b->results.p),
                               ncols, b->stream);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  hip_check(e, "batch kernel launch during capture");
  hip_check(e2, "hipStreamEndCapture");
  b->graph = g;
  hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  b->built = true;
}

// One evaluation: bind, upload, replay, download.
void evaluate(qsv_batch* b, const double* params, double* out_E, double* out_grad) {
  if (!b->built) build(b);
  const size_t nc = b->circ.size();
  const size_t up_bytes = (size_t)b->ctab_total * b->amp();
  const size_t down_bytes = (size_t)b->n_out * sizeof(double);
  char* host = static_cast<char*>(host_buffer(b, std::max(up_bytes, down_bytes) + 256));
  std::vector<cplx> tmp;
  for (size_t i = 0; i < nc; ++i) {
    const qsv_circuit c = b->circ[i].view();
    const double* p = params + b->param_off[i];
    for (int k = 0; k < 2; ++k) {
      const Plan& pl = k == 0 ? b->fwd[i] : b->adj[i];
      const int64_t off = k == 0 ? b->ctab_fwd_off[i] : b->ctab_adj_off[i];
      tmp.assign(pl.ctab_size, cplx(0, 0));
      bind_ctab(pl, &c, p, nullptr, 0, tmp.data());
      for (int32_t e = 0; e < pl.ctab_size; ++e) {
        if (b->dtype == QSV_C64) {
          float* d = reinterpret_cast<float*>(host) + 2 * (off + e);
          d[0] = (float)tmp[e].real();
          d[1] = (float)tmp[e].imag();
        } else {
          double* d = reinterpret_cast<double*>(host) + 2 * (off + e);
          d[0] = tmp[e].real();
          d[1] = tmp[e].imag();
        }
      }
    }
  }
  if (up_bytes) hip_check(hipMemcpyAsync(b->ctab.p, host, up_bytes, hipMemcpyHostToDevice, b->stream), "upload");
  hip_check(hipEventRecord(b->ev0, b->stream), "hipEventRecord");
  hip_check(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
  hip_check(hipEventRecord(b->ev1, b->stream), "hipEventRecord");
  double* res = reinterpret_cast<double*>(host);
  hip_check(hipMemcpyAsync(res, b->results.p, down_bytes, hipMemcpyDeviceToHost, b->stream), "download");
  hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, b->ev0, b->ev1), "hipEventElapsedTime");
  b->last_ms = ms;
  for (size_t i = 0; i < nc; ++i) {
    if (out_E) out_E[i] = res[i];
    if (!out_grad) continue;
    double* g = out_grad + b->param_off[i];
    const int64_t np = b->param_off[i + 1] - b->param_off[i];
    for (int64_t k = 0; k < np; ++k) g[k] = 0.0;
    const Plan& a = b->adj[i];
    for (int32_t s = 0; s < a.n_pslots; ++s) g[a.pslot_param[s]] += res[b->slot_out_off[i] + s];
  }
}

qsv_batch* check_batch(const qsv_batch* b) {
  if (!b) raise(QSV_EINVAL, "batch is NULL");
  return const_cast<qsv_batch*>(b);
}

}  // namespace

extern "C" {

int qsv_batch_create(int32_t dtype, size_t n_circuits, const qsv_circuit* circuits, const qsv_pauli_sum* hams,
                     qsv_batch** out) {
  return guarded([&] {
    if (!out) raise(QSV_EINVAL, "out is NULL");
    *out = nullptr;
    if (dtype != QSV_C64 && dtype != QSV_C128) raise(QSV_EDTYPE, "dtype must be QSV_C64 or QSV_C128");
    if (n_circuits < 1 || n_circuits > 65536) raise(QSV_ERANGE, "n_circuits must be in [1, 65536]");
    if (!circuits || !hams) raise(QSV_EINVAL, "circuits / hams are NULL");
    auto b = std::make_unique<qsv_batch>();
    b->dtype = dtype;
    b->param_off.push_back(0);
    uint64_t total_amps = 0;
    for (size_t i = 0; i < n_circuits; ++i) {
      const qsv_circuit& c = circuits[i];
      validate_circuit(&c, (size_t)1 << 30, -1);
      if (c.n_qubits > 28) raise(QSV_ERANGE, "batched circuits must have at most 28 qubits");
      validate_pauli_sum(&hams[i], c.n_qubits);
      CircuitCopy cc;
      cc.n = c.n_qubits;
      cc.gates.assign(c.gates, c.gates + c.n_gates);
      if (c.matrices) cc.mats.assign(c.matrices, c.matrices + c.n_matrix_doubles);
      int64_t np = 0;
      for (const qsv_gate& g : cc.gates)
        for (int a = 0; a < 3; ++a) np = std::max<int64_t>(np, g.param_index[a] + 1);
      b->param_off.push_back(b->param_off.back() + np);
      b->circ.push_back(std::move(cc));
      HamCopy hc;
      const qsv_pauli_sum& h = hams[i];
      hc.coeffs.assign(h.coeffs, h.coeffs + h.n_terms);
      hc.x.assign(h.x_masks, h.x_masks + h.n_terms);
      hc.z.assign(h.z_masks, h.z_masks + h.n_terms);
      b->ham.push_back(std::move(hc));
      total_amps += 1ull << c.n_qubits;
    }
    (void)total_amps;
    b->tile = dtype == QSV_C64 ? 12 : 12;
    hip_check(hipGetDevice(&b->device), "hipGetDevice");
    hip_check(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipEventCreate(&b->ev0), "hipEventCreate");
    hip_check(hipEventCreate(&b->ev1), "hipEventCreate");
    *out = b.release();
  });
}

int qsv_batch_destroy(qsv_batch* b) {
  if (!b) return QSV_OK;
  return guarded([&] {
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    b->states.release();
    b->statics.release();
    b->ctab.release();
    b->partials.release();
    b->results.release();
    if (b->host) (void)hipHostFree(b->host);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
  });
}

int qsv_batch_info(const qsv_batch* b, size_t* total_params, int64_t* param_offsets, double* last_ms,
                   int32_t* tile_qubits) {
  return guarded([&] {
    check_batch(b);
    if (total_params) *total_params = (size_t)b->param_off.back();
    if (param_offsets) std::copy(b->param_off.begin(), b->param_off.end(), param_offsets);
    if (last_ms) *last_ms = b->last_ms;
    if (tile_qubits) *tile_qubits = b->tile;
  });
}

int qsv_batch_set_tile(qsv_batch* b, int32_t tile_qubits) {
  return guarded([&] {
    check_batch(b);
    if (tile_qubits < 9 || tile_qubits > 13 || (b->dtype == QSV_C128 && tile_qubits > 13))
      raise(QSV_EINVAL, "batch tile width must be in [9, 13]");
    hip_check(hipSetDevice(b->device), "hipSetDevice");
    if (tile_qubits != b->tile || !b->built) {
      b->tile = tile_qubits;
      build(b);
    }
  });
}

int qsv_batch_expectation_and_grad(qsv_batch* b, const double* params, double* out_E, double* out_grad) {
  return guarded([&] {
    check_batch(b);
    if (b->param_off.back() && !params) raise(QSV_EINVAL, "params is NULL");
    if (!out_E) raise(QSV_EINVAL, "out_E is NULL");
    for (int64_t k = 0; k < b->param_off.back(); ++k)
      if (!std::isfinite(params[k])) raise(QSV_EINVAL, "non-finite parameter");
    hip_check(hipSetDevice(b->device), "hipSetDevice");
    evaluate(b, params, out_E, out_grad);
  });
}

int qsv_batch_autotune(qsv_batch* b, const double* params, int32_t* out_tile, int32_t* out_low_qubits) {
  return guarded([&] {
    check_batch(b);
    if (b->param_off.back() && !params) raise(QSV_EINVAL, "params is NULL");
    hip_check(hipSetDevice(b->device), "hipSetDevice");
    // the fusion width and the tile schedule: how many low qubits every tile keeps (dense
    // global accesses) against how many passes the circuits then need
    const int tiles[] = {10, 11, 12, 13}, lows[] = {2, 3, 4};
    int best_t = b->tile, best_l = b->low;
    double best_ms = 1e300;
    std::vector<double> E(b->circ.size());
    for (int t : tiles)
      for (int l : lows) {
        b->tile = t;
        b->low = l;
        build(b);
        evaluate(b, params, E.data(), nullptr);  // warm
        double ms = 1e300;
        for (int r = 0; r < 2; ++r) {
          evaluate(b, params, E.data(), nullptr);
          ms = std::min(ms, b->last_ms);
        }
        if (ms < best_ms) {
          best_ms = ms;
          best_t = t;
          best_l = l;
        }
      }
    b->tile = best_t;
    b->low = best_l;
    build(b);
    if (out_tile) *out_tile = best_t;
    if (out_low_qubits) *out_low_qubits = best_l;
  });
}

}  // extern "C"
