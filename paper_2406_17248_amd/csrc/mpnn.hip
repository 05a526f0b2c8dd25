// Warm-start network for QAOA MaxCut: a 2-layer message-passing network (hidden 64, fp32)
// that maps a 16-node graph to p = 6 QAOA angles (6 gamma then 6 beta), as a correction to
// a linear-ramp schedule.  Hand-written forward, backward and Adam kernels; one workgroup
// per graph (the graph, its activations and its gradient contributions live in LDS), and a
// fixed-order reduction of the per-graph parameter gradients.
//
//   node features  x_v = [1, deg(v) / 4, triangles(v) / 3]
//   layer 1        Z1 = X W1s + (A X) W1n / 4 + b1,   H1 = relu(Z1)
//   layer 2        Z2 = H1 W2s + (A H1) W2n / 4 + b2, H2 = relu(Z2)
//   readout        g = mean_v H2[v];  angles = ramp + g Wo + bo
//   loss           mean over graphs of sum_k (angles_k - label_k)^2 / 12
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "../../include/qsv.h"
#include "hip_util.h"

namespace qsv {
namespace {

constexpr int MN = QSV_MPNN_NODES, MF = QSV_MPNN_FEATURES, MH = QSV_MPNN_HIDDEN, MO = QSV_MPNN_OUTPUTS;
constexpr int O_W1S = 0, O_W1N = O_W1S + MF * MH, O_B1 = O_W1N + MF * MH, O_W2S = O_B1 + MH,
              O_W2N = O_W2S + MH * MH, O_B2 = O_W2N + MH * MH, O_WO = O_B2 + MH, O_BO = O_WO + MH * MO,
              NP = O_BO + MO;
static_assert(NP == QSV_MPNN_PARAMS, "parameter layout");
constexpr int NT = 256;

template <bool BWD>
__global__ __launch_bounds__(NT) void mpnn_graph(const float* __restrict__ W, const uint16_t* __restrict__ adj,
                                                 const float* __restrict__ ramp, const float* __restrict__ labels,
                                                 float* __restrict__ angles, float* __restrict__ loss,
                                                 float* __restrict__ gpart, float inv_batch) {
  const int b = blockIdx.x, t = threadIdx.x;
  __shared__ float A[MN][MN], X[MN][MF], AX[MN][MF];
  __shared__ float Z1[MN][MH], H1[MN][MH], AH1[MN][MH], Z2[MN][MH], D[MN][MH], E[MN][MH];
  __shared__ float g[MH], out[MO], dout[MO], dg[MH];
  for (int i = t; i < MN * MN; i += NT) {
    const int v = i / MN, u = i % MN;
    A[v][u] = (float)((adj[(size_t)b * MN + v] >> u) & 1);
  }
  __syncthreads();
  if (t < MN) {
    float deg = 0.f, tri = 0.f;
    for (int u = 0; u < MN; ++u) {
      deg += A[t][u];
      for (int w = 0; w < MN; ++w) tri += A[t][u] * A[u][w] * A[w][t];
    }
    X[t][0] = 1.f;
    X[t][1] = deg * 0.25f;
    X[t][2] = tri * 0.5f / 3.f;
  }
  __syncthreads();
  if (t < MN * MF) {
    const int v = t / MF, f = t % MF;
    float s = 0.f;
    for (int u = 0; u < MN; ++u) s += A[v][u] * X[u][f];
    AX[v][f] = s;
  }
  __syncthreads();
  for (int i = t; i < MN * MH; i += NT) {
    const int v = i / MH, h = i % MH;
    float z = W[O_B1 + h];
    for (int f = 0; f < MF; ++f) z += X[v][f] * W[O_W1S + f * MH + h] + 0.25f * AX[v][f] * W[O_W1N + f * MH + h];
    Z1[v][h] = z;
    H1[v][h] = z > 0.f ? z : 0.f;
  }
  __syncthreads();
  for (int i = t; i < MN * MH; i += NT) {
    const int v = i / MH, h = i % MH;
    float s = 0.f;
    for (int u = 0; u < MN; ++u) s += A[v][u] * H1[u][h];
    AH1[v][h] = s;
  }
  __syncthreads();
  for (int i = t; i < MN * MH; i += NT) {
    const int v = i / MH, h = i % MH;
    float z = W[O_B2 + h];
    for (int k = 0; k < MH; ++k) z += H1[v][k] * W[O_W2S + k * MH + h] + 0.25f * AH1[v][k] * W[O_W2N + k * MH + h];
    Z2[v][h] = z;
  }
  __syncthreads();
  if (t < MH) {
    float s = 0.f;
    for (int v = 0; v < MN; ++v) s += Z2[v][t] > 0.f ? Z2[v][t] : 0.f;
    g[t] = s / (float)MN;
  }
  __syncthreads();
  if (t < MO) {
    float o = W[O_BO + t] + ramp[t];
    for (int h = 0; h < MH; ++h) o += g[h] * W[O_WO + h * MO + t];
    out[t] = o;
    angles[(size_t)b * MO + t] = o;
  }
  if (!BWD) return;
  __syncthreads();
  if (t < MO) dout[t] = 2.f * (out[t] - labels[(size_t)b * MO + t]) / (float)MO * inv_batch;
  if (t == 0) {
    float l = 0.f;
    for (int o = 0; o < MO; ++o) {
      const float d = out[o] - labels[(size_t)b * MO + o];
      l += d * d;
    }
    loss[b] = l / (float)MO * inv_batch;
  }
  __syncthreads();
  float* G = gpart + (size_t)b * NP;
  if (t < MH) {
    float s = 0.f;
    for (int o = 0; o < MO; ++o) s += W[O_WO + t * MO + o] * dout[o];
    dg[t] = s;
  }
  for (int i = t; i < MH * MO; i += NT) G[O_WO + i] = g[i / MO] * dout[i % MO];
  if (t < MO) G[O_BO + t] = dout[t];
  __syncthreads();
  for (int i = t; i < MN * MH; i += NT) {  // D = dZ2
    const int v = i / MH, h = i % MH;
    D[v][h] = Z2[v][h] > 0.f ? dg[h] / (float)MN : 0.f;
  }
  __syncthreads();
  for (int i = t; i < MH * MH; i += NT) {
    const int k = i / MH, h = i % MH;
    float s = 0.f, sn = 0.f;
    for (int v = 0; v < MN; ++v) {
      s += H1[v][k] * D[v][h];
      sn += AH1[v][k] * D[v][h];
    }
    G[O_W2S + i] = s;
    G[O_W2N + i] = 0.25f * sn;
  }
  if (t < MH) {
    float s = 0.f;
    for (int v = 0; v < MN; ++v) s += D[v][t];
    G[O_B2 + t] = s;
  }
  for (int i = t; i < MN * MH; i += NT) {  // E = dZ2 W2n^T
    const int v = i / MH, k = i % MH;
    float s = 0.f;
    for (int h = 0; h < MH; ++h) s += D[v][h] * W[O_W2N + k * MH + h];
    E[v][k] = s;
  }
  __syncthreads();
  for (int i = t; i < MN * MH; i += NT) {  // dZ1 = (dZ2 W2s^T + A E / 4) masked by Z1 > 0
    const int v = i / MH, k = i % MH;
    float s = 0.f;
    for (int h = 0; h < MH; ++h) s += D[v][h] * W[O_W2S + k * MH + h];
    float a = 0.f;
    for (int u = 0; u < MN; ++u) a += A[v][u] * E[u][k];
    s += 0.25f * a;
    H1[v][k] = Z1[v][k] > 0.f ? s : 0.f;  // H1 is dead after the W2 gradients: reuse for dZ1
  }
  __syncthreads();
  for (int i = t; i < MF * MH; i += NT) {
    const int f = i / MH, h = i % MH;
    float s = 0.f, sn = 0.f;
    for (int v = 0; v < MN; ++v) {
      s += X[v][f] * H1[v][h];
      sn += AX[v][f] * H1[v][h];
    }
    G[O_W1S + i] = s;
    G[O_W1N + i] = 0.25f * sn;
  }
  if (t < MH) {
    float s = 0.f;
    for (int v = 0; v < MN; ++v) s += H1[v][t];
    G[O_B1 + t] = s;
  }
}

// grad[p] = sum_b gpart[b][p]; loss = sum_b loss[b] (fixed order)
__global__ __launch_bounds__(NT) void mpnn_reduce(const float* __restrict__ gpart, const float* __restrict__ lossb,
                                                  int batch, float* __restrict__ grad, float* __restrict__ loss) {
  const int p = blockIdx.x * NT + threadIdx.x;
  if (p < NP) {
    float s = 0.f;
    for (int b = 0; b < batch; ++b) s += gpart[(size_t)b * NP + p];
    grad[p] = s;
  }
  if (p == 0) {
    float s = 0.f;
    for (int b = 0; b < batch; ++b) s += lossb[b];
    *loss = s;
  }
}

__global__ __launch_bounds__(NT) void mpnn_adam(float* __restrict__ W, float* __restrict__ m1, float* __restrict__ m2,
                                                const float* __restrict__ grad, float lr, float b1, float b2, float eps,
                                                float c1, float c2) {
  const int p = blockIdx.x * NT + threadIdx.x;
  if (p >= NP) return;
  const float gr = grad[p];
  const float a = b1 * m1[p] + (1.f - b1) * gr;
  const float v = b2 * m2[p] + (1.f - b2) * gr * gr;
  m1[p] = a;
  m2[p] = v;
  W[p] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

}  // namespace
}  // namespace qsv

using namespace qsv;

struct qsv_mpnn {
  int device = 0;
  hipStream_t stream = nullptr;
  DevBuf W, m1, m2, grad, loss1, gpart, lossb, io;
  int64_t step = 0;
};

namespace {

qsv_mpnn* check_mpnn(const qsv_mpnn* m) {
  if (!m) raise(QSV_EINVAL, "network is NULL");
  return const_cast<qsv_mpnn*>(m);
}

// Upload graphs, ramp and labels; run forward (and backward); returns device pointers.
void run(qsv_mpnn* m, const uint16_t* adj, size_t n, const double* ramp, const double* labels, bool bwd,
         double* out_angles, double* out_loss, float* out_grad) {
  if (!adj || !ramp) raise(QSV_EINVAL, "adjacency / ramp are NULL");
  if (n < 1 || n > 65535) raise(QSV_ERANGE, "n_graphs must be in [1, 65535]");
  if (bwd && !labels) raise(QSV_EINVAL, "labels are NULL");
  for (size_t i = 0; i < n * MN; ++i) {
    const int v = (int)(i % MN);
    if (adj[i] >> v & 1) raise(QSV_EINVAL, "a graph has a self loop");
  }
  hip_check(hipSetDevice(m->device), "hipSetDevice");
  // io layout: adj (n*16 u16) | ramp (12 f32) | labels (n*12 f32) | angles (n*12 f32)
  const size_t o_adj = 0, o_ramp = align_up(n * MN * 2, 256), o_lab = o_ramp + 256,
               o_ang = align_up(o_lab + n * MO * 4, 256), total = align_up(o_ang + n * MO * 4, 256);
  std::vector<char> host(total, 0);
  std::memcpy(host.data() + o_adj, adj, n * MN * 2);
  for (int k = 0; k < MO; ++k) reinterpret_cast<float*>(host.data() + o_ramp)[k] = (float)ramp[k];
  if (labels)
    for (size_t k = 0; k < n * MO; ++k) reinterpret_cast<float*>(host.data() + o_lab)[k] = (float)labels[k];
  m->io.reserve(total);
  char* d = static_cast<char*>(m->io.p);
  hip_check(hipMemcpyAsync(d, host.data(), o_ang, hipMemcpyHostToDevice, m->stream), "upload graphs");
  if (bwd) {
    m->gpart.reserve(n * NP * sizeof(float));
    m->lossb.reserve(n * sizeof(float));
    mpnn_graph<true><<<(unsigned)n, NT, 0, m->stream>>>(
        static_cast<float*>(m->W.p), reinterpret_cast<uint16_t*>(d + o_adj), reinterpret_cast<float*>(d + o_ramp),
        reinterpret_cast<float*>(d + o_lab), reinterpret_cast<float*>(d + o_ang), static_cast<float*>(m->lossb.p),
        static_cast<float*>(m->gpart.p), 1.f / (float)n);
    hip_check(hipGetLastError(), "mpnn forward/backward");
    mpnn_reduce<<<(NP + NT - 1) / NT, NT, 0, m->stream>>>(static_cast<float*>(m->gpart.p),
                                                          static_cast<float*>(m->lossb.p), (int)n,
                                                          static_cast<float*>(m->grad.p), static_cast<float*>(m->loss1.p));
    hip_check(hipGetLastError(), "mpnn reduce");
  } else {
    mpnn_graph<false><<<(unsigned)n, NT, 0, m->stream>>>(
        static_cast<float*>(m->W.p), reinterpret_cast<uint16_t*>(d + o_adj), reinterpret_cast<float*>(d + o_ramp),
        nullptr, reinterpret_cast<float*>(d + o_ang), nullptr, nullptr, 0.f);
    hip_check(hipGetLastError(), "mpnn forward");
  }
  if (out_angles) {
    std::vector<float> a(n * MO);
    hip_check(hipMemcpyAsync(a.data(), d + o_ang, n * MO * 4, hipMemcpyDeviceToHost, m->stream), "download angles");
    hip_check(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    for (size_t k = 0; k < n * MO; ++k) out_angles[k] = a[k];
  }
  if (bwd && (out_loss || out_grad)) {
    float l = 0.f;
    hip_check(hipMemcpyAsync(&l, m->loss1.p, 4, hipMemcpyDeviceToHost, m->stream), "download loss");
    if (out_grad) hip_check(hipMemcpyAsync(out_grad, m->grad.p, NP * 4, hipMemcpyDeviceToHost, m->stream), "download grad");
    hip_check(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    if (out_loss) *out_loss = l;
  }
}

}  // namespace

extern "C" {

int qsv_mpnn_create(const float* init_params, qsv_mpnn** out) {
  return guarded([&] {
    if (!out || !init_params) raise(QSV_EINVAL, "NULL argument");
    *out = nullptr;
    auto m = std::make_unique<qsv_mpnn>();
    hip_check(hipGetDevice(&m->device), "hipGetDevice");
    hip_check(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking), "hipStreamCreate");
    for (DevBuf* b : {&m->W, &m->m1, &m->m2, &m->grad}) b->reserve(NP * sizeof(float));
    m->loss1.reserve(256);
    hip_check(hipMemcpy(m->W.p, init_params, NP * sizeof(float), hipMemcpyHostToDevice), "upload params");
    hip_check(hipMemset(m->m1.p, 0, NP * sizeof(float)), "zero moments");
    hip_check(hipMemset(m->m2.p, 0, NP * sizeof(float)), "zero moments");
    *out = m.release();
  });
}

int qsv_mpnn_destroy(qsv_mpnn* m) {
  if (!m) return QSV_OK;
  return guarded([&] {
    (void)hipSetDevice(m->device);
    (void)hipStreamSynchronize(m->stream);
    for (DevBuf* b : {&m->W, &m->m1, &m->m2, &m->grad, &m->loss1, &m->gpart, &m->lossb, &m->io}) b->release();
    (void)hipStreamDestroy(m->stream);
    delete m;
  });
}

int qsv_mpnn_get_params(const qsv_mpnn* m, float* out) {
  return guarded([&] {
    check_mpnn(m);
    if (!out) raise(QSV_EINVAL, "out is NULL");
    hip_check(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    hip_check(hipMemcpy(out, m->W.p, NP * sizeof(float), hipMemcpyDeviceToHost), "download params");
  });
}

int qsv_mpnn_predict(qsv_mpnn* m, const uint16_t* adj, size_t n_graphs, const double* ramp, double* out_angles) {
  return guarded([&] {
    check_mpnn(m);
    if (!out_angles) raise(QSV_EINVAL, "out_angles is NULL");
    run(m, adj, n_graphs, ramp, nullptr, false, out_angles, nullptr, nullptr);
  });
}

int qsv_mpnn_loss_and_grad(qsv_mpnn* m, const uint16_t* adj, size_t n_graphs, const double* ramp,
                           const double* labels, double* out_loss, float* out_grad) {
  return guarded([&] {
    check_mpnn(m);
    run(m, adj, n_graphs, ramp, labels, true, nullptr, out_loss, out_grad);
  });
}

int qsv_mpnn_train_step(qsv_mpnn* m, const uint16_t* adj, size_t n_graphs, const double* ramp, const double* labels,
                        double lr, double* out_loss) {
  return guarded([&] {
    check_mpnn(m);
    if (!(lr > 0.0) || !std::isfinite(lr)) raise(QSV_EINVAL, "learning rate must be positive");
    run(m, adj, n_graphs, ramp, labels, true, nullptr, nullptr, nullptr);
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
    mpnn_adam<<<(NP + NT - 1) / NT, NT, 0, m->stream>>>(static_cast<float*>(m->W.p), static_cast<float*>(m->m1.p),
                                                        static_cast<float*>(m->m2.p), static_cast<float*>(m->grad.p),
                                                        (float)lr, b1, b2, 1e-8f, c1, c2);
    hip_check(hipGetLastError(), "mpnn adam");
    if (out_loss) {
      float l = 0.f;
      hip_check(hipMemcpyAsync(&l, m->loss1.p, 4, hipMemcpyDeviceToHost, m->stream), "download loss");
      hip_check(hipStreamSynchronize(m->stream), "hipStreamSynchronize");
      *out_loss = l;
    }
  });
}

}  // extern "C"
