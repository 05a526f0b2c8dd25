// HIP kernels of the state-vector engine, written for gfx950 (CDNA4, wave64).
//
//  tile_pass      one fused pass: a workgroup stages a 2^m-amplitude tile (the sub-cube
//                 spanned by the pass's tile qubits, low qubits included so every global
//                 access is a run of >= 128 contiguous bytes) into LDS, applies the pass's
//                 op list there, and writes it back: one HBM read + write of the state for
//                 a whole run of gates.  The adjoint variant stages psi and lambda together,
//                 applies U^dag to both and accumulates Im<lambda|G|psi> per gradient slot
//                 in fp64 (wave shuffles, then LDS across waves, then one partial per tile).
//  gate1/gate2/diag_stream
//                 unfused per-gate passes over HBM (baseline path and tile-width 0).
//  pauli_group    one read pass per group of Pauli terms sharing an x-mask: expectation
//                 partials and, optionally, lambda = H psi.
//  reduce_columns fixed-order fp64 sums of per-block partials (bitwise repeatable).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qsv_kernels.h"

namespace qsv {

template <typename R> struct CT;
template <> struct CT<float>  { using T = float2; };
template <> struct CT<double> { using T = double2; };

__device__ __forceinline__ float  fmaT(float a, float b, float c)    { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = fmaT(a.x, b.x, -a.y * b.y);
  r.y = fmaT(a.x, b.y, a.y * b.x);
  return r;
}
// u0 * v0 + u1 * v1
template <typename C> __device__ __forceinline__ C cdot2(C u0, C v0, C u1, C v1) {
  C r;
  r.x = fmaT(u0.x, v0.x, fmaT(-u0.y, v0.y, fmaT(u1.x, v1.x, -u1.y * v1.y)));
  r.y = fmaT(u0.x, v0.y, fmaT(u0.y, v0.x, fmaT(u1.x, v1.y, u1.y * v1.x)));
  return r;
}
// Im(conj(w) * g) in fp64
template <typename C> __device__ __forceinline__ double im_conj_mul(C w, C g) {
  return (double)w.x * (double)g.y - (double)w.y * (double)g.x;
}

// Register-resident updates.  A pass keeps each amplitude in the same registers from op to
// op only if every op overwrites an input component with the one multiply-add that reads it
// last.  So each output component is finished by a multiply-add on the component it
// replaces; all other reads of the inputs feed partial sums that pass through an empty asm
// first, which orders them before every finishing multiply-add.  That multiply-add is
// itself an asm: the compiler's two-address form would tie the result to the partial sum's
// register instead.
template <typename R> __device__ __forceinline__ void order(R& a, R& b) { asm("" : "+v"(a), "+v"(b)); }
template <typename R> __device__ __forceinline__ void order(R& a, R& b, double& e) {
  asm("" : "+v"(a), "+v"(b), "+v"(e));
}
template <typename R> __device__ __forceinline__ void order(R& a, R& b, R& c, R& d) {
  asm("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
}
template <typename R> __device__ __forceinline__ void order(R& a, R& b, R& c, R& d, double& e) {
  asm("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d), "+v"(e));
}
// a * b + c; fma_s takes a wave-uniform a (an SGPR operand)
__device__ __forceinline__ double fma_s(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "s"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ float fma_s(float a, float b, float c) {
  float r;
  asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "s"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ double fma_v(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ float fma_v(float a, float b, float c) {
  float r;
  asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
// (a0, a1) <- (u00 a0 + u01 a1, u10 a0 + u11 a1) in place, u wave-uniform.  The optional
// `pin` (a value computed from the old inputs, e.g. a gradient term) is held back with
// the partial sums, so it too is computed before any input is overwritten.
template <typename C, typename... Pin>
__device__ __forceinline__ void apply2(C u00, C u01, C u10, C u11, C& a0, C& a1, Pin&... pin) {
  auto p0r = fmaT(-u00.y, a0.y, fmaT(u01.x, a1.x, -u01.y * a1.y));
  auto p0i = fmaT(u00.y, a0.x, fmaT(u01.x, a1.y, u01.y * a1.x));
  auto p1r = fmaT(u10.x, a0.x, fmaT(-u10.y, a0.y, -u11.y * a1.y));
  auto p1i = fmaT(u10.x, a0.y, fmaT(u10.y, a0.x, u11.y * a1.x));
  order(p0r, p0i, p1r, p1i, pin...);
  a0.x = fma_s(u00.x, a0.x, p0r);
  a0.y = fma_s(u00.x, a0.y, p0i);
  a1.x = fma_s(u11.x, a1.x, p1r);
  a1.y = fma_s(u11.x, a1.y, p1i);
}
// a1 <- a1 * p, then (a0, a1) <- (r0.x a0 + r0.y a1, r1.x a0 + r1.y a1) with real r, in place
// (p and r wave-uniform): a phase and a real 2x2 matrix, 12 instructions per pair
template <typename C>
__device__ __forceinline__ void apply2split(C r0, C r1, C p, C& a0, C& a1) {
  {
    auto pr = -a1.y * p.y;
    auto pi = a1.x * p.y;
    order(pr, pi);
    a1.x = fma_s(p.x, a1.x, pr);
    a1.y = fma_s(p.x, a1.y, pi);
  }
  auto p0r = r0.y * a1.x;
  auto p0i = r0.y * a1.y;
  auto p1r = r1.x * a0.x;
  auto p1i = r1.x * a0.y;
  order(p0r, p0i, p1r, p1i);
  a0.x = fma_s(r0.x, a0.x, p0r);
  a0.y = fma_s(r0.x, a0.y, p0i);
  a1.x = fma_s(r1.y, a1.x, p1r);
  a1.y = fma_s(r1.y, a1.y, p1i);
}
// Matrix forms of one-qubit gates (bits 5-6 of TileOp::plain): general, split (a phase then
// a real matrix), real (RY, H, X), and real diagonal with imaginary off-diagonal (RX, Y).
enum MatForm : int { FORM_GENERAL = 0, FORM_SPLIT = 1, FORM_REAL = 2, FORM_XLIKE = 3 };
// apply2 for a form: real U (entries' .x) or U = [[a, i b], [i c, d]] (a, d in .x, b, c in .y)
// in 8 instructions per pair, else the general product
template <int F, typename C, typename... Pin>
__device__ __forceinline__ void apply2f(const C* U, C& a0, C& a1, Pin&... pin) {
  if constexpr (F == FORM_REAL) {
    auto p0r = U[1].x * a1.x;
    auto p0i = U[1].x * a1.y;
    auto p1r = U[2].x * a0.x;
    auto p1i = U[2].x * a0.y;
    order(p0r, p0i, p1r, p1i, pin...);
    a0.x = fma_s(U[0].x, a0.x, p0r);
    a0.y = fma_s(U[0].x, a0.y, p0i);
    a1.x = fma_s(U[3].x, a1.x, p1r);
    a1.y = fma_s(U[3].x, a1.y, p1i);
  } else if constexpr (F == FORM_XLIKE) {
    auto p0r = -U[1].y * a1.y;
    auto p0i = U[1].y * a1.x;
    auto p1r = -U[2].y * a0.y;
    auto p1i = U[2].y * a0.x;
    order(p0r, p0i, p1r, p1i, pin...);
    a0.x = fma_s(U[0].x, a0.x, p0r);
    a0.y = fma_s(U[0].x, a0.y, p0i);
    a1.x = fma_s(U[3].x, a1.x, p1r);
    a1.y = fma_s(U[3].x, a1.y, p1i);
  } else {
    apply2(U[0], U[1], U[2], U[3], a0, a1, pin...);
  }
}
// a <- a * p in place (p per lane), with an optional `pin` as above
template <typename C, typename... Pin> __device__ __forceinline__ void cmul_in(C& a, C p, Pin&... pin) {
  auto pr = -a.y * p.y;
  auto pi = a.x * p.y;
  order(pr, pi, pin...);
  a.x = fma_v(p.x, a.x, pr);
  a.y = fma_v(p.x, a.y, pi);
}

// Negate v when f is 0x80000000 (f = 0: unchanged), by flipping the sign bits.
__device__ __forceinline__ void flip_sign(float2& v, uint32_t f) {
  v.x = __uint_as_float(__float_as_uint(v.x) ^ f);
  v.y = __uint_as_float(__float_as_uint(v.y) ^ f);
}
__device__ __forceinline__ void flip_sign(double2& v, uint32_t f) {
  const uint64_t g = (uint64_t)f << 32;
  v.x = __longlong_as_double(__double_as_longlong(v.x) ^ g);
  v.y = __longlong_as_double(__double_as_longlong(v.y) ^ g);
}

// Deposit the low bits of v into the set positions of mask (ascending).
__device__ __forceinline__ uint64_t pdep64(uint64_t v, uint64_t mask) {
  uint64_t r = 0;
  while (mask && v) {
    const uint64_t low = mask & (~mask + 1);
    if (v & 1) r |= low;
    v >>= 1;
    mask &= mask - 1;
  }
  return r;
}

// The value of a lane chosen by a DPP control (0: where the control selects no lane).
template <int CTRL> __device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// x + (x of lane l ^ 16) (L = 4) or l ^ 32 (L = 5), when x is equal across the 16 (32) lanes
// of each row (half-wave): the row (half-wave) swap of two copies leaves one of each pair.
template <int L> __device__ __forceinline__ double swap_add_f64(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  uint32_t a0 = (uint32_t)u, b0 = a0, a1 = (uint32_t)(u >> 32), b1 = a1;
  if constexpr (L == 5) {
    const auto r0 = __builtin_amdgcn_permlane32_swap(a0, b0, false, false);
    const auto r1 = __builtin_amdgcn_permlane32_swap(a1, b1, false, false);
    a0 = r0[0]; b0 = r0[1]; a1 = r1[0]; b1 = r1[1];
  } else {
    const auto r0 = __builtin_amdgcn_permlane16_swap(a0, b0, false, false);
    const auto r1 = __builtin_amdgcn_permlane16_swap(a1, b1, false, false);
    a0 = r0[0]; b0 = r0[1]; a1 = r1[0]; b1 = r1[1];
  }
  return __longlong_as_double((long long)(((uint64_t)a1 << 32) | a0)) +
         __longlong_as_double((long long)(((uint64_t)b1 << 32) | b0));
}
// Sum over the 64 lanes of a wave, returned in every lane (every lane must be active): a
// butterfly by cross-lane moves that stay out of LDS - quad permutes for lane bits 0 and 1,
// the half-row and row mirrors for bits 2 and 3 (each quad, then each half-row, already
// holds one value), the row and half-wave swaps for bits 4 and 5.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]: lane ^ 1
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]: lane ^ 2
  v += dpp_f64<0x141>(v);  // row_half_mirror: the other quad of the half-row
  v += dpp_f64<0x140>(v);  // row_mirror: the other half of the row
  v = swap_add_f64<4>(v);
  return swap_add_f64<5>(v);
}

// Read-only tables (op lists, diagonal entries, edges, bound matrices, Pauli terms) are
// read through the constant address space: uniform addresses then become scalar loads
// through the scalar cache instead of vector memory instructions.
#define QSV_CONST __attribute__((address_space(4)))
template <typename T> __device__ __forceinline__ T ld(const T* p) { return *(const QSV_CONST T*)p; }
// A whole record through the scalar path, dword by dword (the loads merge into wide
// scalar loads).
template <typename T> __device__ __forceinline__ T ld_record(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "record size must be a multiple of 4 bytes");
  T r;
  uint32_t* d = reinterpret_cast<uint32_t*>(&r);
  const QSV_CONST uint32_t* q = (const QSV_CONST uint32_t*)(const void*)p;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = q[i];
  return r;
}
template <typename C> __device__ __forceinline__ C ldc(const C* p) {
  using R = decltype(p->x);
  const QSV_CONST R* q = (const QSV_CONST R*)p;
  C r;
  r.x = q[0];
  r.y = q[1];
  return r;
}

// ------------------------------------------------------------------------------------------
// Fused tile pass.
// ------------------------------------------------------------------------------------------
template <typename R, int NT, int MAXM, bool ADJ>
__global__ __launch_bounds__(NT) void tile_pass(PassArgs A) {
  using C = typename CT<R>::T;
  constexpr int LGNT = (NT == 1024) ? 10 : (NT == 512) ? 9 : 8;
  constexpr int RA = ((1 << MAXM) + NT - 1) / NT;        // amplitude slots per thread (max)
  constexpr int PP = ((1 << MAXM) / 2 + NT - 1) / NT;    // pairs per thread per 1-qubit op (max)
  constexpr int QP = ((1 << MAXM) / 4 + NT - 1) / NT;    // quads per thread per 2-qubit op (max)
  __shared__ C sp[1 << MAXM];
  __shared__ C sl[ADJ ? (1 << MAXM) : 1];
  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  const int m = A.m;
  const int nloc = 1 << m;
  const int half = nloc >> 1, quarter = nloc >> 2;
  const bool active = tid < nloc;
  const uint64_t tile = blockIdx.x;
  const int b = blockIdx.y;
  const uint64_t full = (A.n_qubits >= 64) ? ~0ull : ((1ull << A.n_qubits) - 1);
  const uint64_t base = pdep64(tile, full & ~A.tile_mask);
  const uint64_t s_tid = pdep64((uint64_t)tid, A.tile_mask);
  uint64_t hmask = A.tile_mask;               // tile bits above the thread bits
  for (int i = 0; i < LGNT; ++i) hmask &= hmask - 1;
  uint64_t xk[RA];                            // global index of each amplitude slot
#pragma unroll
  for (int k = 0; k < RA; ++k) xk[k] = base | s_tid | pdep64((uint64_t)k, hmask);

  C* psi = reinterpret_cast<C*>(A.psi) + (int64_t)b * A.bstride;
  C* lam = ADJ ? reinterpret_cast<C*>(A.lam) + (int64_t)b * A.bstride : nullptr;
  const C* src = A.src ? reinterpret_cast<const C*>(A.src) + (int64_t)b * A.src_bstride : psi;
  const C* T = reinterpret_cast<const C*>(A.ctab) + (int64_t)b * A.ctab_bstride;

  if (active) {
#pragma unroll
    for (int k = 0; k < RA; ++k) {
      const int j = tid + k * NT;
      if (j < nloc) {
        sp[j] = src[xk[k]];
        if (ADJ) sl[j] = lam[xk[k]];
      }
    }
  }
  __syncthreads();

  double acc = 0.0;
  for (int oi = 0; oi < A.n_ops; ++oi) {
    const TileOp* O = A.ops + oi;
    const int type = ld(&O->type);
    const uint64_t omask = ld(&O->omask);
    const bool on = (base & omask) == omask;
    if (on && type == OP_DENSE1) {
      const int mat = ld(&O->mat), gen = ld(&O->gen);
      const C u00 = ldc(T + mat), u01 = ldc(T + mat + 1), u10 = ldc(T + mat + 2), u11 = ldc(T + mat + 3);
      C g00, g01, g10, g11;
      const bool grad = ADJ && gen >= 0;
      if (grad) { g00 = ldc(T + gen); g01 = ldc(T + gen + 1); g10 = ldc(T + gen + 2); g11 = ldc(T + gen + 3); }
      const int a = ld(&O->a);
      const int amask = (1 << a) - 1;
      const uint32_t lm = ld(&O->lmask);
      int j0[PP];
      bool ok[PP];
      C v0[PP], v1[PP], w0[PP], w1[PP];
#pragma unroll
      for (int i = 0; i < PP; ++i) {
        const int p = tid + i * NT;
        j0[i] = ((p >> a) << (a + 1)) | (p & amask);
        ok[i] = p < half && (((uint32_t)j0[i] & lm) == lm);
        if (ok[i]) {
          v0[i] = sp[j0[i]];
          v1[i] = sp[j0[i] | (1 << a)];
          if (ADJ) { w0[i] = sl[j0[i]]; w1[i] = sl[j0[i] | (1 << a)]; }
        }
      }
#pragma unroll
      for (int i = 0; i < PP; ++i) {
        if (!ok[i]) continue;
        if (ADJ) {
          if (grad)
            acc += im_conj_mul(w0[i], cdot2(g00, v0[i], g01, v1[i])) + im_conj_mul(w1[i], cdot2(g10, v0[i], g11, v1[i]));
          sl[j0[i]] = cdot2(u00, w0[i], u01, w1[i]);
          sl[j0[i] | (1 << a)] = cdot2(u10, w0[i], u11, w1[i]);
        }
        sp[j0[i]] = cdot2(u00, v0[i], u01, v1[i]);
        sp[j0[i] | (1 << a)] = cdot2(u10, v0[i], u11, v1[i]);
      }
    } else if (on && type == OP_DENSE2) {
      const int a = ld(&O->a), bb = ld(&O->b);
      const int mat = ld(&O->mat), gen = ld(&O->gen);
      const int lo = a < bb ? a : bb, hi = a < bb ? bb : a;
      const uint32_t lm = ld(&O->lmask);
      const bool grad = ADJ && gen >= 0;
      C U[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) U[r] = ldc(T + mat + r);
#pragma unroll
      for (int i = 0; i < QP; ++i) {
        const int p = tid + i * NT;
        if (p >= quarter) continue;
        int t = ((p >> lo) << (lo + 1)) | (p & ((1 << lo) - 1));
        t = ((t >> hi) << (hi + 1)) | (t & ((1 << hi) - 1));
        if (((uint32_t)t & lm) != lm) continue;
        const int idx[4] = {t, t | (1 << a), t | (1 << bb), t | (1 << a) | (1 << bb)};
        C v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = sp[idx[r]];
        if (ADJ) {
          C w[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) w[r] = sl[idx[r]];
          if (grad) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              C gsum = cdot2(ldc(T + gen + 4 * r), v[0], ldc(T + gen + 4 * r + 1), v[1]);
              gsum = cdot2(C{1, 0}, gsum, ldc(T + gen + 4 * r + 2), v[2]);
              gsum = cdot2(C{1, 0}, gsum, ldc(T + gen + 4 * r + 3), v[3]);
              acc += im_conj_mul(w[r], gsum);
            }
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            C q = cdot2(U[4 * r], w[0], U[4 * r + 1], w[1]);
            q = cdot2(C{1, 0}, q, U[4 * r + 2], w[2]);
            q = cdot2(C{1, 0}, q, U[4 * r + 3], w[3]);
            sl[idx[r]] = q;
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          C o = cdot2(U[4 * r], v[0], U[4 * r + 1], v[1]);
          o = cdot2(C{1, 0}, o, U[4 * r + 2], v[2]);
          o = cdot2(C{1, 0}, o, U[4 * r + 3], v[3]);
          sp[idx[r]] = o;
        }
      }
    } else if (on && type == OP_DIAG) {
      const int first = ld(&O->first), count = ld(&O->count);
      if (active) {
        C v[RA], w[RA];
#pragma unroll
        for (int k = 0; k < RA; ++k) {
          const int j = tid + k * NT;
          if (j < nloc) { v[k] = sp[j]; if (ADJ) w[k] = sl[j]; }
        }
#pragma unroll
        for (int k = 0; k < RA; ++k) {
          const int j = tid + k * NT;
          if (j >= nloc) continue;
          const uint64_t x = xk[k];
          C ph = C{1, 0};
          int sign = 0;
          double gw = 0.0;
          for (int e = 0; e < count; ++e) {
            const DiagEntry* d = A.diag + first + e;
            const uint64_t cm = ld(&d->cmask);
            if (ld(&d->kind) == DIAG_SIGN) {
              sign ^= (int)((x & cm) == cm);
            } else if ((x & cm) == cm) {
              const int q1 = ld(&d->q1);
              const int idx = (int)((x >> ld(&d->q0)) & 1) | (q1 >= 0 ? (int)((x >> q1) & 1) << 1 : 0);
              ph = cmul(ph, ldc(T + ld(&d->mat) + idx));
              if (ADJ) {
                const int dg = ld(&d->gen);
                if (dg >= 0) gw += (double)ldc(T + dg + idx).x;
              }
            }
          }
          if (sign) { ph.x = -ph.x; ph.y = -ph.y; }
          sp[j] = cmul(v[k], ph);
          if (ADJ) {
            acc += gw * im_conj_mul(w[k], v[k]);
            sl[j] = cmul(w[k], ph);
          }
        }
      }
    } else if (on && type == OP_ZZ) {
      const int first = ld(&O->first), count = ld(&O->count), mat = ld(&O->mat), gen = ld(&O->gen);
      if (active) {
        const ZZEdge* ed = A.edges + first;
        C v[RA], w[RA];
#pragma unroll
        for (int k = 0; k < RA; ++k) {
          const int j = tid + k * NT;
          if (j < nloc) { v[k] = sp[j]; if (ADJ) w[k] = sl[j]; }
        }
        int cnt[RA];
#pragma unroll
        for (int k = 0; k < RA; ++k) cnt[k] = 0;
        for (int e = 0; e < count; ++e) {
          const int u = ld(&ed[e].u), vv = ld(&ed[e].v);
#pragma unroll
          for (int k = 0; k < RA; ++k) cnt[k] += (int)(((xk[k] >> u) ^ (xk[k] >> vv)) & 1);
        }
#pragma unroll
        for (int k = 0; k < RA; ++k) {
          const int j = tid + k * NT;
          if (j >= nloc) continue;
          const C ph = ldc(T + mat + cnt[k]);
          sp[j] = cmul(v[k], ph);
          if (ADJ) {
            if (gen >= 0) acc += (double)ldc(T + gen + cnt[k]).x * im_conj_mul(w[k], v[k]);
            sl[j] = cmul(w[k], ph);
          }
        }
      }
    }
    if (ADJ && ld(&O->flush)) {
      const double v = wave_sum(acc);
      if ((tid & 63) == 0) red[tid >> 6] = v;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < NT / 64; ++w) s += red[w];
        A.partials[((int64_t)b * A.n_pslots + ld(&O->pslot)) * (int64_t)gridDim.x + (int64_t)tile] = s;
      }
      acc = 0.0;
    }
    __syncthreads();
  }

  if (active) {
#pragma unroll
    for (int k = 0; k < RA; ++k) {
      const int j = tid + k * NT;
      if (j < nloc) {
        psi[xk[k]] = sp[j];
        if (ADJ) lam[xk[k]] = sl[j];
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Register-blocked tile pass.  Each of the 2^(m-RB) threads keeps 2^RB amplitudes of the
// tile in registers.  The local bits in the current register mask are "register bits":
// a gate on them is pure VALU work inside one thread.  A REMAP op changes which local bits
// are register bits by one write and one read of the tile through LDS (XOR-swizzled so
// every access pattern spreads over the banks).  Gates on other bits are never issued:
// the planner groups each pass's gates into register rounds.
// ------------------------------------------------------------------------------------------
template <int S>  // S = log2(amplitudes per 128-byte LDS row)
__device__ __forceinline__ int swz(int j) {
  int f = 0;
#pragma unroll
  for (int sh = S; sh < 16; sh += S) f ^= j >> sh;
  return j ^ (f & ((1 << S) - 1));
}

// dst <- src in the lanes set in the wave-uniform lane mask, written in place (a select
// whose result the compiler could put in a new register would make it carry the register
// block in two register sets).
__device__ __forceinline__ void sel_in32(uint32_t& d, uint32_t src, uint64_t lanes) {
  asm("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(d) : "v"(src), "s"(lanes));
}
__device__ __forceinline__ void sel_in(float2& d, float2 s, uint64_t lanes) {
  uint32_t x = __float_as_uint(d.x), y = __float_as_uint(d.y);
  sel_in32(x, __float_as_uint(s.x), lanes);
  sel_in32(y, __float_as_uint(s.y), lanes);
  d.x = __uint_as_float(x);
  d.y = __uint_as_float(y);
}
__device__ __forceinline__ void sel_in(double2& d, double2 s, uint64_t lanes) {
  const uint64_t a = (uint64_t)__double_as_longlong(d.x), b = (uint64_t)__double_as_longlong(d.y);
  const uint64_t e = (uint64_t)__double_as_longlong(s.x), f = (uint64_t)__double_as_longlong(s.y);
  uint32_t w[4] = {(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
  sel_in32(w[0], (uint32_t)e, lanes);
  sel_in32(w[1], (uint32_t)(e >> 32), lanes);
  sel_in32(w[2], (uint32_t)f, lanes);
  sel_in32(w[3], (uint32_t)(f >> 32), lanes);
  d.x = __longlong_as_double((long long)((uint64_t)w[1] << 32 | w[0]));
  d.y = __longlong_as_double((long long)((uint64_t)w[3] << 32 | w[2]));
}

template <typename C> __device__ __forceinline__ C csel(bool c, C a, C b) {
  C r;
  r.x = c ? a.x : b.x;
  r.y = c ? a.y : b.y;
  return r;
}

// Cross-lane transposition of a register slot bit and lane bit L (4 or 5) of the wave.  X
// and Y are the two slots that differ in the slot bit.  Afterwards X holds the amplitudes
// whose old lane bit L was 0 and Y those whose old lane bit L was 1, each at the lane whose
// bit L equals their old slot bit:
//   X' = c ? Y(lane ^ 2^L) : X,   Y' = c ? Y : X(lane ^ 2^L)   (c = the lane's bit L),
// which is what gfx950's row swap (bit 4: odd 16-lane rows of the first operand with even
// rows of the second) and half-wave swap (bit 5) do, in place, one 32-bit word each.
template <int L>
__device__ __forceinline__ void xlane32(uint32_t& x, uint32_t& y) {
  static_assert(L == 4 || L == 5, "cross-lane transpositions use lane bits 4 and 5");
  if constexpr (L == 5) {
    const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  }
}
template <int L>
__device__ __forceinline__ void xlane(float2& X, float2& Y) {
  uint32_t x0 = __float_as_uint(X.x), x1 = __float_as_uint(X.y), y0 = __float_as_uint(Y.x), y1 = __float_as_uint(Y.y);
  xlane32<L>(x0, y0);
  xlane32<L>(x1, y1);
  X.x = __uint_as_float(x0); X.y = __uint_as_float(x1);
  Y.x = __uint_as_float(y0); Y.y = __uint_as_float(y1);
}
template <int L>
__device__ __forceinline__ void xlane(double2& X, double2& Y) {
  const uint64_t a = (uint64_t)__double_as_longlong(X.x), b = (uint64_t)__double_as_longlong(X.y);
  const uint64_t e = (uint64_t)__double_as_longlong(Y.x), f = (uint64_t)__double_as_longlong(Y.y);
  uint32_t x[4] = {(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
  uint32_t y[4] = {(uint32_t)e, (uint32_t)(e >> 32), (uint32_t)f, (uint32_t)(f >> 32)};
#pragma unroll
  for (int d = 0; d < 4; ++d) xlane32<L>(x[d], y[d]);
  X.x = __longlong_as_double((long long)((uint64_t)x[1] << 32 | x[0]));
  X.y = __longlong_as_double((long long)((uint64_t)x[3] << 32 | x[2]));
  Y.x = __longlong_as_double((long long)((uint64_t)y[1] << 32 | y[0]));
  Y.y = __longlong_as_double((long long)((uint64_t)y[3] << 32 | y[2]));
}
template <int I, int L, int NR, typename C>
__device__ __forceinline__ void xswap1(C* v) {
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (k & (1 << I)) continue;
    xlane<L>(v[k], v[k | (1 << I)]);
  }
}
// code = slot bit | lane bit << 4 (lane bit 4 or 5)
template <int RB, typename C>
__device__ __forceinline__ void xswap_dispatch(int code, C* v) {
  constexpr int NR = 1 << RB;
  switch (code) {
    case 0 | 4 << 4: xswap1<0, 4, NR>(v); break;
    case 0 | 5 << 4: xswap1<0, 5, NR>(v); break;
    case 1 | 4 << 4: xswap1<1, 4, NR>(v); break;
    case 1 | 5 << 4: xswap1<1, 5, NR>(v); break;
    case 2 | 4 << 4: xswap1<2, 4, NR>(v); break;
    case 2 | 5 << 4: xswap1<2, 5, NR>(v); break;
    default:
      if constexpr (RB > 3) {
        if (code == (3 | 4 << 4)) xswap1<(RB > 3 ? 3 : 0), 4, NR>(v);
        else if (code == (3 | 5 << 4)) xswap1<(RB > 3 ? 3 : 0), 5, NR>(v);
      }
      break;
  }
}

// The local bits of register slot k in a layout whose slot bit i is local bit
// (reg >> 8i) & 255 (wave-uniform).
template <int NR>
__device__ __forceinline__ int spread_of(uint32_t reg, int k) {
  int j = 0;
#pragma unroll
  for (int i = 0; (1 << i) < NR; ++i)
    if ((k >> i) & 1) j |= 1 << (int)((reg >> (8 * i)) & 255);
  return j;
}

// 2x2 gate on register bit I.  Gates without local controls (the common case, a
// wave-uniform test) run straight-line; controlled ones compute every pair and keep the
// old values by select where a control bit is 0, so no lane-divergent branch is formed.
// Re(conj(w) * g) in fp64
template <typename C> __device__ __forceinline__ double re_conj_mul(C w, C g) {
  return (double)w.x * (double)g.x + (double)w.y * (double)g.y;
}
// The adjoint gradient term of a slot pair, Im<w|G|v> over (k, k1): a general 2x2 G, or
// k X / k Y without the multiplications by their zeros (k applied by the caller).
template <int GK, typename C>
__device__ __forceinline__ double grad_term(C w0, C w1, C v0, C v1, const C* G) {
  if constexpr (GK == GEN_X) return im_conj_mul(w0, v1) + im_conj_mul(w1, v0);
  else if constexpr (GK == GEN_Y) return re_conj_mul(w1, v0) - re_conj_mul(w0, v1);
  else return im_conj_mul(w0, cdot2(G[0], v0, G[1], v1)) + im_conj_mul(w1, cdot2(G[2], v0, G[3], v1));
}

template <int I, int NR, bool ADJ, int GK, typename C, int F = FORM_GENERAL>
__device__ __forceinline__ void reg1(C* v, C* w, int jt, uint32_t reg, uint32_t lm, const C* U, bool grad,
                                     const C* G, double& acc) {
  if constexpr (F == FORM_SPLIT) {  // forward, uncontrolled
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (k & (1 << I)) continue;
      apply2split(U[0], U[1], U[2], v[k], v[k | (1 << I)]);
    }
    return;
  }
  if (lm == 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (k & (1 << I)) continue;
      const int k1 = k | (1 << I);
      if (ADJ) {
        double g = 0.0;
        if (grad) g = grad_term<GK>(w[k], w[k1], v[k], v[k1], G);
        apply2f<F>(U, w[k], w[k1], g);
        apply2f<F>(U, v[k], v[k1], g);
        acc += g;
      } else {
        apply2f<F>(U, v[k], v[k1]);
      }
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (k & (1 << I)) continue;
    const int k1 = k | (1 << I);
    const bool ok = ((uint32_t)(jt | spread_of<NR>(reg, k)) & lm) == lm;
    C n0 = v[k], n1 = v[k1];
    if (ADJ) {
      C m0 = w[k], m1 = w[k1];
      double g = 0.0;
      if (grad) g = grad_term<GK>(m0, m1, n0, n1, G);
      apply2(U[0], U[1], U[2], U[3], m0, m1, g);
      acc += ok ? g : 0.0;
      const uint64_t okm = __builtin_amdgcn_ballot_w64(ok);
      sel_in(w[k], m0, okm);
      sel_in(w[k1], m1, okm);
    }
    apply2(U[0], U[1], U[2], U[3], n0, n1);
    const uint64_t okv = __builtin_amdgcn_ballot_w64(ok);
    sel_in(v[k], n0, okv);
    sel_in(v[k1], n1, okv);
  }
}

template <typename C>
__device__ __forceinline__ void mat4(const C* M, const C* x, C* y) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    C o = cdot2(M[4 * r], x[0], M[4 * r + 1], x[1]);
    y[r] = cdot2(C{1, 0}, o, M[4 * r + 2], x[2]);
    y[r] = cdot2(C{1, 0}, y[r], M[4 * r + 3], x[3]);
  }
}

template <int RB, bool ADJ, int GK, typename C, int F = FORM_GENERAL>
__device__ __forceinline__ void reg1_slot(int i, C* v, C* w, int jt, uint32_t reg, uint32_t lm, const C* U,
                                          bool grad, const C* G, double& acc) {
  constexpr int NR = 1 << RB;
  switch (i) {
    case 0: reg1<0, NR, ADJ, GK, C, F>(v, w, jt, reg, lm, U, grad, G, acc); break;
    case 1: reg1<1, NR, ADJ, GK, C, F>(v, w, jt, reg, lm, U, grad, G, acc); break;
    case 2: reg1<2, NR, ADJ, GK, C, F>(v, w, jt, reg, lm, U, grad, G, acc); break;
    default:
      if constexpr (RB > 3) reg1<(RB > 3 ? 3 : 0), NR, ADJ, GK, C, F>(v, w, jt, reg, lm, U, grad, G, acc);
      break;
  }
}
// Forward passes and gradient-free adjoint gates use the general form (its gradient
// code is not reached); gradient-bearing adjoint gates with an X or Y generator get the
// shorter gradient term, scaled by k once per op.
template <int RB, bool ADJ, typename C>
__device__ __forceinline__ void reg1_dispatch(int i, C* v, C* w, int jt, uint32_t reg, uint32_t lm, const C* U,
                                              bool grad, int gkind, const C* G, double& acc) {
  if (ADJ && grad && gkind != GEN_GENERAL) {
    const double kf = gkind == GEN_X ? (double)G[1].x : (double)G[2].y;
    double part = 0.0;
    if (gkind == GEN_X) reg1_slot<RB, ADJ, GEN_X>(i, v, w, jt, reg, lm, U, true, G, part);
    else reg1_slot<RB, ADJ, GEN_Y>(i, v, w, jt, reg, lm, U, true, G, part);
    acc = __builtin_fma(kf, part, acc);
    return;
  }
  reg1_slot<RB, ADJ, GEN_GENERAL>(i, v, w, jt, reg, lm, U, grad, G, acc);
}

// Fused 8x8 block on (lane bit 4, lane bit 5, slot bit I) with the matrix cores.  A lane
// holds, for each pair of slots (k0, k1 = k0 | 2^I), the block components
// (re k0, im k0, re k1, im k1): real rows q + 4i of the 16-row real vector, q = its lane
// bits 4-5, i = 0..3; its lane bits 0-3 select one of 16 columns.  Four 16x16x4 products
// (k-chunk i = component i) give the 16x16 result, whose accumulator layout the planner's
// row order already matches, so every component returns to the register it came from.
typedef float qsv_f4 __attribute__((ext_vector_type(4)));
typedef double qsv_d4 __attribute__((ext_vector_type(4)));
template <int I, int NR>
__device__ __forceinline__ void block16(float2* v, const float* a) {
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (k & (1 << I)) continue;
    const int k1 = k | (1 << I);
    qsv_f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], v[k].x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], v[k].y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], v[k1].x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], v[k1].y, acc, 0, 0, 0);
    v[k].x = acc[0];
    v[k].y = acc[1];
    v[k1].x = acc[2];
    v[k1].y = acc[3];
  }
}
template <int I, int NR>
__device__ __forceinline__ void block16(double2* v, const double* a) {
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    if (k & (1 << I)) continue;
    const int k1 = k | (1 << I);
    qsv_d4 acc = {0.0, 0.0, 0.0, 0.0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], v[k].x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], v[k].y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], v[k1].x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], v[k1].y, acc, 0, 0, 0);
    v[k].x = acc[0];
    v[k].y = acc[1];
    v[k1].x = acc[2];
    v[k1].y = acc[3];
  }
}
template <int RB, typename C, typename R>
__device__ __forceinline__ void block_dispatch(int slot, C* v, const R* a) {
  constexpr int NR = 1 << RB;
  switch (slot) {
    case 0: block16<0, NR>(v, a); break;
    case 1: block16<1, NR>(v, a); break;
    case 2: block16<2, NR>(v, a); break;
    default:
      if constexpr (RB > 3) block16<(RB > 3 ? 3 : 0), NR>(v, a);
      break;
  }
}

__device__ __forceinline__ int insert_zero(int t, int p) { return ((t >> p) << (p + 1)) | (t & ((1 << p) - 1)); }

// Dynamic LDS of the register-blocked passes, sized per launch: the ctab window, then
// (adjoint) the deferred gradient sums.
extern __shared__ __align__(16) unsigned char qsv_dyn_lds[];
template <typename R> __host__ __device__ constexpr size_t win_bytes(int win_n) {
  return ((size_t)(win_n > 0 ? win_n : 0) * 2 * sizeof(R) + 15) & ~(size_t)15;
}
// Enough for every workgroup of a launch whose items have at most win_n window entries and
// pslots gradient slots: an item defers its sums only when pslots x waves fits the cap.
template <typename R> static size_t rb_dyn_lds(int maxm, bool adj, int win_n, int pslots) {
  const int nw = (1 << (maxm - 3)) >= 64 ? (1 << (maxm - 3)) / 64 : 1;
  const int sums = adj ? std::min(pslots * nw, kMaxDeferredSums) : 0;
  return win_bytes<R>(win_n) + (size_t)(sums > 0 ? sums : 0) * sizeof(double);
}

// ZZ edge classes of a register block of RB bits: the register-bit masks with at most two
// bits set, in increasing order (the planner packs class sizes in this order).
template <int RB> __host__ __device__ constexpr int zz_classes() { return RB == 3 ? 7 : 11; }
template <int RB> __host__ __device__ constexpr int zz_class(int i) {
  return RB == 3 ? i : (i < 7 ? i : (i == 7 ? 8 : (i == 8 ? 9 : (i == 9 ? 10 : 12))));
}

// Sign-only diagonal entries in a register-blocked pass: bit k of the result is the
// parity of the entries satisfied by register slot k, from the per-entry thread mask and
// slot set (jt = the thread's local index with its register bits zero).
// The three fields are contiguous (16 bytes), so each entry is one scalar load, and four
// entries are requested before the first is used.
struct SignFields {
  uint64_t ocmask;
  uint32_t tmask, kmask;
};
static_assert(offsetof(DiagEntry, tmask) == offsetof(DiagEntry, ocmask) + 8 &&
                  offsetof(DiagEntry, kmask) == offsetof(DiagEntry, ocmask) + 12,
              "sign fields must be contiguous");
__device__ __forceinline__ SignFields sign_fields(const DiagEntry* d) {
  return ld_record(reinterpret_cast<const SignFields*>(&d->ocmask));
}
// Also returns in `touched` (wave-uniform) the slots any entry of the run can flip.
__device__ __forceinline__ uint32_t sign_slots(const DiagEntry* d, int count, uint64_t base, uint32_t jt,
                                               uint32_t& touched) {
  uint32_t sm = 0, any = 0;
  int e = 0;
  for (; e + 4 <= count; e += 4) {
    SignFields f[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) f[i] = sign_fields(d + e + i);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // entries with an outside control that is 0 in this tile do nothing
      const uint32_t km = f[i].kmask & (0u - (uint32_t)((base & f[i].ocmask) == f[i].ocmask));
      any |= km;
      sm ^= (jt & f[i].tmask) == f[i].tmask ? km : 0u;
    }
  }
  for (; e < count; ++e) {
    const SignFields f = sign_fields(d + e);
    const uint32_t km = f.kmask & (0u - (uint32_t)((base & f.ocmask) == f.ocmask));
    any |= km;
    sm ^= (jt & f.tmask) == f.tmask ? km : 0u;
  }
  touched = any;
  return sm;
}

// FULL: the tile fills the workgroup (m == MAXM), so every thread holds amplitudes.
template <typename R, int RB, int MAXM, bool ADJ, bool FULL>
__device__ __forceinline__ void rb_body(const PassArgs& A, const uint64_t tile, const int b) {
  using C = typename CT<R>::T;
  static_assert(RB == 3 || RB == 4, "register blocks of three or four bits");
  constexpr int NT = 1 << (MAXM - RB);
  constexpr int NR = 1 << RB;
  constexpr int S = sizeof(R) == 8 ? 3 : 4;
  __shared__ C buf[1 << MAXM];
  __shared__ double red[NT >= 64 ? NT / 64 : 1];

  const int tid = threadIdx.x;
  const int m = FULL ? MAXM : A.m;  // single-state launches require a full tile
  const int nloc = 1 << m;
  const bool active = FULL || tid < (nloc >> RB);
  const uint64_t TM = A.tile_mask;
  // The tile's base indices from the planner's runs of tile-index bits: logical (bit q is
  // qubit q: controls and phases read it) and the indices the pass reads and writes (they
  // differ from the logical one when passes relayout the state).
  auto run_base = [&](int at) {
    uint64_t r = 0;
    const int nruns = (int)ld(A.dep + at);
    for (int i = 0; i < nruns; ++i) {
      const uint64_t e = ld(A.dep + at + 1 + i);
      const int lo = (int)(e & 255), len = (int)((e >> 8) & 255), sh = (int)((e >> 16) & 255);
      r |= ((tile >> sh) & ((1ull << len) - 1)) << lo;
    }
    return r;
  };
  const uint64_t base = run_base(kRunsLogical);

  C* psi = reinterpret_cast<C*>(A.psi) + (int64_t)b * A.bstride;
  C* out = A.dst ? reinterpret_cast<C*>(A.dst) + (int64_t)b * A.bstride : psi;
  C* lam = ADJ ? reinterpret_cast<C*>(A.lam) + (int64_t)b * A.bstride : nullptr;
  const C* src = A.src ? reinterpret_cast<const C*>(A.src) + (int64_t)b * A.src_bstride : psi;
  const C* T = reinterpret_cast<const C*>(A.ctab) + (int64_t)b * A.ctab_bstride;

  // Local index of register slot k in a layout: thread bit t of the thread id sits at local
  // bit (thr >> 4t) & 15, slot bit i of k at local bit (reg >> 8i) & 255.  A thread keeps
  // only its own part jt (slot 0); the slot parts are wave-uniform.
  const int nthr = m - RB;  // thread bits in use
  auto layout = [&](uint64_t thr) {
    // an opaque copy of the thread id, so the per-bit terms are not hoisted out of the op
    // loop and kept live in registers for the whole pass
    int tv = tid;
    asm volatile("" : "+v"(tv));
    int j = 0;
#pragma unroll
    for (int t = 0; t < MAXM - RB; ++t)
      if (t < nthr) j |= ((tv >> t) & 1) << (int)((thr >> (4 * t)) & 15);
    return j;
  };
  // LDS byte address of register slot k.  swz is linear over GF(2) and slot k's local index is
  // the thread part (slot 0) with the bits of k spread over the register bits, so the address
  // is a per-thread term, swz(thread part), XOR a wave-uniform term, swz(spread of k): moving
  // a register block through LDS costs one XOR per slot.
  auto slot_offsets = [&](uint32_t reg, int* off) {
    int u[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) u[i] = swz<S>(1 << (int)((reg >> (8 * i)) & 255)) * (int)sizeof(C);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      int o = 0;
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if ((k >> i) & 1) o ^= u[i];
      off[k] = o;
    }
  };
  auto lds_at = [&](int byte_off) -> C& { return *reinterpret_cast<C*>(reinterpret_cast<char*>(buf) + byte_off); };
  // Index a local index is read from: two lookup tables of deposits (local bits 0..6 and
  // 7..13) computed by the planner for the pass; before the stores they are replaced by the
  // tables of the index it is written to when the pass relayouts.
  __shared__ uint64_t dep_lo[128], dep_hi[128];
  for (int i = tid; i < 128; i += NT) {
    dep_lo[i] = A.dep[i];
    dep_hi[i] = A.dep[128 + i];
  }
  // The pass's per-lane table lookups (ZZ phases and generator weights, phase entries) read
  // a copy of their ctab window in dynamic LDS.
  C* win = reinterpret_cast<C*>(qsv_dyn_lds);
  const int win_n = A.win_n;
  // adjoint: per-(slot, wave) gradient sums after the window, reduced at the end of the pass
  constexpr int NW = NT >= 64 ? NT / 64 : 1;
  const bool defer = ADJ && A.pass_pslots * NW <= kMaxDeferredSums;
  double* gsum = reinterpret_cast<double*>(qsv_dyn_lds + win_bytes<R>(win_n));
  const int64_t win_lo = A.win_lo;
  for (int i = tid; i < win_n; i += NT) win[i] = T[win_lo + i];
  __syncthreads();
  auto tab = [&](int off) -> C { return win_n ? win[off - win_lo] : ldc(T + off); };

  int jt = layout(A.lay0_thr);                         // the thread's part of its local indices
  uint32_t reg_cur = A.lay0_reg;                       // register bits of the current layout
  int sw_cur = swz<S>(jt) * (int)sizeof(C);            // per-thread term of its LDS addresses
  auto globals = [&](uint64_t tile_base, uint64_t* xo) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int j = jt | spread_of<NR>(reg_cur, k);
      xo[k] = tile_base | dep_lo[j & 127] | dep_hi[j >> 7];
    }
  };

  C v[NR], w[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    v[k] = C{0, 0};
    if (ADJ) w[k] = C{0, 0};
  }
  if (active) {
    uint64_t xk[NR];
    globals(A.relayout ? run_base(kRunsLoad) : base, xk);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      v[k] = src[xk[k]];
      if (ADJ) w[k] = lam[xk[k]];
    }
  }
  // bit q of the global index of local index j
  auto gbit = [&](int j, int l, int q) -> int { return l >= 0 ? (j >> l) & 1 : (int)((base >> q) & 1); };

  double acc = 0.0;
  const TileOp* O = A.ops;
  for (int oi = 0; oi < A.n_ops; ++oi, ++O) {
    // the record's first 16 bytes (adjoint: 32 bytes) in one scalar load
    const uint64_t* hw = reinterpret_cast<const uint64_t*>(O);
    const uint64_t h0 = ld(hw), h1 = ld(hw + 1), h2 = ADJ ? ld(hw + 2) : 0, h3 = ADJ ? ld(hw + 3) : 0;
    const int plain = (int)(uint32_t)h0, mat = (int)(h0 >> 32);
    const int first = (int)(uint32_t)h1, count = (int)(h1 >> 32);
    const int gen = (int)(uint32_t)h2, pslot = (int)(h2 >> 32);
    const int flush = (int)(uint32_t)h3, gkind = (int)(h3 >> 32);
    if (plain) {
      // the short path: a run of sign flips, then a one-qubit gate on a register slot or a
      // fused block (or nothing), with nothing else to decode
      const int slot = (plain & 7) - 1;
      auto sign_run = [&]() {
        uint32_t touched;
        const uint32_t sm = sign_slots(A.diag + first, count, base, (uint32_t)jt, touched);
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          if (!((touched >> k) & 1u)) continue;
          const uint32_t f = (sm << (31 - k)) & 0x80000000u;
          flip_sign(v[k], f);
          if (ADJ) flip_sign(w[k], f);
        }
      };
      if (!ADJ && (plain & kPlainBlock)) {
        if (active) {
          if (plain & kPlainSigns) sign_run();
          // the lane's four A operands: 4 consecutive reals at 4 * lane of the block's table
          const R* ap = reinterpret_cast<const R*>(T + mat) + 4 * (tid & 63);
          R am[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) am[j] = ap[j];
          block_dispatch<RB>(slot, v, am);
        }
      } else if (slot < 0) {
        if (active) sign_run();
      } else if (active) {
        C U[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) U[r] = ldc(T + mat + r);
        if (plain & kPlainSigns) sign_run();
        const int form = (plain & kPlainForm) / kPlainSplit;
        if (ADJ && gen >= 0) {
          C G[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) G[r] = ldc(T + gen + r);
          // the generator forms of RX and RY come with their gates' matrix forms
          if (gkind == GEN_X && form == FORM_XLIKE) {
            double part = 0.0;
            reg1_slot<RB, ADJ, GEN_X, C, FORM_XLIKE>(slot, v, w, jt, reg_cur, 0u, U, true, G, part);
            acc = __builtin_fma((double)G[1].x, part, acc);
          } else if (gkind == GEN_Y && form == FORM_REAL) {
            double part = 0.0;
            reg1_slot<RB, ADJ, GEN_Y, C, FORM_REAL>(slot, v, w, jt, reg_cur, 0u, U, true, G, part);
            acc = __builtin_fma((double)G[2].y, part, acc);
          } else {
            reg1_dispatch<RB, ADJ>(slot, v, w, jt, reg_cur, 0u, U, true, gkind, G, acc);
          }
        } else if (!ADJ && form == FORM_SPLIT) {
          reg1_slot<RB, ADJ, GEN_GENERAL, C, FORM_SPLIT>(slot, v, w, jt, reg_cur, 0u, U, false, U, acc);
        } else if (form == FORM_REAL) {
          reg1_slot<RB, ADJ, GEN_GENERAL, C, FORM_REAL>(slot, v, w, jt, reg_cur, 0u, U, false, U, acc);
        } else if (form == FORM_XLIKE) {
          reg1_slot<RB, ADJ, GEN_GENERAL, C, FORM_XLIKE>(slot, v, w, jt, reg_cur, 0u, U, false, U, acc);
        } else {
          reg1_slot<RB, ADJ, GEN_GENERAL>(slot, v, w, jt, reg_cur, 0u, U, false, U, acc);
        }
      }
    } else {
      const int type = ld(&O->type);
      const uint32_t lm_raw = ld(&O->lmask);
      bool on = true;
      if (lm_raw & kHasOutsideControls) {
        const uint64_t omask = ld(&O->omask);
        on = (base & omask) == omask;
      }
      const uint32_t lmask = lm_raw & ~kHasOutsideControls;
      // sign flips only (Z, CZ, multi-controlled Z), alone (DIAG with b = 0) or ahead of a
      // gate (DENSE1 with b = 1): the parity of the satisfied entries, as one bit per
      // register slot (slot 0 holds the thread's own local index)
      const int ob = ld(&O->b);
      if (on && active && ((type == OP_DIAG && !ob) || (type == OP_DENSE1 && ob))) {
        uint32_t touched;
        const uint32_t sm = sign_slots(A.diag + first, count, base, (uint32_t)jt, touched);
        // slots no entry can reach are skipped (a wave-uniform test): an entry on a register
        // bit reaches half of them
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          if (!((touched >> k) & 1u)) continue;
          const uint32_t f = (sm << (31 - k)) & 0x80000000u;
          flip_sign(v[k], f);
          if (ADJ) flip_sign(w[k], f);
        }
      }
      if (type == OP_REMAP || type == OP_XSWAP) {
        // the new layout: register slot bits, thread bits, the thread's part of its indices
        const uint32_t lr = (uint32_t)ld(&O->b);
        const int jn = layout(ld(&O->omask));
        const int sw_new = swz<S>(jn) * (int)sizeof(C);
        if (type == OP_XSWAP) {
          // one transposition per op, by cross-lane moves; every lane takes part (partners
          // of active lanes are active)
          const int code = mat & 255;
          xswap_dispatch<RB>(code, v);
          if (ADJ) xswap_dispatch<RB>(code, w);
        } else {
          int uo[NR], un[NR];
          slot_offsets(reg_cur, uo);
          slot_offsets(lr, un);
          if (active) {
#pragma unroll
            for (int k = 0; k < NR; ++k) lds_at(sw_cur ^ uo[k]) = v[k];
          }
          __syncthreads();
          if (active) {
#pragma unroll
            for (int k = 0; k < NR; ++k) v[k] = lds_at(sw_new ^ un[k]);
          }
          if (ADJ) {
            __syncthreads();
            if (active) {
#pragma unroll
              for (int k = 0; k < NR; ++k) lds_at(sw_cur ^ uo[k]) = w[k];
            }
            __syncthreads();
            if (active) {
#pragma unroll
              for (int k = 0; k < NR; ++k) w[k] = lds_at(sw_new ^ un[k]);
            }
          }
          __syncthreads();
        }
        jt = jn;
        reg_cur = lr;
        sw_cur = sw_new;
      } else if (on && active && type == OP_DENSE1) {
        C U[4], G[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) U[r] = ldc(T + mat + r);
        const bool grad = ADJ && gen >= 0;
        if (grad) {
#pragma unroll
          for (int r = 0; r < 4; ++r) G[r] = ldc(T + gen + r);
        }
        reg1_dispatch<RB, ADJ>(ld(&O->a), v, w, jt, reg_cur, lmask, U, grad, ADJ ? gkind : 0, G, acc);
      } else if (on && type == OP_DENSE2) {
        // two-qubit dense gate on local bits a, b, applied to the tile staged in LDS (no
        // gradient: parameterized two-qubit rotations are lowered to RZZ with basis changes)
        const int a = ld(&O->a), bb = ld(&O->b);
        const int lo = a < bb ? a : bb, hi = a < bb ? bb : a;
        const uint32_t lm = lmask;
        int uo[NR];
        slot_offsets(reg_cur, uo);
        auto apply_staged = [&](C (&reg)[NR]) {
          if (active) {
#pragma unroll
            for (int k = 0; k < NR; ++k) lds_at(sw_cur ^ uo[k]) = reg[k];
          }
          __syncthreads();
          for (int p = tid; p < (nloc >> 2); p += NT) {
            const int t = insert_zero(insert_zero(p, lo), hi);
            if (((uint32_t)t & lm) != lm) continue;
            const int idx[4] = {t, t | (1 << a), t | (1 << bb), t | (1 << a) | (1 << bb)};
            C x[4], y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = buf[swz<S>(idx[r])];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              y[r] = cdot2(ldc(T + mat + 4 * r), x[0], ldc(T + mat + 4 * r + 1), x[1]);
              y[r] = cdot2(C{1, 0}, y[r], ldc(T + mat + 4 * r + 2), x[2]);
              y[r] = cdot2(C{1, 0}, y[r], ldc(T + mat + 4 * r + 3), x[3]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) buf[swz<S>(idx[r])] = y[r];
          }
          __syncthreads();
          if (active) {
#pragma unroll
            for (int k = 0; k < NR; ++k) reg[k] = lds_at(sw_cur ^ uo[k]);
          }
          __syncthreads();
        };
        apply_staged(v);
        if (ADJ) apply_staged(w);
      } else if (on && active && type == OP_DIAG && ob) {
        // Slots two at a time, each pair walking the run's entries (scalar loads, cached):
        // phases and generator weights for every slot at once would hold another register
        // block and cut the number of resident waves.
#pragma unroll
        for (int k0 = 0; k0 < NR; k0 += 2) {
          C ph[2] = {C{1, 0}, C{1, 0}};
          double gw[2] = {0.0, 0.0};
          uint32_t sm = 0;
          for (int e = 0; e < count; ++e) {
            const DiagEntry* d = A.diag + first + e;
            const uint64_t ocm = ld(&d->ocmask);
            if ((base & ocm) != ocm) continue;  // an outside control is 0 in this tile
            const uint32_t lcm = ld(&d->lcmask);
            if (ld(&d->kind) == DIAG_SIGN) {
              const uint32_t tm = ld(&d->tmask);
              if (((uint32_t)jt & tm) == tm) sm ^= ld(&d->kmask);
            } else {
              const int l0 = ld(&d->l0), l1 = ld(&d->l1), q0 = ld(&d->q0), q1 = ld(&d->q1);
              const int mat = ld(&d->mat);
              const int dg = ADJ ? ld(&d->gen) : -1;
#pragma unroll
              for (int h = 0; h < 2; ++h) {
                const int j = jt | spread_of<NR>(reg_cur, k0 + h);
                if (((uint32_t)j & lcm) != lcm) continue;
                const int idx = gbit(j, l0, q0) | (q1 >= 0 ? gbit(j, l1, q1) << 1 : 0);
                ph[h] = cmul(ph[h], tab(mat + idx));
                if (ADJ && dg >= 0) gw[h] += (double)tab(dg + idx).x;
              }
            }
          }
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int k = k0 + h;
            C p = ph[h];
            flip_sign(p, (sm << (31 - k)) & 0x80000000u);
            if (ADJ) {
              double g = gw[h] * im_conj_mul(w[k], v[k]);
              cmul_in(w[k], p, g);
              cmul_in(v[k], p, g);
              acc += g;
            } else {
              cmul_in(v[k], p);
            }
          }
        }
      } else if (on && active && type == OP_ZZ) {
        // c(x) = number of edges whose endpoints differ.  Edges come grouped by register
        // class c; an edge of class c differs in slot k iff its thread/outside parity
        // differs from the parity of (k & c), so with a_c = the class's edges whose
        // thread/outside parity is odd, c(slot k) = sum_c a_c + sum_{c: k & c odd} (n_c - 2 a_c).
        // classes are register-bit masks of at most two bits, listed by zz_class<RB>(i); the
        // edge count of class i is byte i of (a, b, lmask)
        const uint32_t cw[3] = {(uint32_t)ld(&O->a), (uint32_t)ld(&O->b), lm_raw};
        const ZZEdge* ed = A.edges + first;
        constexpr int NCLS = zz_classes<RB>();
        int sum_a = 0, dcls[NCLS];
        int e = 0;
#pragma unroll
        for (int c = 0; c < NCLS; ++c) {
          const int nc = (int)((cw[c >> 2] >> (8 * (c & 3))) & 255u);
          int a_c = 0;
          for (int i = 0; i < nc; ++i, ++e) {
            const uint32_t tm = ld(&ed[e].tmask);
            const uint64_t om = ld(&ed[e].omask);
            a_c += (__popc(jt & tm) + __popcll(base & om)) & 1;
          }
          sum_a += a_c;
          dcls[c] = nc - 2 * a_c;
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          int cnt = sum_a;
#pragma unroll
          for (int c = 1; c < NCLS; ++c)
            if (__builtin_popcount(k & zz_class<RB>(c)) & 1) cnt += dcls[c];
          const C p = tab(mat + cnt);
          if (ADJ) {
            double g = 0.0;
            if (gen >= 0) g = (double)tab(gen + cnt).x * im_conj_mul(w[k], v[k]);
            cmul_in(w[k], p, g);
            cmul_in(v[k], p, g);
            acc += g;
          } else {
            cmul_in(v[k], p);
          }
        }
      }
    }
    if (ADJ && flush) {
      const double sv = wave_sum(acc);
      if (defer) {
        if ((tid & 63) == 0) gsum[pslot * NW + (tid >> 6)] = sv;
      } else {
        if ((tid & 63) == 0) red[tid >> 6] = sv;
        __syncthreads();
        if (tid == 0) {
          double s = 0.0;
          for (int q = 0; q < NW; ++q) s += red[q];
          A.partials[((int64_t)b * A.n_pslots + pslot) * A.n_tiles + (int64_t)tile] = s;
        }
        __syncthreads();
      }
      acc = 0.0;
    }
  }
  if (defer) {
    __syncthreads();
    for (int q = tid; q < A.pass_pslots; q += NT) {
      double s = 0.0;
      for (int w2 = 0; w2 < NW; ++w2) s += gsum[q * NW + w2];
      A.partials[((int64_t)b * A.n_pslots + q) * A.n_tiles + (int64_t)tile] = s;
    }
  }

  uint64_t store_base = base;
  if (A.relayout) {
    __syncthreads();
    for (int i = tid; i < 128; i += NT) {
      dep_lo[i] = A.dep[256 + i];
      dep_hi[i] = A.dep[384 + i];
    }
    __syncthreads();
    store_base = run_base(kRunsStore);
  }
  if (active) {
    uint64_t xk[NR];
    globals(store_base, xk);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      out[xk[k]] = v[k];
      if (ADJ) lam[xk[k]] = w[k];
    }
  }
}

template <typename R, int RB, int MAXM, bool ADJ>
__global__ __launch_bounds__(1 << (MAXM - RB)) void tile_pass_rb(PassArgs A) {
  // Workgroups go to the 8 XCDs in turn; give each XCD a contiguous range of tiles, so
  // tiles that share cache lines (they differ only in low qubits outside the tile) run
  // back to back behind the same L2.
  const uint32_t g = gridDim.x, w = blockIdx.x;
  const uint64_t t = (g % 8 == 0) ? (uint64_t)(w & 7) * (g >> 3) + (w >> 3) : w;
  rb_body<R, RB, MAXM, ADJ, true>(A, t, blockIdx.y);
}

// Many circuits in one launch: item i owns workgroups [prefix[i], prefix[i+1]); each
// workgroup finds its item by binary search and runs that circuit's pass on one tile.
template <typename R, int RB, int MAXM, bool ADJ>
__global__ __launch_bounds__(1 << (MAXM - RB)) void tile_pass_rb_multi(const PassArgs* items, const uint32_t* prefix,
                                                                       int n_items) {
  const uint32_t w = blockIdx.x;
  int lo = 0, hi = n_items;  // largest i with prefix[i] <= w
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ld(prefix + mid) <= w) lo = mid; else hi = mid;
  }
  const PassArgs A = items[lo];
  rb_body<R, RB, MAXM, ADJ, false>(A, (uint64_t)(w - ld(prefix + lo)), 0);
}

// ------------------------------------------------------------------------------------------
// Unfused per-gate passes (grid-stride over amplitude pairs / quads / amplitudes).
// ------------------------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void gate1_stream(void* psi_, int64_t bstride, int n, int t,
                                                    uint64_t cmask, const void* ctab_,
                                                    int64_t ctab_bstride, int mat) {
  using C = typename CT<R>::T;
  C* psi = reinterpret_cast<C*>(psi_) + (int64_t)blockIdx.y * bstride;
  const C* T = reinterpret_cast<const C*>(ctab_) + (int64_t)blockIdx.y * ctab_bstride + mat;
  const C u00 = T[0], u01 = T[1], u10 = T[2], u11 = T[3];
  const uint64_t half = 1ull << (n - 1);
  const uint64_t lowm = (1ull << t) - 1;
  for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < half; p += (uint64_t)gridDim.x * 256) {
    const uint64_t x0 = ((p >> t) << (t + 1)) | (p & lowm);
    if ((x0 & cmask) != cmask) continue;
    const uint64_t x1 = x0 | (1ull << t);
    const C v0 = psi[x0], v1 = psi[x1];
    psi[x0] = cdot2(u00, v0, u01, v1);
    psi[x1] = cdot2(u10, v0, u11, v1);
  }
}

template <typename R>
__global__ __launch_bounds__(256) void gate2_stream(void* psi_, int64_t bstride, int n, int ta, int tb,
                                                    uint64_t cmask, const void* ctab_,
                                                    int64_t ctab_bstride, int mat) {
  using C = typename CT<R>::T;
  C* psi = reinterpret_cast<C*>(psi_) + (int64_t)blockIdx.y * bstride;
  const C* U = reinterpret_cast<const C*>(ctab_) + (int64_t)blockIdx.y * ctab_bstride + mat;
  const int lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
  const uint64_t quarter = 1ull << (n - 2);
  for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < quarter; p += (uint64_t)gridDim.x * 256) {
    uint64_t x = ((p >> lo) << (lo + 1)) | (p & ((1ull << lo) - 1));
    x = ((x >> hi) << (hi + 1)) | (x & ((1ull << hi) - 1));
    if ((x & cmask) != cmask) continue;
    const uint64_t idx[4] = {x, x | (1ull << ta), x | (1ull << tb), x | (1ull << ta) | (1ull << tb)};
    C v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = psi[idx[r]];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      C o = cdot2(U[4 * r], v[0], U[4 * r + 1], v[1]);
      o = cdot2(C{1, 0}, o, U[4 * r + 2], v[2]);
      o = cdot2(C{1, 0}, o, U[4 * r + 3], v[3]);
      psi[idx[r]] = o;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void diag_stream(void* psi_, int64_t bstride, int n,
                                                   const DiagEntry* diag, int first, int count,
                                                   const void* ctab_, int64_t ctab_bstride) {
  using C = typename CT<R>::T;
  C* psi = reinterpret_cast<C*>(psi_) + (int64_t)blockIdx.y * bstride;
  const C* T = reinterpret_cast<const C*>(ctab_) + (int64_t)blockIdx.y * ctab_bstride;
  const uint64_t N = 1ull << n;
  for (uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x; x < N; x += (uint64_t)gridDim.x * 256) {
    C ph = C{1, 0};
    int sign = 0;
    for (int e = 0; e < count; ++e) {
      const DiagEntry* d = diag + first + e;
      const uint64_t cm = ld(&d->cmask);
      if (ld(&d->kind) == DIAG_SIGN) {
        sign ^= (int)((x & cm) == cm);
      } else if ((x & cm) == cm) {
        const int q1 = ld(&d->q1);
        const int idx = (int)((x >> ld(&d->q0)) & 1) | (q1 >= 0 ? (int)((x >> q1) & 1) << 1 : 0);
        ph = cmul(ph, ldc(T + ld(&d->mat) + idx));
      }
    }
    if (sign) { ph.x = -ph.x; ph.y = -ph.y; }
    psi[x] = cmul(psi[x], ph);
  }
}

// ------------------------------------------------------------------------------------------
// Pauli-sum group pass.
// ------------------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void group_factor(const PauliGroupArgs& A, uint64_t x, double& fr, double& fi) {
  fr = 0.0;
  fi = 0.0;
  for (int k = 0; k < A.n_terms; ++k) {
    const double s = (__popcll(x & ld(A.zmasks + k)) & 1) ? -1.0 : 1.0;
    fr = __builtin_fma(s, ld(A.cre + k), fr);
    fi = __builtin_fma(s, ld(A.cim + k), fi);
  }
}

// One instantiation per way of walking the group (the host picks it from the group's
// shape), so that each path is allocated registers for itself alone.  Pattern modes (0-3):
// bit 0 the term table staged in LDS once per workgroup, bit 1 lambda written.
enum PauliMode { PG_STAGED = 1, PG_LAM = 2, PG_QUAD = 4, PG_DIAG = 5, PG_XMASK = 6 };
constexpr int kPauliStageTerms = 512;

template <typename R, int MODE>
__global__ __launch_bounds__(256) void pauli_group(PauliGroupArgs A) {
  using C = typename CT<R>::T;
  __shared__ double red[2][4];
  const C* psi = reinterpret_cast<const C*>(A.psi) + (int64_t)blockIdx.y * A.bstride;
  C* lam = A.lam ? reinterpret_cast<C*>(A.lam) + (int64_t)blockIdx.y * A.bstride : nullptr;
  const uint64_t N = 1ull << A.n_qubits;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  double er = 0.0, ei = 0.0;
  if constexpr (MODE < PG_QUAD) {
    // Diagonal group with real coefficients, in chunks of 4096 consecutive amplitudes
    // x = hi | i << 8 | t (t the thread, i = 0..15 its slot).  A term's sign splits into a
    // per-chunk part on hi and a part on the 12 low bits, so per chunk the coefficient of
    // each low pattern p is C_p = sum_k c_k (-1)^{popcount(hi & z_k)} over the terms with
    // that pattern; a thread folds its own bits into E_r = sum over patterns with bits 8-11
    // equal to r of C_p (-1)^{popcount(t & p)}, and a 16-point Walsh-Hadamard transform
    // gives f(x) = sum_r E_r (-1)^{popcount(i & r)} for its 16 slots.  Each term costs a few
    // operations per chunk instead of per amplitude, which leaves the pass bound by HBM.
    // With the term table in LDS the per-chunk sums wait only on LDS, so the chunk's
    // amplitude loads, issued first, stay in flight meanwhile.
    __shared__ double cp[kPauliMaxPatterns];
    constexpr bool staged = (MODE & PG_STAGED) != 0, with_lam = (MODE & PG_LAM) != 0;
    const int P = A.n_pats;
    const int tid = threadIdx.x;
    const uint64_t* tz = A.zmasks;
    const double* tc = A.cre;
    if constexpr (staged) {
      __shared__ uint64_t sz[kPauliStageTerms];
      __shared__ double sc[kPauliStageTerms];
      for (int k = tid; k < A.n_terms; k += 256) {
        sz[k] = A.zmasks[k];
        sc[k] = A.cre[k];
      }
      tz = sz;
      tc = sc;
    }
    const uint64_t n_chunks = N >> 12;
    for (uint64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
      const uint64_t hi = ch << 12;
      C v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = psi[hi | (uint64_t)(i << 8) | (uint64_t)tid];
      __syncthreads();  // the previous chunk's readers of cp are done (and the staging)
      for (int p = tid; p < P; p += 256) {
        const int k0 = (int)(A.pats[p] >> 12);
        const int k1 = p + 1 < P ? (int)(A.pats[p + 1] >> 12) : A.n_terms;
        double sr = 0.0;
        for (int k = k0; k < k1; ++k) {
          const bool neg = __popcll(hi & tz[k]) & 1;
          sr += neg ? -tc[k] : tc[k];
        }
        cp[p] = sr;
      }
      __syncthreads();
      double f[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double a = 0.0;
        const int p0 = ld(A.rfirst + r), p1 = ld(A.rfirst + r + 1);
        for (int p = p0; p < p1; ++p) {
          const uint32_t pat = ld(A.pats + p) & 0xFFu;
          const bool neg = __popc((uint32_t)tid & pat) & 1;
          a += neg ? -cp[p] : cp[p];
        }
        f[r] = a;
      }
      // Walsh-Hadamard transform over the 4 slot bits
#pragma unroll
      for (int h = 1; h < 16; h <<= 1) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          if (r & h) continue;
          const double a = f[r], b = f[r | h];
          f[r] = a + b;
          f[r | h] = a - b;
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        er += ((double)v[i].x * v[i].x + (double)v[i].y * v[i].y) * f[i];
        if constexpr (with_lam) {
          const uint64_t x = hi | (uint64_t)(i << 8) | (uint64_t)tid;
          C o;
          o.x = (R)(f[i] * v[i].x);
          o.y = (R)(f[i] * v[i].y);
          if (A.accumulate) { const C l = lam[x]; o.x += l.x; o.y += l.y; }
          lam[x] = o;
        }
      }
    }
  } else if constexpr (MODE == PG_QUAD) {
    // Diagonal group, four consecutive amplitudes per thread: a term's sign parity on the
    // shared high bits is computed once; the two low bits flip it by the uniform pattern
    // pat(z) (bit j set when popcount(j & z) is odd).
    const bool real_c = A.real_coeffs;
    for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; q < (N >> 2); q += stride) {
      const uint64_t x0 = q << 2;
      C v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = psi[x0 + j];
      double fr[4] = {0.0, 0.0, 0.0, 0.0}, fi[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < A.n_terms; ++k) {
        const uint64_t z = ld(A.zmasks + k);
        const double cr = ld(A.cre + k);
        const uint32_t zl = (uint32_t)z & 3u;
        const uint32_t pat = (zl == 0u) ? 0u : (zl == 1u) ? 0xAu : (zl == 2u) ? 0xCu : 0x6u;
        const uint32_t par = (uint32_t)(__popcll(x0 & z) & 1) ? 0xFu : 0u;
        const uint32_t sg = par ^ pat;
#pragma unroll
        for (int j = 0; j < 4; ++j) fr[j] += ((sg >> j) & 1u) ? -cr : cr;
        if (!real_c) {
          const double ci = ld(A.cim + k);
#pragma unroll
          for (int j = 0; j < 4; ++j) fi[j] += ((sg >> j) & 1u) ? -ci : ci;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double pj = (double)v[j].x * v[j].x + (double)v[j].y * v[j].y;
        er += pj * fr[j];
        ei += pj * fi[j];
        if (lam) {
          C o;
          o.x = (R)(fr[j] * v[j].x - fi[j] * v[j].y);
          o.y = (R)(fr[j] * v[j].y + fi[j] * v[j].x);
          if (A.accumulate) { const C l = lam[x0 + j]; o.x += l.x; o.y += l.y; }
          lam[x0 + j] = o;
        }
      }
    }
  } else if constexpr (MODE == PG_DIAG) {
    for (uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x; x < N; x += stride) {
      double fr, fi;
      group_factor<R>(A, x, fr, fi);
      const C v = psi[x];
      const double p = (double)v.x * v.x + (double)v.y * v.y;
      er += p * fr;
      ei += p * fi;
      if (lam) {
        C o;
        o.x = (R)(fr * v.x - fi * v.y);
        o.y = (R)(fr * v.y + fi * v.x);
        if (A.accumulate) { const C l = lam[x]; o.x += l.x; o.y += l.y; }
        lam[x] = o;
      }
    }
  } else {
    static_assert(MODE == PG_XMASK, "unknown Pauli pass mode");
    const int h = 63 - __clzll(A.xmask);
    const uint64_t lowm = (1ull << h) - 1;
    for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < (N >> 1); p += stride) {
      const uint64_t x = ((p >> h) << (h + 1)) | (p & lowm);
      const uint64_t y = x ^ A.xmask;
      const C vx = psi[x], vy = psi[y];
      double fxr, fxi, fyr, fyi;
      group_factor<R>(A, x, fxr, fxi);
      group_factor<R>(A, y, fyr, fyi);
      // (H psi)[y] += f(x) psi[x];  (H psi)[x] += f(y) psi[y]
      const double axr = fxr * vx.x - fxi * vx.y, axi = fxr * vx.y + fxi * vx.x;
      const double ayr = fyr * vy.x - fyi * vy.y, ayi = fyr * vy.y + fyi * vy.x;
      // E += conj(vy) * a_x + conj(vx) * a_y
      er += (double)vy.x * axr + (double)vy.y * axi + (double)vx.x * ayr + (double)vx.y * ayi;
      ei += (double)vy.x * axi - (double)vy.y * axr + (double)vx.x * ayi - (double)vx.y * ayr;
      if (lam) {
        C oy, ox;
        oy.x = (R)axr; oy.y = (R)axi;
        ox.x = (R)ayr; ox.y = (R)ayi;
        if (A.accumulate) {
          const C ly = lam[y], lx = lam[x];
          oy.x += ly.x; oy.y += ly.y; ox.x += lx.x; ox.y += lx.y;
        }
        lam[y] = oy;
        lam[x] = ox;
      }
    }
  }
  er = wave_sum(er);
  ei = wave_sum(ei);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][w] = er; red[1][w] = ei; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t o = ((int64_t)blockIdx.y * A.ncols + A.col) * gridDim.x + blockIdx.x;
    A.partials[o] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    A.partials[o + gridDim.x] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// out[c] = sum_{i < len} in[c * len + i], fixed order.
__global__ __launch_bounds__(256) void reduce_columns(const double* in, int64_t len, double* out) {
  __shared__ double red[4];
  const double* col = in + (int64_t)blockIdx.x * len;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += 256) s += col[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// psi_b = |index> for every batch item.
template <typename R>
__global__ __launch_bounds__(256) void set_basis(void* psi_, int64_t bstride, uint64_t N, uint64_t index) {
  using C = typename CT<R>::T;
  C* psi = reinterpret_cast<C*>(psi_) + (int64_t)blockIdx.y * bstride;
  // each workgroup writes one contiguous range
  const uint64_t per = (N + gridDim.x - 1) / gridDim.x;
  const uint64_t x0 = (uint64_t)blockIdx.x * per, x1 = x0 + per < N ? x0 + per : N;
  for (uint64_t x = x0 + threadIdx.x; x < x1; x += 256) {
    C v;
    v.x = (x == index) ? (R)1 : (R)0;
    v.y = (R)0;
    psi[x] = v;
  }
}

// dst_b = src (broadcast one state into batch items).
template <typename R>
__global__ __launch_bounds__(256) void broadcast_state(void* dst_, int64_t bstride, const void* src_, uint64_t N) {
  using C = typename CT<R>::T;
  C* dst = reinterpret_cast<C*>(dst_) + (int64_t)blockIdx.y * bstride;
  const C* src = reinterpret_cast<const C*>(src_);
  for (uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x; x < N; x += (uint64_t)gridDim.x * 256) dst[x] = src[x];
}

// ------------------------------------------------------------------------------------------
// Multi-circuit Pauli-sum pass in gather form: each thread owns an output index y and sums
// c_k P_k psi over all terms, (P_k psi)[y] = i^{popcount(x_k & z_k)} (-1)^{popcount((y ^ x_k) & z_k)}
// psi[y ^ x_k]; no two threads write the same lambda entry, so one launch covers every
// term.  Workgroup w handles chunk (w - prefix[i]) of job i (CHUNK amplitudes).
// ------------------------------------------------------------------------------------------
template <typename R, int CHUNK>
__global__ __launch_bounds__(256) void pauli_apply_multi(const PauliJob* jobs, const uint32_t* prefix, int n_jobs) {
  using C = typename CT<R>::T;
  __shared__ double red[2][4];
  const uint32_t w = blockIdx.x;
  int lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ld(prefix + mid) <= w) lo = mid; else hi = mid;
  }
  const PauliJob* J = jobs + lo;
  const uint32_t chunk = w - ld(prefix + lo);
  const C* psi = reinterpret_cast<const C*>(ld(&J->psi));
  C* lam = reinterpret_cast<C*>(ld(&J->lam));
  const uint64_t* xm = ld(&J->xmasks);
  const uint64_t* zm = ld(&J->zmasks);
  const double* cre = ld(&J->cre);
  const double* cim = ld(&J->cim);
  const int nt = ld(&J->n_terms);
  const uint64_t N = 1ull << ld(&J->n_qubits);
  double er = 0.0, ei = 0.0;
  for (uint64_t y = (uint64_t)chunk * CHUNK + threadIdx.x; y < N && y < (uint64_t)(chunk + 1) * CHUNK; y += 256) {
    double lr = 0.0, li = 0.0;
    for (int k = 0; k < nt; ++k) {
      const uint64_t x = y ^ ld(xm + k);
      const C v = psi[x];
      const double sgn = (__popcll(x & ld(zm + k)) & 1) ? -1.0 : 1.0;
      const double ar = sgn * ld(cre + k), ai = sgn * ld(cim + k);
      lr += ar * v.x - ai * v.y;
      li += ar * v.y + ai * v.x;
    }
    const C py = psi[y];
    er += (double)py.x * lr + (double)py.y * li;
    ei += (double)py.x * li - (double)py.y * lr;
    C o;
    o.x = (R)lr;
    o.y = (R)li;
    lam[y] = o;
  }
  er = wave_sum(er);
  ei = wave_sum(ei);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = er; red[1][threadIdx.x >> 6] = ei; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* P = ld(&J->partials);
    P[2 * chunk] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    P[2 * chunk + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// out[c] = sum of in[offs[c] + stride[c] * i] for i < lens[c], fixed order.
__global__ __launch_bounds__(256) void reduce_segments(const double* in, const int64_t* offs, const int32_t* lens,
                                                       const int32_t* strides, double* out) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  const int64_t o = ld(offs + c);
  const int32_t len = ld(lens + c), st = ld(strides + c);
  double s = 0.0;
  for (int32_t i = threadIdx.x; i < len; i += 256) s += in[o + (int64_t)st * i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Fill states with |0...0>: job j covers 2^n[j] amplitudes at ptr[j] in CHUNK-sized pieces.
template <typename R>
__global__ __launch_bounds__(256) void set_zero_multi(void* const* ptrs, const int32_t* nq, const uint32_t* prefix,
                                                      int n_jobs) {
  using C = typename CT<R>::T;
  const uint32_t w = blockIdx.x;
  int lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ld(prefix + mid) <= w) lo = mid; else hi = mid;
  }
  C* psi = reinterpret_cast<C*>(ld(ptrs + lo));
  const uint64_t N = 1ull << ld(nq + lo);
  const uint64_t chunk = w - ld(prefix + lo);
  for (uint64_t x = chunk * 4096 + threadIdx.x; x < N && x < (chunk + 1) * 4096; x += 256) {
    C v;
    v.x = x == 0 ? (R)1 : (R)0;
    v.y = (R)0;
    psi[x] = v;
  }
}

// dst = alpha * src (complex alpha), one state.
template <typename R>
__global__ __launch_bounds__(256) void scale_copy(void* dst_, const void* src_, uint64_t N, double ar, double ai) {
  using C = typename CT<R>::T;
  C* dst = reinterpret_cast<C*>(dst_);
  const C* src = reinterpret_cast<const C*>(src_);
  for (uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x; x < N; x += (uint64_t)gridDim.x * 256) {
    const C v = src[x];
    C o;
    o.x = (R)(ar * v.x - ai * v.y);
    o.y = (R)(ar * v.y + ai * v.x);
    dst[x] = o;
  }
}

// partials[blk] = sum conj(a[x]) b[x] (re at 2 blk, im at 2 blk + 1), fp64.
template <typename R>
__global__ __launch_bounds__(256) void inner_product(const void* a_, const void* b_, uint64_t N, double* partials) {
  using C = typename CT<R>::T;
  __shared__ double red[2][4];
  const C* a = reinterpret_cast<const C*>(a_);
  const C* b = reinterpret_cast<const C*>(b_);
  double re = 0.0, im = 0.0;
  for (uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x; x < N; x += (uint64_t)gridDim.x * 256) {
    const C u = a[x], v = b[x];
    re += (double)u.x * v.x + (double)u.y * v.y;
    im += (double)u.x * v.y - (double)u.y * v.x;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = re; red[1][threadIdx.x >> 6] = im; }
  __syncthreads();
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    partials[gridDim.x + blockIdx.x] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// ------------------------------------------------------------------------------------------
// Host launchers.
// ------------------------------------------------------------------------------------------
static inline unsigned stream_blocks(uint64_t work) {
  const uint64_t b = (work + 255) / 256;
  return (unsigned)(b < 4096 ? (b ? b : 1) : 4096);
}

template <typename R, int NT, int MAXM, bool ADJ>
static hipError_t tile_launch_one(const PassArgs& A, dim3 grid, hipStream_t s) {
  constexpr size_t bytes = (size_t)(2 * sizeof(R)) * ((size_t)1 << MAXM) * (ADJ ? 2 : 1);
  if constexpr (bytes <= 131072) {
    tile_pass<R, NT, MAXM, ADJ><<<grid, NT, 0, s>>>(A);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename R, bool ADJ>
static hipError_t tile_dispatch(int maxm, const PassArgs& A, uint64_t n_tiles, int batch, hipStream_t s) {
  const dim3 grid((unsigned)n_tiles, (unsigned)batch);
  switch (maxm) {
    case 8:  return tile_launch_one<R, 256, 8, ADJ>(A, grid, s);
    case 10: return tile_launch_one<R, 512, 10, ADJ>(A, grid, s);
    case 11: return tile_launch_one<R, 512, 11, ADJ>(A, grid, s);
    case 12: return tile_launch_one<R, 512, 12, ADJ>(A, grid, s);
    case 13: return tile_launch_one<R, 1024, 13, ADJ>(A, grid, s);
    case 14: return tile_launch_one<R, 1024, 14, ADJ>(A, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, int RB, int MAXM, bool ADJ>
static hipError_t rb_launch_one(const PassArgs& A, dim3 grid, hipStream_t s) {
  constexpr size_t bytes = (size_t)(2 * sizeof(R)) * ((size_t)1 << MAXM);
  // four register bits: complex64 forward passes only (their registers allow 4 waves/SIMD)
  if constexpr (bytes <= 131072 && (RB == 3 || (!ADJ && sizeof(R) == 4 && MAXM >= 10))) {
    const size_t dyn = rb_dyn_lds<R>(MAXM, ADJ, A.win_n, A.pass_pslots);
    tile_pass_rb<R, RB, MAXM, ADJ><<<grid, 1 << (MAXM - RB), dyn, s>>>(A);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename R, bool ADJ, int RB>
static hipError_t rb_dispatch_rb(int maxm, const PassArgs& A, dim3 grid, hipStream_t s) {
  switch (maxm) {
    case 9:  return rb_launch_one<R, RB, 9, ADJ>(A, grid, s);
    case 10: return rb_launch_one<R, RB, 10, ADJ>(A, grid, s);
    case 11: return rb_launch_one<R, RB, 11, ADJ>(A, grid, s);
    case 12: return rb_launch_one<R, RB, 12, ADJ>(A, grid, s);
    case 13: return rb_launch_one<R, RB, 13, ADJ>(A, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, bool ADJ>
static hipError_t rb_dispatch(int reg_bits, int maxm, const PassArgs& A, uint64_t n_tiles, int batch,
                              hipStream_t s) {
  const dim3 grid((unsigned)n_tiles, (unsigned)batch);
  if (reg_bits == 3) return rb_dispatch_rb<R, ADJ, 3>(maxm, A, grid, s);
  if (reg_bits == 4) return rb_dispatch_rb<R, ADJ, 4>(maxm, A, grid, s);
  return hipErrorInvalidValue;
}

template <typename R, bool ADJ>
static hipError_t rb_multi_dispatch(int maxm, const PassArgs* items, const uint32_t* prefix, int n_items,
                                    uint32_t n_wg, int max_win, int max_pslots, hipStream_t s) {
  const size_t dyn = rb_dyn_lds<R>(maxm, ADJ, max_win, max_pslots);
  switch (maxm) {
#define QSV_MULTI(M)                                                                                   \
  case M:                                                                                              \
    if constexpr ((size_t)(2 * sizeof(R)) * ((size_t)1 << M) <= 131072) {                              \
      tile_pass_rb_multi<R, 3, M, ADJ><<<n_wg, 1 << (M - 3), dyn, s>>>(items, prefix, n_items);        \
      return hipGetLastError();                                                                        \
    }                                                                                                  \
    return hipErrorInvalidValue;
    QSV_MULTI(9) QSV_MULTI(10) QSV_MULTI(11) QSV_MULTI(12) QSV_MULTI(13)
#undef QSV_MULTI
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tile_pass_rb_multi(int dtype, bool adj, int maxm, const PassArgs* items, const uint32_t* prefix,
                                     int n_items, uint32_t n_wg, int max_win, int max_pslots, hipStream_t s) {
  if (max_win > kMaxWindow) return hipErrorInvalidValue;
  if (dtype == 0)
    return adj ? rb_multi_dispatch<float, true>(maxm, items, prefix, n_items, n_wg, max_win, max_pslots, s)
               : rb_multi_dispatch<float, false>(maxm, items, prefix, n_items, n_wg, max_win, max_pslots, s);
  return adj ? rb_multi_dispatch<double, true>(maxm, items, prefix, n_items, n_wg, max_win, max_pslots, s)
             : rb_multi_dispatch<double, false>(maxm, items, prefix, n_items, n_wg, max_win, max_pslots, s);
}

hipError_t launch_pauli_apply_multi(int dtype, const PauliJob* jobs, const uint32_t* prefix, int n_jobs, uint32_t n_wg,
                                    hipStream_t s) {
  if (dtype == 0) pauli_apply_multi<float, kPauliChunk><<<n_wg, 256, 0, s>>>(jobs, prefix, n_jobs);
  else pauli_apply_multi<double, kPauliChunk><<<n_wg, 256, 0, s>>>(jobs, prefix, n_jobs);
  return hipGetLastError();
}

hipError_t launch_reduce_segments(const double* in, const int64_t* offs, const int32_t* lens, const int32_t* strides,
                                  double* out, int ncols, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  reduce_segments<<<(unsigned)ncols, 256, 0, s>>>(in, offs, lens, strides, out);
  return hipGetLastError();
}

hipError_t launch_set_zero_multi(int dtype, void* const* ptrs, const int32_t* nq, const uint32_t* prefix, int n_jobs,
                                 uint32_t n_wg, hipStream_t s) {
  if (dtype == 0) set_zero_multi<float><<<n_wg, 256, 0, s>>>(ptrs, nq, prefix, n_jobs);
  else set_zero_multi<double><<<n_wg, 256, 0, s>>>(ptrs, nq, prefix, n_jobs);
  return hipGetLastError();
}

hipError_t launch_scale_copy(int dtype, void* dst, const void* src, int n, double ar, double ai, hipStream_t s) {
  const unsigned grid = stream_blocks(1ull << n);
  if (dtype == 0) scale_copy<float><<<grid, 256, 0, s>>>(dst, src, 1ull << n, ar, ai);
  else scale_copy<double><<<grid, 256, 0, s>>>(dst, src, 1ull << n, ar, ai);
  return hipGetLastError();
}

unsigned inner_blocks(int n) {
  const unsigned b = stream_blocks(1ull << n);
  return b < 1024 ? b : 1024;
}

hipError_t launch_inner_product(int dtype, const void* a, const void* b, int n, double* partials, hipStream_t s) {
  const unsigned grid = inner_blocks(n);
  if (dtype == 0) inner_product<float><<<grid, 256, 0, s>>>(a, b, 1ull << n, partials);
  else inner_product<double><<<grid, 256, 0, s>>>(a, b, 1ull << n, partials);
  return hipGetLastError();
}

hipError_t launch_tile_pass_rb(int dtype, bool adj, int reg_bits, int maxm, const PassArgs& A, uint64_t n_tiles,
                               int batch, hipStream_t s) {
  if (A.m != maxm) return hipErrorInvalidValue;  // the kernel assumes a full workgroup
  if (A.win_n > kMaxWindow) return hipErrorInvalidValue;
  if (dtype == 0) return adj ? rb_dispatch<float, true>(reg_bits, maxm, A, n_tiles, batch, s)
                             : rb_dispatch<float, false>(reg_bits, maxm, A, n_tiles, batch, s);
  return adj ? rb_dispatch<double, true>(reg_bits, maxm, A, n_tiles, batch, s)
             : rb_dispatch<double, false>(reg_bits, maxm, A, n_tiles, batch, s);
}

hipError_t launch_tile_pass(int dtype, bool adj, int maxm, const PassArgs& A, uint64_t n_tiles,
                            int batch, hipStream_t s) {
  if (dtype == 0) return adj ? tile_dispatch<float, true>(maxm, A, n_tiles, batch, s)
                             : tile_dispatch<float, false>(maxm, A, n_tiles, batch, s);
  return adj ? tile_dispatch<double, true>(maxm, A, n_tiles, batch, s)
             : tile_dispatch<double, false>(maxm, A, n_tiles, batch, s);
}

hipError_t launch_gate1(int dtype, void* psi, int64_t bstride, int batch, int n, int t, uint64_t cmask,
                        const void* ctab, int64_t ctab_bstride, int mat, hipStream_t s) {
  const dim3 grid(stream_blocks(1ull << (n - 1)), (unsigned)batch);
  if (dtype == 0) gate1_stream<float><<<grid, 256, 0, s>>>(psi, bstride, n, t, cmask, ctab, ctab_bstride, mat);
  else gate1_stream<double><<<grid, 256, 0, s>>>(psi, bstride, n, t, cmask, ctab, ctab_bstride, mat);
  return hipGetLastError();
}

hipError_t launch_gate2(int dtype, void* psi, int64_t bstride, int batch, int n, int ta, int tb,
                        uint64_t cmask, const void* ctab, int64_t ctab_bstride, int mat, hipStream_t s) {
  const dim3 grid(stream_blocks(1ull << (n - 2)), (unsigned)batch);
  if (dtype == 0) gate2_stream<float><<<grid, 256, 0, s>>>(psi, bstride, n, ta, tb, cmask, ctab, ctab_bstride, mat);
  else gate2_stream<double><<<grid, 256, 0, s>>>(psi, bstride, n, ta, tb, cmask, ctab, ctab_bstride, mat);
  return hipGetLastError();
}

hipError_t launch_diag(int dtype, void* psi, int64_t bstride, int batch, int n, const DiagEntry* diag,
                       int first, int count, const void* ctab, int64_t ctab_bstride, hipStream_t s) {
  const dim3 grid(stream_blocks(1ull << n), (unsigned)batch);
  if (dtype == 0) diag_stream<float><<<grid, 256, 0, s>>>(psi, bstride, n, diag, first, count, ctab, ctab_bstride);
  else diag_stream<double><<<grid, 256, 0, s>>>(psi, bstride, n, diag, first, count, ctab, ctab_bstride);
  return hipGetLastError();
}

unsigned pauli_blocks(int n) {
  const uint64_t work = 1ull << (n > 0 ? n - 1 : 0);
  return stream_blocks(work) < 2048 ? stream_blocks(work) : 2048;
}

template <typename R>
void launch_pauli_mode(const PauliGroupArgs& A, dim3 grid, hipStream_t s) {
  if (A.xmask != 0) {
    pauli_group<R, PG_XMASK><<<grid, 256, 0, s>>>(A);
  } else if (A.n_pats > 0 && A.real_coeffs) {
    const int m = (A.n_terms <= kPauliStageTerms ? PG_STAGED : 0) | (A.lam ? PG_LAM : 0);
    switch (m) {
      case 0: pauli_group<R, 0><<<grid, 256, 0, s>>>(A); break;
      case 1: pauli_group<R, 1><<<grid, 256, 0, s>>>(A); break;
      case 2: pauli_group<R, 2><<<grid, 256, 0, s>>>(A); break;
      default: pauli_group<R, 3><<<grid, 256, 0, s>>>(A); break;
    }
  } else if (A.n_qubits >= 2) pauli_group<R, PG_QUAD><<<grid, 256, 0, s>>>(A);
  else pauli_group<R, PG_DIAG><<<grid, 256, 0, s>>>(A);
}

hipError_t launch_pauli_group(int dtype, const PauliGroupArgs& A, int batch, hipStream_t s) {
  const dim3 grid(pauli_blocks(A.n_qubits), (unsigned)batch);
  if (dtype == 0) launch_pauli_mode<float>(A, grid, s);
  else launch_pauli_mode<double>(A, grid, s);
  return hipGetLastError();
}

hipError_t launch_reduce_columns(const double* in, int64_t len, int64_t ncols, double* out, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  reduce_columns<<<(unsigned)ncols, 256, 0, s>>>(in, len, out);
  return hipGetLastError();
}

hipError_t launch_set_basis(int dtype, void* psi, int64_t bstride, int batch, int n, uint64_t index, hipStream_t s) {
  const dim3 grid(stream_blocks(1ull << n), (unsigned)batch);
  if (dtype == 0) set_basis<float><<<grid, 256, 0, s>>>(psi, bstride, 1ull << n, index);
  else set_basis<double><<<grid, 256, 0, s>>>(psi, bstride, 1ull << n, index);
  return hipGetLastError();
}

hipError_t launch_broadcast_state(int dtype, void* dst, int64_t bstride, int batch, const void* src, int n,
                                  hipStream_t s) {
  const dim3 grid(stream_blocks(1ull << n), (unsigned)batch);
  if (dtype == 0) broadcast_state<float><<<grid, 256, 0, s>>>(dst, bstride, src, 1ull << n);
  else broadcast_state<double><<<grid, 256, 0, s>>>(dst, bstride, src, 1ull << n);
  return hipGetLastError();
}

}  // namespace qsv
