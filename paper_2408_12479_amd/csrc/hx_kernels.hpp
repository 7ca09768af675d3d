// Device code: sum-factorised element kernels for the residual, the linearisation update and the
// linearised operator of finite-strain hyperelasticity (material configuration, and the spatial
// configuration as a storage mode of the linearised operator), and the node kernel that sums the
// element vectors.
//
// Thread layout. A workgroup processes EB cells; it has EB * (p+1)^3 threads, one per Gauss
// point of each cell ("q-threads"). The tensor-product contractions run as pencil jobs: a job
// owns one 1D line of one field of one cell, keeps it in registers and applies a 1D matrix whose
// coefficients are uniform across the wavefront (scalar registers). Jobs are spread over all
// threads of the workgroup; fields live in LDS between the sweeps. The q-point physics runs one
// q-point per thread with everything in registers.
//
// Interpolation (Section 6: sum factorisation): values at Gauss points v = (B x B x B) u, then
// reference derivatives g_d = D_d v with the collocation derivative D on the Gauss points. The
// transposed sequence integrates the test-function gradients: s = sum_d D_d^T t_d, out =
// (B^T x B^T x B^T) s. Cost per field: 6 sweeps of n^4 fused multiply-adds (fewer in the even-odd
// form used from n = 5 on).
//
// Assembly: each cell writes its element vector into its own brick of a per-context buffer (no
// atomics); assemble_kernel then sums, in a fixed order, the bricks meeting at every node.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "hx_internal.hpp"
#include "hx_tables.hpp"

namespace hx {

// ------------------------------------------------------------------------------------------
// Storage element types
// ------------------------------------------------------------------------------------------
struct bf16_t {
  uint16_t v;
};

__device__ __forceinline__ double load_val(const double* p) { return *p; }
__device__ __forceinline__ float load_val(const float* p) { return *p; }
__device__ __forceinline__ float load_val(const bf16_t* p) {
  return __uint_as_float(static_cast<uint32_t>(p->v) << 16);
}
__device__ __forceinline__ float load_val(const _Float16* p) { return static_cast<float>(*p); }

// Loads of stored q-point words in the apply when the whole set is larger than the caches: the
// words are read once per apply, and the non-temporal hint keeps them from evicting the vectors
// and the brick buffer, which are reused within the apply.
__device__ __forceinline__ double load_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float load_stream(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ _Float16 load_stream(const _Float16* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ bf16_t load_stream(const bf16_t* p) {
  return bf16_t{__builtin_nontemporal_load(&p->v)};
}

// stored word as held in a register before conversion
__device__ __forceinline__ double as_val(double v) { return v; }
__device__ __forceinline__ float as_val(float v) { return v; }
__device__ __forceinline__ float as_val(bf16_t v) { return __uint_as_float(static_cast<uint32_t>(v.v) << 16); }
__device__ __forceinline__ float as_val(_Float16 v) { return static_cast<float>(v); }

// Layout of the stored q-point words inside a block of EB cells (EBQ = EB (p+1)^3 slots): the
// first W - W mod G words of a slot are packed in groups of G words, group-major, so word w sits
// at (w / G) G EBQ + qi G + w mod G; the remaining W mod G words follow as planes of EBQ words.
// One load per lane then brings a whole group and the lanes of a wavefront read one contiguous
// run, with no word padded. G per word type, as measured (same-GPU A/B of the applies): FP64 one
// word (8-byte loads; 16-byte pairs were 2-8 % slower), FP32 four (16-byte loads: +5 % over pairs,
// which gained up to 5 % over single words), 16-bit four (8-byte loads; 16-byte groups within
// -2 to +3 %). Blocks follow each other at a stride of W EBQ words rounded up to a group, so that
// every group stays aligned to its size.
template <typename ST> struct Pack;
template <> struct Pack<double> { static constexpr int G = 1; };
template <> struct Pack<float> { static constexpr int G = 4; };
template <> struct Pack<bf16_t> { static constexpr int G = 4; };
template <> struct Pack<_Float16> { static constexpr int G = 4; };
template <typename ST>
constexpr int kPack = Pack<ST>::G;
template <typename ST>
__host__ __device__ constexpr int64_t block_words(int W, int EBQ) {
  return (static_cast<int64_t>(W) * EBQ + kPack<ST> - 1) / kPack<ST> * kPack<ST>;
}
template <typename ST, int W>
__device__ __forceinline__ int qword(int w, int EBQ, int qi) {
  constexpr int G = kPack<ST>;
  constexpr int WF = W - W % G;
  return w < WF ? (w / G) * (EBQ * G) + qi * G + w % G : w * EBQ + qi;
}

// one group of one slot by a single load (non-temporal with NT)
typedef unsigned int hx_u2 __attribute__((ext_vector_type(2)));
typedef unsigned int hx_u4 __attribute__((ext_vector_type(4)));
template <typename V, bool NT>
__device__ __forceinline__ V load_vec(const void* p) {
  const V* q = static_cast<const V*>(p);
  if constexpr (NT) return __builtin_nontemporal_load(q);
  else return *q;
}
template <bool NT>
__device__ __forceinline__ void load_group(const double* p, double* out) {
  out[0] = NT ? load_stream(p) : *p;
}
template <bool NT>
__device__ __forceinline__ void load_group(const float* p, float* out) {
  const hx_u4 v = load_vec<hx_u4, NT>(p);
  out[0] = __uint_as_float(v.x);
  out[1] = __uint_as_float(v.y);
  out[2] = __uint_as_float(v.z);
  out[3] = __uint_as_float(v.w);
}
template <bool NT>
__device__ __forceinline__ void load_group(const bf16_t* p, bf16_t* out) {
  const hx_u2 v = load_vec<hx_u2, NT>(p);
  out[0] = bf16_t{static_cast<uint16_t>(v.x & 0xffffu)};
  out[1] = bf16_t{static_cast<uint16_t>(v.x >> 16)};
  out[2] = bf16_t{static_cast<uint16_t>(v.y & 0xffffu)};
  out[3] = bf16_t{static_cast<uint16_t>(v.y >> 16)};
}
template <bool NT>
__device__ __forceinline__ void load_group(const _Float16* p, _Float16* out) {
  const hx_u2 v = load_vec<hx_u2, NT>(p);
  const uint16_t h[4] = {static_cast<uint16_t>(v.x & 0xffffu), static_cast<uint16_t>(v.x >> 16),
                         static_cast<uint16_t>(v.y & 0xffffu), static_cast<uint16_t>(v.y >> 16)};
#pragma unroll
  for (int i = 0; i < 4; ++i) __builtin_memcpy(&out[i], &h[i], sizeof(_Float16));
}

__device__ __forceinline__ void store_val(double* p, double v) { *p = v; }
__device__ __forceinline__ void store_val(float* p, double v) { *p = static_cast<float>(v); }
__device__ __forceinline__ void store_val(bf16_t* p, double v) {
  // round to nearest even from the float value (NaN kept quiet)
  uint32_t u = __float_as_uint(static_cast<float>(v));
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    p->v = static_cast<uint16_t>((u >> 16) | 0x40u);
    return;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  p->v = static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ void store_val(_Float16* p, double v) {
  *p = static_cast<_Float16>(static_cast<float>(v));
}

template <int S> struct StoreOf;
template <> struct StoreOf<kStoreF64> { using T = double; };
template <> struct StoreOf<kStoreF32> { using T = float; };
template <> struct StoreOf<kStoreBF16> { using T = bf16_t; };
template <> struct StoreOf<kStoreF16> { using T = _Float16; };

// ------------------------------------------------------------------------------------------
// Scalar math, per arithmetic type
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
// FP32: the hardware base-2 exponential after scaling by log2(e)
__device__ __forceinline__ float m_exp(float x) { return __expf(x); }

// J^(-2/3): by the cube root in FP64 (also for FP32 arithmetic, see vol_scalars); FP32 by Newton
// steps on f(x) = x^-3 - J^2 from x0 = 1 (Algorithm 2, Section 4) when iters > 0.
__device__ __forceinline__ double jpow(double Jm, int) {
  const double c = cbrt(1.0 + Jm);
  return 1.0 / (c * c);
}
__device__ __forceinline__ float jpow(float Jm, int iters) {
  if (iters > 0) {
    const float alpha = ((Jm + 2.0f) * Jm + 1.0f) * (1.0f / 3.0f);  // J^2 / 3
    float beta = (4.0f / 3.0f) - alpha;                            // first step from x0 = 1
    for (int n = 1; n < iters; ++n) {
      const float b2 = beta * beta;
      beta = (4.0f / 3.0f) * beta - alpha * (b2 * b2);
    }
    return beta;
  }
  return static_cast<float>(jpow(static_cast<double>(Jm), 0));
}

// ------------------------------------------------------------------------------------------
// 3x3 tensors, row-major A[3*i + j]
// ------------------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R det3(const R* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// adjugate (transpose of the cofactor matrix): A^-1 = adj(A) / det(A)
template <typename R>
__device__ __forceinline__ void adj3(const R* A, R* C) {
  C[0] = A[4] * A[8] - A[5] * A[7];
  C[1] = A[2] * A[7] - A[1] * A[8];
  C[2] = A[1] * A[5] - A[2] * A[4];
  C[3] = A[5] * A[6] - A[3] * A[8];
  C[4] = A[0] * A[8] - A[2] * A[6];
  C[5] = A[2] * A[3] - A[0] * A[5];
  C[6] = A[3] * A[7] - A[4] * A[6];
  C[7] = A[1] * A[6] - A[0] * A[7];
  C[8] = A[0] * A[4] - A[1] * A[3];
}

// H[c][J] = sum_d g[c][d] K[d][J]  (reference -> physical gradient, K = J0^-1)
template <typename R>
__device__ __forceinline__ void to_physical(const R* g, const R* K, R* H) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int J = 0; J < 3; ++J)
      H[3 * c + J] = g[3 * c] * K[J] + g[3 * c + 1] * K[3 + J] + g[3 * c + 2] * K[6 + J];
}

// t[c][d] = w sum_J P[c][J] K[d][J]  (stress -> test coefficients on reference gradients)
template <typename R>
__device__ __forceinline__ void to_reference(const R* P, const R* K, R w, R* t) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d)
      t[3 * c + d] =
          w * (P[3 * c] * K[3 * d] + P[3 * c + 1] * K[3 * d + 1] + P[3 * c + 2] * K[3 * d + 2]);
}

// Trilinear geometry at reference point (s, t, r): K = J0^-1, returns det J0.
// X[3*v + c] is coordinate c of vertex v = a + 2b + 4c'.
template <typename R>
__device__ __forceinline__ void trilinear_jacobian(const R* X, R s, R t, R r, R* J) {
  const R s1 = R(1) - s, t1 = R(1) - t, r1 = R(1) - r;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    J[3 * c + 0] = t1 * r1 * (X[3 + c] - X[c]) + t * r1 * (X[9 + c] - X[6 + c]) +
                   t1 * r * (X[15 + c] - X[12 + c]) + t * r * (X[21 + c] - X[18 + c]);
    J[3 * c + 1] = s1 * r1 * (X[6 + c] - X[c]) + s * r1 * (X[9 + c] - X[3 + c]) +
                   s1 * r * (X[18 + c] - X[12 + c]) + s * r * (X[21 + c] - X[15 + c]);
    J[3 * c + 2] = s1 * t1 * (X[12 + c] - X[c]) + s * t1 * (X[15 + c] - X[3 + c]) +
                   s1 * t * (X[18 + c] - X[6 + c]) + s * t * (X[21 + c] - X[9 + c]);
  }
}

// J0 = dX/dxi of the trilinear map at (s, t, r); K = J0^-1, returns det J0
template <typename R>
__device__ __forceinline__ R trilinear_geometry(const R* X, R s, R t, R r, R* K) {
  R J[9];
  trilinear_jacobian(X, s, t, r, J);
  R A[9];
  adj3(J, A);
  const R det = J[0] * A[0] + J[1] * A[3] + J[2] * A[6];
  const R inv = R(1) / det;
#pragma unroll
  for (int i = 0; i < 9; ++i) K[i] = A[i] * inv;
  return det;
}

// ------------------------------------------------------------------------------------------
// Constitutive laws (Sections 3-5), material configuration, stable forms.
// ------------------------------------------------------------------------------------------
// kFIBERC: the fibre law with structure tensors that vary from cell to cell (local frames).
enum : int { kCNH = 0, kINH = 1, kFIBER = 2, kFIBERC = 3 };

template <int LAW>
constexpr bool kIsFiber = LAW == kFIBER || LAW == kFIBERC;

// Structure tensors H_4, H_6 and mean directions M_4, M_6 seen by one q-point: the material's
// (uniform over the workgroup) or those of the thread's cell.
template <typename R>
struct Fib {
  const R* H4;
  const R* H6;
  const R* M4;
  const R* M6;
};

template <typename R>
struct QState {
  R F[9], Fi[9];
  R Jm, lnJ, Jp, c1, c2;
  R c3[2], Ei[2], dfac[2];
  int forced = -1;  // fibre tension switches taken from the update (bit f: family f active), or -1
  int bits = 0;     // the switches as decided (bit f: family f active)
};

template <int LAW, typename R>
__device__ __forceinline__ void fiber_scalars(const MaterialK<R>& m, R Ei, R ImOne, int f, QState<R>& s) {
  // c3 = 2 k1 exp(k2 E_i^2) if I*_i > 1 (strict), else 0  (fibre model, c3 definition). An FP32
  // apply takes the switch as the FP64 update decided it, so that rounding cannot flip it.
  const bool active = s.forced >= 0 ? ((s.forced >> f) & 1) != 0 : ImOne > R(0);
  if (active) s.bits |= 1 << f;
  const R e2 = Ei * Ei;
  s.Ei[f] = Ei;
  s.c3[f] = active ? R(2) * m.k1 * m_exp(m.k2 * e2) : R(0);
  s.dfac[f] = R(2) * m.k2 * e2 + R(1);
}

// iNH and fibre scalars from J - 1 and I1 = tr C (Section 5 definitions): J^-2/3,
// c1 = kappa/2 (J^2 - 1) - mu/3 J^-2/3 I1 and c2 = 2 mu/9 J^-2/3 I1 + kappa J^2, evaluated in FP64
// for both arithmetics and rounded once (FP32 keeps Algorithm 2 for J^-2/3 when asked for).
template <typename R>
__device__ __forceinline__ void vol_scalars(double Jm, double I1, const MaterialK<R>& m, QState<R>& s) {
  const double Jp = (sizeof(R) == 4 && m.jpow_iters > 0) ? static_cast<double>(jpow(static_cast<R>(Jm), m.jpow_iters))
                                                          : jpow(Jm, 0);
  const double kap = static_cast<double>(m.kappa), mu = static_cast<double>(m.mu);
  const double J = 1.0 + Jm;
  s.Jp = static_cast<R>(Jp);
  s.c1 = static_cast<R>(0.5 * kap * Jm * (Jm + 2.0) - mu / 3.0 * Jp * I1);
  s.c2 = static_cast<R>(2.0 * mu / 9.0 * Jp * I1 + kap * J * J);
}

// State from the displacement gradient H = Grad u (stable forms of Section 4):
// E = (H + H^T + H^T H)/2, J - 1 from the invariants of H, C^-1 via F^-1.
// Returns false when J <= 0. E is written to Eout (for the residual).
template <int LAW, typename R>
__device__ __forceinline__ bool state_from_H(const R* H, const MaterialK<R>& m,
                                             const Fib<R>& fb, QState<R>& s, R* E) {
#pragma unroll
  for (int i = 0; i < 9; ++i) s.F[i] = H[i];
  s.F[0] += R(1);
  s.F[4] += R(1);
  s.F[8] += R(1);
  // det(I + H) - 1 = I1(H) + I2(H) + I3(H), in FP64 also for FP32 arithmetic: J and the volumetric
  // terms near J = 1 keep double precision, and the FP32 kernels round their results once
  double Hd[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Hd[i] = static_cast<double>(H[i]);
  const double trH = Hd[0] + Hd[4] + Hd[8];
  const double I2 = Hd[0] * Hd[4] + Hd[0] * Hd[8] + Hd[4] * Hd[8] - Hd[1] * Hd[3] - Hd[2] * Hd[6] - Hd[5] * Hd[7];
  const double Jmd = det3(Hd) + I2 + trH;
  s.Jm = static_cast<R>(Jmd);
  const R J = R(1) + s.Jm;
  R A[9];
  adj3(s.F, A);
  const R invJ = R(1) / J;
#pragma unroll
  for (int i = 0; i < 9; ++i) s.Fi[i] = A[i] * invJ;
  // E = (H + H^T + H^T H) / 2
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      E[3 * i + j] = R(0.5) * (H[3 * i + j] + H[3 * j + i] + H[i] * H[j] + H[3 + i] * H[3 + j] +
                               H[6 + i] * H[6 + j]);
  if constexpr (LAW == kCNH) {
    s.lnJ = static_cast<R>(log1p(Jmd));
  } else {
    vol_scalars<R>(Jmd, static_cast<double>(R(3) + R(2) * (E[0] + E[4] + E[8])), m, s);
    if constexpr (kIsFiber<LAW>) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const R* Hf = f == 0 ? fb.H4 : fb.H6;
        const R* M = f == 0 ? fb.M4 : fb.M6;
        R Ei = R(0), mem = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) Ei += Hf[i] * E[i];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) mem += M[i] * E[3 * i + j] * M[j];
        // E_i = 2 H_i : E,  I*_i - 1 = 2 (M (x) M) : E
        fiber_scalars<LAW>(m, R(2) * Ei, R(2) * mem, f, s);
      }
    }
  }
  return J > R(0);
}

// State from stored F^-1 and J - 1: F = J adj(F^-1).
template <int LAW, typename R>
__device__ __forceinline__ void state_from_finv(const R* Fi, R Jm, const MaterialK<R>& m,
                                                const Fib<R>& fb, QState<R>& s) {
#pragma unroll
  for (int i = 0; i < 9; ++i) s.Fi[i] = Fi[i];
  s.Jm = Jm;
  if constexpr (LAW == kCNH) {
    s.lnJ = static_cast<R>(log1p(static_cast<double>(Jm)));
  } else {
    const R J = R(1) + Jm;
    R A[9];
    adj3(Fi, A);
#pragma unroll
    for (int i = 0; i < 9; ++i) s.F[i] = A[i] * J;
    R I1 = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) I1 += s.F[i] * s.F[i];
    vol_scalars<R>(static_cast<double>(Jm), static_cast<double>(I1), m, s);
    if constexpr (kIsFiber<LAW>) {
      R C[9];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          C[3 * i + j] = s.F[i] * s.F[j] + s.F[3 + i] * s.F[3 + j] + s.F[6 + i] * s.F[6 + j];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const R* Hf = f == 0 ? fb.H4 : fb.H6;
        const R* M = f == 0 ? fb.M4 : fb.M6;
        R Ei = -(Hf[0] + Hf[4] + Hf[8]), mcm = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) Ei += Hf[i] * C[i];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) mcm += M[i] * C[3 * i + j] * M[j];
        fiber_scalars<LAW>(m, Ei, mcm - R(1), f, s);
      }
    }
  }
}

// First Piola-Kirchhoff stress P = F S, stable forms:
//   cNH  P = F^-T (2 mu E + 2 lambda ln J I)
//   iNH  P = F^-T [kappa/2 (J-1)(J+1) I + 2 mu J^-2/3 (E - tr E / 3 I)]
//   fibre adds sum_i c3 E_i F H_i
template <int LAW, typename R>
__device__ __forceinline__ void stress_P(const QState<R>& s, const R* E, const MaterialK<R>& m,
                                         const Fib<R>& fb, R* P) {
  R Sv[9];
  if constexpr (LAW == kCNH) {
#pragma unroll
    for (int i = 0; i < 9; ++i) Sv[i] = R(2) * m.mu * E[i];
    const R d = R(2) * m.lam * s.lnJ;
    Sv[0] += d;
    Sv[4] += d;
    Sv[8] += d;
  } else {
    const R trE3 = (E[0] + E[4] + E[8]) / R(3);
    const R a = R(2) * m.mu * s.Jp;
#pragma unroll
    for (int i = 0; i < 9; ++i) Sv[i] = a * E[i];
    const R d = R(0.5) * m.kappa * s.Jm * (s.Jm + R(2)) - a * trE3;
    Sv[0] += d;
    Sv[4] += d;
    Sv[8] += d;
  }
  // P = F^-T Sv
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      P[3 * i + j] = s.Fi[i] * Sv[j] + s.Fi[3 + i] * Sv[3 + j] + s.Fi[6 + i] * Sv[6 + j];
  if constexpr (kIsFiber<LAW>) {
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const R* Hf = f == 0 ? fb.H4 : fb.H6;
      const R c = s.c3[f] * s.Ei[f];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          P[3 * i + j] += c * (s.F[3 * i] * Hf[j] + s.F[3 * i + 1] * Hf[3 + j] +
                               s.F[3 * i + 2] * Hf[6 + j]);
    }
  }
}

// Linearised stress P' = Grad du S + F D_u S (Section 5 forms, with the c1 sign of the appendix
// derivation), rearranged using F C^-1 = F^-T and S = mu I - a C^-1 (cNH) or
// S = mu J^-2/3 I + c1 C^-1 (iNH) so that no S needs forming:
//   cNH  P' = mu G + a F^-T G^T F^-T + 2 lambda tr(F^-1 G) F^-T,  a = mu - 2 lambda ln J
//   iNH  P' = mu Jp G - c1 F^-T G^T F^-T - 2mu/3 Jp tr(F^-1 G) F
//             + (c2 tr(F^-1 G) - 2mu/3 Jp F:G) F^-T
//   fibre adds sum_i c3 [E_i G H_i + 2 (2 k2 E_i^2 + 1) ((F H_i):G) F H_i]
template <int LAW, typename R>
__device__ __forceinline__ void action(const QState<R>& s, const MaterialK<R>& m,
                                       const Fib<R>& fb, const R* G, R* Pd) {
  // X = (F^-1 G)^T, Y = F^-T X = F^-T G^T F^-T, tr = tr(F^-1 G)
  R X[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      X[3 * i + j] = s.Fi[3 * j] * G[i] + s.Fi[3 * j + 1] * G[3 + i] + s.Fi[3 * j + 2] * G[6 + i];
  const R tr = X[0] + X[4] + X[8];
  R Y[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Y[3 * i + j] = s.Fi[i] * X[j] + s.Fi[3 + i] * X[3 + j] + s.Fi[6 + i] * X[6 + j];
  if constexpr (LAW == kCNH) {
    const R a = m.mu - R(2) * m.lam * s.lnJ;
    const R b = R(2) * m.lam * tr;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Pd[3 * i + j] = m.mu * G[3 * i + j] + a * Y[3 * i + j] + b * s.Fi[3 * j + i];
  } else {
    R FG = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) FG += s.F[i] * G[i];
    const R a = m.mu * s.Jp;
    const R b = R(2) / R(3) * a * tr;
    const R c = s.c2 * tr - R(2) / R(3) * a * FG;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Pd[3 * i + j] = a * G[3 * i + j] - s.c1 * Y[3 * i + j] - b * s.F[3 * i + j] +
                        c * s.Fi[3 * j + i];
    if constexpr (kIsFiber<LAW>) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const R* Hf = f == 0 ? fb.H4 : fb.H6;
        R FH[9], GH[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            FH[3 * i + j] = s.F[3 * i] * Hf[j] + s.F[3 * i + 1] * Hf[3 + j] +
                            s.F[3 * i + 2] * Hf[6 + j];
            GH[3 * i + j] =
                G[3 * i] * Hf[j] + G[3 * i + 1] * Hf[3 + j] + G[3 * i + 2] * Hf[6 + j];
          }
        R fhg = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) fhg += FH[i] * G[i];
        const R ce = s.c3[f] * s.Ei[f];
        const R cf = R(2) * s.c3[f] * s.dfac[f] * fhg;
#pragma unroll
        for (int i = 0; i < 9; ++i) Pd[i] += ce * GH[i] + cf * FH[i];
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Lattice addressing
// ------------------------------------------------------------------------------------------
struct CellPos {
  int ex, ey, ez;
};

__device__ __forceinline__ CellPos cell_pos(const Lattice& L, int e) {
  CellPos c;
  c.ex = e % L.nx;
  const int r = e / L.nx;
  c.ey = r % L.ny;
  c.ez = r / L.ny;
  return c;
}

// position of cell e0 + le from the position of e0 (carry along the lattice; le is small)
__device__ __forceinline__ CellPos cell_advance(const Lattice& L, CellPos c, int le) {
  c.ex += le;
  while (c.ex >= L.nx) {
    c.ex -= L.nx;
    if (++c.ey >= L.ny) {
      c.ey = 0;
      ++c.ez;
    }
  }
  return c;
}

__device__ __forceinline__ int wrap(int I, int n) { return I >= n ? I - n : I; }

// Dirichlet membership split by lattice direction (faces -x,+x | -y,+y,-z,+z)
__device__ __forceinline__ bool cons_x(const Lattice& L, int I) {
  const uint32_t f = L.dir_faces;
  return ((f & 1u) && I == 0) || ((f & 2u) && I == L.Nx - 1);
}
__device__ __forceinline__ bool cons_yz(const Lattice& L, int J, int K) {
  const uint32_t f = L.dir_faces;
  return ((f & 4u) && J == 0) || ((f & 8u) && J == L.Ny - 1) || ((f & 16u) && K == 0) ||
         ((f & 32u) && K == L.Nz - 1);
}

// node index and constraint flag of local node (i, j, k)
__device__ __forceinline__ int64_t node_of(const Lattice& L, const CellPos& c, int i, int j, int k,
                                           bool& cons) {
  const int I = wrap(c.ex * L.p + i, L.Nx), J = wrap(c.ey * L.p + j, L.Ny),
            K = wrap(c.ez * L.p + k, L.Nz);
  cons = cons_x(L, I) || cons_yz(L, J, K);
  return static_cast<int64_t>(I) + static_cast<int64_t>(L.Nx) * (J + static_cast<int64_t>(L.Ny) * K);
}

// ------------------------------------------------------------------------------------------
// Pencil machinery
// ------------------------------------------------------------------------------------------
// LDS layout of one field of an N^3 block: x fastest, rows of N values, planes of PS values; a
// field takes FS values. Q3 pads its planes (16 -> 19 values) and fields (64 -> 73): unpadded,
// the pencils that the lanes of a wavefront read fall on the same banks (4-way conflicts).
template <int N>
struct Lds {
  static constexpr int PS = N == 4 ? 19 : N * N;
  static constexpr int FS = N == 4 ? 73 : N * N * N;
};

// LDS offset of local point q = i + N j + N^2 k within its field
template <int N>
__device__ __forceinline__ int lds_q(int q) {
  return q + (Lds<N>::PS - N * N) * (q / (N * N));
}

// index of point m on pencil (a, b) along direction DIR in a field (x fastest)
template <int N, int DIR>
__device__ __forceinline__ int pidx(int a, int b, int m) {
  constexpr int PS = Lds<N>::PS;
  if constexpr (DIR == 0) return m + N * a + PS * b;
  else if constexpr (DIR == 1) return a + N * m + PS * b;
  else return a + N * b + PS * m;
}

// out = M in (TR: M^T in), M row-major N x N with wave-uniform coefficients
template <int N, bool TR, typename R>
__device__ __forceinline__ void apply1d(const R* M, const R* in, R* out) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R acc = R(0);
#pragma unroll
    for (int m = 0; m < N; ++m) acc = fma(TR ? M[m * N + i] : M[i * N + m], in[m], acc);
    out[i] = acc;
  }
}

// The same contraction in even-odd form. The 1D tables on points symmetric about the middle of
// the interval are centro-symmetric (B: M[N-1-q][N-1-i] = M[q][i]) or centro-antisymmetric (D:
// the same with a minus sign), and so are their transposes. With e_i = in_i + in_(N-1-i) and
// o_i = in_i - in_(N-1-i) (i < N/2), the outputs q and N-1-q come from one even sum E_q and one
// odd sum O_q as E_q + O_q and SGN (E_q - O_q): N = 7 takes 25 multiply-adds and 12 additions
// instead of 49 multiply-adds, N = 5 takes 13 and 8 instead of 25. The folded coefficients form
// compile-time tables read like the plain ones (scalar loads).
template <int N, typename R, bool TR, int SGN>
struct EvenOdd {
  static constexpr int H = N / 2;
  struct Tab {
    R a[H * H];   // (m(q,i) + m(q,N-1-i)) / 2, q, i < H
    R b[H * H];   // (m(q,i) - m(q,N-1-i)) / 2
    R c[H + 1];   // m(q, H) for q < H (odd N), then m(H, H)
    R r[H + 1];   // middle row m(H, i), i < H (odd N)
  };
  static constexpr R m(int q, int i) {
    const R* M = SGN > 0 ? Tab1D<N, R>::B : Tab1D<N, R>::D;
    return TR ? M[i * N + q] : M[q * N + i];
  }
  static constexpr Tab make() {
    Tab t{};
    for (int q = 0; q < H; ++q)
      for (int i = 0; i < H; ++i) {
        t.a[q * H + i] = R(0.5) * (m(q, i) + m(q, N - 1 - i));
        t.b[q * H + i] = R(0.5) * (m(q, i) - m(q, N - 1 - i));
      }
    if (N % 2 == 1) {
      for (int q = 0; q <= H; ++q) t.c[q] = m(q, H);
      for (int i = 0; i < H; ++i) t.r[i] = m(H, i);
    }
    return t;
  }
  static constexpr Tab tab = make();
};

template <int N, bool TR, int SGN, typename R>
__device__ __forceinline__ void apply1d_eo(const R* in, R* out) {
  using EO = EvenOdd<N, R, TR, SGN>;
  constexpr int H = N / 2;
  const auto& T = EO::tab;
  R e[H], o[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    e[i] = in[i] + in[N - 1 - i];
    o[i] = in[i] - in[N - 1 - i];
  }
#pragma unroll
  for (int q = 0; q < H; ++q) {
    R E = R(0), O = R(0);
#pragma unroll
    for (int i = 0; i < H; ++i) {
      E = fma(T.a[q * H + i], e[i], E);
      O = fma(T.b[q * H + i], o[i], O);
    }
    if constexpr (N % 2 == 1) E = fma(T.c[q], in[H], E);
    out[q] = E + O;
    out[N - 1 - q] = SGN > 0 ? E - O : O - E;
  }
  if constexpr (N % 2 == 1) {
    R acc = R(0);
    if constexpr (SGN > 0) {
#pragma unroll
      for (int i = 0; i < H; ++i) acc = fma(T.r[i], e[i], acc);
      acc = fma(T.c[H], in[H], acc);
    } else {
#pragma unroll
      for (int i = 0; i < H; ++i) acc = fma(T.r[i], o[i], acc);
    }
    out[H] = acc;
  }
}

// B (SGN = +1) or D (SGN = -1) contraction: even-odd form from N = 5 on, where it saves work.
template <int N, bool TR, int SGN, typename R>
__device__ __forceinline__ void contract1d(const R* M, const R* in, R* out) {
  if constexpr (N >= 5) apply1d_eo<N, TR, SGN>(in, out);
  else apply1d<N, TR>(M, in, out);
}

// Runs fn(le, set, a, b) for every pencil of NSETS fields of EB cells, spread over the
// workgroup's threads. The job decomposition is computed unconditionally from the thread index
// (the guard comes after it), so that phases with the same NSETS share it instead of repeating
// the integer divisions.
template <int N, int EB, int NSETS, typename Fn>
__device__ __forceinline__ void pencil_jobs(Fn&& fn) {
  constexpr int N2 = N * N;
  constexpr int NT = EB * N * N * N;
  constexpr int PER = NSETS * N2;
  constexpr int TOTAL = EB * PER;
  constexpr int ROUNDS = (TOTAL + NT - 1) / NT;
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const int job = static_cast<int>(threadIdx.x) + r * NT;
    const int le = job / PER;
    const int rr = job - le * PER;
    const int set = rr / N2;
    const int pl = rr - set * N2;
    const int a = pl % N, b = pl / N;
    if (job < TOTAL) fn(le, set, a, b);
  }
}

// Cell and node of a thread in the gather and in the final store: the block's EB cells are
// interleaved along x (thread t: i = t mod N, then the cell, then j and k), so that consecutive
// lanes walk a whole x-row of the block (EB rows of N values side by side in the lattice and in
// the brick buffer) and each load or store instruction covers longer contiguous runs than the
// row of one cell.
// Used for odd N only: with N even the per-cell LDS stride (9 N^3 words) is a multiple of the
// bank count, the cells' rows fall on the same banks and the interleaved LDS writes conflict
// (measured slower at Q3); with N odd they are spread over the banks (Q4: +5 %).
// (The host builds the general meshes' gather map in the same order, with slot_of_thread.)
template <int N, int EB>
__device__ __forceinline__ void interleaved_slot(int t, int& le, int& q) {
  slot_of_thread(N, EB, t, le, q);
}

// Node and constraint flag of gather slot t of block blk of a general mesh (map entry ~node marks
// a constrained node).
template <int N, int EB>
__device__ __forceinline__ int64_t map_node(const int32_t* map, int blk, int t, bool& cons) {
  const int32_t v = map[static_cast<int64_t>(blk) * (EB * N * N * N) + t];
  cons = v < 0;
  return cons ? static_cast<int64_t>(~v) : static_cast<int64_t>(v);
}

// LDS per cell: 9 fields of N^3 values. Forward: values (then d/dx in place) in c, d/dz in
// 3 + c, d/dy in 6 + c; backward: the nine test coefficients.
constexpr int kBuffers = 9;

// Forward pass for one 3-component vector V: writes the 9 reference derivatives at this
// thread's q-point into g[c*3 + d].
template <int N, int EB, bool MASK, int TOPO, typename R>
__device__ __forceinline__ void forward_vector(const KernelArgs<N, R>& a, R* sb, const R* V,
                                               int e0, const CellPos& c0, int le_me, int q_me,
                                               R* g) {
  constexpr int Q = N * N * N;
  constexpr int CB = kBuffers * Lds<N>::FS;  // per-cell stride in LDS
  const Lattice& L = a.L;
  // F0: gather, one node per thread, the block's cells interleaved along x so that the lanes of
  // a wavefront walk contiguous x-rows of the lattice and each load instruction touches few cache
  // lines (a pencil-per-lane gather touches one line per lane and was the most expensive part of
  // the kernel)
  {
    int lg, qg;
    interleaved_slot<N, EB>(le_me * Q + q_me, lg, qg);
    R* cb = sb + lg * CB;
    if (e0 + lg < L.n_cells) {
      bool cons;
      int64_t node;
      if constexpr (TOPO == kTopoMap) {
        node = map_node<N, EB>(a.map, e0 / EB, le_me * Q + q_me, cons);
      } else {
        const int i = qg % N, j = (qg / N) % N, k = qg / (N * N);
        const CellPos cp = cell_advance(L, c0, lg);
        node = node_of(L, cp, i, j, k, cons);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R v = V[c * L.n_nodes + node];
        cb[c * Lds<N>::FS + lds_q<N>(qg)] = (MASK && cons) ? R(0) : v;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) cb[c * Lds<N>::FS + lds_q<N>(qg)] = R(0);
    }
  }
  __syncthreads();
  // F1: interpolate along x
  pencil_jobs<N, EB, 3>([&](int le, int c, int j, int k) __attribute__((always_inline)) {
    R in[N], out[N];
    R* buf = sb + le * CB + c * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 0>(j, k, m)];
    contract1d<N, false, 1>(Tab1D<N, R>::B, in, out);
#pragma unroll
    for (int m = 0; m < N; ++m) buf[pidx<N, 0>(j, k, m)] = out[m];
  });
  __syncthreads();
  // F2: interpolate along y
  pencil_jobs<N, EB, 3>([&](int le, int c, int i, int k) __attribute__((always_inline)) {
    R in[N], out[N];
    R* buf = sb + le * CB + c * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 1>(i, k, m)];
    contract1d<N, false, 1>(Tab1D<N, R>::B, in, out);
#pragma unroll
    for (int m = 0; m < N; ++m) buf[pidx<N, 1>(i, k, m)] = out[m];
  });
  __syncthreads();
  // F3: interpolate along z (values at Gauss points, in place) and differentiate along z
  pencil_jobs<N, EB, 3>([&](int le, int c, int i, int j) __attribute__((always_inline)) {
    R in[N], v[N], d[N];
    R* buf = sb + le * CB + c * Lds<N>::FS;
    R* bz = sb + le * CB + (3 + c) * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 2>(i, j, m)];
    contract1d<N, false, 1>(Tab1D<N, R>::B, in, v);
    contract1d<N, false, -1>(Tab1D<N, R>::D, v, d);
#pragma unroll
    for (int m = 0; m < N; ++m) {
      buf[pidx<N, 2>(i, j, m)] = v[m];
      bz[pidx<N, 2>(i, j, m)] = d[m];
    }
  });
  __syncthreads();
  // F4: differentiate along y (into 6 + c)
  pencil_jobs<N, EB, 3>([&](int le, int c, int a1, int b1) __attribute__((always_inline)) {
    R in[N], d[N];
    const R* buf = sb + le * CB + c * Lds<N>::FS;
    R* by = sb + le * CB + (6 + c) * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 1>(a1, b1, m)];
    contract1d<N, false, -1>(Tab1D<N, R>::D, in, d);
#pragma unroll
    for (int m = 0; m < N; ++m) by[pidx<N, 1>(a1, b1, m)] = d[m];
  });
  __syncthreads();
  // F5: differentiate along x, in place
  pencil_jobs<N, EB, 3>([&](int le, int c, int a1, int b1) __attribute__((always_inline)) {
    R in[N], d[N];
    R* buf = sb + le * CB + c * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 0>(a1, b1, m)];
    contract1d<N, false, -1>(Tab1D<N, R>::D, in, d);
#pragma unroll
    for (int m = 0; m < N; ++m) buf[pidx<N, 0>(a1, b1, m)] = d[m];
  });
  __syncthreads();
  // F6: this thread's q-point
  const R* cb = sb + le_me * CB;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    g[3 * c + 0] = cb[c * Lds<N>::FS + lds_q<N>(q_me)];
    g[3 * c + 1] = cb[(6 + c) * Lds<N>::FS + lds_q<N>(q_me)];
    g[3 * c + 2] = cb[(3 + c) * Lds<N>::FS + lds_q<N>(q_me)];
  }
}

// Backward pass: integrates the test coefficients t[c*3 + d] of every q-thread against the
// reference gradients of the basis and writes the element vector.
// The last contraction is written back to LDS so that the output runs one node per thread, the
// lanes of a wavefront covering contiguous x-rows. The element vector goes, without atomics, to
// the broken lattice a.ework, where every cell owns an N^3 brick: the value of local node
// (i, j, k) of cell (ex, ey, ez) sits at (ex N + i, ey N + j, ez N + k) of an
// (nx N) x (ny N) x (nz N) array per component; assemble_kernel then sums the bricks that meet
// at each node and writes every row of the output once, in whole cache lines. (Device-scope
// FP64 atomics on the shared nodes cost about a third of the apply on MI355X; storing the
// cell-interior rows directly from here, interleaved with the other kernel's rows, was slower.)
template <int N, int EB, int TOPO, typename R>
__device__ __forceinline__ void backward_scatter(const KernelArgs<N, R>& a, R* sb, int e0,
                                                 const CellPos& c0, int le_me, int q_me,
                                                 const R* t) {
  constexpr int Q = N * N * N;
  constexpr int CB = kBuffers * Lds<N>::FS;
  const Lattice& L = a.L;
  __syncthreads();  // buffers may still be read by the forward pass
  {
    R* cb = sb + le_me * CB;
#pragma unroll
    for (int i = 0; i < 9; ++i) cb[i * Lds<N>::FS + lds_q<N>(q_me)] = t[i];
  }
  __syncthreads();
  // B2: D^T along x on t[c][0], D^T along y on t[c][1]
  pencil_jobs<N, EB, 6>([&](int le, int set, int a1, int b1) __attribute__((always_inline)) {
    const int c = set >> 1;
    R in[N], out[N];
    if ((set & 1) == 0) {
      R* buf = sb + le * CB + (3 * c) * Lds<N>::FS;
#pragma unroll
      for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 0>(a1, b1, m)];
      contract1d<N, true, -1>(Tab1D<N, R>::D, in, out);
#pragma unroll
      for (int m = 0; m < N; ++m) buf[pidx<N, 0>(a1, b1, m)] = out[m];
    } else {
      R* buf = sb + le * CB + (3 * c + 1) * Lds<N>::FS;
#pragma unroll
      for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 1>(a1, b1, m)];
      contract1d<N, true, -1>(Tab1D<N, R>::D, in, out);
#pragma unroll
      for (int m = 0; m < N; ++m) buf[pidx<N, 1>(a1, b1, m)] = out[m];
    }
  });
  __syncthreads();
  // B3: along z: s = tx' + ty' + D^T tz, then B^T
  pencil_jobs<N, EB, 3>([&](int le, int c, int i, int j) __attribute__((always_inline)) {
    R tz[N], s[N], out[N];
    R* bx = sb + le * CB + (3 * c) * Lds<N>::FS;
    const R* by = sb + le * CB + (3 * c + 1) * Lds<N>::FS;
    const R* bzp = sb + le * CB + (3 * c + 2) * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) tz[m] = bzp[pidx<N, 2>(i, j, m)];
    contract1d<N, true, -1>(Tab1D<N, R>::D, tz, s);
#pragma unroll
    for (int m = 0; m < N; ++m) s[m] += bx[pidx<N, 2>(i, j, m)] + by[pidx<N, 2>(i, j, m)];
    contract1d<N, true, 1>(Tab1D<N, R>::B, s, out);
#pragma unroll
    for (int m = 0; m < N; ++m) bx[pidx<N, 2>(i, j, m)] = out[m];
  });
  __syncthreads();
  // B4: B^T along y
  pencil_jobs<N, EB, 3>([&](int le, int c, int i, int k) __attribute__((always_inline)) {
    R in[N], out[N];
    R* buf = sb + le * CB + (3 * c) * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 1>(i, k, m)];
    contract1d<N, true, 1>(Tab1D<N, R>::B, in, out);
#pragma unroll
    for (int m = 0; m < N; ++m) buf[pidx<N, 1>(i, k, m)] = out[m];
  });
  __syncthreads();
  // B5: B^T along x in place, then one node per thread scatters (contiguous rows per wave)
  pencil_jobs<N, EB, 3>([&](int le, int c, int j, int k) __attribute__((always_inline)) {
    R in[N], out[N];
    R* buf = sb + le * CB + (3 * c) * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 0>(j, k, m)];
    contract1d<N, true, 1>(Tab1D<N, R>::B, in, out);
#pragma unroll
    for (int m = 0; m < N; ++m) buf[pidx<N, 0>(j, k, m)] = out[m];
  });
  __syncthreads();
  {
    // the store runs with the block's cells interleaved along x, like the gather
    int lg, qg;
    interleaved_slot<N, EB>(le_me * Q + q_me, lg, qg);
    const int e = e0 + lg;
    if constexpr (TOPO == kTopoMap) {
      // general mesh: the brick of a cell is its workgroup's slots, in the gather's order, so
      // that the store is one contiguous run per workgroup; the node kernel finds each node's
      // slots through its slot list
      if (e < L.n_cells) {
        bool cons;
        (void)map_node<N, EB>(a.map, e0 / EB, le_me * Q + q_me, cons);
        if (!cons) {
          const int64_t ES = static_cast<int64_t>(gridDim.x) * (EB * Q);
          const int64_t pos = static_cast<int64_t>(e0 / EB) * (EB * Q) + le_me * Q + q_me;
#pragma unroll
          for (int c = 0; c < 3; ++c) a.ework[c * ES + pos] = sb[lg * CB + (3 * c) * Lds<N>::FS + lds_q<N>(qg)];
        }
      }
    } else if (e < L.n_cells) {
      const int i = qg % N, j = (qg / N) % N, k = qg / (N * N);
      const CellPos cp = cell_advance(L, c0, lg);
      bool cons;
      (void)node_of(L, cp, i, j, k, cons);
      if (!cons) {
        const int64_t EX = static_cast<int64_t>(L.nx) * N, EY = static_cast<int64_t>(L.ny) * N;
        const int64_t ES = EX * EY * (static_cast<int64_t>(L.nz) * N);
        const int64_t pos = (cp.ex * N + i) + EX * ((cp.ey * N + j) + EY * (static_cast<int64_t>(cp.ez) * N + k));
#pragma unroll
        for (int c = 0; c < 3; ++c) a.ework[c * ES + pos] = sb[lg * CB + (3 * c) * Lds<N>::FS + lds_q<N>(qg)];
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Assembly of the element vectors at the lattice nodes
// ------------------------------------------------------------------------------------------
// Cells meeting at lattice index Ig along one direction (ncell cells, Nn nodes; periodic if
// Nn == ncell * P): up to two (cell, local index) pairs, the lower cell first.
template <int P>
__device__ __forceinline__ int cells_at(int Ig, int ncell, int Nn, int* cc, int* ll) {
  const int ec = Ig / P, il = Ig - ec * P;
  if (il) {
    cc[0] = ec;
    ll[0] = il;
    return 1;
  }
  int cnt = 0;
  if (ec > 0) {
    cc[0] = ec - 1;
    ll[0] = P;
    cnt = 1;
  } else if (Nn == ncell * P) {
    cc[0] = ncell - 1;
    ll[0] = P;
    cnt = 1;
  }
  if (ec < ncell) {
    cc[cnt] = ec;
    ll[cnt] = 0;
    ++cnt;
  }
  return cnt;
}

// One thread per lattice node, in node order (consecutive lanes walk the x-rows and continue on
// the next row, so no lane idles at the end of a row). Every node gets the sum of the bricks of
// the 1, 2, 4 or 8 cells that share it, in a fixed order (the apply is deterministic), or, on
// constrained rows, cons_src (du of the apply: identity rows) or zero (residual).
// the node kernel's last step on component row idx with assembled value t (see NodeEpilogue)
// The epilogue's operands at one component row (b, the inverse diagonal, the previous direction
// and x), requested before the node's bricks so that their memory latency overlaps the brick loads.
template <typename R>
struct EpiIn {
  R b, dinv, d, x;
};

template <typename R>
__device__ __forceinline__ EpiIn<R> epi_load(const Epi<R>& ep, int64_t idx) {
  EpiIn<R> v{R(0), R(0), R(0), R(0)};
  if (ep.kind == kEpiStore) return v;
  v.b = ep.b[idx];
  if (ep.kind == kEpiChebyshev || ep.kind == kEpiChebyshevFirst) {
    v.dinv = ep.dinv[idx];
    v.x = ep.x[idx];
    if (ep.kind == kEpiChebyshev) v.d = ep.d[idx];
  }
  return v;
}

// the node kernel's last step on component row idx with assembled value t (see NodeEpilogue)
template <typename R>
__device__ __forceinline__ void node_epilogue(const Epi<R>& ep, int64_t idx, R t, R* __restrict__ out,
                                              const EpiIn<R>& v) {
  if (ep.kind == kEpiChebyshev) {
    const R di = ep.c1 * v.d + ep.c2 * v.dinv * (v.b - t);
    ep.d[idx] = di;
    ep.x[idx] = v.x + di;
  } else if (ep.kind == kEpiChebyshevFirst) {
    const R di = ep.c2 * v.dinv * (v.b - t);
    ep.d[idx] = di;
    ep.x[idx] = v.x + di;
  } else if (ep.kind == kEpiResidual) {
    out[idx] = v.b - t;
  } else {
    out[idx] = t;
  }
}

template <typename R>
__device__ __forceinline__ void node_epilogue(const Epi<R>& ep, int64_t idx, R t, R* __restrict__ out) {
  node_epilogue(ep, idx, t, out, epi_load(ep, idx));
}

// EPI: the apply carries a smoother or residual epilogue (a separate instantiation, so that the
// plain store keeps the lean kernel).
template <int N, typename R, bool EPI>
__global__ void __launch_bounds__(256) assemble_kernel(Lattice L, const R* __restrict__ E,
                                                       const R* cons_src, R* out, Epi<R> ep) {
  constexpr int P = N - 1;
  const int64_t n = L.n_nodes;
  // n_nodes < 2^31 (the setup bounds cells * (p+1)^3), so the index arithmetic is 32-bit
  const uint32_t nd = blockIdx.x * 256u + threadIdx.x;
  if (nd >= static_cast<uint64_t>(n)) return;
  const int64_t node = nd;
  const uint32_t row = nd / static_cast<uint32_t>(L.Nx);
  const int I = static_cast<int>(nd - row * static_cast<uint32_t>(L.Nx));
  const int K = static_cast<int>(row / static_cast<uint32_t>(L.Ny)), J = static_cast<int>(row) - K * L.Ny;
  if (cons_x(L, I) || cons_yz(L, J, K)) {
#pragma unroll
    for (int c = 0; c < 3; ++c) node_epilogue(ep, c * n + node, cons_src ? cons_src[c * n + node] : R(0), out);
    return;
  }
  int cx[2], lx[2], cy[2], ly[2], cz[2], lz[2];
  const int nxc = cells_at<P>(I, L.nx, L.Nx, cx, lx);
  const int nyc = cells_at<P>(J, L.ny, L.Ny, cy, ly);
  const int nzc = cells_at<P>(K, L.nz, L.Nz, cz, lz);
  const int64_t EX = static_cast<int64_t>(L.nx) * N, EY = static_cast<int64_t>(L.ny) * N;
  const int64_t ES = EX * EY * (static_cast<int64_t>(L.nz) * N);
  // positions of the one or two bricks along x in a brick row (the same position twice if one)
  const int x0 = cx[0] * N + lx[0];
  const int x1 = nxc > 1 ? cx[1] * N + lx[1] : x0;
  // all loads are issued before the first sum: summing each value as it arrives would wait for
  // up to eight memory round trips one after the other
  EpiIn<R> pre[3] = {};
  R off[3] = {R(0), R(0), R(0)};  // nodal block smoother: the inverse block's entries 01, 02, 12
  if constexpr (EPI) {
    pre[0] = epi_load(ep, node);
    pre[1] = epi_load(ep, n + node);
    pre[2] = epi_load(ep, 2 * n + node);
    if (ep.blocks && ep.kind != kEpiResidual) {
      off[0] = ep.dinv[3 * n + node];
      off[1] = ep.dinv[4 * n + node];
      off[2] = ep.dinv[5 * n + node];
    }
  }
  R v[4][3][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int k = 2 * a + b;
      if (a < nzc && b < nyc) {
        const int64_t rowpos = EX * ((cy[b] * N + ly[b]) + EY * (static_cast<int64_t>(cz[a]) * N + lz[a]));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          v[k][c][0] = E[c * ES + rowpos + x0];
          v[k][c][1] = E[c * ES + rowpos + x1];
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) v[k][c][0] = v[k][c][1] = R(0);
      }
    }
  R s0 = R(0), s1 = R(0), s2 = R(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    s0 += v[k][0][0];
    s1 += v[k][1][0];
    s2 += v[k][2][0];
    if (nxc > 1) {
      s0 += v[k][0][1];
      s1 += v[k][1][1];
      s2 += v[k][2][1];
    }
  }
  if constexpr (EPI) {
    if (ep.blocks && ep.kind != kEpiResidual) {
      // nodal block Jacobi: the three residual components of the node times the inverse block
      // (diagonal entries in pre[c].dinv), then the Chebyshev update of each component
      const R r0 = pre[0].b - s0, r1 = pre[1].b - s1, r2 = pre[2].b - s2;
      const R w[3] = {pre[0].dinv * r0 + off[0] * r1 + off[1] * r2,
                      off[0] * r0 + pre[1].dinv * r1 + off[2] * r2,
                      off[1] * r0 + off[2] * r1 + pre[2].dinv * r2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R di = (ep.kind == kEpiChebyshev ? ep.c1 * pre[c].d : R(0)) + ep.c2 * w[c];
        ep.d[c * n + node] = di;
        ep.x[c * n + node] = pre[c].x + di;
      }
    } else {
      node_epilogue(ep, node, s0, out, pre[0]);
      node_epilogue(ep, n + node, s1, out, pre[1]);
      node_epilogue(ep, 2 * n + node, s2, out, pre[2]);
    }
  } else {
    out[node] = s0;
    out[n + node] = s1;
    out[2 * n + node] = s2;
  }
}

// General meshes: one thread per node sums the element-vector slots of its list (increasing slot
// order, so repeated applies are bit-identical); constrained rows receive cons_src or zero.
template <typename R>
__global__ void __launch_bounds__(256) assemble_map_kernel(int64_t n, const int32_t* __restrict__ nptr,
                                                           const int32_t* __restrict__ nslot,
                                                           const uint8_t* __restrict__ cmask, int64_t ES,
                                                           const R* __restrict__ E, const R* cons_src,
                                                           R* out, Epi<R> ep) {
  const int64_t node = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (node >= n) return;
  if (cmask[node]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) node_epilogue(ep, c * n + node, cons_src ? cons_src[c * n + node] : R(0), out);
    return;
  }
  const int s0 = nptr[node], s1 = nptr[node + 1];
  R s[3] = {R(0), R(0), R(0)};
  for (int k = s0; k < s1; ++k) {
    const int64_t sl = nslot[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] += E[c * ES + sl];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) node_epilogue(ep, c * n + node, s[c], out);
}

// ------------------------------------------------------------------------------------------
// Operations (what happens at the q-point)
// ------------------------------------------------------------------------------------------
// Geometry of this q-point from the cell's vertices in LDS.
// arr[idx] for a lane-dependent idx without dynamic indexing of kernel arguments (which would
// force a private copy of the argument block)
template <int N, typename R>
__device__ __forceinline__ R pick(const R* arr, int idx) {
  R v = arr[0];
#pragma unroll
  for (int i = 1; i < N; ++i) v = idx == i ? arr[i] : v;
  return v;
}

template <int N, typename R>
__device__ __forceinline__ R qpoint_geometry(const R* X, int q, R* K) {
  const int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
  const R det = trilinear_geometry(X, pick<N>(Tab1D<N, R>::x, qx), pick<N>(Tab1D<N, R>::x, qy), pick<N>(Tab1D<N, R>::x, qz), K);
  return det * (pick<N>(Tab1D<N, R>::w, qx) * pick<N>(Tab1D<N, R>::w, qy) * pick<N>(Tab1D<N, R>::w, qz));
}

template <int N, typename R>
__device__ __forceinline__ void qpoint_jacobian(const R* X, int q, R* J0) {
  const int qx = q % N, qy = (q / N) % N, qz = q / (N * N);
  trilinear_jacobian(X, pick<N>(Tab1D<N, R>::x, qx), pick<N>(Tab1D<N, R>::x, qy), pick<N>(Tab1D<N, R>::x, qz), J0);
}

// ------------------------------------------------------------------------------------------
// Spatial configuration (Section 2, spatial residual and its linearisation; Section 5 spatial
// forms). Stored words per q-point: K = sqrt(w det J0) J_t^-1 (9, row-major, J_t = dx/dxi of the
// deformed map x = X + u_k), the Kirchhoff stress tau (6: xx yy zz xy xz yz), then
//   cNH   a2 = 2 (mu - 2 lambda ln J)                       J c:e = a2 e + 2 lambda tr(e) I
//   iNH   c1, c2, beta_b = (2 mu / 3) J^-2/3 b (6)        J c:e = -[beta_b tr(e) + (beta_b:e) I]
//                                                                 - 2 c1 e + c2 tr(e) I
//   fibre iNH, then per family h_i = F H_i F^T (6), d_i = 2 c3 (2 k2 E_i^2 + 1):
//                                                         J c:e += sum_i d_i (h_i:e) h_i
// The b-term is the push-forward of the symmetrised iNH second derivative (b, not C).
// The apply: with g' = (d du/dxi) K = sqrt(w det J0) grad du and e' = sym(g'), everything is
// linear in g', so t = [ g' tau + J c:e' ] K^T = w det J0 [ (grad du) tau + J c:e ] J_t^-T: the
// weight rides on the stored inverse Jacobian and costs no word.
// ------------------------------------------------------------------------------------------
template <int LAW>
constexpr int kSpatialWords = spatial_words(LAW == kCNH ? 0 : (LAW == kINH ? 1 : 2));

template <typename R>
__device__ __forceinline__ void sym_to_full(const R* v, R* A) {
  A[0] = v[0];
  A[4] = v[1];
  A[8] = v[2];
  A[1] = A[3] = v[3];
  A[2] = A[6] = v[4];
  A[5] = A[7] = v[5];
}

template <typename R>
__device__ __forceinline__ void full_to_sym(const R* A, R* v) {
  v[0] = A[0];
  v[1] = A[4];
  v[2] = A[8];
  v[3] = R(0.5) * (A[1] + A[3]);
  v[4] = R(0.5) * (A[2] + A[6]);
  v[5] = R(0.5) * (A[5] + A[7]);
}

// Spatial data at a q-point (update): H = Grad u, F, state, J0 and the reference gradient g of u.
template <int LAW, typename R>
__device__ __forceinline__ void spatial_words_at(const R* H, const QState<R>& st, const MaterialK<R>& m,
                                                 const Fib<R>& fb, const R* J0, const R* g, R wdet, R* out) {
  R Jt[9], A[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Jt[i] = J0[i] + g[i];
  adj3(Jt, A);
  const R inv = sqrt(wdet) / (Jt[0] * A[0] + Jt[1] * A[3] + Jt[2] * A[6]);
#pragma unroll
  for (int i = 0; i < 9; ++i) out[i] = A[i] * inv;
  // b~ = (H + H^T + H H^T) / 2 (stable Green-Euler strain)
  R bt[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      bt[3 * i + j] = R(0.5) * (H[3 * i + j] + H[3 * j + i] + H[3 * i] * H[3 * j] + H[3 * i + 1] * H[3 * j + 1] +
                                H[3 * i + 2] * H[3 * j + 2]);
  R tau[9];
  if constexpr (LAW == kCNH) {
    // tau = 2 mu b~ + 2 lambda ln J I
    const R d = R(2) * m.lam * st.lnJ;
#pragma unroll
    for (int i = 0; i < 9; ++i) tau[i] = R(2) * m.mu * bt[i];
    tau[0] += d;
    tau[4] += d;
    tau[8] += d;
    out[15] = R(2) * (m.mu - R(2) * m.lam * st.lnJ);
  } else {
    // tau = kappa/2 (J - 1)(J + 1) I + 2 mu J^-2/3 (b~ - tr(b~)/3 I)
    const R tr3 = (bt[0] + bt[4] + bt[8]) / R(3);
    const R a = R(2) * m.mu * st.Jp;
    const R d = R(0.5) * m.kappa * st.Jm * (st.Jm + R(2)) - a * tr3;
#pragma unroll
    for (int i = 0; i < 9; ++i) tau[i] = a * bt[i];
    tau[0] += d;
    tau[4] += d;
    tau[8] += d;
    out[15] = st.c1;
    out[16] = st.c2;
    R bb[9];
    const R beta = R(2) / R(3) * m.mu * st.Jp;
#pragma unroll
    for (int i = 0; i < 9; ++i) bb[i] = beta * R(2) * bt[i];
    bb[0] += beta;
    bb[4] += beta;
    bb[8] += beta;
    full_to_sym(bb, out + 17);
    if constexpr (kIsFiber<LAW>) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const R* Hf = f == 0 ? fb.H4 : fb.H6;
        R FH[9], h[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            FH[3 * i + j] = st.F[3 * i] * Hf[j] + st.F[3 * i + 1] * Hf[3 + j] + st.F[3 * i + 2] * Hf[6 + j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            h[3 * i + j] = FH[3 * i] * st.F[3 * j] + FH[3 * i + 1] * st.F[3 * j + 1] + FH[3 * i + 2] * st.F[3 * j + 2];
        const R ce = st.c3[f] * st.Ei[f];
#pragma unroll
        for (int i = 0; i < 9; ++i) tau[i] += ce * h[i];
        full_to_sym(h, out + 23 + 7 * f);
        out[29 + 7 * f] = R(2) * st.c3[f] * st.dfac[f];
      }
    }
  }
  full_to_sym(tau, out + 9);
}

// Spatial apply at a q-point: reference gradient g of du -> test coefficients t.
template <int LAW, typename R>
__device__ __forceinline__ void spatial_action(const R* d, const MaterialK<R>& m, const R* g, R* t) {
  const R* Kt = d;
  R gd[9];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j) gd[3 * c + j] = g[3 * c] * Kt[j] + g[3 * c + 1] * Kt[3 + j] + g[3 * c + 2] * Kt[6 + j];
  R tau[9];
  sym_to_full(d + 9, tau);
  R e[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) e[3 * i + j] = R(0.5) * (gd[3 * i + j] + gd[3 * j + i]);
  const R tr = gd[0] + gd[4] + gd[8];
  R sg[9];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 3; ++j) sg[3 * c + j] = gd[3 * c] * tau[j] + gd[3 * c + 1] * tau[3 + j] + gd[3 * c + 2] * tau[6 + j];
  if constexpr (LAW == kCNH) {
    const R a2 = d[15];
#pragma unroll
    for (int i = 0; i < 9; ++i) sg[i] += a2 * e[i];
    const R l = R(2) * m.lam * tr;
    sg[0] += l;
    sg[4] += l;
    sg[8] += l;
  } else {
    const R c1 = d[15], c2 = d[16];
    R bb[9];
    sym_to_full(d + 17, bb);
    R be = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) be += bb[i] * e[i];
#pragma unroll
    for (int i = 0; i < 9; ++i) sg[i] += -bb[i] * tr - R(2) * c1 * e[i];
    const R diag = c2 * tr - be;
    sg[0] += diag;
    sg[4] += diag;
    sg[8] += diag;
    if constexpr (kIsFiber<LAW>) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        R h[9];
        sym_to_full(d + 23 + 7 * f, h);
        R he = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) he += h[i] * e[i];
        const R cf = d[29 + 7 * f] * he;
#pragma unroll
        for (int i = 0; i < 9; ++i) sg[i] += cf * h[i];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int dd = 0; dd < 3; ++dd)
      t[3 * c + dd] = sg[3 * c] * Kt[3 * dd] + sg[3 * c + 1] * Kt[3 * dd + 1] + sg[3 * c + 2] * Kt[3 * dd + 2];
}

// ------------------------------------------------------------------------------------------
// The stored-scalar and stored-tensor stages of the reference-configuration operator (Section 5:
// the weak forms with the stored quantities marked; Tab. overview_precompute).
// SCALARS: the law's scalars are stored and F is formed from u_k at every apply, as with nothing
// stored; F^-1 = adj(F) / J. Words:
//   cNH   ln J
//   iNH   J - 1, J^-2/3, c1, c2
//   fibre the iNH words, then c3 and E_i of each family (c3 carries the tension switch)
// TENSORS: F, S, F^-1 and C^-1 are stored with the scalars of D_u S, and the apply evaluates
// P' = G S + F D_u S[G] (G = Grad du) term by term:
//   cNH   D_u S = 2 (mu - 2 lambda ln J) sym(F^-1 G C^-1) + 2 lambda tr(F^-1 G) C^-1
//   iNH   D_u S = -2 c1 sym(F^-1 G C^-1) + (c2 tr(F^-1 G) - 2mu/3 J^-2/3 F:G) C^-1
//                 - 2mu/3 J^-2/3 tr(F^-1 G) I
//   fibre adds sum_i 2 c3 (2 k2 E_i^2 + 1) ((F H_i):G) H_i
// with the c1 sign of the appendix derivation (as in `action`). Words: F 9, S 6 (symmetric),
// F^-1 9, C^-1 6 (symmetric), then cNH ln J; iNH J^-2/3, c1, c2; fibre adds 2 c3 (2 k2 E_i^2 + 1)
// per family.
// ------------------------------------------------------------------------------------------
template <int LAW>
constexpr int kScalarWords = LAW == kCNH ? 1 : (LAW == kINH ? 4 : 8);
template <int LAW>
constexpr int kTensorWords = LAW == kCNH ? 31 : (LAW == kINH ? 33 : 35);

template <int LAW, typename R>
__device__ __forceinline__ void scalar_words(const QState<R>& s, R* d) {
  if constexpr (LAW == kCNH) {
    d[0] = s.lnJ;
  } else {
    d[0] = s.Jm;
    d[1] = s.Jp;
    d[2] = s.c1;
    d[3] = s.c2;
    if constexpr (kIsFiber<LAW>) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        d[4 + 2 * f] = s.c3[f];
        d[5 + 2 * f] = s.Ei[f];
      }
    }
  }
}

// State of an apply from H = Grad u_k and the stored scalars. cNH forms J - 1 from the invariants
// of H in FP64, as the update does.
template <int LAW, typename R>
__device__ __forceinline__ void state_from_scalars(const R* H, const R* d, const MaterialK<R>& m, QState<R>& s) {
#pragma unroll
  for (int i = 0; i < 9; ++i) s.F[i] = H[i];
  s.F[0] += R(1);
  s.F[4] += R(1);
  s.F[8] += R(1);
  if constexpr (LAW == kCNH) {
    double Hd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Hd[i] = static_cast<double>(H[i]);
    const double trH = Hd[0] + Hd[4] + Hd[8];
    const double I2 = Hd[0] * Hd[4] + Hd[0] * Hd[8] + Hd[4] * Hd[8] - Hd[1] * Hd[3] - Hd[2] * Hd[6] - Hd[5] * Hd[7];
    s.Jm = static_cast<R>(det3(Hd) + I2 + trH);
    s.lnJ = d[0];
  } else {
    s.Jm = d[0];
    s.Jp = d[1];
    s.c1 = d[2];
    s.c2 = d[3];
    if constexpr (kIsFiber<LAW>) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        s.c3[f] = d[4 + 2 * f];
        s.Ei[f] = d[5 + 2 * f];
        s.dfac[f] = R(2) * m.k2 * s.Ei[f] * s.Ei[f] + R(1);
      }
    }
  }
  R A[9];
  adj3(s.F, A);
  const R invJ = R(1) / (R(1) + s.Jm);
#pragma unroll
  for (int i = 0; i < 9; ++i) s.Fi[i] = A[i] * invJ;
}

template <int LAW, typename R>
__device__ __forceinline__ void tensor_words(const QState<R>& s, const R* E, const MaterialK<R>& m,
                                             const Fib<R>& fb, R* d) {
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i] = s.F[i];
  // S = F^-1 P, symmetrised (P from the stable stress of the residual)
  R P[9], S[9];
  stress_P<LAW>(s, E, m, fb, P);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) S[3 * i + j] = s.Fi[3 * i] * P[j] + s.Fi[3 * i + 1] * P[3 + j] + s.Fi[3 * i + 2] * P[6 + j];
  R Ss[9], Ci[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Ss[3 * i + j] = R(0.5) * (S[3 * i + j] + S[3 * j + i]);
      Ci[3 * i + j] = s.Fi[3 * i] * s.Fi[3 * j] + s.Fi[3 * i + 1] * s.Fi[3 * j + 1] + s.Fi[3 * i + 2] * s.Fi[3 * j + 2];
    }
  full_to_sym(Ss, d + 9);
#pragma unroll
  for (int i = 0; i < 9; ++i) d[15 + i] = s.Fi[i];
  full_to_sym(Ci, d + 24);
  if constexpr (LAW == kCNH) {
    d[30] = s.lnJ;
  } else {
    d[30] = s.Jp;
    d[31] = s.c1;
    d[32] = s.c2;
    if constexpr (kIsFiber<LAW>) {
#pragma unroll
      for (int f = 0; f < 2; ++f) d[33 + f] = R(2) * s.c3[f] * s.dfac[f];
    }
  }
}

template <int LAW, typename R>
__device__ __forceinline__ void tensor_action(const R* d, const MaterialK<R>& m, const Fib<R>& fb, const R* G,
                                              R* Pd) {
  const R* F = d;
  const R* Fi = d + 15;
  R S[9], Ci[9];
  sym_to_full(d + 9, S);
  sym_to_full(d + 24, Ci);
  // Y = F^-1 G, M = Y C^-1
  R Y[9], M[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Y[3 * i + j] = Fi[3 * i] * G[j] + Fi[3 * i + 1] * G[3 + j] + Fi[3 * i + 2] * G[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[3 * i + j] = Y[3 * i] * Ci[j] + Y[3 * i + 1] * Ci[3 + j] + Y[3 * i + 2] * Ci[6 + j];
  const R tr = Y[0] + Y[4] + Y[8];
  R DS[9];
  if constexpr (LAW == kCNH) {
    const R a = m.mu - R(2) * m.lam * d[30];   // 2 a sym(M) = a (M + M^T)
    const R b = R(2) * m.lam * tr;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) DS[3 * i + j] = a * (M[3 * i + j] + M[3 * j + i]) + b * Ci[3 * i + j];
  } else {
    const R Jp = d[30], c1 = d[31], c2 = d[32];
    R FG = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) FG += F[i] * G[i];
    const R two3 = R(2) / R(3) * m.mu * Jp;
    const R cc = c2 * tr - two3 * FG;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) DS[3 * i + j] = -c1 * (M[3 * i + j] + M[3 * j + i]) + cc * Ci[3 * i + j];
    DS[0] -= two3 * tr;
    DS[4] -= two3 * tr;
    DS[8] -= two3 * tr;
    if constexpr (kIsFiber<LAW>) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const R* Hf = f == 0 ? fb.H4 : fb.H6;
        R fhg = R(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            fhg += (F[3 * i] * Hf[j] + F[3 * i + 1] * Hf[3 + j] + F[3 * i + 2] * Hf[6 + j]) * G[3 * i + j];
        const R w = d[33 + f] * fhg;
#pragma unroll
        for (int i = 0; i < 9; ++i) DS[i] += w * Hf[i];
      }
    }
  }
  // P' = G S + F D_u S
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Pd[3 * i + j] = G[3 * i] * S[j] + G[3 * i + 1] * S[3 + j] + G[3 * i + 2] * S[6 + j] + F[3 * i] * DS[j] +
                      F[3 * i + 1] * DS[3 + j] + F[3 * i + 2] * DS[6 + j];
}

template <int N, int EB, typename R>
__device__ __forceinline__ void load_vertices(const KernelArgs<N, R>& a, R* sv, int e0,
                                              const CellPos& c0) {
  // 24 values per cell (8 vertices x 3 coordinates), spread over the workgroup, relative to the
  // cell's first vertex and formed in FP64: the map uses only vertex differences, and differences
  // of FP32 absolute coordinates would lose digits in proportion to |X| / h
  constexpr int NT = EB * N * N * N;
  for (int idx = threadIdx.x; idx < EB * 24; idx += NT) {
    const int le = idx / 24, q = idx - 24 * le;
    const int e = e0 + le;
    if (e >= a.L.n_cells) continue;
    const CellPos cp = cell_advance(a.L, c0, le);
    const int v = q / 3, comp = q - 3 * v;
    int vx = cp.ex + (v & 1), vy = cp.ey + ((v >> 1) & 1), vz = cp.ez + (v >> 2);
    vx = vx >= a.L.Vx ? vx - a.L.Vx : vx;
    vy = vy >= a.L.Vy ? vy - a.L.Vy : vy;
    vz = vz >= a.L.Vz ? vz - a.L.Vz : vz;
    const int64_t vid = vx + static_cast<int64_t>(a.L.Vx) * (vy + static_cast<int64_t>(a.L.Vy) * vz);
    const int64_t v0 = cp.ex + static_cast<int64_t>(a.L.Vx) * (cp.ey + static_cast<int64_t>(a.L.Vy) * cp.ez);
    sv[le * 24 + q] = static_cast<R>(a.vert[3 * vid + comp] - a.vert[3 * v0 + comp]);
  }
}

// Block of cells of workgroup b in a grid of g: the hardware deals workgroups to the 8 XCDs in
// turn (b mod 8), so the blocks are renumbered to give each XCD a contiguous range of them (a
// slab of the lattice): neighbouring blocks, which gather the nodes on their common faces, then
// mostly run on one XCD and share its L2. A bijection of [0, g) for any g.
__device__ __forceinline__ int xcd_block(int b, int g) {
  constexpr int kXcd = 8;
  const int per = g / kXcd, rem = g - per * kXcd;
  const int x = b % kXcd;
  return x * per + (x < rem ? x : rem) + b / kXcd;
}

// Waves per SIMD the kernel is compiled for: the update may use the whole register file; the FP64
// applies that re-evaluate the law from u_k at every apply with nothing or only scalars stored
// (NONE, SPATIAL_RECOMPUTE, SPATIAL_SCALARS) hold more than 128 registers' worth of state and run
// at 2 waves rather than spill (measured, with the autotuner's cells per workgroup: Q3 / Q4 / Q6
// +2-3 % NONE, +16 / +4 / +17 % SPATIAL_RECOMPUTE, +5 / +8 / +14 % SPATIAL_SCALARS; the same bound
// made SCALARS, F^-1 + J and TENSORS no faster or slower); the others keep 4.
template <int KIND, int MODE, typename R>
constexpr int kMinWaves = KIND == 2 ? 1
                          : (KIND == 0 && sizeof(R) == 8 &&
                             (MODE == HX_STORE_SPATIAL_RECOMPUTE || MODE == HX_STORE_SPATIAL_SCALARS ||
                              MODE == HX_STORE_NONE))
                                ? 2
                                : 4;

// Kernel: ops = residual, apply (four storage modes) and update (four storage modes).
//   KIND 0 apply, 1 residual, 2 update; MODE = hx_storage; S = StoreType; LAW
// The apply and residual kernels are held to at most 128 VGPRs (4 waves per SIMD; forcing 8
// waves spills and is slower) except the FP64 applies of kMinWaves; the update runs once per
// Newton step and may use the whole register file.
template <int N, int EB, typename R, int KIND, int MODE, int LAW, int S, bool NT = false,
          int TOPO = kTopoLattice>
__global__ void __launch_bounds__(EB * N * N * N, (kMinWaves<KIND, MODE, R>))
    element_kernel(KernelArgs<N, R> a) {
  constexpr int Q = N * N * N;
  using ST = typename StoreOf<S>::T;
  __shared__ R sb[EB * kBuffers * Lds<N>::FS];
  __shared__ R sv[EB * 24];
  __shared__ float sred[EB];
  const int le = threadIdx.x / Q;
  const int q = threadIdx.x - le * Q;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int e0 = blk * EB;
  const int e = e0 + le;
  const bool valid = e < a.L.n_cells;
  const CellPos c0 = cell_pos(a.L, e0);
  // stored data: blocks of W words per slot, packed in 8-byte groups (qword); the block base is
  // uniform across the workgroup and the lane offset follows the thread index
  constexpr int W = MODE == HX_STORE_TANGENT          ? 45
                    : MODE == HX_STORE_FINV_J         ? 10
                    : MODE == HX_STORE_SPATIAL        ? kSpatialWords<LAW>
                    : MODE == HX_STORE_SCALARS        ? kScalarWords<LAW>
                    : MODE == HX_STORE_SPATIAL_SCALARS ? kScalarWords<LAW>
                    : MODE == HX_STORE_TENSORS        ? kTensorWords<LAW>
                                                      : 0;
  constexpr int EBQ = EB * Q;
  const int64_t qblk = static_cast<int64_t>(blk) * block_words<ST>(W, EBQ);
  const int qi = threadIdx.x;

  // stored q-point data of this thread (apply), requested before the sum factorisation so that
  // its HBM latency overlaps the gather and the forward sweeps (the tensor stage's 31-35 words
  // would stay live through the sweeps and spill: they are loaded where they are used)
  constexpr int WA = KIND == 0 && MODE != HX_STORE_TENSORS ? W : 0;
  ST qv[WA > 0 ? WA : 1];
  if constexpr (WA > 0) {
    if (valid) {
      const ST* qd = static_cast<const ST*>(a.qdata) + qblk;
      constexpr int G = kPack<ST>;
#pragma unroll
      for (int g = 0; g < WA / G; ++g) load_group<NT>(qd + qword<ST, W>(g * G, EBQ, qi), qv + g * G);
#pragma unroll
      for (int w = WA / G * G; w < WA; ++w) {
        if constexpr (NT)
          qv[w] = load_stream(qd + qword<ST, W>(w, EBQ, qi));
        else
          qv[w] = qd[qword<ST, W>(w, EBQ, qi)];
      }
    }
  }

  constexpr bool kGeom = !(KIND == 0 && (MODE == HX_STORE_TANGENT || MODE == HX_STORE_SPATIAL));
  // stored geometry of this thread's q-point (curved or general meshes), requested early like the
  // stored data; the lattice of trilinear cells forms it from the vertices instead
  constexpr bool kGeoStored = kGeom && TOPO != kTopoLattice;
  R gq[kGeoStored ? kGeoWords : 1];
  if constexpr (kGeoStored) {
    const R* gp = a.geo + static_cast<int64_t>(blk) * kGeoWords * EBQ;
#pragma unroll
    for (int w = 0; w < kGeoWords; ++w) gq[w] = valid ? gp[w * EBQ + qi] : R(0);
  }
  if constexpr (kGeom && TOPO == kTopoLattice) load_vertices<N, EB>(a, sv, e0, c0);
  // K = J0^-1 and w det J0 at this thread's q-point
  auto geometry = [&](R* K) -> R {
    if constexpr (!kGeoStored) {
      return valid ? qpoint_geometry<N>(sv + le * 24, q, K) : R(0);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) K[i] = gq[i];
      return gq[9];
    }
  };
  // J0 itself (the spatial data): from the vertices, or as the inverse of the stored J0^-1
  auto jacobian_at = [&](const R* K, R* J0) {
    if constexpr (!kGeoStored) {
      qpoint_jacobian<N>(sv + le * 24, q, J0);
    } else {
      R A[9];
      adj3(K, A);
      const R inv = R(1) / (K[0] * A[0] + K[1] * A[3] + K[2] * A[6]);
#pragma unroll
      for (int i = 0; i < 9; ++i) J0[i] = A[i] * inv;
    }
  };
  if constexpr (KIND == 2 && S == kStoreF16) {
    if (q == 0) sred[le] = 0.0f;
  }

  R g0[9], g1[9], t[9];
  // the apply modes that interpolate the linearisation point u_k at every apply
  constexpr bool kRecompute = MODE == HX_STORE_NONE || MODE == HX_STORE_SPATIAL_RECOMPUTE ||
                              MODE == HX_STORE_SCALARS || MODE == HX_STORE_SPATIAL_SCALARS;
  if constexpr (KIND == 0 && kRecompute) {
    // linearisation point first (not masked), then the direction (masked)
    forward_vector<N, EB, false, TOPO>(a, sb, a.in1, e0, c0, le, q, g1);
    __syncthreads();
    forward_vector<N, EB, true, TOPO>(a, sb, a.in0, e0, c0, le, q, g0);
  } else if constexpr (KIND == 0) {
    forward_vector<N, EB, true, TOPO>(a, sb, a.in0, e0, c0, le, q, g0);
  } else {
    forward_vector<N, EB, false, TOPO>(a, sb, a.in0, e0, c0, le, q, g0);
  }

  const MaterialK<R>& m = a.c->m;
  Fib<R> fb{m.H4, m.H6, m.M4, m.M6};
  if constexpr (LAW == kFIBERC) {
    const R* f = a.fib + static_cast<int64_t>(valid ? e : e0) * kFibWords;
    fb = Fib<R>{f, f + 9, f + 18, f + 21};
  }
  if constexpr (KIND == 0 && MODE == HX_STORE_TANGENT) {
    // t = D g with the stored symmetric 9x9 tangent (45 planes, upper triangle row by row)
    R Dv[45];
    if (valid) {
#pragma unroll
      for (int w = 0; w < 45; ++w) Dv[w] = static_cast<R>(as_val(qv[w]));
    } else {
#pragma unroll
      for (int w = 0; w < 45; ++w) Dv[w] = R(0);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) t[i] = R(0);
    int w = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      t[i] += Dv[w] * g0[i];
      ++w;
#pragma unroll
      for (int j = i + 1; j < 9; ++j) {
        t[i] += Dv[w] * g0[j];
        t[j] += Dv[w] * g0[i];
        ++w;
      }
    }
    if constexpr (S == kStoreF16) {
      if (valid) {
        const R inv = R(1) / static_cast<R>(a.cscale[e]);
#pragma unroll
        for (int i = 0; i < 9; ++i) t[i] *= inv;
      }
    }
  } else if constexpr (KIND == 0 && MODE == HX_STORE_SPATIAL) {
    R d[W];
#pragma unroll
    for (int w = 0; w < W; ++w) d[w] = valid ? static_cast<R>(as_val(qv[w])) : R(0);
    spatial_action<LAW>(d, m, g0, t);
  } else if constexpr (KIND == 0 && (MODE == HX_STORE_SPATIAL_RECOMPUTE || MODE == HX_STORE_SPATIAL_SCALARS)) {
    // the spatial data formed from u_k at this apply (with the law's scalars recomputed, or as
    // stored), then the spatial action
    R K[9], H[9];
    const R wdet = geometry(K);
    to_physical(g1, K, H);
    QState<R> st;
    if constexpr (MODE == HX_STORE_SPATIAL_SCALARS) {
      R ds[W];
#pragma unroll
      for (int w = 0; w < W; ++w) ds[w] = valid ? static_cast<R>(as_val(qv[w])) : R(0);
      state_from_scalars<LAW>(H, ds, m, st);
    } else {
      if constexpr (kIsFiber<LAW>) {
        if (a.act && valid) st.forced = a.act[static_cast<int64_t>(blk) * EBQ + qi];
      }
      R E[9];
      state_from_H<LAW>(H, m, fb, st, E);
    }
    R J0[9];
    jacobian_at(K, J0);
    constexpr int WS = kSpatialWords<LAW>;
    R d[WS];
    spatial_words_at<LAW>(H, st, m, fb, J0, g1, wdet, d);
    if (!valid) {
#pragma unroll
      for (int w = 0; w < WS; ++w) d[w] = R(0);
    }
    spatial_action<LAW>(d, m, g0, t);
  } else if constexpr (KIND == 0 && MODE == HX_STORE_TENSORS) {
    R K[9];
    const R wdet = geometry(K);
    R d[W];
    const ST* qd = static_cast<const ST*>(a.qdata) + qblk;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if constexpr (NT)
        d[w] = valid ? static_cast<R>(as_val(load_stream(qd + qword<ST, W>(w, EBQ, qi)))) : R(0);
      else
        d[w] = valid ? static_cast<R>(as_val(qd[qword<ST, W>(w, EBQ, qi)])) : R(0);
    }
    R G[9], Pd[9];
    to_physical(g0, K, G);
    tensor_action<LAW>(d, m, fb, G, Pd);
    to_reference(Pd, K, wdet, t);
  } else if constexpr (KIND == 0) {
    R K[9];
    const R wdet = geometry(K);
    QState<R> st;
    if constexpr (kIsFiber<LAW>) {
      if (a.act && valid) st.forced = a.act[static_cast<int64_t>(blk) * EBQ + qi];
    }
    if constexpr (MODE == HX_STORE_NONE) {
      R H[9], E[9];
      to_physical(g1, K, H);
      state_from_H<LAW>(H, m, fb, st, E);
    } else if constexpr (MODE == HX_STORE_SCALARS) {
      R H[9], d[W];
      to_physical(g1, K, H);
#pragma unroll
      for (int w = 0; w < W; ++w) d[w] = valid ? static_cast<R>(as_val(qv[w])) : R(0);
      state_from_scalars<LAW>(H, d, m, st);
    } else {
      R Fi[9], Jm;
      if (valid) {
#pragma unroll
        for (int w = 0; w < 9; ++w) Fi[w] = static_cast<R>(as_val(qv[w]));
        Jm = static_cast<R>(as_val(qv[9]));
      } else {
#pragma unroll
        for (int w = 0; w < 9; ++w) Fi[w] = R(w % 4 == 0);
        Jm = R(0);
      }
      state_from_finv<LAW>(Fi, Jm, m, fb, st);
    }
    R G[9], Pd[9];
    to_physical(g0, K, G);
    action<LAW>(st, m, fb, G, Pd);
    to_reference(Pd, K, wdet, t);
  } else if constexpr (KIND == 1) {
    R K[9], H[9], E[9];
    const R wdet = geometry(K);
    to_physical(g0, K, H);
    QState<R> st;
    state_from_H<LAW>(H, m, fb, st, E);
    if constexpr (MODE == HX_STORE_SPATIAL) {
      // over the spatial configuration: t = w det J0 tau J_t^-T; the spatial data carries
      // sqrt(w det J0) J_t^-1 and tau
      R J0[9];
      jacobian_at(K, J0);
      constexpr int WS = kSpatialWords<LAW>;
      R d[WS], tau[9];
      spatial_words_at<LAW>(H, st, m, fb, J0, g0, wdet, d);
      sym_to_full(d + 9, tau);
      to_reference(tau, d, sqrt(wdet), t);
    } else {
      R P[9];
      stress_P<LAW>(st, E, m, fb, P);
      to_reference(P, K, wdet, t);
    }
  } else {
    // linearisation update (always FP64 arithmetic)
    R K[9], H[9], E[9];
    const R wdet = geometry(K);
    to_physical(g0, K, H);
    QState<R> st;
    const bool ok = state_from_H<LAW>(H, m, fb, st, E);
    int bad = 0;
    if (valid && !ok) bad |= kFlagInverted;
    if constexpr (kIsFiber<LAW>) {
      if (a.act_w && valid) a.act_w[static_cast<int64_t>(blk) * EBQ + qi] = static_cast<uint8_t>(st.bits);
    }
    ST* qw = static_cast<ST*>(a.qdata_w) + qblk;
    if constexpr (MODE == HX_STORE_FINV_J) {
      R chk = st.Jm;
#pragma unroll
      for (int w = 0; w < 9; ++w) chk += st.Fi[w];
      if (valid && !isfinite(chk)) bad |= kFlagNonFinite;
      if (valid) {
#pragma unroll
        for (int w = 0; w < 9; ++w) store_val(qw + qword<ST, W>(w, EBQ, qi), st.Fi[w]);
        store_val(qw + qword<ST, W>(9, EBQ, qi), st.Jm);
      }
    } else if constexpr (MODE == HX_STORE_TANGENT) {
      // columns of the reference tangent: unit reference gradient e_k (x) e_b maps to the
      // physical gradient G[k][J] = K[b][J]
      R Dm[81];
#pragma unroll
      for (int col = 0; col < 9; ++col) {
        const int kk = col / 3, bb = col % 3;
        R G[9], Pd[9], tc[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) G[i] = R(0);
#pragma unroll
        for (int J = 0; J < 3; ++J) G[3 * kk + J] = K[3 * bb + J];
        action<LAW>(st, m, fb, G, Pd);
        to_reference(Pd, K, wdet, tc);
#pragma unroll
        for (int r = 0; r < 9; ++r) Dm[9 * r + col] = tc[r];
      }
      R Dsym[45];
      int w = 0;
      R chk = R(0), amax = R(0);
#pragma unroll
      for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = i; j < 9; ++j) {
          Dsym[w] = R(0.5) * (Dm[9 * i + j] + Dm[9 * j + i]);
          chk += Dsym[w];
          amax = fmax(amax, fabs(Dsym[w]));
          ++w;
        }
      if (valid && !isfinite(chk)) bad |= kFlagNonFinite;
      R scale = R(1);
      if constexpr (S == kStoreF16) {
        // per-cell power-of-two scale: largest magnitude maps below 2^14
        if (valid && isfinite(amax)) atomicMax(reinterpret_cast<unsigned*>(&sred[le]),
                                               __float_as_uint(static_cast<float>(amax)));
        __syncthreads();
        const float cm = sred[le];
        int ex2 = 0;
        if (cm > 0.0f) frexpf(cm, &ex2);
        const float sc = ldexpf(1.0f, 14 - ex2);
        scale = static_cast<R>(sc);
        if (valid && q == 0) a.cscale_w[e] = sc;
      }
      if (valid) {
#pragma unroll
        for (int i = 0; i < 45; ++i) store_val(qw + qword<ST, W>(i, EBQ, qi), Dsym[i] * scale);
      }
    } else if constexpr (MODE == HX_STORE_SCALARS || MODE == HX_STORE_TENSORS) {
      R dw[W];
      if constexpr (MODE == HX_STORE_SCALARS)
        scalar_words<LAW>(st, dw);
      else
        tensor_words<LAW>(st, E, m, fb, dw);
      R chk = R(0);
#pragma unroll
      for (int w = 0; w < W; ++w) chk += dw[w];
      if (valid && !isfinite(chk)) bad |= kFlagNonFinite;
      if (valid) {
#pragma unroll
        for (int w = 0; w < W; ++w) store_val(qw + qword<ST, W>(w, EBQ, qi), dw[w]);
      }
    } else if constexpr (MODE == HX_STORE_SPATIAL) {
      R J0[9], dw[W];
      jacobian_at(K, J0);
      spatial_words_at<LAW>(H, st, m, fb, J0, g0, wdet, dw);
      R chk = R(0);
#pragma unroll
      for (int w = 0; w < W; ++w) chk += dw[w];
      if (valid && !isfinite(chk)) bad |= kFlagNonFinite;
      if (valid) {
#pragma unroll
        for (int w = 0; w < W; ++w) store_val(qw + qword<ST, W>(w, EBQ, qi), dw[w]);
      }
    } else {
      R chk = st.Jm;
      if (valid && !isfinite(chk)) bad |= kFlagNonFinite;
    }
    if (bad) atomicOr(a.flag, bad);
    return;
  }
  if constexpr (KIND != 2) {
    if (!valid) {
#pragma unroll
      for (int i = 0; i < 9; ++i) t[i] = R(0);
    }
    backward_scatter<N, EB, TOPO>(a, sb, e0, c0, le, q, t);
  }
}

// ------------------------------------------------------------------------------------------
// Diagonal and nodal 3x3 blocks of the linearised operator from the stored reference tangent
// (multigrid smoothers). For node a = (i,j,k) and components c, d:
//   K_(c a)(d a) = sum_q sum_{al,be} D_(c al)(d be)(q) dphi_a/dxi_al(q) dphi_a/dxi_be(q),
// and dphi_a/dxi_al dphi_a/dxi_be factorises per direction into products of the 1D tables
// B (values) and G (derivatives of the nodal basis at the Gauss points), so each of the six
// unique (al, be) pairs (the product is symmetric in al, be) is three transposed 1D sweeps, with
// the coefficient D_(c al)(d be) + D_(c be)(d al) for al < be. The three fields of a pass are the
// components c = d (OFF false: the diagonal) or the pairs (0,1), (0,2), (1,2) (OFF true).
// ------------------------------------------------------------------------------------------
template <int N, int AL, int BE, int DIR, typename R>
__device__ __forceinline__ R diag_coef(int q, int i) {
  const R x = (DIR == AL) ? Tab1D<N, R>::G[q * N + i] : Tab1D<N, R>::B[q * N + i];
  const R y = (DIR == BE) ? Tab1D<N, R>::G[q * N + i] : Tab1D<N, R>::B[q * N + i];
  return x * y;
}

template <int N, int AL, int BE, int DIR, typename R>
__device__ __forceinline__ void diag_apply1d(const R* in, R* out) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R acc = R(0);
#pragma unroll
    for (int m = 0; m < N; ++m) acc = fma(diag_coef<N, AL, BE, DIR, R>(m, i), in[m], acc);
    out[i] = acc;
  }
}

__host__ __device__ constexpr int packed_index(int a, int b) { return a * 9 - a * (a + 1) / 2 + b; }

// components (c, d) of field f of a diagonal (OFF false) or off-diagonal (OFF true) pass
template <bool OFF>
__host__ __device__ constexpr int pair_c(int f) { return OFF ? (f == 2 ? 1 : 0) : f; }
template <bool OFF>
__host__ __device__ constexpr int pair_d(int f) { return OFF ? (f == 0 ? 1 : 2) : f; }

template <int N, int EB, int AL, int BE, bool OFF, typename R>
__device__ __forceinline__ void diag_pair(R* sb, const R* Dv, int le_me, int q_me) {
  constexpr int Q = N * N * N;
  constexpr int CB = 6 * Lds<N>::FS;
  R* cb = sb + le_me * CB;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int c = pair_c<OFF>(f), d = pair_d<OFF>(f);
    // D is symmetric, stored as its upper triangle; 3c + AL <= 3d + BE always holds here
    R coef = Dv[packed_index(3 * c + AL, 3 * d + BE)];
    if constexpr (AL != BE) {
      const int r = 3 * c + BE, k = 3 * d + AL;
      coef += r <= k ? Dv[packed_index(r, k)] : Dv[packed_index(k, r)];
    }
    cb[f * Lds<N>::FS + lds_q<N>(q_me)] = coef;
  }
  __syncthreads();
  pencil_jobs<N, EB, 3>([&](int le, int c, int i, int j) __attribute__((always_inline)) {
    R in[N], out[N];
    R* buf = sb + le * CB + c * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 2>(i, j, m)];
    diag_apply1d<N, AL, BE, 2>(in, out);
#pragma unroll
    for (int m = 0; m < N; ++m) buf[pidx<N, 2>(i, j, m)] = out[m];
  });
  __syncthreads();
  pencil_jobs<N, EB, 3>([&](int le, int c, int i, int k) __attribute__((always_inline)) {
    R in[N], out[N];
    R* buf = sb + le * CB + c * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 1>(i, k, m)];
    diag_apply1d<N, AL, BE, 1>(in, out);
#pragma unroll
    for (int m = 0; m < N; ++m) buf[pidx<N, 1>(i, k, m)] = out[m];
  });
  __syncthreads();
  pencil_jobs<N, EB, 3>([&](int le, int c, int j, int k) __attribute__((always_inline)) {
    R in[N], out[N];
    R* buf = sb + le * CB + c * Lds<N>::FS;
    R* acc = sb + le * CB + (3 + c) * Lds<N>::FS;
#pragma unroll
    for (int m = 0; m < N; ++m) in[m] = buf[pidx<N, 0>(j, k, m)];
    diag_apply1d<N, AL, BE, 0>(in, out);
#pragma unroll
    for (int m = 0; m < N; ++m) acc[pidx<N, 0>(j, k, m)] += out[m];
  });
  __syncthreads();
}

template <int N, int EB, typename R, int S, bool OFF>
__global__ void __launch_bounds__(EB * N * N * N) diag_kernel(KernelArgs<N, R> a) {
  constexpr int Q = N * N * N;
  constexpr int EBQ = EB * Q;
  using ST = typename StoreOf<S>::T;
  __shared__ R sb[EB * 6 * Lds<N>::FS];
  const int le = threadIdx.x / Q;
  const int q = threadIdx.x - le * Q;
  const int e0 = blockIdx.x * EB;
  const int e = e0 + le;
  const bool valid = e < a.L.n_cells;
  const CellPos c0 = cell_pos(a.L, e0);
  const ST* qd = static_cast<const ST*>(a.qdata) + static_cast<int64_t>(blockIdx.x) * block_words<ST>(45, EBQ);
  R Dv[45];
  R inv = R(1);
  if constexpr (S == kStoreF16) {
    if (valid) inv = R(1) / static_cast<R>(a.cscale[e]);
  }
#pragma unroll
  for (int w = 0; w < 45; ++w)
    Dv[w] = valid ? static_cast<R>(load_val(qd + qword<ST, 45>(w, EBQ, threadIdx.x))) * inv : R(0);
  R* cb = sb + le * 6 * Lds<N>::FS;
#pragma unroll
  for (int c = 0; c < 3; ++c) cb[(3 + c) * Lds<N>::FS + lds_q<N>(q)] = R(0);
  diag_pair<N, EB, 0, 0, OFF>(sb, Dv, le, q);
  diag_pair<N, EB, 1, 1, OFF>(sb, Dv, le, q);
  diag_pair<N, EB, 2, 2, OFF>(sb, Dv, le, q);
  diag_pair<N, EB, 0, 1, OFF>(sb, Dv, le, q);
  diag_pair<N, EB, 0, 2, OFF>(sb, Dv, le, q);
  diag_pair<N, EB, 1, 2, OFF>(sb, Dv, le, q);
  if (!valid) return;
  const Lattice& L = a.L;
  const int i = q % N, j = (q / N) % N, k = q / (N * N);
  constexpr int P = N - 1;
  const CellPos cp = cell_advance(L, c0, le);
  bool cons;
  const int64_t node = node_of(L, cp, i, j, k, cons);
  if (cons) return;
  const bool inner = i > 0 && i < P && j > 0 && j < P && k > 0 && k < P;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const R v = cb[(3 + c) * Lds<N>::FS + lds_q<N>(q)];
    R* dst = a.out + c * L.n_nodes + node;
    if (inner)
      *dst = v;
    else
      unsafeAtomicAdd(dst, v);
  }
}

}  // namespace hx
