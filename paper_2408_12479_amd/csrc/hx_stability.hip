// Forward-stability evaluation of the q-point functions (Section 7.1).
//
// One thread per sampled displacement gradient H: the first Piola-Kirchhoff stress P(I + H) and
// its directional derivative P'(H)[G], in FP64 or FP32, either with the stable forms of Section 4
// (the very functions the operator kernels run) or with the standard forms of Section 3:
// C = F^T F, J = det F, C^-1 by inversion of C, ln J and J^(-2/3) evaluated from J itself.
#include <hip/hip_runtime.h>

#include <cmath>

#include "hx.h"
#include "hx_kernels.hpp"

namespace hx {
namespace {

template <typename R>
__device__ __forceinline__ void matmul3(const R* A, const R* B, R* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

template <typename R>
__device__ __forceinline__ void matmul3_tn(const R* A, const R* B, R* C) {  // C = A^T B
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}

template <typename R>
__device__ __forceinline__ void inv3(const R* A, R* Ai) {
  R adj[9];
  adj3(A, adj);
  const R inv = R(1) / (A[0] * adj[0] + A[1] * adj[3] + A[2] * adj[6]);
#pragma unroll
  for (int i = 0; i < 9; ++i) Ai[i] = adj[i] * inv;
}

__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __forceinline__ double m_cbrt(double x) { return cbrt(x); }
__device__ __forceinline__ float m_cbrt(float x) { return cbrtf(x); }

// Standard forms: S and D_u S[G] from C, J = det F and C^-1 = inv(C) (Section 3 and the chain
// rule: D C = F^T G + G^T F, D C^-1 = -C^-1 (D C) C^-1, D ln J = C^-1 : (F^T G)).
template <int LAW, typename R>
__device__ void standard_forms(const R* H, const R* G, const MaterialK<R>& m, R* P, R* Pd) {
  R F[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) F[i] = H[i];
  F[0] += R(1);
  F[4] += R(1);
  F[8] += R(1);
  R C[9], Ci[9], FtG[9], dC[9];
  matmul3_tn(F, F, C);
  inv3(C, Ci);
  const R J = det3(F);
  const R lnJ = m_log(J);
  matmul3_tn(F, G, FtG);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dC[3 * i + j] = FtG[3 * i + j] + FtG[3 * j + i];
  R tr = R(0);  // D ln J = C^-1 : F^T G
#pragma unroll
  for (int i = 0; i < 9; ++i) tr += Ci[i] * FtG[i];
  R T[9], dCi[9];
  matmul3(Ci, dC, T);
  matmul3(T, Ci, dCi);
#pragma unroll
  for (int i = 0; i < 9; ++i) dCi[i] = -dCi[i];
  R S[9], dS[9];
  if constexpr (LAW == kCNH) {
    // S = mu (I - C^-1) + 2 lambda ln J C^-1
    const R a = R(2) * m.lam * lnJ - m.mu;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      S[i] = a * Ci[i];
      dS[i] = R(2) * m.lam * tr * Ci[i] + a * dCi[i];
    }
    S[0] += m.mu;
    S[4] += m.mu;
    S[8] += m.mu;
  } else {
    // S = mu J^-2/3 I + c1 C^-1, c1 = kappa/2 (J^2 - 1) - mu/3 J^-2/3 I1, I1 = tr C
    const R cb = m_cbrt(J);
    const R Jp = R(1) / (cb * cb);
    const R I1 = C[0] + C[4] + C[8];
    const R c1 = R(0.5) * m.kappa * (J * J - R(1)) - m.mu / R(3) * Jp * I1;
    const R dJp = -R(2) / R(3) * Jp * tr;
    const R dI1 = dC[0] + dC[4] + dC[8];
    const R dc1 = m.kappa * J * J * tr - m.mu / R(3) * (dJp * I1 + Jp * dI1);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      S[i] = c1 * Ci[i];
      dS[i] = dc1 * Ci[i] + c1 * dCi[i];
    }
    S[0] += m.mu * Jp;
    S[4] += m.mu * Jp;
    S[8] += m.mu * Jp;
    dS[0] += m.mu * dJp;
    dS[4] += m.mu * dJp;
    dS[8] += m.mu * dJp;
    if constexpr (kIsFiber<LAW>) {
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const R* Hf = f == 0 ? m.H4 : m.H6;
        const R* M = f == 0 ? m.M4 : m.M6;
        R Ei = -(Hf[0] + Hf[4] + Hf[8]), dEi = R(0), Istar = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          Ei += Hf[i] * C[i];
          dEi += Hf[i] * dC[i];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) Istar += M[i] * C[3 * i + j] * M[j];
        if (Istar > R(1)) {
          const R c3 = R(2) * m.k1 * m_exp(m.k2 * Ei * Ei);
          const R dcoef = c3 * (R(2) * m.k2 * Ei * Ei + R(1)) * dEi;
#pragma unroll
          for (int i = 0; i < 9; ++i) {
            S[i] += c3 * Ei * Hf[i];
            dS[i] += dcoef * Hf[i];
          }
        }
      }
    }
  }
  // P = F S, P' = G S + F D_u S
  R GS[9], FdS[9];
  matmul3(F, S, P);
  matmul3(G, S, GS);
  matmul3(F, dS, FdS);
#pragma unroll
  for (int i = 0; i < 9; ++i) Pd[i] = GS[i] + FdS[i];
}

template <typename R, int LAW, int FORM>
__global__ void qpoint_eval_kernel(MaterialK<R> m, int64_t n, const double* __restrict__ Hin,
                                   const double* __restrict__ Gin, double* __restrict__ Pout,
                                   double* __restrict__ dPout) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n) return;
  R H[9], G[9], P[9], Pd[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    H[i] = static_cast<R>(Hin[9 * s + i]);
    G[i] = static_cast<R>(Gin[9 * s + i]);
  }
  if constexpr (FORM == 0) {
    const Fib<R> fb{m.H4, m.H6, m.M4, m.M6};
    QState<R> st;
    R E[9];
    state_from_H<LAW>(H, m, fb, st, E);
    stress_P<LAW>(st, E, m, fb, P);
    action<LAW>(st, m, fb, G, Pd);
  } else {
    standard_forms<LAW>(H, G, m, P, Pd);
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    Pout[9 * s + i] = static_cast<double>(P[i]);
    dPout[9 * s + i] = static_cast<double>(Pd[i]);
  }
}

template <typename R>
MaterialK<R> material_k(const hx_material& mat, int jpow_iters) {
  MaterialK<R> m{};
  m.mu = static_cast<R>(mat.mu);
  m.lam = static_cast<R>(mat.lambda);
  m.kappa = static_cast<R>(mat.kappa);
  m.k1 = static_cast<R>(mat.k1);
  m.k2 = static_cast<R>(mat.k2);
  for (int i = 0; i < 9; ++i) {
    m.H4[i] = static_cast<R>(mat.H4[i]);
    m.H6[i] = static_cast<R>(mat.H6[i]);
  }
  for (int i = 0; i < 3; ++i) {
    m.M4[i] = static_cast<R>(mat.M4[i]);
    m.M6[i] = static_cast<R>(mat.M6[i]);
  }
  m.jpow_iters = jpow_iters;
  return m;
}

template <typename R, int LAW>
hipError_t launch_eval(const hx_material& mat, int form, int jpow, int64_t n, const double* H, const double* G,
                       double* P, double* dP, hipStream_t s) {
  const MaterialK<R> m = material_k<R>(mat, jpow);
  const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
  if (form == 0)
    qpoint_eval_kernel<R, LAW, 0><<<blocks, 256, 0, s>>>(m, n, H, G, P, dP);
  else
    qpoint_eval_kernel<R, LAW, 1><<<blocks, 256, 0, s>>>(m, n, H, G, P, dP);
  return hipGetLastError();
}

template <typename R>
hipError_t by_law(const hx_material& mat, int form, int jpow, int64_t n, const double* H, const double* G,
                  double* P, double* dP, hipStream_t s) {
  switch (mat.law) {
    case HX_LAW_CNH: return launch_eval<R, kCNH>(mat, form, jpow, n, H, G, P, dP, s);
    case HX_LAW_INH: return launch_eval<R, kINH>(mat, form, jpow, n, H, G, P, dP, s);
    case HX_LAW_FIBER: return launch_eval<R, kFIBER>(mat, form, jpow, n, H, G, P, dP, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace
}  // namespace hx

extern "C" hx_status hx_qpoint_eval(const hx_material* mat, int32_t form, hx_precision prec, int32_t jpow_iters,
                                    int64_t n, const double* H, const double* G, double* P, double* dP,
                                    void* stream) {
  if (!mat || n < 0 || (n > 0 && (!H || !G || !P || !dP))) return HX_E_ARG;
  if (form != 0 && form != 1) return HX_E_ARG;
  if (prec != HX_FP64 && prec != HX_FP32) return HX_E_ARG;
  if (jpow_iters < 0 || jpow_iters > 16) return HX_E_ARG;
  if (mat->law != HX_LAW_CNH && mat->law != HX_LAW_INH && mat->law != HX_LAW_FIBER) return HX_E_ARG;
  if (n == 0) return HX_OK;
  if (n > (int64_t(1) << 31) * 256) return HX_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const hipError_t e = prec == HX_FP64 ? hx::by_law<double>(*mat, form, jpow_iters, n, H, G, P, dP, s)
                                       : hx::by_law<float>(*mat, form, jpow_iters, n, H, G, P, dP, s);
  return e == hipSuccess ? HX_OK : HX_E_HIP;
}
