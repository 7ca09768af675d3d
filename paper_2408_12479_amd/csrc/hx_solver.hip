// p-multigrid preconditioner and mixed-precision Newton-Krylov solve (Section 6; Algorithm 1).
//
// Levels share one structured mesh and differ in degree (p -> ... -> 1). Transfers are the
// polynomial embedding of the coarse space into the fine space (prolongation) and its transpose
// (restriction); the linearisation point is moved down by interpolation at the coarse nodes.
// Smoothing is Chebyshev-accelerated Jacobi with the inverse diagonal of the level operator
// (computed matrix-free from the stored tangent) and a power-iteration estimate of the largest
// eigenvalue; the coarsest level is solved approximately by a higher-degree Chebyshev iteration,
// which keeps the V-cycle a fixed linear operator. The V-cycle runs in FP32 or FP64 and is
// captured once per linearisation into a HIP graph. The outer Krylov solver is a flexible
// preconditioned CG in FP64 on the finest FP64 operator.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "hx.h"
#include "hx_context.hpp"
#include "hx_kernels.hpp"
#include "hx_tables.hpp"

namespace hx {
namespace {

int grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, 8192)));
}

#define HX_GRID_LOOP(i, n)                                                               \
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < (n); \
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)

// ---------------------------------------------------------------- vector kernels
template <typename T>
__global__ void k_fill(T* x, T v, int64_t n) {
  HX_GRID_LOOP(i, n) x[i] = v;
}

template <typename T>
__global__ void k_axpby(T* y, T a, const T* x, T b, int64_t n) {  // y = a x + b y
  HX_GRID_LOOP(i, n) y[i] = a * x[i] + b * y[i];
}

template <typename S, typename T>
__global__ void k_convert(const S* in, T* out, int64_t n) {
  HX_GRID_LOOP(i, n) out[i] = static_cast<T>(in[i]);
}

// Chebyshev: d = c * dinv * (b - t); x = (first ? d : x + d)     (t may be null: t = 0)
template <typename T>
__global__ void k_cheb_first(T* x, T* d, const T* b, const T* t, const T* dinv, T c, int first,
                             int64_t n) {
  HX_GRID_LOOP(i, n) {
    const T r = b[i] - (t ? t[i] : T(0));
    const T di = c * dinv[i] * r;
    d[i] = di;
    x[i] = first ? di : x[i] + di;
  }
}

// Chebyshev: d = c1 d + c2 dinv (b - t); x += d
template <typename T>
__global__ void k_cheb_step(T* x, T* d, const T* b, const T* t, const T* dinv, T c1, T c2,
                            int64_t n) {
  HX_GRID_LOOP(i, n) {
    const T di = c1 * d[i] + c2 * dinv[i] * (b[i] - t[i]);
    d[i] = di;
    x[i] += di;
  }
}

// out[k] += sum a_k b_k for up to three pairs, FP64 accumulation
template <typename T>
__global__ void k_dots(const T* a0, const T* b0, const T* a1, const T* b1, const T* a2,
                       const T* b2, int npairs, double* out, int64_t n) {
  double s[3] = {0.0, 0.0, 0.0};
  HX_GRID_LOOP(i, n) {
    s[0] += static_cast<double>(a0[i]) * b0[i];
    if (npairs > 1) s[1] += static_cast<double>(a1[i]) * b1[i];
    if (npairs > 2) s[2] += static_cast<double>(a2[i]) * b2[i];
  }
  __shared__ double red[3][256];
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < npairs; ++k) unsafeAtomicAdd(out + k, red[k][0]);
}

__device__ __forceinline__ bool node_constrained(const Lattice& L, int64_t node) {
  const int I = static_cast<int>(node % L.Nx);
  const int J = static_cast<int>((node / L.Nx) % L.Ny);
  const int K = static_cast<int>(node / (static_cast<int64_t>(L.Nx) * L.Ny));
  return cons_x(L, I) || cons_yz(L, J, K);
}

template <typename T>
__global__ void k_zero_constrained(T* x, Lattice L) {
  HX_GRID_LOOP(i, 3 * L.n_nodes) if (node_constrained(L, i % L.n_nodes)) x[i] = T(0);
}

// inverse diagonal: constrained rows are identity rows
template <typename T>
__global__ void k_diag_finish(T* d, Lattice L) {
  HX_GRID_LOOP(i, 3 * L.n_nodes) {
    const T v = node_constrained(L, i % L.n_nodes) ? T(1) : d[i];
    d[i] = T(1) / v;
  }
}

// deterministic pseudo-random start vector (integer hash), constrained entries zero
template <typename T>
__global__ void k_hash_vector(T* x, Lattice L) {
  HX_GRID_LOOP(i, 3 * L.n_nodes) {
    uint32_t h = static_cast<uint32_t>(i) * 2654435761u + 0x9e3779b9u;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    const T v = static_cast<T>(h & 0xffffff) / static_cast<T>(0x1000000) - T(0.5);
    x[i] = node_constrained(L, i % L.n_nodes) ? T(0) : v;
  }
}

// ---------------------------------------------------------------- transfers between degrees
// does cell (cp) own its local node with index l along a direction with nc cells, degree p?
__device__ __forceinline__ bool owns(int l, int p, int cell, int ncell, bool periodic) {
  return l < p || (!periodic && cell == ncell - 1);
}

__device__ __forceinline__ bool owns_node(const Lattice& L, const CellPos& cp, int i, int j,
                                          int k, int periodic) {
  return owns(i, L.p, cp.ex, L.nx, periodic & 1) && owns(j, L.p, cp.ey, L.ny, periodic & 2) &&
         owns(k, L.p, cp.ez, L.nz, periodic & 4);
}

// xf += P xc: each fine node written once, by its owning cell
template <int NF, int NC, typename T>
__global__ void __launch_bounds__(NF* NF* NF) k_prolong_add(const T* __restrict__ xc,
                                                            T* __restrict__ xf, Lattice Lf,
                                                            Lattice Lc, int periodic) {
  constexpr int QF = NF * NF * NF, QC = NC * NC * NC;
  __shared__ T sc[3 * QC];
  const int e = blockIdx.x;
  const CellPos cp = cell_pos(Lf, e);
  const int t = threadIdx.x;
  if (t < QC) {
    bool cons;
    const int64_t node = node_of(Lc, cp, t % NC, (t / NC) % NC, t / (NC * NC), cons);
    for (int c = 0; c < 3; ++c) sc[c * QC + t] = xc[c * Lc.n_nodes + node];
  }
  __syncthreads();
  const int i = t % NF, j = (t / NF) % NF, k = t / (NF * NF);
  if (!owns_node(Lf, cp, i, j, k, periodic)) return;
  T v[3] = {T(0), T(0), T(0)};
  for (int cc = 0; cc < NC; ++cc)
    for (int b = 0; b < NC; ++b) {
      const T wjk = Transfer1D<NF, NC, T>::Icf[j * NC + b] * Transfer1D<NF, NC, T>::Icf[k * NC + cc];
      for (int a = 0; a < NC; ++a) {
        const T w = wjk * Transfer1D<NF, NC, T>::Icf[i * NC + a];
        const int l = a + NC * (b + NC * cc);
        v[0] += w * sc[l];
        v[1] += w * sc[QC + l];
        v[2] += w * sc[2 * QC + l];
      }
    }
  bool cons;
  const int64_t node = node_of(Lf, cp, i, j, k, cons);
  for (int c = 0; c < 3; ++c) xf[c * Lf.n_nodes + node] += v[c];
  (void)QF;
}

// rc += P^T rf (rc zeroed by the caller)
template <int NF, int NC, typename T>
__global__ void __launch_bounds__(NF* NF* NF) k_restrict_add(const T* __restrict__ rf,
                                                             T* __restrict__ rc, Lattice Lf,
                                                             Lattice Lc, int periodic) {
  constexpr int QF = NF * NF * NF, QC = NC * NC * NC;
  __shared__ T sf[3 * QF];
  const int e = blockIdx.x;
  const CellPos cp = cell_pos(Lf, e);
  const int t = threadIdx.x;
  {
    const int i = t % NF, j = (t / NF) % NF, k = t / (NF * NF);
    const bool own = owns_node(Lf, cp, i, j, k, periodic);
    bool cons;
    const int64_t node = node_of(Lf, cp, i, j, k, cons);
    for (int c = 0; c < 3; ++c) sf[c * QF + t] = own ? rf[c * Lf.n_nodes + node] : T(0);
  }
  __syncthreads();
  if (t >= QC) return;
  const int a = t % NC, b = (t / NC) % NC, cc = t / (NC * NC);
  T v[3] = {T(0), T(0), T(0)};
  for (int k = 0; k < NF; ++k)
    for (int j = 0; j < NF; ++j) {
      const T wjk = Transfer1D<NF, NC, T>::Icf[j * NC + b] * Transfer1D<NF, NC, T>::Icf[k * NC + cc];
      for (int i = 0; i < NF; ++i) {
        const T w = wjk * Transfer1D<NF, NC, T>::Icf[i * NC + a];
        const int l = i + NF * (j + NF * k);
        v[0] += w * sf[l];
        v[1] += w * sf[QF + l];
        v[2] += w * sf[2 * QF + l];
      }
    }
  bool cons;
  const int64_t node = node_of(Lc, cp, a, b, cc, cons);
  if (cons) return;
  for (int c = 0; c < 3; ++c) unsafeAtomicAdd(rc + c * Lc.n_nodes + node, v[c]);
}

// uc = uf at the coarse nodes (each coarse node written once, by its owning cell)
template <int NF, int NC>
__global__ void __launch_bounds__(NF* NF* NF) k_interp_down(const double* __restrict__ uf,
                                                            double* __restrict__ uc, Lattice Lf,
                                                            Lattice Lc, int periodic) {
  constexpr int QF = NF * NF * NF, QC = NC * NC * NC;
  __shared__ double sf[3 * QF];
  const int e = blockIdx.x;
  const CellPos cp = cell_pos(Lf, e);
  const int t = threadIdx.x;
  {
    bool cons;
    const int64_t node = node_of(Lf, cp, t % NF, (t / NF) % NF, t / (NF * NF), cons);
    for (int c = 0; c < 3; ++c) sf[c * QF + t] = uf[c * Lf.n_nodes + node];
  }
  __syncthreads();
  if (t >= QC) return;
  const int a = t % NC, b = (t / NC) % NC, cc = t / (NC * NC);
  if (!owns_node(Lc, cp, a, b, cc, periodic)) return;
  double v[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < NF; ++k)
    for (int j = 0; j < NF; ++j) {
      const double wjk = Transfer1D<NF, NC, double>::Jfc[b * NF + j] * Transfer1D<NF, NC, double>::Jfc[cc * NF + k];
      for (int i = 0; i < NF; ++i) {
        const double w = wjk * Transfer1D<NF, NC, double>::Jfc[a * NF + i];
        const int l = i + NF * (j + NF * k);
        v[0] += w * sf[l];
        v[1] += w * sf[QF + l];
        v[2] += w * sf[2 * QF + l];
      }
    }
  bool cons;
  const int64_t node = node_of(Lc, cp, a, b, cc, cons);
  for (int c = 0; c < 3; ++c) uc[c * Lc.n_nodes + node] = v[c];
}

// kind: 0 prolong_add, 1 restrict_add, 2 interp_down
template <int NF, int NC, typename T>
hipError_t launch_transfer(int kind, const void* in, void* out, const Lattice& Lf,
                           const Lattice& Lc, int periodic, hipStream_t s) {
  const dim3 grid(Lf.n_cells), block(NF * NF * NF);
  if (kind == 0)
    k_prolong_add<NF, NC, T><<<grid, block, 0, s>>>(static_cast<const T*>(in), static_cast<T*>(out), Lf, Lc, periodic);
  else if (kind == 1)
    k_restrict_add<NF, NC, T><<<grid, block, 0, s>>>(static_cast<const T*>(in), static_cast<T*>(out), Lf, Lc, periodic);
  else
    k_interp_down<NF, NC><<<grid, block, 0, s>>>(static_cast<const double*>(in), static_cast<double*>(out), Lf, Lc, periodic);
  return hipGetLastError();
}

template <typename T, int NF>
hipError_t transfer_nc(int nc, int kind, const void* in, void* out, const Lattice& Lf,
                       const Lattice& Lc, int periodic, hipStream_t s) {
  switch (nc) {
    case 2: if constexpr (NF > 2) return launch_transfer<NF, 2, T>(kind, in, out, Lf, Lc, periodic, s); break;
    case 3: if constexpr (NF > 3) return launch_transfer<NF, 3, T>(kind, in, out, Lf, Lc, periodic, s); break;
    case 4: if constexpr (NF > 4) return launch_transfer<NF, 4, T>(kind, in, out, Lf, Lc, periodic, s); break;
    case 5: if constexpr (NF > 5) return launch_transfer<NF, 5, T>(kind, in, out, Lf, Lc, periodic, s); break;
    case 6: if constexpr (NF > 6) return launch_transfer<NF, 6, T>(kind, in, out, Lf, Lc, periodic, s); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t transfer(int kind, const void* in, void* out, const Lattice& Lf, const Lattice& Lc,
                    int periodic, hipStream_t s) {
  const int nf = Lf.p + 1, nc = Lc.p + 1;
  switch (nf) {
    case 3: return transfer_nc<T, 3>(nc, kind, in, out, Lf, Lc, periodic, s);
    case 4: return transfer_nc<T, 4>(nc, kind, in, out, Lf, Lc, periodic, s);
    case 5: return transfer_nc<T, 5>(nc, kind, in, out, Lf, Lc, periodic, s);
    case 6: return transfer_nc<T, 6>(nc, kind, in, out, Lf, Lc, periodic, s);
    case 7: return transfer_nc<T, 7>(nc, kind, in, out, Lf, Lc, periodic, s);
    default: return hipErrorInvalidValue;
  }
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t b) {
    if (p && bytes >= b) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) bytes = b;
    return e;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

}  // namespace
}  // namespace hx

using namespace hx;

struct hx_mg_s {
  std::vector<hx_ctx> lv;
  hx_mg_options opt{};
  bool fp32 = true;
  int periodic = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // per level: b, x, t (operator output), d (Chebyshev direction), dinv; u (FP64 linearisation)
  std::vector<std::unique_ptr<DevBuf[]>> buf;
  std::vector<double> lmax;
  DevBuf dots;  // 3 doubles
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ready = false;
  int vcycles = 0;
  std::string err;
  // Newton / Krylov work vectors (FP64, finest level)
  DevBuf r, x, p, q, z, zold, f;
};

namespace {

enum { B_B = 0, B_X, B_T, B_D, B_DINV, B_U, B_COUNT };

hx_status mg_fail(hx_mg mg, hx_status s, const std::string& m) {
  if (mg) mg->err = m;
  return s;
}

hx_precision mg_prec(const hx_mg mg) { return mg->fp32 ? HX_FP32 : HX_FP64; }

size_t vec_bytes(const hx_mg mg, int l) {
  return static_cast<size_t>(3 * mg->lv[l]->L.n_nodes) * (mg->fp32 ? sizeof(float) : sizeof(double));
}

template <typename T>
hipError_t level_apply(hx_mg mg, int l, const T* x, T* y) {
  const hx_status st = hx_apply_tangent(mg->lv[l], x, y, mg_prec(mg), mg->stream);
  return st == HX_OK ? hipSuccess : hipErrorLaunchFailure;
}

// Chebyshev-Jacobi on level l: x <- approximately A^-1 b, degree `deg`, starting from x (zero_init:
// from 0). Eigenvalue interval [lmax / range, lmax].
template <typename T>
hipError_t chebyshev(hx_mg mg, int l, int deg, bool zero_init) {
  const hx_ctx c = mg->lv[l];
  const int64_t n = 3 * c->L.n_nodes;
  DevBuf* B = mg->buf[l].get();
  T* b = B[B_B].as<T>();
  T* x = B[B_X].as<T>();
  T* t = B[B_T].as<T>();
  T* d = B[B_D].as<T>();
  const T* dinv = B[B_DINV].as<T>();
  const double lmax = mg->lmax[l], lmin = lmax / mg->opt.smoothing_range;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho_old = 1.0 / sigma;
  hipError_t e;
  if (zero_init) {
    k_cheb_first<T><<<grid_for(n), 256, 0, mg->stream>>>(x, d, b, nullptr, dinv, static_cast<T>(1.0 / theta), 1, n);
  } else {
    if ((e = level_apply<T>(mg, l, x, t)) != hipSuccess) return e;
    k_cheb_first<T><<<grid_for(n), 256, 0, mg->stream>>>(x, d, b, t, dinv, static_cast<T>(1.0 / theta), 0, n);
  }
  for (int k = 1; k < deg; ++k) {
    if ((e = level_apply<T>(mg, l, x, t)) != hipSuccess) return e;
    const double rho = 1.0 / (2.0 * sigma - rho_old);
    k_cheb_step<T><<<grid_for(n), 256, 0, mg->stream>>>(x, d, b, t, dinv, static_cast<T>(rho * rho_old),
                                                        static_cast<T>(2.0 * rho / delta), n);
    rho_old = rho;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t vcycle_level(hx_mg mg, int l) {
  const int L = static_cast<int>(mg->lv.size());
  hipError_t e;
  if (l == L - 1) return chebyshev<T>(mg, l, mg->opt.coarse_degree, true);
  if ((e = chebyshev<T>(mg, l, mg->opt.smoother_degree, true)) != hipSuccess) return e;
  const hx_ctx cf = mg->lv[l], cc = mg->lv[l + 1];
  DevBuf* Bf = mg->buf[l].get();
  DevBuf* Bc = mg->buf[l + 1].get();
  const int64_t nf = 3 * cf->L.n_nodes, nc = 3 * cc->L.n_nodes;
  // t = b - A x (residual of the smoothed iterate)
  if ((e = level_apply<T>(mg, l, Bf[B_X].as<T>(), Bf[B_T].as<T>())) != hipSuccess) return e;
  k_axpby<T><<<grid_for(nf), 256, 0, mg->stream>>>(Bf[B_T].as<T>(), T(1), Bf[B_B].as<T>(), T(-1), nf);
  k_fill<T><<<grid_for(nc), 256, 0, mg->stream>>>(Bc[B_B].as<T>(), T(0), nc);
  if ((e = transfer<T>(1, Bf[B_T].p, Bc[B_B].p, cf->L, cc->L, mg->periodic, mg->stream)) != hipSuccess) return e;
  if ((e = vcycle_level<T>(mg, l + 1)) != hipSuccess) return e;
  if ((e = transfer<T>(0, Bc[B_X].p, Bf[B_X].p, cf->L, cc->L, mg->periodic, mg->stream)) != hipSuccess) return e;
  return chebyshev<T>(mg, l, mg->opt.smoother_degree, false);
}

hipError_t vcycle_enqueue(hx_mg mg) {
  return mg->fp32 ? vcycle_level<float>(mg, 0) : vcycle_level<double>(mg, 0);
}

hipError_t read_dots(hx_mg mg, int npairs, double* host) {
  hipError_t e = hipMemcpyAsync(host, mg->dots.p, npairs * sizeof(double), hipMemcpyDeviceToHost, mg->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(mg->stream);
}

template <typename T>
hipError_t dots(hx_mg mg, int64_t n, int npairs, const T* a0, const T* b0, const T* a1,
                const T* b1, const T* a2, const T* b2, double* host) {
  k_fill<double><<<1, 64, 0, mg->stream>>>(mg->dots.as<double>(), 0.0, 3);
  k_dots<T><<<std::min(grid_for(n), 1024), 256, 0, mg->stream>>>(a0, b0, a1, b1, a2, b2, npairs, mg->dots.as<double>(), n);
  return read_dots(mg, npairs, host);
}

// largest eigenvalue of D^-1 A on level l by power iteration
template <typename T>
hipError_t estimate_lmax(hx_mg mg, int l, double* out) {
  const hx_ctx c = mg->lv[l];
  const int64_t n = 3 * c->L.n_nodes;
  DevBuf* B = mg->buf[l].get();
  T* v = B[B_X].as<T>();
  T* w = B[B_T].as<T>();
  const T* dinv = B[B_DINV].as<T>();
  k_hash_vector<T><<<grid_for(n), 256, 0, mg->stream>>>(v, c->L);
  double h[3], lam = 0.0;
  hipError_t e = dots<T>(mg, n, 1, v, v, nullptr, nullptr, nullptr, nullptr, h);
  if (e != hipSuccess) return e;
  double nv = std::sqrt(h[0]);
  for (int it = 0; it < mg->opt.eig_iters; ++it) {
    if ((e = level_apply<T>(mg, l, v, w)) != hipSuccess) return e;
    // w = dinv * w (the constrained identity rows keep eigenvalue 1)
    k_cheb_first<T><<<grid_for(n), 256, 0, mg->stream>>>(w, B[B_D].as<T>(), w, nullptr, dinv, T(1), 1, n);
    if ((e = dots<T>(mg, n, 1, w, w, nullptr, nullptr, nullptr, nullptr, h)) != hipSuccess) return e;
    const double nw = std::sqrt(h[0]);
    lam = nw / nv;
    k_axpby<T><<<grid_for(n), 256, 0, mg->stream>>>(v, static_cast<T>(1.0 / nw), w, T(0), n);
    nv = 1.0;
  }
  *out = lam * mg->opt.eig_safety;
  return hipGetLastError();
}

template <typename T>
hipError_t level_diagonal(hx_mg mg, int l) {
  const hx_ctx c = mg->lv[l];
  const int64_t n = 3 * c->L.n_nodes;
  T* dinv = mg->buf[l][B_DINV].as<T>();
  k_fill<T><<<grid_for(n), 256, 0, mg->stream>>>(dinv, T(0), n);
  const Slot& sl = c->slot[mg->fp32 ? 1 : 0];
  HostArgs h = args_for(c);
  h.out = dinv;
  h.qdata = sl.qdata;
  h.cscale = sl.cscale;
  HostOp op{OpKind::Diagonal, c->base.mat.law, HX_STORE_TANGENT, sl.store, mg->fp32};
  bool ok = false;
  hipError_t e = dispatch(c->p, op, h, mg->stream, &ok);
  if (!ok) return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  k_diag_finish<T><<<grid_for(n), 256, 0, mg->stream>>>(dinv, c->L);
  return hipGetLastError();
}

}  // namespace

extern "C" {

hx_status hx_mg_create(const hx_ctx* levels, int32_t n_levels, const hx_mg_options* opt,
                       hx_mg* out) {
  if (!out) return HX_E_ARG;
  *out = nullptr;
  if (!levels || n_levels < 1) return HX_E_ARG;
  for (int l = 0; l < n_levels; ++l) {
    if (!levels[l]) return HX_E_ARG;
    if (l > 0) {
      const Lattice& a = levels[l - 1]->L;
      const Lattice& b = levels[l]->L;
      if (a.nx != b.nx || a.ny != b.ny || a.nz != b.nz || b.p >= a.p || a.dir_faces != b.dir_faces)
        return HX_E_ARG;
    }
  }
  hx_mg_s* mg = new (std::nothrow) hx_mg_s();
  if (!mg) return HX_E_NOMEM;
  mg->lv.assign(levels, levels + n_levels);
  hx_mg_options o{};
  o.smoother_degree = 4;
  o.coarse_degree = 30;
  o.smoothing_range = 20.0;
  o.eig_iters = 20;
  o.eig_safety = 1.2;
  o.precision = HX_FP32;
  o.use_graph = 1;
  if (opt) {
    o = *opt;
    if (o.smoother_degree < 1 || o.coarse_degree < 1 || o.eig_iters < 1 || !(o.smoothing_range > 1.0) ||
        !(o.eig_safety >= 1.0) || (o.precision != HX_FP32 && o.precision != HX_FP64)) {
      delete mg;
      return HX_E_ARG;
    }
  }
  mg->opt = o;
  mg->fp32 = o.precision == HX_FP32;
  // periodic flags: recovered from the lattice (periodic direction has N = n p)
  const Lattice& L0 = levels[0]->L;
  mg->periodic = (L0.Nx == L0.nx * L0.p ? 1 : 0) | (L0.Ny == L0.ny * L0.p ? 2 : 0) | (L0.Nz == L0.nz * L0.p ? 4 : 0);
  hipError_t e = hipStreamCreateWithFlags(&mg->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&mg->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&mg->ev_out, hipEventDisableTiming);
  if (e == hipSuccess) e = mg->dots.alloc(4 * sizeof(double));
  for (int l = 0; l < n_levels && e == hipSuccess; ++l) {
    mg->buf.emplace_back(new DevBuf[B_COUNT]);
    for (int k = 0; k < B_COUNT && e == hipSuccess; ++k) {
      const size_t b = k == B_U ? 3 * levels[l]->L.n_nodes * sizeof(double) : vec_bytes(mg, l);
      e = mg->buf[l][k].alloc(b);
    }
  }
  mg->lmax.assign(n_levels, 1.0);
  if (e != hipSuccess) {
    hx_mg_destroy(mg);
    return e == hipErrorOutOfMemory ? HX_E_NOMEM : HX_E_HIP;
  }
  *out = mg;
  return HX_OK;
}

hx_status hx_mg_destroy(hx_mg mg) {
  if (!mg) return HX_OK;
  if (mg->stream) (void)hipStreamSynchronize(mg->stream);
  if (mg->exec) (void)hipGraphExecDestroy(mg->exec);
  if (mg->graph) (void)hipGraphDestroy(mg->graph);
  if (mg->ev_in) (void)hipEventDestroy(mg->ev_in);
  if (mg->ev_out) (void)hipEventDestroy(mg->ev_out);
  if (mg->stream) (void)hipStreamDestroy(mg->stream);
  delete mg;
  return HX_OK;
}

const char* hx_mg_last_error(hx_mg mg) { return mg ? mg->err.c_str() : ""; }

hx_status hx_mg_update(hx_mg mg, const double* u, void* stream) {
  if (!mg || !u) return HX_E_ARG;
  hipStream_t caller = static_cast<hipStream_t>(stream);
  hipError_t e = hipEventRecord(mg->ev_in, caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(mg->stream, mg->ev_in, 0);
  if (e != hipSuccess) return mg_fail(mg, HX_E_HIP, "hx_mg_update: stream order");
  const int L = static_cast<int>(mg->lv.size());
  const int64_t n0 = 3 * mg->lv[0]->L.n_nodes;
  k_convert<double, double><<<grid_for(n0), 256, 0, mg->stream>>>(u, mg->buf[0][B_U].as<double>(), n0);
  for (int l = 1; l < L; ++l) {
    if ((e = transfer<double>(2, mg->buf[l - 1][B_U].p, mg->buf[l][B_U].p, mg->lv[l - 1]->L,
                              mg->lv[l]->L, mg->periodic, mg->stream)) != hipSuccess)
      return mg_fail(mg, HX_E_HIP, "hx_mg_update: transfer of the linearisation point");
  }
  for (int l = 0; l < L; ++l) {
    const hx_status st = hx_update_linearization(mg->lv[l], mg->buf[l][B_U].as<double>(), HX_STORE_TANGENT,
                                                 mg_prec(mg), mg->stream);
    if (st != HX_OK) return mg_fail(mg, st, std::string("hx_mg_update: level update: ") + hx_last_error(mg->lv[l]));
    e = mg->fp32 ? level_diagonal<float>(mg, l) : level_diagonal<double>(mg, l);
    if (e != hipSuccess) return mg_fail(mg, HX_E_HIP, "hx_mg_update: diagonal");
    double lm = 1.0;
    e = mg->fp32 ? estimate_lmax<float>(mg, l, &lm) : estimate_lmax<double>(mg, l, &lm);
    if (e != hipSuccess) return mg_fail(mg, HX_E_HIP, "hx_mg_update: eigenvalue estimate");
    if (!(lm > 0.0) || !std::isfinite(lm)) return mg_fail(mg, HX_E_NONFINITE, "hx_mg_update: eigenvalue estimate");
    mg->lmax[l] = lm;
  }
  // capture one V-cycle (internal buffers only) into a graph
  if (mg->exec) {
    (void)hipGraphExecDestroy(mg->exec);
    mg->exec = nullptr;
  }
  if (mg->graph) {
    (void)hipGraphDestroy(mg->graph);
    mg->graph = nullptr;
  }
  if (mg->opt.use_graph) {
    if ((e = hipStreamSynchronize(mg->stream)) != hipSuccess) return mg_fail(mg, HX_E_HIP, "hx_mg_update: sync");
    if ((e = hipStreamBeginCapture(mg->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return mg_fail(mg, HX_E_HIP, "hx_mg_update: begin capture");
    const hipError_t ev = vcycle_enqueue(mg);
    e = hipStreamEndCapture(mg->stream, &mg->graph);
    if (ev != hipSuccess || e != hipSuccess) return mg_fail(mg, HX_E_HIP, "hx_mg_update: capture");
    if ((e = hipGraphInstantiate(&mg->exec, mg->graph, nullptr, nullptr, 0)) != hipSuccess)
      return mg_fail(mg, HX_E_HIP, "hx_mg_update: instantiate");
  }
  mg->ready = true;
  if ((e = hipEventRecord(mg->ev_out, mg->stream)) != hipSuccess || (e = hipStreamWaitEvent(caller, mg->ev_out, 0)) != hipSuccess)
    return mg_fail(mg, HX_E_HIP, "hx_mg_update: stream order");
  return HX_OK;
}

static hx_status vcycle_internal(hx_mg mg) {
  hipError_t e = mg->exec ? hipGraphLaunch(mg->exec, mg->stream) : vcycle_enqueue(mg);
  ++mg->vcycles;
  return e == hipSuccess ? HX_OK : mg_fail(mg, HX_E_HIP, "V-cycle launch");
}

hx_status hx_mg_vcycle(hx_mg mg, const void* r, void* z, void* stream) {
  if (!mg || !r || !z) return HX_E_ARG;
  if (!mg->ready) return mg_fail(mg, HX_E_STATE, "hx_mg_vcycle: no hx_mg_update yet");
  hipStream_t caller = static_cast<hipStream_t>(stream);
  hipError_t e = hipEventRecord(mg->ev_in, caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(mg->stream, mg->ev_in, 0);
  const int64_t n0 = 3 * mg->lv[0]->L.n_nodes;
  DevBuf* B = mg->buf[0].get();
  if (mg->fp32)
    k_convert<float, float><<<grid_for(n0), 256, 0, mg->stream>>>(static_cast<const float*>(r), B[B_B].as<float>(), n0);
  else
    k_convert<double, double><<<grid_for(n0), 256, 0, mg->stream>>>(static_cast<const double*>(r), B[B_B].as<double>(), n0);
  hx_status st = vcycle_internal(mg);
  if (st != HX_OK) return st;
  if (mg->fp32)
    k_convert<float, float><<<grid_for(n0), 256, 0, mg->stream>>>(B[B_X].as<float>(), static_cast<float*>(z), n0);
  else
    k_convert<double, double><<<grid_for(n0), 256, 0, mg->stream>>>(B[B_X].as<double>(), static_cast<double*>(z), n0);
  if (e == hipSuccess) e = hipEventRecord(mg->ev_out, mg->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(caller, mg->ev_out, 0);
  return e == hipSuccess ? HX_OK : mg_fail(mg, HX_E_HIP, "hx_mg_vcycle: launch");
}

int64_t hx_mg_vcycle_count(hx_mg mg) { return mg ? mg->vcycles : -1; }

hx_status hx_mg_transfer(hx_mg mg, int32_t level, int32_t kind, const void* in, void* out,
                         void* stream) {
  if (!mg || !in || !out || level < 0 || level + 1 >= static_cast<int>(mg->lv.size()) || kind < 0 || kind > 2)
    return HX_E_ARG;
  const hx_ctx cf = mg->lv[level], cc = mg->lv[level + 1];
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (kind == 2)
    e = transfer<double>(2, in, out, cf->L, cc->L, mg->periodic, s);
  else if (mg->fp32)
    e = transfer<float>(kind, in, out, cf->L, cc->L, mg->periodic, s);
  else
    e = transfer<double>(kind, in, out, cf->L, cc->L, mg->periodic, s);
  return e == hipSuccess ? HX_OK : mg_fail(mg, HX_E_HIP, "hx_mg_transfer: launch");
}

hx_status hx_mg_inverse_diagonal(hx_mg mg, int32_t level, void* out, void* stream) {
  if (!mg || !out || level < 0 || level >= static_cast<int>(mg->lv.size())) return HX_E_ARG;
  if (!mg->ready) return mg_fail(mg, HX_E_STATE, "hx_mg_inverse_diagonal: no hx_mg_update yet");
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipStreamSynchronize(mg->stream);
  const hipError_t e = hipMemcpyAsync(out, mg->buf[level][B_DINV].p, vec_bytes(mg, level), hipMemcpyDeviceToDevice, s);
  return e == hipSuccess ? HX_OK : mg_fail(mg, HX_E_HIP, "hx_mg_inverse_diagonal: copy");
}

double hx_mg_lambda_max(hx_mg mg, int32_t level) {
  if (!mg || level < 0 || level >= static_cast<int>(mg->lv.size())) return -1.0;
  return mg->lmax[level];
}

// Preconditioner application on FP64 vectors: z = M^-1 r (conversion to the V-cycle precision).
static hx_status precondition(hx_mg mg, const double* r, double* z) {
  const int64_t n0 = 3 * mg->lv[0]->L.n_nodes;
  DevBuf* B = mg->buf[0].get();
  if (mg->fp32)
    k_convert<double, float><<<grid_for(n0), 256, 0, mg->stream>>>(r, B[B_B].as<float>(), n0);
  else
    k_convert<double, double><<<grid_for(n0), 256, 0, mg->stream>>>(r, B[B_B].as<double>(), n0);
  hx_status st = vcycle_internal(mg);
  if (st != HX_OK) return st;
  if (mg->fp32)
    k_convert<float, double><<<grid_for(n0), 256, 0, mg->stream>>>(B[B_X].as<float>(), z, n0);
  else
    k_convert<double, double><<<grid_for(n0), 256, 0, mg->stream>>>(B[B_X].as<double>(), z, n0);
  return hipGetLastError() == hipSuccess ? HX_OK : mg_fail(mg, HX_E_HIP, "precondition");
}

hx_status hx_newton_solve(hx_mg mg, double* u, const double* f_ext, const hx_newton_opts* opt,
                          hx_newton_report* rep, void* stream) {
  if (!mg || !u || !opt) return HX_E_ARG;
  if (opt->load_steps < 1 || opt->max_newton < 0 || opt->max_krylov < 1 || !(opt->krylov_rel_tol > 0.0))
    return mg_fail(mg, HX_E_ARG, "hx_newton_solve: invalid options");
  const auto t0 = std::chrono::steady_clock::now();
  hx_ctx fine = mg->lv[0];
  const int64_t n = 3 * fine->L.n_nodes;
  const size_t nb = n * sizeof(double);
  hipError_t e = hipSuccess;
  DevBuf* W[] = {&mg->r, &mg->x, &mg->p, &mg->q, &mg->z, &mg->zold, &mg->f};
  for (DevBuf* b : W)
    if ((e = b->alloc(nb)) != hipSuccess) return mg_fail(mg, HX_E_NOMEM, "hx_newton_solve: work vectors");
  hipStream_t caller = static_cast<hipStream_t>(stream);
  if ((e = hipEventRecord(mg->ev_in, caller)) != hipSuccess || (e = hipStreamWaitEvent(mg->stream, mg->ev_in, 0)) != hipSuccess)
    return mg_fail(mg, HX_E_HIP, "hx_newton_solve: stream order");
  double* r = mg->r.as<double>();
  double* x = mg->x.as<double>();
  double* p = mg->p.as<double>();
  double* q = mg->q.as<double>();
  double* z = mg->z.as<double>();
  double* zo = mg->zold.as<double>();
  double* f = mg->f.as<double>();
  hx_newton_report R{};
  const int vc0 = mg->vcycles;
  double h[3];
  auto residual = [&](double scale) -> hx_status {
    hx_status st = hx_residual(fine, u, r, mg->stream);
    if (st != HX_OK) return st;
    if (f_ext) {
      k_convert<double, double><<<grid_for(n), 256, 0, mg->stream>>>(f_ext, f, n);
      k_zero_constrained<double><<<grid_for(n), 256, 0, mg->stream>>>(f, fine->L);
      k_axpby<double><<<grid_for(n), 256, 0, mg->stream>>>(r, -scale, f, 1.0, n);
    }
    return hipGetLastError() == hipSuccess ? HX_OK : HX_E_HIP;
  };
  hx_status status = HX_OK;
  for (int step = 1; step <= opt->load_steps && status == HX_OK; ++step) {
    const double scale = static_cast<double>(step) / opt->load_steps;
    if ((status = residual(scale)) != HX_OK) break;
    if ((e = dots<double>(mg, n, 1, r, r, nullptr, nullptr, nullptr, nullptr, h)) != hipSuccess) { status = HX_E_HIP; break; }
    double rn = std::sqrt(h[0]);
    const double r0 = rn;
    if (step == 1) R.initial_residual = r0;
    int it = 0;
    bool converged = rn <= std::max(opt->newton_abs_tol, opt->newton_rel_tol * r0);
    while (!converged && it < opt->max_newton) {
      // linearisation of the outer FP64 operator and of every multigrid level
      if (mg->fp32) {
        status = hx_update_linearization(fine, u, opt->outer_mode, HX_FP64, mg->stream);
        if (status != HX_OK) break;
      }
      if ((status = hx_mg_update(mg, u, mg->stream)) != HX_OK) break;
      // flexible PCG on K dx = -r
      k_fill<double><<<grid_for(n), 256, 0, mg->stream>>>(x, 0.0, n);
      k_axpby<double><<<grid_for(n), 256, 0, mg->stream>>>(r, 0.0, r, -1.0, n);  // r <- -r (the right-hand side)
      if ((status = precondition(mg, r, z)) != HX_OK) break;
      k_convert<double, double><<<grid_for(n), 256, 0, mg->stream>>>(z, p, n);
      if ((e = dots<double>(mg, n, 2, r, z, r, r, nullptr, nullptr, h)) != hipSuccess) { status = HX_E_HIP; break; }
      double rz = h[0];
      const double bn = std::sqrt(h[1]);
      const double tol = opt->krylov_rel_tol * bn;
      int k = 0;
      for (; k < opt->max_krylov; ++k) {
        const hx_precision op = HX_FP64;
        if ((status = hx_apply_tangent(fine, p, q, op, mg->stream)) != HX_OK) break;
        if ((e = dots<double>(mg, n, 1, p, q, nullptr, nullptr, nullptr, nullptr, h)) != hipSuccess) { status = HX_E_HIP; break; }
        const double pq = h[0];
        if (!(pq > 0.0)) break;  // loss of positive definiteness: keep the current iterate
        const double alpha = rz / pq;
        k_axpby<double><<<grid_for(n), 256, 0, mg->stream>>>(x, alpha, p, 1.0, n);
        k_axpby<double><<<grid_for(n), 256, 0, mg->stream>>>(r, -alpha, q, 1.0, n);
        if ((e = dots<double>(mg, n, 1, r, r, nullptr, nullptr, nullptr, nullptr, h)) != hipSuccess) { status = HX_E_HIP; break; }
        if (std::sqrt(h[0]) <= tol) {
          ++k;
          break;
        }
        k_convert<double, double><<<grid_for(n), 256, 0, mg->stream>>>(z, zo, n);
        if ((status = precondition(mg, r, z)) != HX_OK) break;
        if ((e = dots<double>(mg, n, 2, r, z, r, zo, nullptr, nullptr, h)) != hipSuccess) { status = HX_E_HIP; break; }
        const double beta = (h[0] - h[1]) / rz;  // flexible (Polak-Ribiere) update
        rz = h[0];
        k_axpby<double><<<grid_for(n), 256, 0, mg->stream>>>(p, 1.0, z, beta, n);
      }
      if (status != HX_OK) break;
      R.krylov_iters += k;
      k_axpby<double><<<grid_for(n), 256, 0, mg->stream>>>(u, 1.0, x, 1.0, n);
      ++it;
      if ((status = residual(scale)) != HX_OK) break;
      if ((e = dots<double>(mg, n, 1, r, r, nullptr, nullptr, nullptr, nullptr, h)) != hipSuccess) { status = HX_E_HIP; break; }
      rn = std::sqrt(h[0]);
      if (!std::isfinite(rn)) { status = HX_E_NONFINITE; break; }
      converged = rn <= std::max(opt->newton_abs_tol, opt->newton_rel_tol * r0);
    }
    R.newton_iters += it;
    R.final_residual = rn;
    if (status == HX_OK) {
      R.load_steps_done = step;
      if (!converged) status = HX_E_NOT_CONVERGED;
    }
  }
  (void)hipStreamSynchronize(mg->stream);
  R.vcycles = mg->vcycles - vc0;
  R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = R;
  (void)hipEventRecord(mg->ev_out, mg->stream);
  (void)hipStreamWaitEvent(caller, mg->ev_out, 0);
  if (status == HX_E_HIP) return mg_fail(mg, status, "hx_newton_solve: HIP error");
  if (status == HX_E_NOT_CONVERGED) return mg_fail(mg, status, "hx_newton_solve: Newton did not converge");
  return status;
}

// Dead-load pressure on one boundary face (Section 2 residual, Neumann term):
// f_(c,a) = -p * int_face phi_a N_c dA, N the outward unit normal of the reference body.
hx_status hx_surface_load(hx_ctx ctx, int32_t face, double pressure, double* f) {
  if (!ctx || !f || face < 0 || face > 5) return HX_E_ARG;
  const Lattice& L = ctx->L;
  const int d = face / 2, side = face % 2;
  const int per = (L.Nx == L.nx * L.p ? 1 : 0) | (L.Ny == L.ny * L.p ? 2 : 0) | (L.Nz == L.nz * L.p ? 4 : 0);
  if (per & (1 << d)) return set_error(ctx, HX_E_ARG, "hx_surface_load: face of a periodic direction");
  const int n = ctx->p + 1;
  const int64_t nn = L.n_nodes;
  std::memset(f, 0, 3 * nn * sizeof(double));
  const double* xq = ctx->base.x;
  const double* wq = ctx->base.w;
  const int da = (d + 1) % 3, db = (d + 2) % 3;  // tangential reference directions (cyclic)
  const int nc[3] = {L.nx, L.ny, L.nz};
  const int cd = side ? nc[d] - 1 : 0;
  std::vector<double> la(n * n);  // la[q*n + i] = l_i(x_q) on the GLL nodes
  for (int qq = 0; qq < n; ++qq)
    for (int i = 0; i < n; ++i) {
      double v = 1.0;
      for (int m = 0; m < n; ++m)
        if (m != i) v *= (xq[qq] - ctx->gll[m]) / (ctx->gll[i] - ctx->gll[m]);
      la[qq * n + i] = v;
    }
  int cell[3];
  for (int c2 = 0; c2 < nc[db]; ++c2)
    for (int c1 = 0; c1 < nc[da]; ++c1) {
      cell[d] = cd;
      cell[da] = c1;
      cell[db] = c2;
      const int e = cell[0] + L.nx * (cell[1] + L.ny * cell[2]);
      (void)e;
      double X8[8][3];
      for (int v = 0; v < 8; ++v) {
        int vx = cell[0] + (v & 1), vy = cell[1] + ((v >> 1) & 1), vz = cell[2] + (v >> 2);
        vx = vx >= L.Vx ? vx - L.Vx : vx;
        vy = vy >= L.Vy ? vy - L.Vy : vy;
        vz = vz >= L.Vz ? vz - L.Vz : vz;
        const double* P = &ctx->vert_host[3 * (vx + static_cast<int64_t>(L.Vx) * (vy + static_cast<int64_t>(L.Vy) * vz))];
        for (int k = 0; k < 3; ++k) X8[v][k] = P[k];
      }
      for (int q2 = 0; q2 < n; ++q2)
        for (int q1 = 0; q1 < n; ++q1) {
          double xi[3];
          xi[d] = side ? 1.0 : 0.0;
          xi[da] = xq[q1];
          xi[db] = xq[q2];
          // tangent vectors dX/dxi_da, dX/dxi_db of the trilinear map
          double ta[3] = {0, 0, 0}, tb[3] = {0, 0, 0};
          for (int v = 0; v < 8; ++v) {
            const int bit[3] = {v & 1, (v >> 1) & 1, v >> 2};
            double phi[3], dphi[3];
            for (int k = 0; k < 3; ++k) {
              phi[k] = bit[k] ? xi[k] : 1.0 - xi[k];
              dphi[k] = bit[k] ? 1.0 : -1.0;
            }
            const double ga = dphi[da] * phi[db] * phi[d];
            const double gb = phi[da] * dphi[db] * phi[d];
            for (int k = 0; k < 3; ++k) {
              ta[k] += ga * X8[v][k];
              tb[k] += gb * X8[v][k];
            }
          }
          // ta x tb points along +xi_d for a positively oriented map: outward on the max side
          double nda[3] = {ta[1] * tb[2] - ta[2] * tb[1], ta[2] * tb[0] - ta[0] * tb[2], ta[0] * tb[1] - ta[1] * tb[0]};
          const double sgn = side ? 1.0 : -1.0;
          const double w = wq[q1] * wq[q2];
          for (int j2 = 0; j2 < n; ++j2)
            for (int j1 = 0; j1 < n; ++j1) {
              int loc[3];
              loc[d] = side ? n - 1 : 0;
              loc[da] = j1;
              loc[db] = j2;
              int I[3] = {cell[0] * L.p + loc[0], cell[1] * L.p + loc[1], cell[2] * L.p + loc[2]};
              I[0] = I[0] >= L.Nx ? I[0] - L.Nx : I[0];
              I[1] = I[1] >= L.Ny ? I[1] - L.Ny : I[1];
              I[2] = I[2] >= L.Nz ? I[2] - L.Nz : I[2];
              const int64_t node = I[0] + static_cast<int64_t>(L.Nx) * (I[1] + static_cast<int64_t>(L.Ny) * I[2]);
              const double phi = la[q1 * n + j1] * la[q2 * n + j2];
              for (int k = 0; k < 3; ++k) f[k * nn + node] += -pressure * sgn * nda[k] * w * phi;
            }
        }
    }
  return HX_OK;
}

}  // extern "C"
