// p-multigrid preconditioner and mixed-precision Newton-Krylov solve (Section 6; Algorithm 1).
//
// Levels share one structured mesh and differ in degree (p -> ... -> 1). Transfers are the
// polynomial embedding of the coarse space into the fine space (prolongation) and its transpose
// (restriction); the linearisation point is moved down by interpolation at the coarse nodes.
// Smoothing is Chebyshev-accelerated Jacobi with the inverse diagonal of the level operator
// (computed matrix-free from the stored tangent) and Lanczos estimates of the extreme
// eigenvalues; the coarsest level is solved approximately by a higher-degree Chebyshev iteration,
// which keeps the V-cycle a fixed linear operator. The V-cycle runs in FP32 or FP64 and is
// captured once per linearisation into a HIP graph. The outer Krylov solver is a flexible
// preconditioned CG in FP64 on the finest FP64 operator.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <chrono>
#include <cmath>
#include <cstdio>
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

// The nodal block smoother's D^-1 r at node i: dinv holds the inverse blocks as planes
// (00, 11, 22, 01, 02, 12) of nn nodes; r_c = b[c nn + i] - t[c nn + i] (t may be null).
template <typename T>
__device__ __forceinline__ void block_solve(const T* dinv, const T* b, const T* t, int64_t i, int64_t nn, T w[3]) {
  T r[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = b[c * nn + i] - (t ? t[c * nn + i] : T(0));
  const T a00 = dinv[i], a11 = dinv[nn + i], a22 = dinv[2 * nn + i];
  const T a01 = dinv[3 * nn + i], a02 = dinv[4 * nn + i], a12 = dinv[5 * nn + i];
  w[0] = a00 * r[0] + a01 * r[1] + a02 * r[2];
  w[1] = a01 * r[0] + a11 * r[1] + a12 * r[2];
  w[2] = a02 * r[0] + a12 * r[1] + a22 * r[2];
}

// k_cheb_first with the nodal block smoother (one thread per node, nn nodes)
template <typename T>
__global__ void k_cheb_first_blk(T* x, T* d, const T* b, const T* t, const T* dinv, T c, int first,
                                 int64_t nn) {
  HX_GRID_LOOP(i, nn) {
    T w[3];
    block_solve(dinv, b, t, i, nn, w);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T di = c * w[k];
      const T xo = first ? T(0) : x[k * nn + i];
      d[k * nn + i] = di;
      x[k * nn + i] = first ? di : xo + di;
    }
  }
}

// k_cheb_step with the nodal block smoother
template <typename T>
__global__ void k_cheb_step_blk(T* x, T* d, const T* b, const T* t, const T* dinv, T c1, T c2, int64_t nn) {
  HX_GRID_LOOP(i, nn) {
    T w[3];
    block_solve(dinv, b, t, i, nn, w);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T di = c1 * d[k * nn + i] + c2 * w[k];
      d[k * nn + i] = di;
      x[k * nn + i] += di;
    }
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

// ---------------------------------------------------------------- PCG with device-side scalars
// Scalars of the device-resident PCG: inner products of the running iteration, the stop flag
// (1: loss of positive definiteness, the iterate is kept; 2: converged), the count of completed
// iterations and the squared stopping threshold.
enum { CG_RZ = 0, CG_PQ, CG_RR, CG_RZN, CG_RZO, CG_STOP, CG_ITERS, CG_TOL2, CG_COUNT };

// x += alpha p, r -= alpha q with alpha = rz / pq, and in the same pass the inner products of the
// new residual with itself and with the previous preconditioned residual z (still in z: the
// preconditioner has not run yet), so that the flexible beta needs no copy of z. Nothing moves
// once the iteration has stopped or pq <= 0 (then the iterate is kept, as the host-driven loop
// does); the condition is uniform over the grid.
__global__ void __launch_bounds__(256) k_cg_alpha(double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ p, const double* __restrict__ q,
                                                  const double* __restrict__ z, double* __restrict__ sc,
                                                  int64_t n) {
  const double pq = sc[CG_PQ];
  if (sc[CG_STOP] != 0.0 || !(pq > 0.0)) return;
  const double alpha = sc[CG_RZ] / pq;
  double rr = 0.0, rz = 0.0;
  HX_GRID_LOOP(i, n) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    rr += ri * ri;
    rz += ri * z[i];
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = rr;
  red[1][threadIdx.x] = rz;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    unsafeAtomicAdd(sc + CG_RR, red[0][0]);
    unsafeAtomicAdd(sc + CG_RZO, red[1][0]);
  }
}

// p = z + beta p with the flexible (Polak-Ribiere) beta = (r.z - r.z_old) / rz
__global__ void k_cg_beta(double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ sc,
                          int64_t n) {
  if (sc[CG_STOP] != 0.0 || !(sc[CG_PQ] > 0.0) || sc[CG_RZ] == 0.0) return;
  const double beta = (sc[CG_RZN] - sc[CG_RZO]) / sc[CG_RZ];
  HX_GRID_LOOP(i, n) p[i] = z[i] + beta * p[i];
}

// End of an iteration: count it, set the stop flag (pq <= 0, or ||r||^2 at or below the threshold),
// rz <- r.z, and clear the accumulators of the next iteration's inner products.
__global__ void k_cg_roll(double* sc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (sc[CG_STOP] == 0.0) {
    if (!(sc[CG_PQ] > 0.0)) {
      sc[CG_STOP] = 1.0;
    } else {
      sc[CG_ITERS] += 1.0;
      if (sc[CG_RR] <= sc[CG_TOL2]) sc[CG_STOP] = 2.0;
      sc[CG_RZ] = sc[CG_RZN];
    }
  }
  sc[CG_PQ] = sc[CG_RR] = sc[CG_RZN] = sc[CG_RZO] = 0.0;
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

// nodal blocks (planes 00, 11, 22, 01, 02, 12) -> their inverses, in FP64 by the adjugate; the
// identity at constrained nodes
template <typename T>
__global__ void k_block_finish(T* d, Lattice L) {
  const int64_t nn = L.n_nodes;
  HX_GRID_LOOP(i, nn) {
    if (node_constrained(L, i)) {
      d[i] = d[nn + i] = d[2 * nn + i] = T(1);
      d[3 * nn + i] = d[4 * nn + i] = d[5 * nn + i] = T(0);
      continue;
    }
    const double a00 = d[i], a11 = d[nn + i], a22 = d[2 * nn + i];
    const double a01 = d[3 * nn + i], a02 = d[4 * nn + i], a12 = d[5 * nn + i];
    const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
    const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
    const double inv = 1.0 / (a00 * c00 + a01 * c01 + a02 * c02);
    d[i] = static_cast<T>(c00 * inv);
    d[nn + i] = static_cast<T>(c11 * inv);
    d[2 * nn + i] = static_cast<T>(c22 * inv);
    d[3 * nn + i] = static_cast<T>(c01 * inv);
    d[4 * nn + i] = static_cast<T>(c02 * inv);
    d[5 * nn + i] = static_cast<T>(c12 * inv);
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

// ---------------------------------------------------------------- dense coarse solve
// Probe vector of colour class (cx, cy, cz) and component cc: 1 on the nodes whose lattice index
// is congruent to the class modulo the colour counts (kx, ky, kz), 0 elsewhere.
template <typename T>
__global__ void k_probe(T* x, Lattice L, int kx, int ky, int kz, int cx, int cy, int cz, int cc) {
  HX_GRID_LOOP(i, 3 * L.n_nodes) {
    const int64_t node = i % L.n_nodes;
    const int c = static_cast<int>(i / L.n_nodes);
    const int I = static_cast<int>(node % L.Nx);
    const int J = static_cast<int>((node / L.Nx) % L.Ny);
    const int K = static_cast<int>(node / (static_cast<int64_t>(L.Nx) * L.Ny));
    x[i] = (c == cc && I % kx == cx && J % ky == cy && K % kz == cz) ? T(1) : T(0);
  }
}

// index in {I-p, ..., I+p} (wrapped if periodic, skipped if outside) congruent to col mod k; -1 if
// none. Nodes of degree-p cells couple with the nodes up to p lattice indices away, and k >= 2p + 1
// colours (or k = N, one colour per index) leave at most one candidate in that window.
__device__ __forceinline__ int probe_hit(int I, int N, bool periodic, int k, int col, int p) {
  if (k == N) return col;
  for (int d = -p; d <= p; ++d) {
    int J = I + d;
    if (periodic) {
      J = J < 0 ? J + N : (J >= N ? J - N : J);
    } else if (J < 0 || J >= N) {
      continue;
    }
    if (J % k == col) return J;
  }
  return -1;
}

// y = A x for a probe x: row i of A has its only entry of this colour class in the column of the
// neighbour node of that class, so A[i][col(i)] = y[i]. A is column-major n x n (FP64).
template <typename T>
__global__ void k_probe_extract(const T* __restrict__ y, double* __restrict__ A, Lattice L, int kx, int ky,
                                int kz, int cx, int cy, int cz, int cc) {
  const int64_t n = 3 * L.n_nodes;
  HX_GRID_LOOP(i, n) {
    const int64_t node = i % L.n_nodes;
    const int I = static_cast<int>(node % L.Nx);
    const int J = static_cast<int>((node / L.Nx) % L.Ny);
    const int K = static_cast<int>(node / (static_cast<int64_t>(L.Nx) * L.Ny));
    const int a = probe_hit(I, L.Nx, L.Nx == L.nx * L.p, kx, cx, L.p);
    const int b = probe_hit(J, L.Ny, L.Ny == L.ny * L.p, ky, cy, L.p);
    const int c = probe_hit(K, L.Nz, L.Nz == L.nz * L.p, kz, cz, L.p);
    if (a < 0 || b < 0 || c < 0) continue;
    const int64_t col = cc * L.n_nodes + a + static_cast<int64_t>(L.Nx) * (b + static_cast<int64_t>(L.Ny) * c);
    A[col * n + i] = static_cast<double>(y[i]);
  }
}

__global__ void k_identity(double* B, int64_t n) {
  HX_GRID_LOOP(i, n * n) B[i] = (i / n == i % n) ? 1.0 : 0.0;
}

// x = M b with the dense symmetric n x n matrix M (column j = row j): one wavefront per row.
template <typename T>
__global__ void __launch_bounds__(256) k_dense_mv(const T* __restrict__ M, const T* __restrict__ b,
                                                  T* __restrict__ x, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (row >= n) return;
  const T* m = M + row * n;
  T acc = T(0);
  for (int64_t j = lane; j < n; j += 64) acc += m[j] * b[j];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) x[row] = acc;
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

// Sum-factorised transfers between degrees on one cell: the 3D interpolation matrix is the tensor
// product of the 1D table Icf (fine GLL point x coarse basis function), applied as three 1D
// contractions through LDS; every pencil's coefficients are compile-time constants.
// in: NI values per pencil with stride SI, out: NO values with stride SO (TR: Icf^T, i.e. from the
// fine to the coarse points).
template <int NF, int NC, bool TR, typename T>
__device__ __forceinline__ void transfer_pencil(const T* in, int si, T* out, int so) {
  constexpr int NI = TR ? NF : NC, NO = TR ? NC : NF;
  T v[NI];
#pragma unroll
  for (int m = 0; m < NI; ++m) v[m] = in[m * si];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < NI; ++m)
      acc += (TR ? Transfer1D<NF, NC, T>::Icf[m * NC + o] : Transfer1D<NF, NC, T>::Icf[o * NC + m]) * v[m];
    out[o * so] = acc;
  }
}

// xf += P xc: each fine node written once, by its owning cell. Contractions along x, y, z:
// [NC^3] -> [NF NC^2] -> [NF^2 NC] -> [NF^3] per component.
template <int NF, int NC, typename T>
__global__ void __launch_bounds__(NF* NF* NF) k_prolong_add(const T* __restrict__ xc,
                                                            T* __restrict__ xf, Lattice Lf,
                                                            Lattice Lc, int periodic) {
  constexpr int QF = NF * NF * NF, QC = NC * NC * NC;
  constexpr int S1 = NF * NC * NC, S2 = NF * NF * NC;
  __shared__ T s0[3 * QC];
  __shared__ T s1[3 * S1];
  __shared__ T s2[3 * S2];
  __shared__ T s3[3 * QF];
  const int e = blockIdx.x;
  const CellPos cp = cell_pos(Lf, e);
  const int t = threadIdx.x;
  // this thread's fine node: its current values are requested first, so that the read half of the
  // update overlaps the gather and the contractions
  const int i = t % NF, j = (t / NF) % NF, k = t / (NF * NF);
  const bool own = owns_node(Lf, cp, i, j, k, periodic);
  bool fcons;
  const int64_t fnode = node_of(Lf, cp, i, j, k, fcons);
  T xo[3] = {T(0), T(0), T(0)};
  if (own)
    for (int c = 0; c < 3; ++c) xo[c] = xf[c * Lf.n_nodes + fnode];
  if (t < QC) {
    bool cons;
    const int64_t node = node_of(Lc, cp, t % NC, (t / NC) % NC, t / (NC * NC), cons);
    for (int c = 0; c < 3; ++c) s0[c * QC + t] = xc[c * Lc.n_nodes + node];
  }
  __syncthreads();
  // along x: pencils (c, b, cc), coarse a -> fine i
  for (int job = t; job < 3 * NC * NC; job += QF) {
    const int c = job / (NC * NC), r = job - c * (NC * NC);
    transfer_pencil<NF, NC, false>(s0 + c * QC + NC * r, 1, s1 + c * S1 + NF * r, 1);
  }
  __syncthreads();
  // along y: pencils (c, i, cc), coarse b -> fine j
  for (int job = t; job < 3 * NF * NC; job += QF) {
    const int c = job / (NF * NC), r = job - c * (NF * NC);
    const int i = r % NF, cc = r / NF;
    transfer_pencil<NF, NC, false>(s1 + c * S1 + i + NF * NC * cc, NF, s2 + c * S2 + i + NF * NF * cc, NF);
  }
  __syncthreads();
  // along z: pencils (c, i, j), coarse cc -> fine k
  for (int job = t; job < 3 * NF * NF; job += QF) {
    const int c = job / (NF * NF), r = job - c * (NF * NF);
    transfer_pencil<NF, NC, false>(s2 + c * S2 + r, NF * NF, s3 + c * QF + r, NF * NF);
  }
  __syncthreads();
  if (!own) return;
  for (int c = 0; c < 3; ++c) xf[c * Lf.n_nodes + fnode] = xo[c] + s3[c * QF + t];
}

// rc += P^T rf (rc zeroed by the caller): the owned fine values of the cell contracted along z,
// y, x: [NF^3] -> [NF^2 NC] -> [NF NC^2] -> [NC^3], then added atomically at the coarse nodes.
template <int NF, int NC, typename T>
__global__ void __launch_bounds__(NF* NF* NF) k_restrict_add(const T* __restrict__ rf,
                                                             T* __restrict__ rc, Lattice Lf,
                                                             Lattice Lc, int periodic) {
  constexpr int QF = NF * NF * NF, QC = NC * NC * NC;
  constexpr int S1 = NF * NC * NC, S2 = NF * NF * NC;
  __shared__ T sf[3 * QF];
  __shared__ T s2[3 * S2];
  __shared__ T s1[3 * S1];
  __shared__ T s0[3 * QC];
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
  // along z: pencils (c, i, j), fine k -> coarse cc
  for (int job = t; job < 3 * NF * NF; job += QF) {
    const int c = job / (NF * NF), r = job - c * (NF * NF);
    transfer_pencil<NF, NC, true>(sf + c * QF + r, NF * NF, s2 + c * S2 + r, NF * NF);
  }
  __syncthreads();
  // along y: pencils (c, i, cc), fine j -> coarse b
  for (int job = t; job < 3 * NF * NC; job += QF) {
    const int c = job / (NF * NC), r = job - c * (NF * NC);
    const int i = r % NF, cc = r / NF;
    transfer_pencil<NF, NC, true>(s2 + c * S2 + i + NF * NF * cc, NF, s1 + c * S1 + i + NF * NC * cc, NF);
  }
  __syncthreads();
  // along x: pencils (c, b, cc), fine i -> coarse a
  for (int job = t; job < 3 * NC * NC; job += QF) {
    const int c = job / (NC * NC), r = job - c * (NC * NC);
    transfer_pencil<NF, NC, true>(s1 + c * S1 + NF * r, 1, s0 + c * QC + NC * r, 1);
  }
  __syncthreads();
  if (t >= QC) return;
  const int a = t % NC, b = (t / NC) % NC, cc = t / (NC * NC);
  bool cons;
  const int64_t node = node_of(Lc, cp, a, b, cc, cons);
  if (cons) return;
  for (int c = 0; c < 3; ++c) unsafeAtomicAdd(rc + c * Lc.n_nodes + node, s0[c * QC + t]);
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

// ---------------------------------------------------------------- transfers between lattices
// Two degree-1 lattices where the coarse one has half the cells in some directions (factor 2)
// and the same cells in the others (factor 1). The coarse cell covers 2 fine cells per halved
// direction; the coarse Q1 basis, evaluated at the fine node in the coarse cell's reference
// coordinates, is 1 at coincident nodes and 1/2 at midpoints. The fine geometry is not required
// to be the coarse geometry refined (curved bodies): the transfer lives in reference space.

// coarse neighbours of fine node index I along one direction: a (weight wa), b (weight 1 - wa)
__device__ __forceinline__ void h_up(int I, int fac, int Nc, bool periodic, int& a, int& b, bool& two) {
  if (fac == 1 || (I & 1) == 0) {
    a = fac == 1 ? I : I >> 1;
    b = a;
    two = false;
    return;
  }
  a = (I - 1) >> 1;
  b = a + 1;
  if (periodic && b >= Nc) b -= Nc;
  two = true;
}

template <typename T>
__global__ void k_h_prolong_add(const T* __restrict__ xc, T* __restrict__ xf, Lattice Lf, Lattice Lc,
                                int fx, int fy, int fz, int periodic) {
  HX_GRID_LOOP(node, Lf.n_nodes) {
    const int I = static_cast<int>(node % Lf.Nx);
    const int J = static_cast<int>((node / Lf.Nx) % Lf.Ny);
    const int K = static_cast<int>(node / (static_cast<int64_t>(Lf.Nx) * Lf.Ny));
    int ia[2], ja[2], ka[2];
    bool ti, tj, tk;
    h_up(I, fx, Lc.Nx, periodic & 1, ia[0], ia[1], ti);
    h_up(J, fy, Lc.Ny, periodic & 2, ja[0], ja[1], tj);
    h_up(K, fz, Lc.Nz, periodic & 4, ka[0], ka[1], tk);
    const T wi = ti ? T(0.5) : T(1), wj = tj ? T(0.5) : T(1), wk = tk ? T(0.5) : T(1);
    T v[3] = {T(0), T(0), T(0)};
    for (int c2 = 0; c2 < (tk ? 2 : 1); ++c2)
      for (int b2 = 0; b2 < (tj ? 2 : 1); ++b2)
        for (int a2 = 0; a2 < (ti ? 2 : 1); ++a2) {
          const int64_t cn = ia[a2] + static_cast<int64_t>(Lc.Nx) * (ja[b2] + static_cast<int64_t>(Lc.Ny) * ka[c2]);
          const T w = wi * wj * wk;
          for (int c = 0; c < 3; ++c) v[c] += w * xc[c * Lc.n_nodes + cn];
        }
    for (int c = 0; c < 3; ++c) xf[c * Lf.n_nodes + node] += v[c];
  }
}

// fine indices feeding coarse index Ic along one direction: f[0..cnt), weights w
__device__ __forceinline__ int h_down(int Ic, int fac, int Nf, bool periodic, int* f, float* w) {
  if (fac == 1) {
    f[0] = Ic;
    w[0] = 1.0f;
    return 1;
  }
  int cnt = 0;
  for (int d = -1; d <= 1; ++d) {
    int I = 2 * Ic + d;
    if (periodic) {
      I = I < 0 ? I + Nf : (I >= Nf ? I - Nf : I);
    } else if (I < 0 || I >= Nf) {
      continue;
    }
    f[cnt] = I;
    w[cnt] = d == 0 ? 1.0f : 0.5f;
    ++cnt;
  }
  return cnt;
}

// rc += P^T rf, gathered per coarse node (no atomics); constrained coarse rows untouched
template <typename T>
__global__ void k_h_restrict_add(const T* __restrict__ rf, T* __restrict__ rc, Lattice Lf, Lattice Lc,
                                 int fx, int fy, int fz, int periodic) {
  HX_GRID_LOOP(node, Lc.n_nodes) {
    if (node_constrained(Lc, node)) continue;
    const int I = static_cast<int>(node % Lc.Nx);
    const int J = static_cast<int>((node / Lc.Nx) % Lc.Ny);
    const int K = static_cast<int>(node / (static_cast<int64_t>(Lc.Nx) * Lc.Ny));
    int fi[3], fj[3], fk[3];
    float wi[3], wj[3], wk[3];
    const int ni = h_down(I, fx, Lf.Nx, periodic & 1, fi, wi);
    const int nj = h_down(J, fy, Lf.Ny, periodic & 2, fj, wj);
    const int nk = h_down(K, fz, Lf.Nz, periodic & 4, fk, wk);
    T v[3] = {T(0), T(0), T(0)};
    for (int c2 = 0; c2 < nk; ++c2)
      for (int b2 = 0; b2 < nj; ++b2)
        for (int a2 = 0; a2 < ni; ++a2) {
          const int64_t fn = fi[a2] + static_cast<int64_t>(Lf.Nx) * (fj[b2] + static_cast<int64_t>(Lf.Ny) * fk[c2]);
          const T w = static_cast<T>(wi[a2] * wj[b2] * wk[c2]);
          for (int c = 0; c < 3; ++c) v[c] += w * rf[c * Lf.n_nodes + fn];
        }
    for (int c = 0; c < 3; ++c) rc[c * Lc.n_nodes + node] += v[c];
  }
}

// uc = uf at the coarse nodes (every coarse node is a fine node)
__global__ void k_h_inject(const double* __restrict__ uf, double* __restrict__ uc, Lattice Lf, Lattice Lc,
                           int fx, int fy, int fz) {
  HX_GRID_LOOP(node, Lc.n_nodes) {
    const int64_t I = node % Lc.Nx;
    const int64_t J = (node / Lc.Nx) % Lc.Ny;
    const int64_t K = node / (static_cast<int64_t>(Lc.Nx) * Lc.Ny);
    const int64_t fn = fx * I + Lf.Nx * (fy * J + Lf.Ny * (fz * K));
    for (int c = 0; c < 3; ++c) uc[c * Lc.n_nodes + node] = uf[c * Lf.n_nodes + fn];
  }
}

// coarsening factor per direction between two degree-1 lattices (1 or 2), 0 if not related
int h_factor(int nf, int nc) { return nf == nc ? 1 : (nf == 2 * nc ? 2 : 0); }

template <typename T>
hipError_t h_transfer(int kind, const void* in, void* out, const Lattice& Lf, const Lattice& Lc, int periodic,
                      hipStream_t s) {
  const int fx = h_factor(Lf.nx, Lc.nx), fy = h_factor(Lf.ny, Lc.ny), fz = h_factor(Lf.nz, Lc.nz);
  if (!fx || !fy || !fz) return hipErrorInvalidValue;
  if (kind == 0)
    k_h_prolong_add<T><<<grid_for(Lf.n_nodes), 256, 0, s>>>(static_cast<const T*>(in), static_cast<T*>(out), Lf, Lc,
                                                            fx, fy, fz, periodic);
  else if (kind == 1)
    k_h_restrict_add<T><<<grid_for(Lc.n_nodes), 256, 0, s>>>(static_cast<const T*>(in), static_cast<T*>(out), Lf, Lc,
                                                              fx, fy, fz, periodic);
  else
    k_h_inject<<<grid_for(Lc.n_nodes), 256, 0, s>>>(static_cast<const double*>(in), static_cast<double*>(out), Lf, Lc,
                                                    fx, fy, fz);
  return hipGetLastError();
}

template <typename T>
hipError_t transfer(int kind, const void* in, void* out, const Lattice& Lf, const Lattice& Lc,
                    int periodic, hipStream_t s) {
  if (Lf.p == 1 && Lc.p == 1) return h_transfer<T>(kind, in, out, Lf, Lc, periodic, s);
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
  std::vector<double> lmax;   // Chebyshev upper bound: largest Ritz value times the safety factor
  std::vector<double> lmin;   // smallest Ritz value
  std::vector<int> mode;  // storage mode of each level's operator (-1 before the first update)
  DevBuf dots;  // 3 doubles
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ready = false;
  int vcycles = 0;
  std::string err;
  // Newton / Krylov work vectors (FP64, finest level)
  DevBuf r, x, p, q, z, f;
  DevBuf us, du;                      // load stepping: displacement at the step's start, last increment
  DevBuf cg;                          // device scalars of the PCG (CG_*), with the ||r||^2 history
  hipGraphExec_t cg_exec = nullptr;   // one PCG iteration, captured per linearisation
  // dense coarse solve: the coarsest operator is assembled by probing, factored by Cholesky and
  // kept as its explicit inverse (hierarchy precision)
  bool dense = false;
  rocblas_handle blas = nullptr;
  DevBuf cA, cB, cinv, cinfo;
};

namespace {

enum { B_B = 0, B_X, B_T, B_D, B_DINV, B_U, B_COUNT };

// PCG iterations between two reads of the residual history by the host
constexpr int kCgChunk = 4;

// largest coarsest level (DoFs) that the dense coarse solve accepts
// the automatic choice takes the dense solve up to 8192 DoFs; asked for explicitly, up to 32768
// (the factor, the identity/inverse and the FP32 or FP64 inverse take 20 n^2 bytes at most: 21 GB)
constexpr int64_t kDenseCoarseAuto = 8192;
constexpr int64_t kDenseCoarseMax = 32768;

hx_status mg_fail(hx_mg mg, hx_status s, const std::string& m) {
  if (mg) mg->err = m;
  return s;
}

// Storage precision of level l: the hierarchy's, except that the coarsest level of a hierarchy
// with 16-bit data keeps FP32 data (its operator is assembled and factored).
hx_precision level_prec(const hx_mg mg, int l) {
  if (!mg->fp32) return HX_FP64;
  const bool coarsest = l == static_cast<int>(mg->lv.size()) - 1;
  return coarsest ? HX_FP32 : mg->opt.precision;
}

bool sixteen_bit(hx_precision p) { return p == HX_FP32_BF16DATA || p == HX_FP32_FP16DATA; }

size_t vec_bytes(const hx_mg mg, int l) {
  return static_cast<size_t>(3 * mg->lv[l]->L.n_nodes) * (mg->fp32 ? sizeof(float) : sizeof(double));
}

template <typename T>
hipError_t level_apply(hx_mg mg, int l, const T* x, T* y) {
  const hx_status st = hx_apply_tangent(mg->lv[l], x, y, level_prec(mg, l), mg->stream);
  return st == HX_OK ? hipSuccess : hipErrorLaunchFailure;
}

// The level apply followed, in its node kernel, by a smoother step or the residual (see
// NodeEpilogue); y receives the residual (kEpiResidual) and is otherwise not written.
template <typename T>
hipError_t level_apply_epi(hx_mg mg, int l, T* x, T* y, int kind, const T* b, T* d, const T* dinv, double c1,
                           double c2) {
  const NodeEpilogue epi{kind, b, x, d, dinv, c1, c2, mg->opt.smoother_blocks};
  const hx_status st = hx::apply_with_epilogue(mg->lv[l], x, y, level_prec(mg, l), mg->stream, epi);
  return st == HX_OK ? hipSuccess : hipErrorLaunchFailure;
}

// Chebyshev-Jacobi on level l: x <- approximately A^-1 b, degree `deg`, starting from x (zero_init:
// from 0). Eigenvalue interval [lmax / range, lmax] for smoothing; the coarse solve widens it down
// to the smallest Ritz value (modes below the interval are still damped, never amplified).
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
  const bool coarse = l == static_cast<int>(mg->lv.size()) - 1;
  const double lmax = mg->lmax[l];
  const double lmin = coarse ? std::min(lmax / mg->opt.smoothing_range, mg->lmin[l]) : lmax / mg->opt.smoothing_range;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho_old = 1.0 / sigma;
  hipError_t e;
  const bool fuse = mg->opt.fuse_smoother != 0;
  const bool blk = mg->opt.smoother_blocks != 0;
  const int64_t nn = c->L.n_nodes;
  // separate smoother steps: point or nodal block Jacobi
  auto first_step = [&](const T* tt, int first) {
    if (blk)
      k_cheb_first_blk<T><<<grid_for(nn), 256, 0, mg->stream>>>(x, d, b, tt, dinv, static_cast<T>(1.0 / theta), first, nn);
    else
      k_cheb_first<T><<<grid_for(n), 256, 0, mg->stream>>>(x, d, b, tt, dinv, static_cast<T>(1.0 / theta), first, n);
  };
  if (zero_init) {
    first_step(nullptr, 1);
  } else if (fuse) {
    // the step in the apply's node kernel (no separate pass over the vectors)
    if ((e = level_apply_epi<T>(mg, l, x, t, kEpiChebyshevFirst, b, d, dinv, 0.0, 1.0 / theta)) != hipSuccess)
      return e;
  } else {
    if ((e = level_apply<T>(mg, l, x, t)) != hipSuccess) return e;
    first_step(t, 0);
  }
  for (int k = 1; k < deg; ++k) {
    const double rho = 1.0 / (2.0 * sigma - rho_old);
    const double c1 = rho * rho_old, c2 = 2.0 * rho / delta;
    if (fuse) {
      if ((e = level_apply_epi<T>(mg, l, x, t, kEpiChebyshev, b, d, dinv, c1, c2)) != hipSuccess) return e;
    } else {
      if ((e = level_apply<T>(mg, l, x, t)) != hipSuccess) return e;
      if (blk)
        k_cheb_step_blk<T><<<grid_for(nn), 256, 0, mg->stream>>>(x, d, b, t, dinv, static_cast<T>(c1),
                                                                 static_cast<T>(c2), nn);
      else
        k_cheb_step<T><<<grid_for(n), 256, 0, mg->stream>>>(x, d, b, t, dinv, static_cast<T>(c1), static_cast<T>(c2), n);
    }
    rho_old = rho;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t vcycle_level(hx_mg mg, int l) {
  const int L = static_cast<int>(mg->lv.size());
  hipError_t e;
  if (l == L - 1) {
    if (!mg->dense) return chebyshev<T>(mg, l, mg->opt.coarse_degree, true);
    const int64_t n = 3 * mg->lv[l]->L.n_nodes;
    DevBuf* B = mg->buf[l].get();
    const int64_t blocks = (n * 64 + 255) / 256;
    k_dense_mv<T><<<static_cast<unsigned>(blocks), 256, 0, mg->stream>>>(mg->cinv.as<T>(), B[B_B].as<T>(),
                                                                         B[B_X].as<T>(), n);
    return hipGetLastError();
  }
  if ((e = chebyshev<T>(mg, l, mg->opt.smoother_degree, true)) != hipSuccess) return e;
  const hx_ctx cf = mg->lv[l], cc = mg->lv[l + 1];
  DevBuf* Bf = mg->buf[l].get();
  DevBuf* Bc = mg->buf[l + 1].get();
  const int64_t nf = 3 * cf->L.n_nodes, nc = 3 * cc->L.n_nodes;
  // t = b - A x (residual of the smoothed iterate)
  if (mg->opt.fuse_smoother) {
    if ((e = level_apply_epi<T>(mg, l, Bf[B_X].as<T>(), Bf[B_T].as<T>(), kEpiResidual, Bf[B_B].as<T>(), nullptr,
                                nullptr, 0.0, 0.0)) != hipSuccess)
      return e;
  } else {
    if ((e = level_apply<T>(mg, l, Bf[B_X].as<T>(), Bf[B_T].as<T>())) != hipSuccess) return e;
    k_axpby<T><<<grid_for(nf), 256, 0, mg->stream>>>(Bf[B_T].as<T>(), T(1), Bf[B_B].as<T>(), T(-1), nf);
  }
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

// Number of eigenvalues below x of the symmetric tridiagonal matrix (diagonal a, off-diagonal b),
// by the Sturm sequence of its leading principal minors.
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int c = 0;
  double q = a[0] - x;
  if (q < 0.0) ++c;
  for (size_t i = 1; i < a.size(); ++i) {
    const double qp = q != 0.0 ? q : 1e-300;
    q = a[i] - x - b[i - 1] * b[i - 1] / qp;
    if (q < 0.0) ++c;
  }
  return c;
}

// k-th smallest eigenvalue (k = 0 .. m-1) of the tridiagonal matrix by bisection inside the
// Gershgorin interval.
double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int k) {
  double lo = 1e300, hi = -1e300;
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(a, b, mid) > k) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Extreme eigenvalues of D^-1 A on level l: Lanczos through eig_iters steps of Jacobi-
// preconditioned CG from a fixed pseudo-random start (zero on constrained rows). The Ritz values
// of the CG tridiagonal matrix, T_kk = 1/alpha_k + beta_(k-1)/alpha_(k-1),
// T_k,k+1 = sqrt(beta_k)/alpha_k, bound the spectrum from inside; the largest converges fast.
template <typename T>
hipError_t estimate_spectrum(hx_mg mg, int l, double* lmax, double* lmin) {
  const hx_ctx c = mg->lv[l];
  const int64_t n = 3 * c->L.n_nodes;
  DevBuf* B = mg->buf[l].get();
  T* r = B[B_B].as<T>();
  T* z = B[B_X].as<T>();
  T* q = B[B_T].as<T>();
  T* p = B[B_D].as<T>();
  const T* dinv = B[B_DINV].as<T>();
  const int64_t nn = c->L.n_nodes;
  // z = D^-1 r (point or nodal block Jacobi)
  auto precond = [&]() {
    if (mg->opt.smoother_blocks)
      k_cheb_first_blk<T><<<grid_for(nn), 256, 0, mg->stream>>>(z, z, r, nullptr, dinv, T(1), 1, nn);
    else
      k_cheb_first<T><<<grid_for(n), 256, 0, mg->stream>>>(z, z, r, nullptr, dinv, T(1), 1, n);
  };
  k_hash_vector<T><<<grid_for(n), 256, 0, mg->stream>>>(r, c->L);
  precond();
  k_convert<T, T><<<grid_for(n), 256, 0, mg->stream>>>(z, p, n);
  double h[3];
  hipError_t e = dots<T>(mg, n, 1, r, z, nullptr, nullptr, nullptr, nullptr, h);
  if (e != hipSuccess) return e;
  double rz = h[0];
  std::vector<double> alpha, beta;
  for (int it = 0; it < mg->opt.eig_iters && rz > 0.0; ++it) {
    if ((e = level_apply<T>(mg, l, p, q)) != hipSuccess) return e;
    if ((e = dots<T>(mg, n, 1, p, q, nullptr, nullptr, nullptr, nullptr, h)) != hipSuccess) return e;
    if (!(h[0] > 0.0)) break;
    const double a = rz / h[0];
    k_axpby<T><<<grid_for(n), 256, 0, mg->stream>>>(r, static_cast<T>(-a), q, T(1), n);
    precond();
    if ((e = dots<T>(mg, n, 1, r, z, nullptr, nullptr, nullptr, nullptr, h)) != hipSuccess) return e;
    const double bta = h[0] / rz;
    alpha.push_back(a);
    beta.push_back(bta);
    rz = h[0];
    k_axpby<T><<<grid_for(n), 256, 0, mg->stream>>>(p, T(1), z, static_cast<T>(bta), n);
  }
  if (alpha.empty()) return hipErrorInvalidValue;
  const size_t m = alpha.size();
  std::vector<double> da(m), ob(m > 1 ? m - 1 : 0);
  for (size_t k = 0; k < m; ++k) {
    da[k] = 1.0 / alpha[k] + (k > 0 ? beta[k - 1] / alpha[k - 1] : 0.0);
    if (k + 1 < m) ob[k] = std::sqrt(beta[k]) / alpha[k];
  }
  *lmax = tridiag_eig(da, ob, static_cast<int>(m) - 1);
  *lmin = tridiag_eig(da, ob, 0);
  return hipGetLastError();
}

// smallest colour count >= 2p + 1 along a lattice direction that keeps probe columns apart (a node
// couples with the nodes up to p indices away): any such k for an open direction (at most N, where
// every index is its own colour), a divisor of N for a periodic one (so the wrap keeps
// same-coloured nodes 2p + 1 or more indices apart), else N
int probe_colours(int N, bool periodic, int p) {
  const int k0 = 2 * p + 1;
  if (!periodic) return std::min(k0, N);
  for (int k = k0; k <= N; ++k)
    if (N % k == 0) return k;
  return N;
}

// Assembles the coarsest operator by probing (3 * kx * ky * kz applies, k >= 2p + 1 colours per
// direction), factors it by Cholesky (rocSOLVER, FP64) and stores its inverse in the hierarchy
// precision.
template <typename T>
hx_status dense_coarse_update(hx_mg mg) {
  const int l = static_cast<int>(mg->lv.size()) - 1;
  const Lattice& L = mg->lv[l]->L;
  const int64_t n = 3 * L.n_nodes;
  DevBuf* B = mg->buf[l].get();
  T* x = B[B_X].as<T>();
  T* y = B[B_T].as<T>();
  double* A = mg->cA.as<double>();
  const int kx = probe_colours(L.Nx, L.Nx == L.nx * L.p, L.p), ky = probe_colours(L.Ny, L.Ny == L.ny * L.p, L.p),
            kz = probe_colours(L.Nz, L.Nz == L.nz * L.p, L.p);
  k_fill<double><<<grid_for(n * n), 256, 0, mg->stream>>>(A, 0.0, n * n);
  for (int cc = 0; cc < 3; ++cc)
    for (int cz = 0; cz < kz; ++cz)
      for (int cy = 0; cy < ky; ++cy)
        for (int cx = 0; cx < kx; ++cx) {
          k_probe<T><<<grid_for(n), 256, 0, mg->stream>>>(x, L, kx, ky, kz, cx, cy, cz, cc);
          if (level_apply<T>(mg, l, x, y) != hipSuccess) return HX_E_HIP;
          k_probe_extract<T><<<grid_for(n), 256, 0, mg->stream>>>(y, A, L, kx, ky, kz, cx, cy, cz, cc);
        }
  k_identity<<<grid_for(n * n), 256, 0, mg->stream>>>(mg->cB.as<double>(), n);
  if (hipGetLastError() != hipSuccess) return HX_E_HIP;
  const rocblas_int nn = static_cast<rocblas_int>(n);
  rocblas_int* info = mg->cinfo.as<rocblas_int>();
  if (rocblas_set_stream(mg->blas, mg->stream) != rocblas_status_success ||
      rocsolver_dpotrf(mg->blas, rocblas_fill_lower, nn, A, nn, info) != rocblas_status_success)
    return HX_E_HIP;
  rocblas_int h_info = 0;
  if (hipMemcpyAsync(&h_info, info, sizeof(h_info), hipMemcpyDeviceToHost, mg->stream) != hipSuccess ||
      hipStreamSynchronize(mg->stream) != hipSuccess)
    return HX_E_HIP;
  if (h_info != 0) return HX_E_NONFINITE;  // not positive definite
  if (rocsolver_dpotrs(mg->blas, rocblas_fill_lower, nn, nn, A, nn, mg->cB.as<double>(), nn) != rocblas_status_success)
    return HX_E_HIP;
  k_convert<double, T><<<grid_for(n * n), 256, 0, mg->stream>>>(mg->cB.as<double>(), mg->cinv.as<T>(), n * n);
  return hipGetLastError() == hipSuccess ? HX_OK : HX_E_HIP;
}

template <typename T>
hipError_t level_diagonal(hx_mg mg, int l) {
  const hx_ctx c = mg->lv[l];
  const int64_t n = 3 * c->L.n_nodes;
  T* dinv = mg->buf[l][B_DINV].as<T>();
  const bool blk = mg->opt.smoother_blocks != 0;
  k_fill<T><<<grid_for(blk ? 2 * n : n), 256, 0, mg->stream>>>(dinv, T(0), blk ? 2 * n : n);
  const Slot& sl = c->slot[mg->fp32 ? 1 : 0];
  if (sl.variant != 0) return hipErrorInvalidValue;  // the diagonal reads the default layout
  HostArgs h = args_for(c);
  h.out = dinv;
  h.qdata = sl.qdata;
  h.cscale = sl.cscale;
  HostOp op{blk ? OpKind::DiagonalBlocks : OpKind::Diagonal, c->base.mat.law, HX_STORE_TANGENT, sl.store, mg->fp32};
  bool ok = false;
  hipError_t e = dispatch(c->p, op, h, mg->stream, &ok);
  if (!ok) return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  if (blk)
    k_block_finish<T><<<grid_for(c->L.n_nodes), 256, 0, mg->stream>>>(dinv, c->L);
  else
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
    // transfers, the diagonal and the coarse assembly address lattices
    if (levels[l]->topo == kTopoMap) return HX_E_UNSUPPORTED;
    if (l > 0) {
      const Lattice& a = levels[l - 1]->L;
      const Lattice& b = levels[l]->L;
      const int pa = (a.Nx == a.nx * a.p ? 1 : 0) | (a.Ny == a.ny * a.p ? 2 : 0) | (a.Nz == a.nz * a.p ? 4 : 0);
      const int pb = (b.Nx == b.nx * b.p ? 1 : 0) | (b.Ny == b.ny * b.p ? 2 : 0) | (b.Nz == b.nz * b.p ? 4 : 0);
      if (a.dir_faces != b.dir_faces || pa != pb) return HX_E_ARG;
      const bool same = a.nx == b.nx && a.ny == b.ny && a.nz == b.nz;
      if (same) {
        if (b.p >= a.p) return HX_E_ARG;  // degree transfer
      } else {
        // lattice transfer: degree 1 on both, every direction kept or halved
        if (a.p != 1 || b.p != 1 || !h_factor(a.nx, b.nx) || !h_factor(a.ny, b.ny) || !h_factor(a.nz, b.nz))
          return HX_E_ARG;
      }
    }
  }
  hx_mg_s* mg = new (std::nothrow) hx_mg_s();
  if (!mg) return HX_E_NOMEM;
  mg->lv.assign(levels, levels + n_levels);
  hx_mg_options o{};
  hx_mg_default_options(&o);
  if (opt) {
    o = *opt;
    const bool mode_ok = (o.level_mode >= HX_STORE_NONE && o.level_mode < kModes) || o.level_mode == HX_STORE_AUTO;
    if (o.smoother_degree < 1 || o.coarse_degree < 1 || o.eig_iters < 1 || !(o.smoothing_range > 1.0) ||
        !(o.eig_safety >= 1.0) ||
        (o.precision != HX_FP32 && o.precision != HX_FP64 && o.precision != HX_FP32_BF16DATA &&
         o.precision != HX_FP32_FP16DATA) ||
        !mode_ok ||
        o.coarse_solver < 0 || o.coarse_solver > 2 || o.fuse_smoother < 0 || o.fuse_smoother > 1 ||
        o.smoother_blocks < 0 || o.smoother_blocks > 1) {
      delete mg;
      return HX_E_ARG;
    }
  }
  mg->opt = o;
  mg->fp32 = o.precision != HX_FP64;
  const int64_t n_coarse = 3 * levels[n_levels - 1]->L.n_nodes;
  if (o.coarse_solver == 2 && n_coarse > kDenseCoarseMax) {
    delete mg;
    return HX_E_UNSUPPORTED;
  }
  mg->dense = o.coarse_solver == 2 || (o.coarse_solver == 0 && n_coarse <= kDenseCoarseAuto);
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
      // D^-1: 3 values per node (point Jacobi) or 6 (nodal blocks)
      const size_t b = k == B_U      ? 3 * levels[l]->L.n_nodes * sizeof(double)
                       : k == B_DINV ? vec_bytes(mg, l) * (o.smoother_blocks ? 2 : 1)
                                     : vec_bytes(mg, l);
      e = mg->buf[l][k].alloc(b);
    }
  }
  if (e == hipSuccess && mg->dense) {
    const size_t nn = static_cast<size_t>(n_coarse) * n_coarse;
    e = mg->cA.alloc(nn * sizeof(double));
    if (e == hipSuccess) e = mg->cB.alloc(nn * sizeof(double));
    if (e == hipSuccess) e = mg->cinv.alloc(nn * (mg->fp32 ? sizeof(float) : sizeof(double)));
    if (e == hipSuccess) e = mg->cinfo.alloc(sizeof(rocblas_int));
    if (e == hipSuccess && rocblas_create_handle(&mg->blas) != rocblas_status_success) e = hipErrorUnknown;
  }
  mg->lmax.assign(n_levels, 1.0);
  mg->lmin.assign(n_levels, 1.0);
  mg->mode.assign(n_levels, -1);
  if (e != hipSuccess) {
    hx_mg_destroy(mg);
    return e == hipErrorOutOfMemory ? HX_E_NOMEM : HX_E_HIP;
  }
  *out = mg;
  return HX_OK;
}

hx_status hx_mg_default_options(hx_mg_options* o) {
  if (!o) return HX_E_ARG;
  *o = hx_mg_options{};
  o->smoother_degree = 4;
  o->coarse_degree = 30;
  o->smoothing_range = 100.0;
  o->eig_iters = 20;
  o->eig_safety = 1.2;
  o->precision = HX_FP32;
  o->use_graph = 1;
  o->level_mode = HX_STORE_TANGENT;
  o->coarse_solver = 0;
  o->fuse_smoother = 1;
  o->smoother_blocks = 1;
  return HX_OK;
}

int32_t hx_mg_level_mode(hx_mg mg, int32_t level) {
  if (!mg || level < 0 || level >= static_cast<int32_t>(mg->mode.size())) return -1;
  return mg->mode[level];
}

hx_status hx_mg_destroy(hx_mg mg) {
  if (!mg) return HX_OK;
  if (mg->stream) (void)hipStreamSynchronize(mg->stream);
  if (mg->exec) (void)hipGraphExecDestroy(mg->exec);
  if (mg->graph) (void)hipGraphDestroy(mg->graph);
  if (mg->cg_exec) (void)hipGraphExecDestroy(mg->cg_exec);
  if (mg->ev_in) (void)hipEventDestroy(mg->ev_in);
  if (mg->ev_out) (void)hipEventDestroy(mg->ev_out);
  if (mg->blas) (void)rocblas_destroy_handle(mg->blas);
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
    const hx_precision lp = level_prec(mg, l);
    // the default configuration: the diagonal kernel reads the tangent in its block layout
    const hx_status st = hx::update_linearization(mg->lv[l], mg->buf[l][B_U].as<double>(), HX_STORE_TANGENT,
                                                  lp, mg->stream, 0, -1);
    if (st != HX_OK) return mg_fail(mg, st, std::string("hx_mg_update: level update: ") + hx_last_error(mg->lv[l]));
    e = mg->fp32 ? level_diagonal<float>(mg, l) : level_diagonal<double>(mg, l);
    if (e != hipSuccess) return mg_fail(mg, HX_E_HIP, "hx_mg_update: diagonal");
    // the level operator's own storage mode (the diagonal above needed the tangent); binary16
    // data exists for the stored tangent only
    hx_status sm = HX_OK;
    if (lp == HX_FP32_FP16DATA) {
      mg->mode[l] = HX_STORE_TANGENT;
    } else if (mg->mode[l] < 0 && mg->opt.level_mode == HX_STORE_AUTO) {
      hx_storage best = HX_STORE_TANGENT;
      sm = hx_autotune_storage(mg->lv[l], mg->buf[l][B_U].as<double>(), lp, 5, &best, nullptr, mg->stream);
      if (sm == HX_OK) mg->mode[l] = best;
    } else {
      if (mg->mode[l] < 0) mg->mode[l] = mg->opt.level_mode;
      if (mg->mode[l] != HX_STORE_TANGENT)
        sm = hx::update_linearization(mg->lv[l], mg->buf[l][B_U].as<double>(), static_cast<hx_storage>(mg->mode[l]),
                                      lp, mg->stream, 0, -1);
    }
    if (sm != HX_OK) return mg_fail(mg, sm, std::string("hx_mg_update: level mode: ") + hx_last_error(mg->lv[l]));
    double lm = 1.0, ln = 1.0;
    e = mg->fp32 ? estimate_spectrum<float>(mg, l, &lm, &ln) : estimate_spectrum<double>(mg, l, &lm, &ln);
    if (e != hipSuccess) return mg_fail(mg, HX_E_HIP, "hx_mg_update: eigenvalue estimate");
    if (!(lm > 0.0) || !std::isfinite(lm) || !(ln > 0.0))
      return mg_fail(mg, HX_E_NONFINITE, "hx_mg_update: eigenvalue estimate");
    mg->lmax[l] = lm * mg->opt.eig_safety;
    mg->lmin[l] = ln;
  }
  if (mg->dense) {
    const hx_status sd = mg->fp32 ? dense_coarse_update<float>(mg) : dense_coarse_update<double>(mg);
    if (sd != HX_OK)
      return mg_fail(mg, sd, sd == HX_E_NONFINITE ? "hx_mg_update: coarse matrix not positive definite"
                                                  : "hx_mg_update: dense coarse factorisation");
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
  const size_t bytes = vec_bytes(mg, level) * (mg->opt.smoother_blocks ? 2 : 1);
  const hipError_t e = hipMemcpyAsync(out, mg->buf[level][B_DINV].p, bytes, hipMemcpyDeviceToDevice, s);
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

// The preconditioner's kernels enqueued directly (for the capture of a whole PCG iteration).
static hx_status precondition_enqueue(hx_mg mg, const double* r, double* z) {
  const int64_t n0 = 3 * mg->lv[0]->L.n_nodes;
  DevBuf* B = mg->buf[0].get();
  if (mg->fp32)
    k_convert<double, float><<<grid_for(n0), 256, 0, mg->stream>>>(r, B[B_B].as<float>(), n0);
  else
    k_convert<double, double><<<grid_for(n0), 256, 0, mg->stream>>>(r, B[B_B].as<double>(), n0);
  if (vcycle_enqueue(mg) != hipSuccess) return HX_E_HIP;
  if (mg->fp32)
    k_convert<float, double><<<grid_for(n0), 256, 0, mg->stream>>>(B[B_X].as<float>(), z, n0);
  else
    k_convert<double, double><<<grid_for(n0), 256, 0, mg->stream>>>(B[B_X].as<double>(), z, n0);
  return hipGetLastError() == hipSuccess ? HX_OK : HX_E_HIP;
}

// One flexible PCG iteration (apply, inner products, updates, preconditioner) whose scalars live in
// mg->cg: nothing in it waits for the host.
static hx_status cg_iteration_enqueue(hx_mg mg, hx_ctx fine) {
  const int64_t n = 3 * fine->L.n_nodes;
  double* r = mg->r.as<double>();
  double* x = mg->x.as<double>();
  double* p = mg->p.as<double>();
  double* q = mg->q.as<double>();
  double* z = mg->z.as<double>();
  double* sc = mg->cg.as<double>();
  const int dg = std::min(grid_for(n), 1024);
  hx_status st = hx_apply_tangent(fine, p, q, HX_FP64, mg->stream);
  if (st != HX_OK) return st;
  k_dots<double><<<dg, 256, 0, mg->stream>>>(p, q, nullptr, nullptr, nullptr, nullptr, 1, sc + CG_PQ, n);
  k_cg_alpha<<<dg, 256, 0, mg->stream>>>(x, r, p, q, z, sc, n);
  if ((st = precondition_enqueue(mg, r, z)) != HX_OK) return st;
  k_dots<double><<<dg, 256, 0, mg->stream>>>(r, z, nullptr, nullptr, nullptr, nullptr, 1, sc + CG_RZN, n);
  k_cg_beta<<<grid_for(n), 256, 0, mg->stream>>>(p, z, sc, n);
  k_cg_roll<<<1, 64, 0, mg->stream>>>(sc);
  return hipGetLastError() == hipSuccess ? HX_OK : HX_E_HIP;
}

// Captures cg_iteration_enqueue into mg->cg_exec (the buffers of the current linearisation).
static hx_status capture_cg_iteration(hx_mg mg, hx_ctx fine) {
  if (mg->cg_exec) {
    (void)hipGraphExecDestroy(mg->cg_exec);
    mg->cg_exec = nullptr;
  }
  hipError_t e = hipStreamSynchronize(mg->stream);
  if (e == hipSuccess) e = hipStreamBeginCapture(mg->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return HX_E_HIP;
  const hx_status st = cg_iteration_enqueue(mg, fine);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(mg->stream, &g);
  if (st != HX_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != HX_OK ? st : HX_E_HIP;
  }
  e = hipGraphInstantiate(&mg->cg_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e == hipSuccess ? HX_OK : HX_E_HIP;
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
  DevBuf* W[] = {&mg->r, &mg->x, &mg->p, &mg->q, &mg->z, &mg->f};
  for (DevBuf* b : W)
    if ((e = b->alloc(nb)) != hipSuccess) return mg_fail(mg, HX_E_NOMEM, "hx_newton_solve: work vectors");
  if (opt->predictor && ((e = mg->us.alloc(nb)) != hipSuccess || (e = mg->du.alloc(nb)) != hipSuccess))
    return mg_fail(mg, HX_E_NOMEM, "hx_newton_solve: predictor vectors");
  if ((e = mg->cg.alloc(CG_COUNT * sizeof(double))) != hipSuccess)
    return mg_fail(mg, HX_E_NOMEM, "hx_newton_solve: scalars");
  hipStream_t caller = static_cast<hipStream_t>(stream);
  if ((e = hipEventRecord(mg->ev_in, caller)) != hipSuccess || (e = hipStreamWaitEvent(mg->stream, mg->ev_in, 0)) != hipSuccess)
    return mg_fail(mg, HX_E_HIP, "hx_newton_solve: stream order");
  double* r = mg->r.as<double>();
  double* x = mg->x.as<double>();
  double* p = mg->p.as<double>();
  double* z = mg->z.as<double>();
  double* f = mg->f.as<double>();
  hx_newton_report R{};
  const int vc0 = mg->vcycles;
  double h[CG_COUNT];
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
  const bool mode_ok = (opt->outer_mode >= HX_STORE_NONE && opt->outer_mode < kModes) ||
                       opt->outer_mode == HX_STORE_AUTO;
  if (!mode_ok) return mg_fail(mg, HX_E_ARG, "hx_newton_solve: unknown outer_mode");
  int outer = opt->outer_mode == HX_STORE_AUTO ? -1 : opt->outer_mode;
  double* us = opt->predictor ? mg->us.as<double>() : nullptr;
  double* du = opt->predictor ? mg->du.as<double>() : nullptr;
  for (int step = 1; step <= opt->load_steps && status == HX_OK; ++step) {
    const double scale = static_cast<double>(step) / opt->load_steps;
    if ((status = residual(scale)) != HX_OK) break;
    if ((e = dots<double>(mg, n, 1, r, r, nullptr, nullptr, nullptr, nullptr, h)) != hipSuccess) { status = HX_E_HIP; break; }
    double rn = std::sqrt(h[0]);
    const double r0 = rn;
    if (us) {
      k_convert<double, double><<<grid_for(n), 256, 0, mg->stream>>>(u, us, n);
      if (step > 1) {
        // secant predictor u_k + (u_k - u_(k-1)). Its residual is often larger than at u_k (the
        // extrapolation's error sits in the stiff volumetric modes), yet Newton converges from it
        // in fewer steps, because one linear solve removes that error; it is dropped only where
        // the residual is not finite (a state that inverts cells)
        k_axpby<double><<<grid_for(n), 256, 0, mg->stream>>>(u, 1.0, du, 1.0, n);
        if ((status = residual(scale)) != HX_OK) break;
        if ((e = dots<double>(mg, n, 1, r, r, nullptr, nullptr, nullptr, nullptr, h)) != hipSuccess) { status = HX_E_HIP; break; }
        const double rp = std::sqrt(h[0]);
        const bool keep = std::isfinite(rp);
        if (keep) {
          rn = rp;
        } else {
          k_convert<double, double><<<grid_for(n), 256, 0, mg->stream>>>(us, u, n);
          if ((status = residual(scale)) != HX_OK) break;
        }
        if (opt->verbose) {
          std::fprintf(stderr, "[hx_newton] load step %d/%d  predictor |r|/|r0| %.3e (%s)\n", step, opt->load_steps,
                       rp / r0, keep ? "kept" : "dropped");
          std::fflush(stderr);
        }
      }
    }
    if (step == 1) R.initial_residual = r0;
    int it = 0;
    bool converged = rn <= std::max(opt->newton_abs_tol, opt->newton_rel_tol * r0);
    while (!converged && it < opt->max_newton) {
      const auto t_lin = std::chrono::steady_clock::now();
      // linearisation of the outer FP64 operator and of every multigrid level
      if (mg->fp32) {
        if (outer < 0) {
          // storage mode and configuration of the outer operator by the autotuner (recorded in the
          // context, so that the following updates of that mode use the same configuration)
          hx_tune_entry best{};
          status = hx_autotune(fine, u, HX_FP64, 5, nullptr, 0, nullptr, &best, mg->stream);
          outer = best.mode;
        } else {
          status = hx_update_linearization(fine, u, static_cast<hx_storage>(outer), HX_FP64, mg->stream);
        }
        if (status != HX_OK) break;
      }
      if ((status = hx_mg_update(mg, u, mg->stream)) != HX_OK) break;
      // flexible PCG on K dx = -r; the scalars stay on the device, every iteration is one graph
      // launch, and the host reads the residual history every kCgChunk iterations
      k_fill<double><<<grid_for(n), 256, 0, mg->stream>>>(x, 0.0, n);
      k_axpby<double><<<grid_for(n), 256, 0, mg->stream>>>(r, 0.0, r, -1.0, n);  // r <- -r (the right-hand side)
      if ((status = precondition(mg, r, z)) != HX_OK) break;
      k_convert<double, double><<<grid_for(n), 256, 0, mg->stream>>>(z, p, n);
      double* sc = mg->cg.as<double>();
      k_fill<double><<<1, 64, 0, mg->stream>>>(sc, 0.0, CG_COUNT);
      {
        const int dg = std::min(grid_for(n), 1024);
        k_dots<double><<<dg, 256, 0, mg->stream>>>(r, z, nullptr, nullptr, nullptr, nullptr, 1, sc + CG_RZ, n);
        k_dots<double><<<dg, 256, 0, mg->stream>>>(r, r, nullptr, nullptr, nullptr, nullptr, 1, sc + CG_RR, n);
      }
      if ((e = hipMemcpyAsync(h, sc, CG_COUNT * sizeof(double), hipMemcpyDeviceToHost, mg->stream)) != hipSuccess ||
          (e = hipStreamSynchronize(mg->stream)) != hipSuccess) {
        status = HX_E_HIP;
        break;
      }
      const double tol = opt->krylov_rel_tol * std::sqrt(h[CG_RR]);
      k_fill<double><<<1, 64, 0, mg->stream>>>(sc + CG_RR, 0.0, 1);
      k_fill<double><<<1, 64, 0, mg->stream>>>(sc + CG_TOL2, tol * tol, 1);
      // the graph holds the buffers of this linearisation: captured again at every Newton step
      if (mg->opt.use_graph && (status = capture_cg_iteration(mg, fine)) != HX_OK) break;
      const double lin_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_lin).count();
      int k = 0;
      double stop = 0.0;
      while (stop == 0.0 && k < opt->max_krylov) {
        const int m = std::min(kCgChunk, opt->max_krylov - k);
        for (int i = 0; i < m && status == HX_OK; ++i) {
          if (mg->cg_exec && mg->opt.use_graph)
            status = hipGraphLaunch(mg->cg_exec, mg->stream) == hipSuccess ? HX_OK : HX_E_HIP;
          else
            status = cg_iteration_enqueue(mg, fine);
        }
        mg->vcycles += m;
        if (status != HX_OK) break;
        if ((e = hipMemcpyAsync(h, sc, CG_COUNT * sizeof(double), hipMemcpyDeviceToHost, mg->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(mg->stream)) != hipSuccess) {
          status = HX_E_HIP;
          break;
        }
        k = static_cast<int>(h[CG_ITERS]);
        stop = h[CG_STOP];
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
      if (opt->verbose) {
        std::fprintf(stderr, "[hx_newton] load step %d/%d  Newton %d  CG %d  |r|/|r0| %.3e  %.2f s (linearisation %.3f s)\n",
                     step, opt->load_steps, it, k, rn / r0,
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(), lin_s);
        std::fflush(stderr);
      }
    }
    R.newton_iters += it;
    R.final_residual = rn;
    if (us && status == HX_OK) {
      // this step's increment, from the previous converged displacement
      k_convert<double, double><<<grid_for(n), 256, 0, mg->stream>>>(u, du, n);
      k_axpby<double><<<grid_for(n), 256, 0, mg->stream>>>(du, -1.0, us, 1.0, n);
    }
    if (status == HX_OK) {
      R.load_steps_done = step;
      if (!converged) status = HX_E_NOT_CONVERGED;
    }
  }
  (void)hipStreamSynchronize(mg->stream);
  R.vcycles = mg->vcycles - vc0;
  R.outer_mode = mg->fp32 ? outer : mg->mode[0];
  R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = R;
  (void)hipEventRecord(mg->ev_out, mg->stream);
  (void)hipStreamWaitEvent(caller, mg->ev_out, 0);
  if (status == HX_E_HIP) return mg_fail(mg, status, "hx_newton_solve: HIP error");
  if (status == HX_E_NOT_CONVERGED) return mg_fail(mg, status, "hx_newton_solve: Newton did not converge");
  return status;
}

}  // extern "C"
