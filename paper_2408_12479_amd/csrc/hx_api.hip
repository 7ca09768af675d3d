// Host runtime of libhx.so: context setup, device memory, 1D basis tables and the C ABI of hx.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "hx.h"
#include "hx_context.hpp"
#include "hx_internal.hpp"

namespace hx {

// ------------------------------------------------------------------------------------------
// 1D rules on [0, 1] (host, long double Newton iterations)
// ------------------------------------------------------------------------------------------
static void legendre_ld(int n, long double x, long double& P, long double& dP) {
  long double p0 = 1.0L, p1 = x;
  if (n == 0) {
    P = 1.0L;
    dP = 0.0L;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = n * (p0 - x * p1) / (1.0L - x * x);
}

// Gauss-Legendre points/weights of n points on [0, 1] (roots of P_n by Newton).
static void gauss_points(int n, std::vector<double>& x, std::vector<double>& w) {
  const long double pi = 3.141592653589793238462643383279503L;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    long double z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    long double P, dP;
    for (int it = 0; it < 100; ++it) {
      legendre_ld(n, z, P, dP);
      const long double dz = P / dP;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    legendre_ld(n, z, P, dP);
    // z descends with i; store ascending on [0, 1]
    x[n - 1 - i] = static_cast<double>(0.5L * (1.0L + z));
    w[n - 1 - i] = static_cast<double>(1.0L / ((1.0L - z * z) * dP * dP));
  }
}

// Gauss-Lobatto points of degree p on [0, 1]: end points and the roots of P_p'.
static std::vector<double> gll_points(int p) {
  std::vector<double> x(p + 1);
  x[0] = 0.0;
  x[p] = 1.0;
  const long double pi = 3.141592653589793238462643383279503L;
  for (int i = 1; i < p; ++i) {
    long double z = -std::cos(pi * i / p);  // Chebyshev-Lobatto guess, ascending
    for (int it = 0; it < 100; ++it) {
      long double P, dP;
      legendre_ld(p, z, P, dP);
      const long double d2P = (2.0L * z * dP - p * (p + 1) * P) / (1.0L - z * z);
      const long double dz = dP / d2P;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    x[i] = static_cast<double>(0.5L * (1.0L + z));
  }
  return x;
}

static long double lagrange(const std::vector<double>& nodes, int i, long double x) {
  long double v = 1.0L;
  for (size_t m = 0; m < nodes.size(); ++m)
    if (static_cast<int>(m) != i) v *= (x - nodes[m]) / ((long double)nodes[i] - nodes[m]);
  return v;
}

static long double lagrange_deriv(const std::vector<double>& nodes, int i, long double x) {
  long double s = 0.0L;
  const int n = static_cast<int>(nodes.size());
  for (int m = 0; m < n; ++m) {
    if (m == i) continue;
    long double t = 1.0L / ((long double)nodes[i] - nodes[m]);
    for (int l = 0; l < n; ++l)
      if (l != i && l != m) t *= (x - nodes[l]) / ((long double)nodes[i] - nodes[l]);
    s += t;
  }
  return s;
}

static void basis_tables(int p, HostArgs& h, std::vector<double>& gll) {
  const int n = p + 1;
  std::vector<double> xq, wq;
  gauss_points(n, xq, wq);
  gll = gll_points(p);
  for (int q = 0; q < n; ++q) {
    h.x[q] = xq[q];
    h.w[q] = wq[q];
    for (int i = 0; i < n; ++i) {
      h.B[q * n + i] = static_cast<double>(lagrange(gll, i, xq[q]));
      h.D[q * n + i] = static_cast<double>(lagrange_deriv(xq, i, xq[q]));
    }
  }
}

// Modified Bessel functions I0, I1 by their power series (all terms positive).
static double bessel_i(int order, double a) {
  const double h = 0.5 * a;
  double term = order == 0 ? 1.0 : h, sum = term;
  for (int k = 1; k < 500; ++k) {
    term *= h * h / (static_cast<double>(k) * (k + order));
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

}  // namespace hx

using namespace hx;

namespace {

thread_local std::string g_setup_error;

// Element-vector buffer of hx_apply_tangent_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends). Host code never passes the array's
// name to a kernel: it is a host-side stand-in, not a device address. The device address of each
// GPU's copy is looked up once, with that device current, by the setup calls.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first call per device)
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace

namespace {

hx_status fail(hx_ctx ctx, hx_status s, const std::string& msg) {
  if (ctx)
    ctx->err = msg;
  else
    g_setup_error = msg;
  return s;
}

hx_status hip_fail(hx_ctx ctx, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(ctx, e == hipErrorOutOfMemory ? HX_E_NOMEM : HX_E_HIP, m);
}

}  // namespace

hipError_t hx::dispatch(int p, const HostOp& op, const HostArgs& h, hipStream_t s, bool* ok) {
#define HX_CASE(d)                                                       \
  case d:                                                                \
    switch (h.topo) {                                                    \
      case kTopoLattice: return dispatch_p##d##_t0(op, h, s, ok);        \
      case kTopoLatticeG: return dispatch_p##d##_t1(op, h, s, ok);       \
      case kTopoMap: return dispatch_p##d##_t2(op, h, s, ok);            \
      default: break;                                                    \
    }                                                                    \
    break;
  switch (p) {
    HX_CASE(1)
    HX_CASE(2)
    HX_CASE(3)
    HX_CASE(4)
    HX_CASE(5)
    HX_CASE(6)
    default: break;
  }
#undef HX_CASE
  *ok = false;
  return hipSuccess;
}

int hx::cells_per_block(int p, int variant) {
  switch (p) {
    case 1: return cells_per_block_p1(variant);
    case 2: return cells_per_block_p2(variant);
    case 3: return cells_per_block_p3(variant);
    case 4: return cells_per_block_p4(variant);
    case 5: return cells_per_block_p5(variant);
    case 6: return cells_per_block_p6(variant);
    default: return 1;
  }
}

namespace {

hipError_t write_consts(int p, const HostArgs& h) {
  switch (p) {
    case 1: return consts_p1(h);
    case 2: return consts_p2(h);
    case 3: return consts_p3(h);
    case 4: return consts_p4(h);
    case 5: return consts_p5(h);
    case 6: return consts_p6(h);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool hx::host_constrained(const hx_ctx_s* c, int64_t node) {
  if (c->topo == kTopoMap) return c->cons_host[static_cast<size_t>(node)] != 0;
  const Lattice& L = c->L;
  const int I = static_cast<int>(node % L.Nx);
  const int J = static_cast<int>((node / L.Nx) % L.Ny);
  const int K = static_cast<int>(node / (static_cast<int64_t>(L.Nx) * L.Ny));
  const uint32_t f = L.dir_faces;
  return ((f & 1u) && I == 0) || ((f & 2u) && I == L.Nx - 1) || ((f & 4u) && J == 0) ||
         ((f & 8u) && J == L.Ny - 1) || ((f & 16u) && K == 0) || ((f & 32u) && K == L.Nz - 1);
}

namespace {

// vertex v = a + 2b + 4c of cell (ex, ey, ez)
const double* cell_vertex(const hx_ctx_s* c, int ex, int ey, int ez, int v) {
  const Lattice& L = c->L;
  int vx = ex + (v & 1), vy = ey + ((v >> 1) & 1), vz = ez + (v >> 2);
  vx = vx >= L.Vx ? vx - L.Vx : vx;
  vy = vy >= L.Vy ? vy - L.Vy : vy;
  vz = vz >= L.Vz ? vz - L.Vz : vz;
  return &c->vert_host[3 * (vx + static_cast<int64_t>(L.Vx) * (vy + static_cast<int64_t>(L.Vy) * vz))];
}

void trilinear(const hx_ctx_s* c, int ex, int ey, int ez, double s, double t, double r, double* X) {
  X[0] = X[1] = X[2] = 0.0;
  for (int v = 0; v < 8; ++v) {
    const double wv = ((v & 1) ? s : 1 - s) * (((v >> 1) & 1) ? t : 1 - t) * ((v >> 2) ? r : 1 - r);
    const double* P = cell_vertex(c, ex, ey, ez, v);
    for (int k = 0; k < 3; ++k) X[k] += wv * P[k];
  }
}

// smallest det J0 over all Gauss points of all cells (trilinear maps)
double min_detJ0(const hx_ctx_s* c) {
  const Lattice& L = c->L;
  const int n = c->p + 1;
  double mn = 1e300;
  for (int ez = 0; ez < L.nz; ++ez)
    for (int ey = 0; ey < L.ny; ++ey)
      for (int ex = 0; ex < L.nx; ++ex) {
        const double* X[8];
        for (int v = 0; v < 8; ++v) X[v] = cell_vertex(c, ex, ey, ez, v);
        for (int qz = 0; qz < n; ++qz)
          for (int qy = 0; qy < n; ++qy)
            for (int qx = 0; qx < n; ++qx) {
              const double s = c->base.x[qx], t = c->base.x[qy], r = c->base.x[qz];
              double J[9];
              for (int k = 0; k < 3; ++k) {
                J[3 * k + 0] = (1 - t) * (1 - r) * (X[1][k] - X[0][k]) + t * (1 - r) * (X[3][k] - X[2][k]) +
                               (1 - t) * r * (X[5][k] - X[4][k]) + t * r * (X[7][k] - X[6][k]);
                J[3 * k + 1] = (1 - s) * (1 - r) * (X[2][k] - X[0][k]) + s * (1 - r) * (X[3][k] - X[1][k]) +
                               (1 - s) * r * (X[6][k] - X[4][k]) + s * r * (X[7][k] - X[5][k]);
                J[3 * k + 2] = (1 - s) * (1 - t) * (X[4][k] - X[0][k]) + s * (1 - t) * (X[5][k] - X[1][k]) +
                               (1 - s) * t * (X[6][k] - X[2][k]) + s * t * (X[7][k] - X[3][k]);
              }
              const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                                 J[2] * (J[3] * J[7] - J[4] * J[6]);
              mn = std::min(mn, det);
            }
      }
  return mn;
}

template <typename T>
__global__ void copy_convert(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = static_cast<T>(src[i]);
}

__global__ void clear_flag(int* f) { *f = 0; }

// A fixed non-trivial direction for timing runs: x_i = 1 + (i mod 7) / 8.
template <typename T>
__global__ void fill_timing_direction(T* __restrict__ x, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = T(1) + T(i % 7) * T(0.125);
}

// STREAM triad, two elements per thread with 16-byte loads and stores (the last thread of an odd
// n takes one element)
__global__ void stream_triad(double* __restrict__ a, const double* __restrict__ b,
                             const double* __restrict__ c, double s, int64_t n) {
  const int64_t i = 2 * (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x);
  if (i + 1 < n) {
    const double2 x = *reinterpret_cast<const double2*>(b + i);
    const double2 y = *reinterpret_cast<const double2*>(c + i);
    *reinterpret_cast<double2*>(a + i) = make_double2(x.x + s * y.x, x.y + s * y.y);
  } else if (i < n) {
    a[i] = b[i] + s * c[i];
  }
}

// FP64 issue-rate probe: per thread, independent dependency chains of vector fused multiply-adds
// (kind 0), of 16x16x4 FP64 matrix instructions (kind 1), or both in every wave with equal flops of
// each (kind 2). Per wave and iteration: 64 vector FMA instructions (8 chains x 8 steps, 64 lanes
// x 2 flops each = 8192 flops) and 4 matrix instructions (16 x 16 x 4 x 2 = 2048 flops each).
constexpr int kProbeBlocks = 2048, kProbeThreads = 256;
typedef double probe_d4 __attribute__((ext_vector_type(4)));

template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) fp64_pipe_probe(int64_t iters, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const double y = 0.999999, z = 1e-6;
  double x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = 1e-3 * c;
  probe_d4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = probe_d4{0.0, 0.0, 0.0, 0.0};
  const double a = 1e-3 * lane, b = 1e-3;
  for (int64_t it = 0; it < iters; ++it) {
    if constexpr (KIND != 1) {
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = fma(x[c], y, z);
    }
    if constexpr (KIND != 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
  }
  double s = 0.0;
  if constexpr (KIND != 1) {
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
  }
  if constexpr (KIND != 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) s += (acc[c][0] + acc[c][1]) + (acc[c][2] + acc[c][3]);
  }
  out[static_cast<int64_t>(blockIdx.x) * kProbeThreads + threadIdx.x] = s;
}

int grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, 8192)));
}

}  // namespace

HostArgs hx::args_for(const hx_ctx_s* c) {
  HostArgs h = c->base;
  h.vert64 = c->vert64;
  h.flag = c->flag;
  h.ework = c->ework;
  h.cblk64 = c->cblk64;
  h.cblk32 = c->cblk32;
  h.fib64 = c->fib64;
  h.fib32 = c->fib32;
  h.topo = c->topo;
  h.map = c->map;
  h.nptr = c->nptr;
  h.nslot = c->nslot;
  h.cmask = c->cmask;
  h.geo64 = c->geo64;
  h.geo32 = c->geo32;
  return h;
}

hx_status hx::set_error(hx_ctx_s* ctx, hx_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

namespace {

int store_of(hx_precision p) {
  switch (p) {
    case HX_FP64: return kStoreF64;
    case HX_FP32: return kStoreF32;
    case HX_FP32_BF16DATA: return kStoreBF16;
    case HX_FP32_FP16DATA: return kStoreF16;
  }
  return -1;
}

size_t store_bytes(int s) { return s == kStoreF64 ? 8 : (s == kStoreF32 ? 4 : 2); }

void release_slot(Slot& s) {
  if (s.qdata) (void)hipFree(s.qdata);
  if (s.cscale) (void)hipFree(s.cscale);
  if (s.uk) (void)hipFree(s.uk);
  if (s.act) (void)hipFree(s.act);
  s = Slot();
}

// Per-cell structure tensors in global coordinates from the local frames (rows E1, E2, E3) and
// the material's local components: H = Q^T H_loc Q and M = Q^T M_loc with Q[a][i] = (E_a)_i.
// Output [cell][kFibWords] = H4 (9), H6 (9), M4 (3), M6 (3). False if a frame is not orthonormal
// to 1e-8 or not right-handed.
bool cell_fibers(const double* frames, int64_t cells, const hx_material& m, std::vector<double>& out) {
  out.assign(static_cast<size_t>(cells) * kFibWords, 0.0);
  for (int64_t e = 0; e < cells; ++e) {
    const double* Q = frames + 9 * e;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double d = 0.0;
        for (int i = 0; i < 3; ++i) d += Q[3 * a + i] * Q[3 * b + i];
        if (!(std::fabs(d - (a == b ? 1.0 : 0.0)) <= 1e-8)) return false;
      }
    const double det = Q[0] * (Q[4] * Q[8] - Q[5] * Q[7]) - Q[1] * (Q[3] * Q[8] - Q[5] * Q[6]) +
                       Q[2] * (Q[3] * Q[7] - Q[4] * Q[6]);
    if (!(det > 0.0)) return false;
    double* o = out.data() + kFibWords * e;
    const double* Hl[2] = {m.H4, m.H6};
    const double* Ml[2] = {m.M4, m.M6};
    for (int f = 0; f < 2; ++f) {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) v += Q[3 * a + i] * Hl[f][3 * a + b] * Q[3 * b + j];
          o[9 * f + 3 * i + j] = v;
        }
      for (int i = 0; i < 3; ++i) {
        double v = 0.0;
        for (int a = 0; a < 3; ++a) v += Q[3 * a + i] * Ml[f][a];
        o[18 + 3 * f + i] = v;
      }
    }
  }
  return true;
}

}  // namespace

extern "C" {

const char* hx_status_string(hx_status s) {
  switch (s) {
    case HX_OK: return "ok";
    case HX_E_ARG: return "invalid argument";
    case HX_E_HIP: return "HIP runtime error";
    case HX_E_NOMEM: return "out of device memory";
    case HX_E_STATE: return "call out of order";
    case HX_E_INVERTED: return "inverted element or deformation (det <= 0)";
    case HX_E_NONFINITE: return "non-finite linearisation data";
    case HX_E_NOT_CONVERGED: return "not converged";
    case HX_E_UNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

const char* hx_last_error(hx_ctx ctx) { return ctx ? ctx->err.c_str() : g_setup_error.c_str(); }

hx_status hx_fiber_structure(double a, double b, double phi, const double* E, double* H4,
                             double* H6, double* M4, double* M6) {
  if (!E || !H4 || !H6 || !M4 || !M6 || !(a >= 0.0) || !(b > 0.0) || !std::isfinite(phi))
    return fail(nullptr, HX_E_ARG, "hx_fiber_structure: invalid argument");
  const double pi = 3.14159265358979323846;
  const double H33 = 1.0 / (4.0 * b) - std::exp(-2.0 * b) / (std::sqrt(2.0 * pi * b) * std::erf(std::sqrt(2.0 * b)));
  const double ratio = bessel_i(1, a) / bessel_i(0, a);
  const double H11 = 0.5 * (1.0 - H33) * (1.0 + ratio);
  const double H22 = 0.5 * (1.0 - H33) * (1.0 - ratio);
  for (int fam = 0; fam < 2; ++fam) {
    const double ang = fam == 0 ? phi : -phi;
    const double c = std::cos(ang), s = std::sin(ang);
    double M1[3], M2[3], M3[3];
    for (int k = 0; k < 3; ++k) {
      M1[k] = c * E[k] + s * E[3 + k];
      M2[k] = -s * E[k] + c * E[3 + k];
      M3[k] = E[6 + k];
    }
    double* H = fam == 0 ? H4 : H6;
    double* M = fam == 0 ? M4 : M6;
    for (int i = 0; i < 3; ++i) {
      M[i] = M1[i];
      for (int j = 0; j < 3; ++j)
        H[3 * i + j] = H11 * M1[i] * M1[j] + H22 * M2[i] * M2[j] + H33 * M3[i] * M3[j];
    }
  }
  return HX_OK;
}

}  // extern "C"

// Setup steps shared by the lattice and the general meshes: basis tables, device buffers, fibre
// frames, constants, stored geometry (curved or general meshes) and the static buffer's address.
// On failure the context is destroyed.
hx_status hx::finish_setup(hx_ctx_s* c, const hx_material* mat, const hx_options* opt, const double* frames,
                           hx_ctx* out) {
  const int p = c->p;
  HostArgs& h = c->base;
  std::memset(&h, 0, sizeof(h));
  h.L = c->L;
  h.topo = c->topo;
  basis_tables(p, h, c->gll);
  h.mat = *mat;
  h.jpow_iters = opt ? opt->jpow_newton_iters : 0;
  const int64_t cells = c->L.n_cells;
  const int64_t q = static_cast<int64_t>(p + 1) * (p + 1) * (p + 1);
  const int64_t eb = cells_per_block(p);
  const int64_t padded = (cells + eb - 1) / eb * eb;
  hipError_t e;
  if ((e = hipMalloc(&c->flag, sizeof(int))) != hipSuccess ||
      (e = hipMalloc(&c->ework, 3 * padded * q * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&c->cblk64, kConstBlockBytes)) != hipSuccess ||
      (e = hipMalloc(&c->cblk32, kConstBlockBytes)) != hipSuccess) {
    hx_destroy(c);
    return hip_fail(nullptr, e, "hx_setup: allocation");
  }
  if ((e = hipMemset(c->flag, 0, sizeof(int))) != hipSuccess) {
    hx_destroy(c);
    return hip_fail(nullptr, e, "hx_setup: clear");
  }
  if (mat->law == HX_LAW_FIBER && frames) {
    std::vector<double> fib;
    if (!cell_fibers(frames, cells, *mat, fib)) {
      hx_destroy(c);
      return fail(nullptr, HX_E_ARG, "hx_setup: a cell frame is not orthonormal and right-handed");
    }
    std::vector<float> fib32(fib.begin(), fib.end());
    if ((e = hipMalloc(&c->fib64, fib.size() * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&c->fib32, fib.size() * sizeof(float))) != hipSuccess ||
        (e = hipMemcpy(c->fib64, fib.data(), fib.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->fib32, fib32.data(), fib.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) {
      hx_destroy(c);
      return hip_fail(nullptr, e, "hx_setup: cell frames");
    }
  }
  if (c->topo != kTopoLattice) {
    const hx_status st = build_stored_geometry(c);
    if (st != HX_OK) {
      const std::string msg = c->err;
      hx_destroy(c);
      return fail(nullptr, st, msg);
    }
  }
  HostArgs ha = args_for(c);
  if ((e = write_consts(p, ha)) != hipSuccess) {
    hx_destroy(c);
    return hip_fail(nullptr, e, "hx_setup: constants");
  }
  void* sp = nullptr;
  if ((e = scratch_address(c->device, &sp)) != hipSuccess) {
    hx_destroy(c);
    return hip_fail(nullptr, e, "hx_setup: address of the static element-vector buffer");
  }
  *out = c;
  return HX_OK;
}

hx_status hx::setup_fail(hx_status s, const std::string& msg) { return fail(nullptr, s, msg); }

bool hx::check_options(const hx_options* opt, const char* who) {
  if (!opt) return true;
  for (int i = 0; i < 6; ++i)
    if (opt->reserved[i]) {
      fail(nullptr, HX_E_ARG, std::string(who) + ": reserved option fields must be zero");
      return false;
    }
  if (opt->jpow_newton_iters < 0 || opt->jpow_newton_iters > 16) {
    fail(nullptr, HX_E_ARG, std::string(who) + ": jpow_newton_iters out of [0, 16]");
    return false;
  }
  return true;
}

extern "C" {

hx_status hx_setup_lattice(const hx_lattice* mesh, int32_t p, const hx_material* mat, const hx_options* opt,
                           hx_ctx* out) {
  if (!out) return fail(nullptr, HX_E_ARG, "hx_setup_lattice: out is NULL");
  *out = nullptr;
  if (!mesh || !mat) return fail(nullptr, HX_E_ARG, "hx_setup_lattice: NULL mesh or material");
  const bool curved = mesh->geom_nodes != nullptr;
  if (!curved && !mesh->vertices) return fail(nullptr, HX_E_ARG, "hx_setup_lattice: NULL vertices (and no geometry points)");
  if (p < 1 || p > kMaxDegree) return fail(nullptr, HX_E_UNSUPPORTED, "hx_setup_lattice: degree must be in [1, 6]");
  if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1) return fail(nullptr, HX_E_ARG, "hx_setup_lattice: empty lattice");
  if (mat->law != HX_LAW_CNH && mat->law != HX_LAW_INH && mat->law != HX_LAW_FIBER)
    return fail(nullptr, HX_E_ARG, "hx_setup_lattice: unknown law");
  if (!check_options(opt, "hx_setup_lattice")) return HX_E_ARG;
  if (mesh->dirichlet_faces >> 6) return fail(nullptr, HX_E_ARG, "hx_setup_lattice: dirichlet_faces has bits above 5");
  if (curved && (mesh->geom_degree < 1 || mesh->geom_degree > kMaxGeomDegree))
    return fail(nullptr, HX_E_ARG, "hx_setup_lattice: geom_degree out of [1, 8]");
  if (!curved && mesh->geom_degree > 1)
    return fail(nullptr, HX_E_ARG, "hx_setup_lattice: geom_degree > 1 needs geom_nodes");

  hx_ctx_s* c = new (std::nothrow) hx_ctx_s();
  if (!c) return fail(nullptr, HX_E_NOMEM, "hx_setup_lattice: host allocation failed");
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, HX_E_HIP, "hx_setup_lattice: no HIP device");
  }
  c->p = p;
  c->topo = curved ? kTopoLatticeG : kTopoLattice;
  Lattice& L = c->L;
  L.nx = mesh->nx;
  L.ny = mesh->ny;
  L.nz = mesh->nz;
  L.p = p;
  const int per = mesh->periodic;
  const int64_t cells = static_cast<int64_t>(L.nx) * L.ny * L.nz;
  L.Vx = L.nx + ((per & 1) ? 0 : 1);
  L.Vy = L.ny + ((per & 2) ? 0 : 1);
  L.Vz = L.nz + ((per & 4) ? 0 : 1);
  const int64_t Nx = static_cast<int64_t>(L.nx) * p + ((per & 1) ? 0 : 1);
  const int64_t Ny = static_cast<int64_t>(L.ny) * p + ((per & 2) ? 0 : 1);
  const int64_t Nz = static_cast<int64_t>(L.nz) * p + ((per & 4) ? 0 : 1);
  const int64_t nodes = Nx * Ny * Nz;
  const int64_t q = static_cast<int64_t>(p + 1) * (p + 1) * (p + 1);
  const int64_t eb = cells_per_block(p);
  if ((cells + eb) * q > (int64_t(1) << 31) - 1 || Nx > (1 << 30) || Ny > (1 << 30) || Nz > (1 << 30)) {
    delete c;
    return fail(nullptr, HX_E_ARG, "hx_setup_lattice: mesh too large (cells * (p+1)^3 must fit in int32)");
  }
  L.Nx = static_cast<int32_t>(Nx);
  L.Ny = static_cast<int32_t>(Ny);
  L.Nz = static_cast<int32_t>(Nz);
  L.n_cells = static_cast<int32_t>(cells);
  L.n_nodes = nodes;
  uint32_t faces = mesh->dirichlet_faces;
  if (per & 1) faces &= ~3u;
  if (per & 2) faces &= ~12u;
  if (per & 4) faces &= ~48u;
  L.dir_faces = faces;

  if (curved) {
    const int g = mesh->geom_degree;
    c->geom_degree = g;
    const size_t m3 = static_cast<size_t>(g + 1) * (g + 1) * (g + 1);
    c->geom_host.assign(mesh->geom_nodes, mesh->geom_nodes + 3 * m3 * cells);
    for (double v : c->geom_host)
      if (!std::isfinite(v)) {
        delete c;
        return fail(nullptr, HX_E_ARG, "hx_setup_lattice: non-finite geometry point");
      }
  } else {
    const int64_t nv = static_cast<int64_t>(L.Vx) * L.Vy * L.Vz;
    c->vert_host.assign(mesh->vertices, mesh->vertices + 3 * nv);
    for (double v : c->vert_host)
      if (!std::isfinite(v)) {
        delete c;
        return fail(nullptr, HX_E_ARG, "hx_setup_lattice: non-finite vertex coordinate");
      }
    HostArgs tmp{};  // the Gauss points for the check (finish_setup fills the context's tables)
    basis_tables(p, tmp, c->gll);
    std::memcpy(c->base.x, tmp.x, sizeof(tmp.x));
    if (!(min_detJ0(c) > 0.0)) {
      delete c;
      return fail(nullptr, HX_E_INVERTED, "hx_setup_lattice: det J0 <= 0 at a Gauss point of some cell");
    }
    hipError_t e;
    if ((e = hipMalloc(&c->vert64, 3 * nv * sizeof(double))) != hipSuccess ||
        (e = hipMemcpy(c->vert64, c->vert_host.data(), 3 * nv * sizeof(double), hipMemcpyHostToDevice)) !=
            hipSuccess) {
      hx_destroy(c);
      return hip_fail(nullptr, e, "hx_setup_lattice: vertices");
    }
  }
  return finish_setup(c, mat, opt, mesh->frames, out);
}

hx_status hx_destroy(hx_ctx ctx) {
  if (!ctx) return HX_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(ctx->device);
  for (Slot& s : ctx->slot) release_slot(s);
  if (ctx->vert64) (void)hipFree(ctx->vert64);
  if (ctx->flag) (void)hipFree(ctx->flag);
  if (ctx->ework) (void)hipFree(ctx->ework);
  if (ctx->cblk64) (void)hipFree(ctx->cblk64);
  if (ctx->cblk32) (void)hipFree(ctx->cblk32);
  if (ctx->fib64) (void)hipFree(ctx->fib64);
  if (ctx->fib32) (void)hipFree(ctx->fib32);
  if (ctx->geo64) (void)hipFree(ctx->geo64);
  if (ctx->geo32) (void)hipFree(ctx->geo32);
  if (ctx->map) (void)hipFree(ctx->map);
  if (ctx->nptr) (void)hipFree(ctx->nptr);
  if (ctx->nslot) (void)hipFree(ctx->nslot);
  if (ctx->cmask) (void)hipFree(ctx->cmask);
  (void)hipSetDevice(cur);
  delete ctx;
  return HX_OK;
}

int64_t hx_num_nodes(hx_ctx ctx) { return ctx ? ctx->L.n_nodes : -1; }
int64_t hx_num_dofs(hx_ctx ctx) { return ctx ? 3 * ctx->L.n_nodes : -1; }
int64_t hx_num_cells(hx_ctx ctx) { return ctx ? ctx->L.n_cells : -1; }

hx_status hx_node_coords(hx_ctx ctx, double* xyz) {
  if (!ctx || !xyz) return fail(ctx, HX_E_ARG, "hx_node_coords: NULL argument");
  const Lattice& L = ctx->L;
  const int p = ctx->p;
  if (ctx->topo == kTopoMap) {
    // the map of the cell where the node is first met (cells in order, local nodes x fastest)
    const int n = p + 1, Q = n * n * n;
    std::vector<uint8_t> seen(static_cast<size_t>(L.n_nodes), 0);
    for (int64_t e = 0; e < L.n_cells; ++e)
      for (int a = 0; a < Q; ++a) {
        const int64_t node = ctx->cell_nodes[static_cast<size_t>(e) * Q + a];
        if (seen[node]) continue;
        seen[node] = 1;
        const double xi[3] = {ctx->gll[a % n], ctx->gll[(a / n) % n], ctx->gll[a / (n * n)]};
        host_map(ctx, e, xi, xyz + 3 * node, nullptr);
      }
    return HX_OK;
  }
  for (int64_t node = 0; node < L.n_nodes; ++node) {
    const int lat[3] = {static_cast<int>(node % L.Nx), static_cast<int>((node / L.Nx) % L.Ny),
                        static_cast<int>(node / (static_cast<int64_t>(L.Nx) * L.Ny))};
    const int nc[3] = {L.nx, L.ny, L.nz};
    int cell[3];
    double loc[3];
    for (int d = 0; d < 3; ++d) {
      cell[d] = std::min(lat[d] / p, nc[d] - 1);
      loc[d] = ctx->gll[lat[d] - cell[d] * p];
    }
    if (ctx->topo == kTopoLattice)
      trilinear(ctx, cell[0], cell[1], cell[2], loc[0], loc[1], loc[2], xyz + 3 * node);
    else
      host_map(ctx, cell[0] + static_cast<int64_t>(L.nx) * (cell[1] + static_cast<int64_t>(L.ny) * cell[2]), loc,
               xyz + 3 * node, nullptr);
  }
  return HX_OK;
}

hx_status hx_constrained_mask(hx_ctx ctx, uint8_t* mask) {
  if (!ctx || !mask) return fail(ctx, HX_E_ARG, "hx_constrained_mask: NULL argument");
  for (int64_t node = 0; node < ctx->L.n_nodes; ++node) mask[node] = host_constrained(ctx, node) ? 1 : 0;
  return HX_OK;
}

hx_status hx_residual(hx_ctx ctx, const double* u, double* r, void* stream) {
  if (!ctx || !u || !r) return fail(ctx, HX_E_ARG, "hx_residual: NULL argument");
  if (static_cast<const void*>(u) == static_cast<const void*>(r)) return fail(ctx, HX_E_ARG, "hx_residual: u and r alias");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HostArgs h = args_for(ctx);
  h.in0 = u;
  h.out = r;
  HostOp op{OpKind::Residual, ctx->base.mat.law, HX_STORE_NONE, kStoreF64, false};
  bool ok = false;
  const hipError_t e = dispatch(ctx->p, op, h, s, &ok);
  if (!ok) return fail(ctx, HX_E_UNSUPPORTED, "hx_residual: not built");
  if (e != hipSuccess) return hip_fail(ctx, e, "hx_residual: launch");
  return HX_OK;
}

hx_status hx_residual_spatial(hx_ctx ctx, const double* u, double* r, void* stream) {
  if (!ctx || !u || !r) return fail(ctx, HX_E_ARG, "hx_residual_spatial: NULL argument");
  if (static_cast<const void*>(u) == static_cast<const void*>(r))
    return fail(ctx, HX_E_ARG, "hx_residual_spatial: u and r alias");
  HostArgs h = args_for(ctx);
  h.in0 = u;
  h.out = r;
  HostOp op{OpKind::Residual, ctx->base.mat.law, HX_STORE_SPATIAL, kStoreF64, false};
  bool ok = false;
  const hipError_t e = dispatch(ctx->p, op, h, static_cast<hipStream_t>(stream), &ok);
  if (!ok) return fail(ctx, HX_E_UNSUPPORTED, "hx_residual_spatial: not built");
  if (e != hipSuccess) return hip_fail(ctx, e, "hx_residual_spatial: launch");
  return HX_OK;
}

hx_status hx_update_linearization(hx_ctx ctx, const double* u, hx_storage mode, hx_precision prec,
                                  void* stream) {
  if (!ctx || !u) return fail(ctx, HX_E_ARG, "hx_update_linearization: NULL argument");
  int variant = 0, nt = -1;
  if (mode >= HX_STORE_NONE && mode < kModes && store_of(prec) >= 0) {
    const Tuning& t = ctx->tuned[prec == HX_FP64 ? 0 : 1][mode];
    if (t.set) {
      variant = t.variant;
      nt = t.nt;
    }
  }
  return hx::update_linearization(ctx, u, mode, prec, stream, variant, nt);
}

}  // extern "C"

hx_status hx::update_linearization(hx_ctx_s* ctx, const double* u, hx_storage mode, hx_precision prec,
                                   void* stream, int variant, int nt) {
  if (!ctx || !u) return fail(ctx, HX_E_ARG, "hx_update_linearization: NULL argument");
  if (variant < 0 || variant >= kVariants || (variant != 0 && ctx->topo != kTopoLattice))
    return fail(ctx, HX_E_ARG, "hx_update_linearization: cells-per-workgroup variant not available for this mesh");
  if (mode < HX_STORE_NONE || mode >= kModes) return fail(ctx, HX_E_ARG, "hx_update_linearization: unknown storage mode");
  // the modes that re-interpolate the linearisation point at every apply keep a copy of it
  const bool keeps_uk = mode == HX_STORE_NONE || mode == HX_STORE_SPATIAL_RECOMPUTE || mode == HX_STORE_SCALARS ||
                        mode == HX_STORE_SPATIAL_SCALARS;
  const int st = store_of(prec);
  if (st < 0) return fail(ctx, HX_E_ARG, "hx_update_linearization: unknown precision");
  // bfloat16 data (FP32 range) for every mode that stores data; binary16 (range limited, scaled per
  // cell by a power of two) for the stored tangent only; the modes that store nothing run as FP32
  if (st == kStoreF16 && (mode == HX_STORE_FINV_J || mode == HX_STORE_SPATIAL))
    return fail(ctx, HX_E_UNSUPPORTED, "hx_update_linearization: binary16 data only for the stored tangent");
  if ((st == kStoreF16 || st == kStoreBF16) &&
      (mode == HX_STORE_SCALARS || mode == HX_STORE_TENSORS || mode == HX_STORE_SPATIAL_SCALARS))
    return fail(ctx, HX_E_UNSUPPORTED, "hx_update_linearization: the scalar and tensor stages store FP64 or FP32 data");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Slot& sl = ctx->slot[prec == HX_FP64 ? 0 : 1];
  const Lattice& L = ctx->L;
  const int64_t Q = static_cast<int64_t>(ctx->p + 1) * (ctx->p + 1) * (ctx->p + 1);
  // whole workgroup blocks of cells (the last one may be partly unused)
  const int64_t eb = cells_per_block(ctx->p, variant);
  const int64_t padded_cells = (L.n_cells + eb - 1) / eb * eb;
  // blocks of eb cells, each rounded up to whole groups of stored words (the kernels' block
  // stride: one FP64 word, four FP32 or 16-bit words)
  const int64_t group = st == kStoreF64 ? 1 : 4;
  const int64_t block = (mode_words(mode, ctx->base.mat.law) * eb * Q + group - 1) / group * group;
  const size_t need = static_cast<size_t>(block) * (padded_cells / eb) * store_bytes(st);
  hipError_t e = hipStreamSynchronize(s);  // the slot's buffers may still be in use
  if (e != hipSuccess) return hip_fail(ctx, e, "hx_update_linearization: sync");
  // the slot is unusable from here until the new data has been written: a failure below leaves it
  // invalid (an apply then returns HX_E_STATE instead of reading stale or partial data)
  sl.valid = false;
  if (need > sl.qcap) {
    if (sl.qdata) (void)hipFree(sl.qdata);
    sl.qdata = nullptr;
    sl.qcap = 0;
    if ((e = hipMalloc(&sl.qdata, need)) != hipSuccess) {
      sl.qbytes = 0;
      return hip_fail(ctx, e, "hx_update_linearization: q-point data");
    }
    sl.qcap = need;
  }
  sl.qbytes = need;
  if (st == kStoreF16 && !sl.cscale) {
    if ((e = hipMalloc(&sl.cscale, L.n_cells * sizeof(float))) != hipSuccess) {
      return hip_fail(ctx, e, "hx_update_linearization: cell scales");
    }
  }
  const int64_t n = 3 * L.n_nodes;
  if (keeps_uk) {
    const size_t ub = n * (prec == HX_FP64 ? sizeof(double) : sizeof(float));
    if (!sl.uk) {
      if ((e = hipMalloc(&sl.uk, ub)) != hipSuccess) {
          return hip_fail(ctx, e, "hx_update_linearization: u_k");
      }
    }
    if (prec == HX_FP64)
      copy_convert<double><<<grid_for(n), 256, 0, s>>>(u, static_cast<double*>(sl.uk), n);
    else
      copy_convert<float><<<grid_for(n), 256, 0, s>>>(u, static_cast<float*>(sl.uk), n);
  }
  // FP32 recompute and F^-1+J modes of the fibre law: the tension switches are decided here in
  // FP64 and kept, so that the FP32 apply cannot flip them by rounding
  const bool keep_act = ctx->base.mat.law == HX_LAW_FIBER && prec != HX_FP64 &&
                        (mode == HX_STORE_NONE || mode == HX_STORE_SPATIAL_RECOMPUTE || mode == HX_STORE_FINV_J);
  if (keep_act) {
    const size_t ab = static_cast<size_t>(padded_cells) * Q;
    if (sl.act_bytes < ab) {
      if (sl.act) (void)hipFree(sl.act);
      sl.act = nullptr;
      sl.act_bytes = 0;
      if ((e = hipMalloc(&sl.act, ab)) != hipSuccess) {
          return hip_fail(ctx, e, "hx_update_linearization: fibre switches");
      }
      sl.act_bytes = ab;
    }
  }
  sl.keep_act = keep_act;
  clear_flag<<<1, 1, 0, s>>>(ctx->flag);
  HostArgs h = args_for(ctx);
  h.in0 = u;
  h.qdata_w = sl.qdata;
  h.cscale_w = sl.cscale;
  h.act_w = keep_act ? sl.act : nullptr;
  h.variant = variant;
  HostOp op{OpKind::Update, ctx->base.mat.law, mode, st, false};
  bool ok = false;
  e = dispatch(ctx->p, op, h, s, &ok);
  if (!ok) return fail(ctx, HX_E_UNSUPPORTED, "hx_update_linearization: combination not built");
  if (e != hipSuccess) return hip_fail(ctx, e, "hx_update_linearization: launch");
  int flag = 0;
  if ((e = hipMemcpyAsync(&flag, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(ctx, e, "hx_update_linearization: status read");
  sl.valid = true;
  sl.mode = mode;
  sl.store = st;
  sl.variant = variant;
  sl.nt = nt;
  if (flag & kFlagInverted) return fail(ctx, HX_E_INVERTED, "hx_update_linearization: J <= 0 at a q-point");
  if (flag & kFlagNonFinite) return fail(ctx, HX_E_NONFINITE, "hx_update_linearization: non-finite data");
  return HX_OK;
}

extern "C" {

}  // extern "C"

namespace {

// The apply with a given element-vector buffer (the context's, or the static one).
// (messages are formed only on failure: the successful path allocates nothing, host or device)
hx_status apply_with(hx_ctx ctx, const void* du, void* dst, hx_precision prec, void* stream, void* ework,
                     const char* who, const NodeEpilogue* epi = nullptr) {
  if (!ctx || !du || !dst) return fail(ctx, HX_E_ARG, std::string(who) + ": NULL argument");
  if (du == dst) return fail(ctx, HX_E_ARG, std::string(who) + ": du and dst alias");
  if (store_of(prec) < 0) return fail(ctx, HX_E_ARG, std::string(who) + ": unknown precision");
  const bool fp32 = prec != HX_FP64;
  const Slot& sl = ctx->slot[fp32 ? 1 : 0];
  if (!sl.valid) return fail(ctx, HX_E_STATE, std::string(who) + ": no linearisation stored for this precision");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HostArgs h = args_for(ctx);
  h.ework = ework;
  if (epi) h.epi = *epi;
  h.in0 = du;
  h.in1 = sl.uk;
  h.out = dst;
  h.qdata = sl.qdata;
  // stored data larger than the last-level cache is streamed (non-temporal loads); smaller data
  // may stay cached between applies (unless the autotuner chose otherwise)
  h.stream_qdata = sl.nt >= 0 ? sl.nt : (sl.qbytes > (size_t(128) << 20) ? 1 : 0);
  h.variant = sl.variant;
  h.cscale = sl.cscale;
  h.act = sl.keep_act ? sl.act : nullptr;
  HostOp op{OpKind::Apply, ctx->base.mat.law, sl.mode, sl.store, fp32};
  bool ok = false;
  const hipError_t e = dispatch(ctx->p, op, h, s, &ok);
  if (!ok) return fail(ctx, HX_E_UNSUPPORTED, std::string(who) + ": combination not built");
  if (e != hipSuccess) return hip_fail(ctx, e, (std::string(who) + ": launch").c_str());
  return HX_OK;
}

}  // namespace

hx_status hx::apply_with_epilogue(hx_ctx_s* ctx, const void* du, void* dst, hx_precision prec, void* stream,
                                  const NodeEpilogue& epi) {
  return apply_with(ctx, du, dst, prec, stream, ctx ? ctx->ework : nullptr, "level apply", &epi);
}

extern "C" {

hx_status hx_apply_tangent(hx_ctx ctx, const void* du, void* dst, hx_precision prec, void* stream) {
  return apply_with(ctx, du, dst, prec, stream, ctx ? ctx->ework : nullptr, "hx_apply_tangent");
}

hx_status hx_apply_tangent_noalloc(hx_ctx ctx, const void* du, void* dst, hx_precision prec, void* stream) {
  if (!ctx) return fail(ctx, HX_E_ARG, "hx_apply_tangent_noalloc: NULL context");
  // the element vectors of every cell: 3 components x cells (whole workgroups) x (p+1)^3 values of
  // the apply's type
  const int64_t q = static_cast<int64_t>(ctx->p + 1) * (ctx->p + 1) * (ctx->p + 1);
  const int64_t eb = cells_per_block(ctx->p);
  const int64_t padded = (static_cast<int64_t>(ctx->L.n_cells) + eb - 1) / eb * eb;
  const size_t need = static_cast<size_t>(3 * padded * q) * (prec == HX_FP64 ? sizeof(double) : sizeof(float));
  if (need > kScratchBytes)
    return fail(ctx, HX_E_ARG, "hx_apply_tangent_noalloc: the element vectors need " + std::to_string(need) +
                                   " bytes, more than the static buffer's " + std::to_string(kScratchBytes));
  void* sp = nullptr;
  const hipError_t e = scratch_address(ctx->device, &sp);  // set at hx_setup: a table read
  if (e != hipSuccess) return hip_fail(ctx, e, "hx_apply_tangent_noalloc: static buffer");
  return apply_with(ctx, du, dst, prec, stream, sp, "hx_apply_tangent_noalloc");
}

}  // extern "C"

namespace {

// Timing buffers of the autotuners: a fixed direction, an output and two events.
struct TuneBench {
  hx_ctx ctx;
  hx_precision prec;
  hipStream_t s;
  void* du = nullptr;
  void* dst = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~TuneBench() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (du) (void)hipFree(du);
    if (dst) (void)hipFree(dst);
  }
  hipError_t init() {
    const int64_t n = 3 * ctx->L.n_nodes;
    const size_t vb = n * (prec == HX_FP64 ? sizeof(double) : sizeof(float));
    hipError_t e = hipMalloc(&du, vb);
    if (e == hipSuccess) e = hipMalloc(&dst, vb);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return e;
    if (prec == HX_FP64)
      fill_timing_direction<double><<<grid_for(n), 256, 0, s>>>(static_cast<double*>(du), n);
    else
      fill_timing_direction<float><<<grid_for(n), 256, 0, s>>>(static_cast<float*>(du), n);
    return hipGetLastError();
  }
  // updates the slot in (mode, variant, nt), applies once to warm up, then times reps applies
  hx_status time(const double* u, hx_storage mode, int variant, int nt, int reps, double* ms_out) {
    hx_status st = hx::update_linearization(ctx, u, mode, prec, s, variant, nt);
    if (st == HX_OK) st = hx_apply_tangent(ctx, du, dst, prec, s);
    if (st != HX_OK) return st;
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == HX_OK; ++r) st = hx_apply_tangent(ctx, du, dst, prec, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (st != HX_OK) return st;
    if (e != hipSuccess) return hip_fail(ctx, e, "autotuner: timing");
    *ms_out = ms / reps;
    return HX_OK;
  }
};

const hx_storage kTuneModes[kModes] = {HX_STORE_NONE,    HX_STORE_FINV_J,
                                       HX_STORE_TANGENT, HX_STORE_SPATIAL,
                                       HX_STORE_SPATIAL_RECOMPUTE, HX_STORE_SCALARS,
                                       HX_STORE_TENSORS, HX_STORE_SPATIAL_SCALARS};

}  // namespace

extern "C" {

hx_status hx_autotune_storage(hx_ctx ctx, const double* u, hx_precision prec, int32_t reps,
                              hx_storage* best, double* ms_per_apply, void* stream) {
  if (!ctx || !u || !best) return fail(ctx, HX_E_ARG, "hx_autotune_storage: NULL argument");
  if (prec != HX_FP64 && prec != HX_FP32 && prec != HX_FP32_BF16DATA)
    return fail(ctx, HX_E_ARG, "hx_autotune_storage: precision must be HX_FP64, HX_FP32 or HX_FP32_BF16DATA");
  if (reps < 1 || reps > 1000) return fail(ctx, HX_E_ARG, "hx_autotune_storage: reps out of [1, 1000]");
  TuneBench tb{ctx, prec, static_cast<hipStream_t>(stream)};
  const hipError_t e = tb.init();
  if (e != hipSuccess) return hip_fail(ctx, e, "hx_autotune_storage: allocation");
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  int arg = 0;
  for (int k = 0; k < 4; ++k) {
    // the default configuration (the multigrid's levels rely on it for their diagonal)
    const hx_status st = tb.time(u, kTuneModes[k], 0, -1, reps, &t[k]);
    if (st != HX_OK) return st;
    if (t[k] < t[arg]) arg = k;
  }
  if (ms_per_apply)
    for (int k = 0; k < 4; ++k) ms_per_apply[k] = t[k];
  *best = kTuneModes[arg];
  if (arg != 3) return hx::update_linearization(ctx, u, kTuneModes[arg], prec, stream, 0, -1);
  return HX_OK;
}

int32_t hx_cells_per_workgroup(int32_t p, int32_t variant) {
  if (p < 1 || p > kMaxDegree || variant < 0 || variant >= kVariants) return -1;
  return cells_per_block(p, variant);
}

hx_status hx_autotune(hx_ctx ctx, const double* u, hx_precision prec, int32_t reps, hx_tune_entry* table,
                      int32_t max_entries, int32_t* n_entries, hx_tune_entry* best, void* stream) {
  if (!ctx || !u || !best) return fail(ctx, HX_E_ARG, "hx_autotune: NULL argument");
  if (prec != HX_FP64 && prec != HX_FP32) return fail(ctx, HX_E_ARG, "hx_autotune: precision must be HX_FP64 or HX_FP32");
  if (reps < 1 || reps > 1000) return fail(ctx, HX_E_ARG, "hx_autotune: reps out of [1, 1000]");
  if (table && max_entries < 0) return fail(ctx, HX_E_ARG, "hx_autotune: max_entries < 0");
  TuneBench tb{ctx, prec, static_cast<hipStream_t>(stream)};
  const hipError_t e = tb.init();
  if (e != hipSuccess) return hip_fail(ctx, e, "hx_autotune: allocation");
  const int cls = prec == HX_FP64 ? 0 : 1;
  const int nvar = ctx->topo == kTopoLattice ? kVariants : 1;
  int count = 0;
  hx_tune_entry overall{};
  overall.ms = -1.0;
  for (int k = 0; k < kModes; ++k) {
    const hx_storage mode = kTuneModes[k];
    const bool stored = mode != HX_STORE_NONE && mode != HX_STORE_SPATIAL_RECOMPUTE;
    hx_tune_entry mode_best{};
    mode_best.ms = -1.0;
    for (int v = 0; v < nvar; ++v)
      for (int nt = 0; nt < 2; ++nt) {
        if (!stored && nt == 1) continue;  // no stored data to stream
        double ms = 0.0;
        const hx_status st = tb.time(u, mode, v, nt, reps, &ms);
        if (st != HX_OK) return st;
        hx_tune_entry en{mode, v, cells_per_block(ctx->p, v), nt, ms};
        if (table && count < max_entries) table[count] = en;
        ++count;
        if (mode_best.ms < 0.0 || ms < mode_best.ms) mode_best = en;
      }
    ctx->tuned[cls][mode] = Tuning{true, mode_best.variant, mode_best.nontemporal};
    if (overall.ms < 0.0 || mode_best.ms < overall.ms) overall = mode_best;
  }
  if (n_entries) *n_entries = count;
  *best = overall;
  return hx::update_linearization(ctx, u, overall.mode, prec, stream, overall.variant, overall.nontemporal);
}

hx_status hx_set_tuning(hx_ctx ctx, hx_precision prec, hx_storage mode, int32_t variant, int32_t nontemporal) {
  if (!ctx) return HX_E_ARG;
  if (prec != HX_FP64 && prec != HX_FP32 && prec != HX_FP32_BF16DATA && prec != HX_FP32_FP16DATA)
    return fail(ctx, HX_E_ARG, "hx_set_tuning: unknown precision");
  if (mode < HX_STORE_NONE || mode >= kModes) return fail(ctx, HX_E_ARG, "hx_set_tuning: unknown storage mode");
  if (variant < 0 || variant >= kVariants || (variant != 0 && ctx->topo != kTopoLattice))
    return fail(ctx, HX_E_ARG, "hx_set_tuning: variant not available for this mesh");
  if (nontemporal < -1 || nontemporal > 1) return fail(ctx, HX_E_ARG, "hx_set_tuning: nontemporal out of [-1, 1]");
  ctx->tuned[prec == HX_FP64 ? 0 : 1][mode] = Tuning{true, variant, nontemporal};
  return HX_OK;
}

int64_t hx_linearization_bytes(hx_ctx ctx, hx_precision prec) {
  if (!ctx || store_of(prec) < 0) return -1;
  const Slot& sl = ctx->slot[prec == HX_FP64 ? 0 : 1];
  return sl.valid ? static_cast<int64_t>(sl.qbytes) : 0;
}

hx_status hx_fp64_pipe_probe(int32_t kind, int64_t iters, double* out, void* stream) {
  if (kind < 0 || kind > 2 || iters < 1 || iters > 1000000 || !out || (reinterpret_cast<uintptr_t>(out) & 7))
    return HX_E_ARG;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (kind == 0)
    hipLaunchKernelGGL(fp64_pipe_probe<0>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, iters, out);
  else if (kind == 1)
    hipLaunchKernelGGL(fp64_pipe_probe<1>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, iters, out);
  else
    hipLaunchKernelGGL(fp64_pipe_probe<2>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, iters, out);
  return hipGetLastError() == hipSuccess ? HX_OK : HX_E_HIP;
}

hx_status hx_stream_triad(int64_t n, double* a, const double* b, const double* c, double s, void* stream) {
  const auto misaligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) != 0; };
  if (n < 0 || n > (int64_t(1) << 39)) return HX_E_ARG;
  if (n == 0) return HX_OK;
  if (!a || !b || !c || misaligned(a) || misaligned(b) || misaligned(c)) return HX_E_ARG;
  const int64_t blocks = (n + 511) / 512;  // 256 threads x 2 elements
  hipLaunchKernelGGL(stream_triad, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), a, b, c, s, n);
  return hipGetLastError() == hipSuccess ? HX_OK : HX_E_HIP;
}

}  // extern "C"
