// Internal declarations shared by the host runtime (hx_api.cpp) and the per-degree kernel
// translation units (hx_degree.hip, compiled once per polynomial degree).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hx.h"

namespace hx {

constexpr int kMaxDegree = 6;

// Structured lattice: cells, node lattice (Gauss-Lobatto points) and vertex lattice.
struct Lattice {
  int32_t nx, ny, nz;     // cells per direction
  int32_t Nx, Ny, Nz;     // nodes per direction
  int32_t Vx, Vy, Vz;     // vertices per direction
  int32_t p;              // polynomial degree
  uint32_t dir_faces;     // Dirichlet face bits, periodic directions cleared
  int32_t n_cells;
  int64_t n_nodes;
};

// 1D tables of degree p = N-1 on [0, 1]. B maps nodal values at the N Gauss-Lobatto points to
// values at the N Gauss points; D differentiates a degree-p polynomial given by its values at
// the Gauss points (collocation derivative), so grad = (D_d)(B x B x B) u.
template <int N, typename R>
struct Basis1D {
  R B[N * N];  // B[q*N + i] = l_i(x_q)
  R D[N * N];  // D[q*N + r] = l~_r'(x_q), l~ the Lagrange basis on the Gauss points
  R w[N];      // Gauss weights
  R x[N];      // Gauss points
};

template <typename R>
struct MaterialK {
  R mu, lam, kappa, k1, k2;
  R H4[9], H6[9];
  R M4[3], M6[3];
  int32_t jpow_iters;
};

// Degree- and material-dependent constants, kept in device memory per context and read by
// the kernels through a wave-uniform pointer (scalar loads).
template <int N, typename R>
struct Consts {
  Basis1D<N, R> b;
  MaterialK<R> m;
};

constexpr size_t kConstBlockBytes = 4096;

// How a context addresses its nodes and finds its geometry (a template parameter of the kernels):
//   kTopoLattice  structured lattice, geometry = trilinear map of the 8 cell vertices, evaluated
//                 at every q-point from the vertex lattice
//   kTopoLatticeG structured lattice, geometry stored per q-point (curved cells)
//   kTopoMap      general mesh: node of every gather slot from an int32 map, geometry stored per
//                 q-point, element vectors summed per node through a node -> slot list
enum Topo : int { kTopoLattice = 0, kTopoLatticeG = 1, kTopoMap = 2 };

// Words of stored geometry per q-point: K = J0^-1 (9, row-major K[3 d + J] = dxi_d / dX_J) and
// w_q det J0.
constexpr int kGeoWords = 10;

// Gather/store slot of thread t of a workgroup of EB cells of n^3 points: the cell le of the block
// and the local node q. With several cells of odd n per workgroup, the cells are interleaved along
// x (t: i = t mod n, then the cell, then j and k) so that consecutive lanes walk a whole x-row of
// the block; otherwise t = le n^3 + q.
__host__ __device__ inline void slot_of_thread(int n, int EB, int t, int& le, int& q) {
  if (EB > 1 && (n & 1)) {
    const int i = t % n;
    const int r = t / n;
    le = r % EB;
    q = i + n * (r / EB);
  } else {
    le = t / (n * n * n);
    q = t - le * n * n * n;
  }
}

// Everything a kernel needs, passed by value.
template <int N, typename R>
struct KernelArgs {
  Lattice L;
  const Consts<N, R>* __restrict__ c;
  const double* vert;   // vertices [Vz][Vy][Vx][3] (FP64 in every arithmetic)
  const int32_t* map;   // general meshes: node of gather slot [block][EB n^3] (~node if constrained)
  const R* geo;         // stored geometry planes [block][kGeoWords][EB n^3] (curved or general meshes)
  const R* in0;         // gathered vector (du, or u for residual/update)
  const R* in1;         // linearisation point u_k (recompute mode)
  R* out;               // output vector (apply, residual)
  R* ework;             // element vectors on the broken lattice [3][nz*N][ny*N][nx*N]
                        // (apply, residual; summed by assemble_kernel)
  const void* qdata;    // stored per-q-point planes [block][W][cells_per_block * Q]
  void* qdata_w;        // planes written by the update
  const float* cscale;  // per-cell power-of-two scale of binary16 data
  float* cscale_w;
  int* flag;            // status bits (kFlagInverted | kFlagNonFinite)
  const R* fib;         // per-cell fibre tensors [cell][kFibWords] (fibre law with cell frames)
  const uint8_t* act;   // fibre switches per q-point [block][cells_per_block * Q] (FP32 apply), or NULL
  uint8_t* act_w;       // written by the update, or NULL
};

// Per-cell fibre data: H4 (3x3), H6 (3x3), M4, M6 in global coordinates.
constexpr int kFibWords = 24;

constexpr int kFlagInverted = 1;
constexpr int kFlagNonFinite = 2;

enum StoreType : int { kStoreF64 = 0, kStoreF32 = 1, kStoreBF16 = 2, kStoreF16 = 3 };
// Diagonal: the operator's diagonal [3][n_nodes]; DiagonalBlocks: its nodal 3x3 blocks
// [6][n_nodes] (00, 11, 22, 01, 02, 12)
enum class OpKind : int { Apply = 0, Residual = 1, Update = 2, Diagonal = 3, DiagonalBlocks = 4 };

// Host-side description of one launch.
struct HostOp {
  OpKind kind;
  hx_law law;
  hx_storage mode;
  int store;         // StoreType of the data (apply, update)
  bool fp32;         // apply arithmetic and vector type (Apply only)
};

// Number of cells-per-workgroup variants of the lattice of trilinear cells.
constexpr int kVariants = 2;

// What the node kernel of an apply does with the assembled row t (the sum of the element vectors at
// the node, or the input on constrained rows):
//   kEpiStore      out = t
//   kEpiChebyshev  d = c1 d + c2 dinv (b - t), x += d   (one Chebyshev step of the smoother, with x
//                  the apply's input; out is not written)
//   kEpiResidual   out = b - t                           (the residual of the smoothed iterate)
//   kEpiChebyshevFirst  d = c2 dinv (b - t), x += d      (the first step from a nonzero iterate)
enum EpiKind : int { kEpiStore = 0, kEpiChebyshev = 1, kEpiResidual = 2, kEpiChebyshevFirst = 3 };

// dinv: the smoother's D^-1, point Jacobi [3][n_nodes] (blocks = 0) or the inverses of the nodal
// 3x3 blocks [6][n_nodes], entries (00, 11, 22, 01, 02, 12) (blocks = 1)
struct NodeEpilogue {
  int kind;
  const void* b;
  void* x;
  void* d;
  const void* dinv;
  double c1, c2;
  int blocks;
};

// the same with the apply's arithmetic type, as the node kernel receives it
template <typename R>
struct Epi {
  int kind;
  const R* b;
  R* x;
  R* d;
  const R* dinv;
  R c1, c2;
  int blocks;
};

struct HostArgs {
  Lattice L;
  NodeEpilogue epi;     // node kernel of an apply (zero: plain store)
  int topo;             // Topo of the context
  int variant;          // cells-per-workgroup variant of an apply or update (0 default, 1 the
                        // alternative; lattices of trilinear cells only): the stored data is laid
                        // out in blocks of that many cells
  const int32_t* map;   // kTopoMap: gather slot -> node (device)
  const int32_t* nptr;  // kTopoMap: node -> first entry of its slot list [n_nodes + 1] (device)
  const int32_t* nslot; // kTopoMap: slot lists, increasing within a node (device)
  const uint8_t* cmask; // kTopoMap: constrained nodes [n_nodes] (device)
  const double* geo64;  // stored geometry planes, FP64 (kTopoLatticeG, kTopoMap)
  const float* geo32;   // the same rounded to FP32
  double B[64], D[64], w[8], x[8];   // 1D tables, row-major N x N
  hx_material mat;
  int32_t jpow_iters;
  const double* vert64;
  const void* in0;
  const void* in1;
  void* out;
  void* ework;    // 3 * n_cells * (p+1)^3 FP64 words, reused as FP32 by FP32 applies
  const void* qdata;
  int stream_qdata;   // nonzero: the apply loads the planes with the non-temporal hint (large data)
  void* qdata_w;
  const float* cscale;
  float* cscale_w;
  int* flag;
  void* cblk64;   // device block holding Consts<N, double>
  void* cblk32;   // device block holding Consts<N, float>
  const uint8_t* act;   // fibre switches decided by the FP64 update (FP32 recompute modes)
  uint8_t* act_w;
  const double* fib64;  // per-cell fibre tensors, or NULL (material tensors everywhere)
  const float* fib32;
};

// Words per q-point of the spatial storage mode: sqrt(w det J0) J_t^-1 (9), tau (6) and the law's
// data (cNH 1; iNH 2 + 6; fibre iNH + 2 x 7).
constexpr int spatial_words(int law) { return law == 0 ? 16 : (law == 1 ? 23 : 37); }

// Words per q-point of each storage mode.
inline int mode_words(hx_storage m, hx_law law) {
  switch (m) {
    case HX_STORE_TANGENT: return 45;
    case HX_STORE_FINV_J: return 10;
    case HX_STORE_SPATIAL: return spatial_words(law);
    case HX_STORE_SCALARS:
    case HX_STORE_SPATIAL_SCALARS: return law == 0 ? 1 : (law == 1 ? 4 : 8);
    case HX_STORE_TENSORS: return law == 0 ? 31 : (law == 1 ? 33 : 35);
    default: return 0;
  }
}

// One per degree, defined in hx_degree.hip compiled with HX_DEGREE = p.
int cells_per_block_p1(int variant);
int cells_per_block_p2(int variant);
int cells_per_block_p3(int variant);
int cells_per_block_p4(int variant);
int cells_per_block_p5(int variant);
int cells_per_block_p6(int variant);
hipError_t consts_p1(const HostArgs&);
hipError_t consts_p2(const HostArgs&);
hipError_t consts_p3(const HostArgs&);
hipError_t consts_p4(const HostArgs&);
hipError_t consts_p5(const HostArgs&);
hipError_t consts_p6(const HostArgs&);
#define HX_DECLARE_DISPATCH(p)                                                  \
  hipError_t dispatch_p##p##_t0(const HostOp&, const HostArgs&, hipStream_t, bool*); \
  hipError_t dispatch_p##p##_t1(const HostOp&, const HostArgs&, hipStream_t, bool*); \
  hipError_t dispatch_p##p##_t2(const HostOp&, const HostArgs&, hipStream_t, bool*);
HX_DECLARE_DISPATCH(1)
HX_DECLARE_DISPATCH(2)
HX_DECLARE_DISPATCH(3)
HX_DECLARE_DISPATCH(4)
HX_DECLARE_DISPATCH(5)
HX_DECLARE_DISPATCH(6)
#undef HX_DECLARE_DISPATCH

}  // namespace hx
