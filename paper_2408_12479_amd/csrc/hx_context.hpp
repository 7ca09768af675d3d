// Library context shared by the host translation units (operators and solvers).
#pragma once

#include <string>
#include <vector>

#include "hx_internal.hpp"

namespace hx {

// One linearisation slot (FP64 class or FP32 class).
struct Slot {
  bool valid = false;
  hx_storage mode = HX_STORE_NONE;
  int store = kStoreF64;
  void* qdata = nullptr;
  size_t qbytes = 0;   // bytes of the current mode's data
  size_t qcap = 0;     // bytes allocated (kept across mode switches)
  float* cscale = nullptr;
  void* uk = nullptr;  // linearisation point (recompute mode): double or float
  uint8_t* act = nullptr;  // fibre switches per q-point (FP32 slot, recompute and F^-1+J modes)
  size_t act_bytes = 0;
  bool keep_act = false;   // the apply reads act
  int variant = 0;         // cells-per-workgroup variant the data is laid out for
  int nt = -1;             // stored data loaded non-temporally: -1 by size, 0 no, 1 yes
};

// Storage modes NONE .. SPATIAL_SCALARS (the hx_storage values 0 .. kModes - 1).
constexpr int kModes = 8;

// A configuration the autotuner chose (or the caller set) for one storage mode of one slot.
struct Tuning {
  bool set = false;
  int variant = 0;
  int nt = -1;
};

int cells_per_block(int p, int variant = 0);
hipError_t dispatch(int p, const HostOp& op, const HostArgs& h, hipStream_t s, bool* ok);

}  // namespace hx

struct hx_ctx_s {
  int device = 0;
  int p = 0;
  int topo = hx::kTopoLattice;    // hx::Topo
  hx::Lattice L{};
  hx::HostArgs base{};
  std::vector<double> gll;
  std::vector<double> vert_host;  // [V][3] (lattice of trilinear cells)
  double* vert64 = nullptr;
  // curved or general meshes: every cell's map as degree-g points (host copy, [cells][(g+1)^3][3])
  // and the stored geometry planes of the kernels
  int geom_degree = 1;
  std::vector<double> geom_host;
  double* geo64 = nullptr;
  float* geo32 = nullptr;
  // general meshes: first-touch node of every local node [cells][(p+1)^3], constraint flags,
  // face boundary ids [cells][6]; device gather map, node -> slot lists, constraint flags
  std::vector<int32_t> cell_nodes;
  std::vector<uint8_t> cons_host;
  std::vector<uint8_t> face_bid;
  int32_t* map = nullptr;
  int32_t* nptr = nullptr;
  int32_t* nslot = nullptr;
  uint8_t* cmask = nullptr;
  int* flag = nullptr;
  void* ework = nullptr;  // element vectors on the broken lattice (apply, residual)
  void* cblk64 = nullptr;
  void* cblk32 = nullptr;
  double* fib64 = nullptr;  // per-cell fibre tensors (frames given), else NULL
  float* fib32 = nullptr;
  hx::Slot slot[2];  // 0: FP64 class, 1: FP32 class
  hx::Tuning tuned[2][hx::kModes];  // per slot and storage mode (hx_storage value)
  std::string err;
};

namespace hx {
// largest degree of a cell's geometry map
constexpr int kMaxGeomDegree = 8;

// argument block of a context's kernels (pointers filled in)
HostArgs args_for(const hx_ctx_s* c);
hx_status set_error(hx_ctx_s* ctx, hx_status s, const std::string& msg);
// setup steps shared by the lattice and the general meshes (destroys c on failure)
hx_status finish_setup(hx_ctx_s* c, const hx_material* mat, const hx_options* opt, const double* frames,
                       hx_ctx* out);
// error of a failed setup (read by hx_last_error(NULL))
hx_status setup_fail(hx_status s, const std::string& msg);
bool check_options(const hx_options* opt, const char* who);
// the apply with a node-kernel epilogue (a Chebyshev step or the residual fused into the node
// kernel; dst may be NULL for a Chebyshev step)
hx_status apply_with_epilogue(hx_ctx_s* ctx, const void* du, void* dst, hx_precision prec, void* stream,
                              const NodeEpilogue& epi);
// the linearisation update in a given configuration (variant, non-temporal policy); the public
// update uses the configuration recorded for the mode, the multigrid the default one
hx_status update_linearization(hx_ctx_s* ctx, const double* u, hx_storage mode, hx_precision prec,
                               void* stream, int variant, int nt);
// stored geometry planes (K = J0^-1, w det J0 per q-point, FP64 and FP32) from c->geom_host;
// HX_E_INVERTED if det J0 <= 0 at some Gauss point (message in c->err)
hx_status build_stored_geometry(hx_ctx_s* c);
// node of local index (i, j, k) of cell e (any topology), and whether it is constrained
int64_t host_node(const hx_ctx_s* c, int64_t e, int i, int j, int k);
bool host_constrained(const hx_ctx_s* c, int64_t node);
// the map of cell e at reference point xi (any topology): position X and, if dX is not NULL,
// dX[3 c + d] = dX_c / dxi_d
void host_map(const hx_ctx_s* c, int64_t e, const double* xi, double* X, double* dX);
}  // namespace hx
