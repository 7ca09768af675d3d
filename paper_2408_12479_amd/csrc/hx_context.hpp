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
};

int cells_per_block(int p);
hipError_t dispatch(int p, const HostOp& op, const HostArgs& h, hipStream_t s, bool* ok);

}  // namespace hx

struct hx_ctx_s {
  int device = 0;
  int p = 0;
  hx::Lattice L{};
  hx::HostArgs base{};
  std::vector<double> gll;
  std::vector<double> vert_host;  // [V][3]
  double* vert64 = nullptr;
  int* flag = nullptr;
  void* ework = nullptr;  // element vectors on the broken lattice (apply, residual)
  void* cblk64 = nullptr;
  void* cblk32 = nullptr;
  double* fib64 = nullptr;  // per-cell fibre tensors (frames given), else NULL
  float* fib32 = nullptr;
  hx::Slot slot[2];  // 0: FP64 class, 1: FP32 class
  std::string err;
};

namespace hx {
// argument block of a context's kernels (pointers filled in)
HostArgs args_for(const hx_ctx_s* c);
hx_status set_error(hx_ctx_s* ctx, hx_status s, const std::string& msg);
}  // namespace hx
