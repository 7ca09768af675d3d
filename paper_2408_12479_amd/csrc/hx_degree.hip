// Kernel instantiations and launch dispatch for one polynomial degree (HX_DEGREE) and one kind of
// mesh topology (HX_TOPO: 0 lattice of trilinear cells, 1 lattice with stored geometry, 2 general
// mesh), both set by the build. Each (degree, topology) pair is its own translation unit so that
// they compile in parallel.
#include <type_traits>

#include "hx_kernels.hpp"

#ifndef HX_DEGREE
#error "HX_DEGREE must be defined"
#endif
#ifndef HX_TOPO
#error "HX_TOPO must be defined"
#endif

#define HX_CAT2(a, b) a##b
#define HX_CAT(a, b) HX_CAT2(a, b)
#define HX_CAT4(a, b, c, d) HX_CAT(HX_CAT(a, b), HX_CAT(c, d))
#define HX_DISPATCH_NAME(t) HX_CAT4(dispatch_p, HX_DEGREE, _t, t)

namespace hx {
namespace {

constexpr int N = HX_DEGREE + 1;
constexpr int TOPO = HX_TOPO;

// Cells per workgroup: the workgroup holds EB * N^3 q-threads; chosen so that the thread count
// is close to a multiple of the 64-wide wavefront. Q3 and Q4 take 4 cells: their pencil phases
// (3 N^2 jobs per cell) then fill whole wavefronts better than with 2, which measured faster in
// the stored-data modes; Q6 stays at one cell (two were slower). Variant 1 is the alternative the
// autotuner times against the default on the lattice of trilinear cells (other meshes lay their
// stored geometry and gather map out for the default).
template <int n, int V = 0> struct Blocking { static constexpr int EB = 1; };
template <> struct Blocking<2> { static constexpr int EB = 8; };   //  64 threads
template <> struct Blocking<3> { static constexpr int EB = 7; };   // 189 of 192
template <> struct Blocking<4> { static constexpr int EB = 4; };   // 256
template <> struct Blocking<5> { static constexpr int EB = 4; };   // 500 of 512
template <> struct Blocking<6> { static constexpr int EB = 1; };   // 216 of 256
template <> struct Blocking<7> { static constexpr int EB = 1; };   // 343 of 384
template <> struct Blocking<2, 1> { static constexpr int EB = 16; };  // 128
template <> struct Blocking<3, 1> { static constexpr int EB = 9; };   // 243 of 256
template <> struct Blocking<4, 1> { static constexpr int EB = 2; };   // 128
template <> struct Blocking<5, 1> { static constexpr int EB = 2; };   // 250 of 256
template <> struct Blocking<6, 1> { static constexpr int EB = 2; };   // 432 of 448
template <> struct Blocking<7, 1> { static constexpr int EB = 2; };   // 686 of 704

template <typename R>
Consts<N, R> make_consts(const HostArgs& h) {
  Consts<N, R> c{};
  for (int i = 0; i < N * N; ++i) {
    c.b.B[i] = static_cast<R>(h.B[i]);
    c.b.D[i] = static_cast<R>(h.D[i]);
  }
  for (int i = 0; i < N; ++i) {
    c.b.w[i] = static_cast<R>(h.w[i]);
    c.b.x[i] = static_cast<R>(h.x[i]);
  }
  c.m.mu = static_cast<R>(h.mat.mu);
  c.m.lam = static_cast<R>(h.mat.lambda);
  c.m.kappa = static_cast<R>(h.mat.kappa);
  c.m.k1 = static_cast<R>(h.mat.k1);
  c.m.k2 = static_cast<R>(h.mat.k2);
  for (int i = 0; i < 9; ++i) {
    c.m.H4[i] = static_cast<R>(h.mat.H4[i]);
    c.m.H6[i] = static_cast<R>(h.mat.H6[i]);
  }
  for (int i = 0; i < 3; ++i) {
    c.m.M4[i] = static_cast<R>(h.mat.M4[i]);
    c.m.M6[i] = static_cast<R>(h.mat.M6[i]);
  }
  c.m.jpow_iters = h.jpow_iters;
  return c;
}

static_assert(sizeof(Consts<N, double>) <= kConstBlockBytes, "constant block too small");

template <typename R>
KernelArgs<N, R> make_args(const HostArgs& h) {
  KernelArgs<N, R> a{};
  a.L = h.L;
  if constexpr (std::is_same<R, double>::value) {
    a.c = static_cast<const Consts<N, R>*>(h.cblk64);
    a.fib = h.fib64;
  } else {
    a.c = static_cast<const Consts<N, R>*>(h.cblk32);
    a.fib = h.fib32;
  }
  a.vert = h.vert64;
  a.map = h.map;
  if constexpr (std::is_same<R, double>::value)
    a.geo = h.geo64;
  else
    a.geo = h.geo32;
  a.in0 = static_cast<const R*>(h.in0);
  a.in1 = static_cast<const R*>(h.in1);
  a.out = static_cast<R*>(h.out);
  a.ework = static_cast<R*>(h.ework);
  a.qdata = h.qdata;
  a.qdata_w = h.qdata_w;
  a.cscale = h.cscale;
  a.cscale_w = h.cscale_w;
  a.flag = h.flag;
  a.act = h.act;
  a.act_w = h.act_w;
  return a;
}

template <typename R, int KIND, int MODE, int LAW, int S, int V = 0>
hipError_t launch_v(const HostArgs& h, hipStream_t s) {
  constexpr int EB = Blocking<N, V>::EB;
  const KernelArgs<N, R> a = make_args<R>(h);
  const int nblk = (h.L.n_cells + EB - 1) / EB;
  if (nblk == 0) return hipSuccess;
  if constexpr (KIND == 0 && MODE != HX_STORE_NONE && MODE != HX_STORE_SPATIAL_RECOMPUTE) {
    // stored data larger than the last-level cache: non-temporal loads (a separate instantiation,
    // since a run-time choice between the two loads is merged into one by the compiler)
    if (h.stream_qdata)
      element_kernel<N, EB, R, KIND, MODE, LAW, S, true, TOPO><<<dim3(nblk), dim3(EB * N * N * N), 0, s>>>(a);
    else
      element_kernel<N, EB, R, KIND, MODE, LAW, S, false, TOPO><<<dim3(nblk), dim3(EB * N * N * N), 0, s>>>(a);
  } else {
    element_kernel<N, EB, R, KIND, MODE, LAW, S, false, TOPO><<<dim3(nblk), dim3(EB * N * N * N), 0, s>>>(a);
  }
  if constexpr (KIND == 0 || KIND == 1) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // every row: sum of the element vectors at the node; constrained rows du (apply) or 0; then the
    // node epilogue of the apply (plain store, or a smoother step fused into the node kernel)
    const dim3 grid(static_cast<unsigned>((h.L.n_nodes + 255) / 256));
    Epi<R> ep{};
    if constexpr (KIND == 0) {
      ep = Epi<R>{h.epi.kind, static_cast<const R*>(h.epi.b), static_cast<R*>(h.epi.x), static_cast<R*>(h.epi.d),
                  static_cast<const R*>(h.epi.dinv), static_cast<R>(h.epi.c1), static_cast<R>(h.epi.c2),
                  h.epi.blocks};
    }
    if constexpr (TOPO == kTopoMap) {
      const int64_t ES = static_cast<int64_t>(nblk) * EB * N * N * N;
      assemble_map_kernel<R><<<grid, dim3(256), 0, s>>>(h.L.n_nodes, h.nptr, h.nslot, h.cmask, ES, a.ework,
                                                         KIND == 0 ? a.in0 : nullptr, a.out, ep);
    } else {
      if (ep.kind != kEpiStore)
        assemble_kernel<N, R, true><<<grid, dim3(256), 0, s>>>(h.L, a.ework, KIND == 0 ? a.in0 : nullptr, a.out, ep);
      else
        assemble_kernel<N, R, false><<<grid, dim3(256), 0, s>>>(h.L, a.ework, KIND == 0 ? a.in0 : nullptr, a.out, ep);
    }
  }
  return hipGetLastError();
}

// the apply and the update of the lattice of trilinear cells come in two cells-per-workgroup variants
template <typename R, int KIND, int MODE, int LAW, int S>
hipError_t launch(const HostArgs& h, hipStream_t s) {
#if HX_TOPO == 0
  if constexpr (KIND == 0 || KIND == 2) {
    if (h.variant == 1) return launch_v<R, KIND, MODE, LAW, S, 1>(h, s);
  }
#endif
  return launch_v<R, KIND, MODE, LAW, S, 0>(h, s);
}

template <int LAW>
hipError_t by_law(const HostOp& op, const HostArgs& h, hipStream_t s, bool* ok) {
  *ok = true;
  switch (op.kind) {
    case OpKind::Residual:
      // material form, or (mode SPATIAL) the spatial form
      if (op.mode == HX_STORE_SPATIAL) return launch<double, 1, HX_STORE_SPATIAL, LAW, kStoreF64>(h, s);
      return launch<double, 1, HX_STORE_NONE, LAW, kStoreF64>(h, s);
    case OpKind::Update:
      // nothing stored: the update checks the state (and decides the fibre switches of FP32 applies)
      if (op.mode == HX_STORE_NONE || op.mode == HX_STORE_SPATIAL_RECOMPUTE)
        return launch<double, 2, HX_STORE_NONE, LAW, kStoreF64>(h, s);
      if (op.mode == HX_STORE_FINV_J) {
        if (op.store == kStoreF64) return launch<double, 2, HX_STORE_FINV_J, LAW, kStoreF64>(h, s);
        if (op.store == kStoreF32) return launch<double, 2, HX_STORE_FINV_J, LAW, kStoreF32>(h, s);
        if (op.store == kStoreBF16) return launch<double, 2, HX_STORE_FINV_J, LAW, kStoreBF16>(h, s);
      }
      if (op.mode == HX_STORE_SCALARS || op.mode == HX_STORE_SPATIAL_SCALARS) {
        // the same stored scalars for both configurations
        if (op.store == kStoreF64) return launch<double, 2, HX_STORE_SCALARS, LAW, kStoreF64>(h, s);
        if (op.store == kStoreF32) return launch<double, 2, HX_STORE_SCALARS, LAW, kStoreF32>(h, s);
      }
      if (op.mode == HX_STORE_TENSORS) {
        if (op.store == kStoreF64) return launch<double, 2, HX_STORE_TENSORS, LAW, kStoreF64>(h, s);
        if (op.store == kStoreF32) return launch<double, 2, HX_STORE_TENSORS, LAW, kStoreF32>(h, s);
      }
      if (op.mode == HX_STORE_SPATIAL) {
        if (op.store == kStoreF64) return launch<double, 2, HX_STORE_SPATIAL, LAW, kStoreF64>(h, s);
        if (op.store == kStoreF32) return launch<double, 2, HX_STORE_SPATIAL, LAW, kStoreF32>(h, s);
        if (op.store == kStoreBF16) return launch<double, 2, HX_STORE_SPATIAL, LAW, kStoreBF16>(h, s);
      }
      if (op.mode == HX_STORE_TANGENT) {
        switch (op.store) {
          case kStoreF64: return launch<double, 2, HX_STORE_TANGENT, LAW, kStoreF64>(h, s);
          case kStoreF32: return launch<double, 2, HX_STORE_TANGENT, LAW, kStoreF32>(h, s);
          case kStoreBF16: return launch<double, 2, HX_STORE_TANGENT, LAW, kStoreBF16>(h, s);
          case kStoreF16: return launch<double, 2, HX_STORE_TANGENT, LAW, kStoreF16>(h, s);
          default: break;
        }
      }
      break;
    case OpKind::Diagonal:
    case OpKind::DiagonalBlocks:
      break;
    case OpKind::Apply:
      if (op.mode == HX_STORE_NONE) {
        return op.fp32 ? launch<float, 0, HX_STORE_NONE, LAW, kStoreF32>(h, s)
                       : launch<double, 0, HX_STORE_NONE, LAW, kStoreF64>(h, s);
      }
      if (op.mode == HX_STORE_SPATIAL_RECOMPUTE) {
        return op.fp32 ? launch<float, 0, HX_STORE_SPATIAL_RECOMPUTE, LAW, kStoreF32>(h, s)
                       : launch<double, 0, HX_STORE_SPATIAL_RECOMPUTE, LAW, kStoreF64>(h, s);
      }
      if (op.mode == HX_STORE_SCALARS) {
        if (!op.fp32 && op.store == kStoreF64) return launch<double, 0, HX_STORE_SCALARS, LAW, kStoreF64>(h, s);
        if (op.fp32 && op.store == kStoreF32) return launch<float, 0, HX_STORE_SCALARS, LAW, kStoreF32>(h, s);
      }
      if (op.mode == HX_STORE_SPATIAL_SCALARS) {
        if (!op.fp32 && op.store == kStoreF64) return launch<double, 0, HX_STORE_SPATIAL_SCALARS, LAW, kStoreF64>(h, s);
        if (op.fp32 && op.store == kStoreF32) return launch<float, 0, HX_STORE_SPATIAL_SCALARS, LAW, kStoreF32>(h, s);
      }
      if (op.mode == HX_STORE_TENSORS) {
        if (!op.fp32 && op.store == kStoreF64) return launch<double, 0, HX_STORE_TENSORS, LAW, kStoreF64>(h, s);
        if (op.fp32 && op.store == kStoreF32) return launch<float, 0, HX_STORE_TENSORS, LAW, kStoreF32>(h, s);
      }
      if (op.mode == HX_STORE_FINV_J) {
        if (!op.fp32 && op.store == kStoreF64)
          return launch<double, 0, HX_STORE_FINV_J, LAW, kStoreF64>(h, s);
        if (op.fp32 && op.store == kStoreF32)
          return launch<float, 0, HX_STORE_FINV_J, LAW, kStoreF32>(h, s);
        if (op.fp32 && op.store == kStoreBF16)
          return launch<float, 0, HX_STORE_FINV_J, LAW, kStoreBF16>(h, s);
      }
#if HX_TOPO != 1
      if (op.mode == HX_STORE_SPATIAL) {
        // the stored words carry the frames: one apply kernel per law family
        constexpr int AL = LAW == kFIBERC ? kFIBER : LAW;
        if (!op.fp32 && op.store == kStoreF64)
          return launch<double, 0, HX_STORE_SPATIAL, AL, kStoreF64>(h, s);
        if (op.fp32 && op.store == kStoreF32)
          return launch<float, 0, HX_STORE_SPATIAL, AL, kStoreF32>(h, s);
        if (op.fp32 && op.store == kStoreBF16)
          return launch<float, 0, HX_STORE_SPATIAL, AL, kStoreBF16>(h, s);
      }
#endif
      break;
  }
  *ok = false;
  return hipSuccess;
}

// the diagonal blocks of the three components; with blocks, also the three off-diagonal
// component pairs into planes 3..5 of the output
template <typename R, int S>
hipError_t launch_diag(const HostArgs& h, bool blocks, hipStream_t s) {
  constexpr int EB = Blocking<N>::EB;
  KernelArgs<N, R> a = make_args<R>(h);
  const int nblk = (h.L.n_cells + EB - 1) / EB;
  if (nblk == 0) return hipSuccess;
  diag_kernel<N, EB, R, S, false><<<dim3(nblk), dim3(EB * N * N * N), 0, s>>>(a);
  if (blocks) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    a.out += 3 * h.L.n_nodes;
    diag_kernel<N, EB, R, S, true><<<dim3(nblk), dim3(EB * N * N * N), 0, s>>>(a);
  }
  return hipGetLastError();
}

// The diagonal (multigrid on lattices) and the apply modes that never read the geometry are
// built in the translation unit of the lattice of trilinear cells; the lattice with stored
// geometry forwards them there (see the dispatch below), general meshes have no diagonal.
#if HX_TOPO == 0
hipError_t diagonal(const HostOp& op, const HostArgs& h, hipStream_t s, bool* ok) {
  *ok = true;
  const bool blocks = op.kind == OpKind::DiagonalBlocks;
  if (op.mode == HX_STORE_TANGENT) {
    if (!op.fp32 && op.store == kStoreF64) return launch_diag<double, kStoreF64>(h, blocks, s);
    if (op.fp32) {
      switch (op.store) {
        case kStoreF32: return launch_diag<float, kStoreF32>(h, blocks, s);
        case kStoreBF16: return launch_diag<float, kStoreBF16>(h, blocks, s);
        case kStoreF16: return launch_diag<float, kStoreF16>(h, blocks, s);
        default: break;
      }
    }
  }
  *ok = false;
  return hipSuccess;
}
#endif

#if HX_TOPO != 1
// The stored-tangent apply does not depend on the law.
hipError_t apply_tangent_mode(const HostOp& op, const HostArgs& h, hipStream_t s, bool* ok) {
  *ok = true;
  if (!op.fp32 && op.store == kStoreF64)
    return launch<double, 0, HX_STORE_TANGENT, kCNH, kStoreF64>(h, s);
  if (op.fp32) {
    switch (op.store) {
      case kStoreF32: return launch<float, 0, HX_STORE_TANGENT, kCNH, kStoreF32>(h, s);
      case kStoreBF16: return launch<float, 0, HX_STORE_TANGENT, kCNH, kStoreBF16>(h, s);
      case kStoreF16: return launch<float, 0, HX_STORE_TANGENT, kCNH, kStoreF16>(h, s);
      default: break;
    }
  }
  *ok = false;
  return hipSuccess;
}
#endif

}  // namespace

#if HX_TOPO == 0
// Cells per workgroup: the stored q-point data is laid out in blocks of this many cells.
int HX_CAT(cells_per_block_p, HX_DEGREE)(int variant) {
  return variant == 1 ? Blocking<N, 1>::EB : Blocking<N>::EB;
}

// Writes the constant blocks of a context (synchronous; called once at setup).
hipError_t HX_CAT(consts_p, HX_DEGREE)(const HostArgs& h) {
  const Consts<N, double> c64 = make_consts<double>(h);
  const Consts<N, float> c32 = make_consts<float>(h);
  hipError_t e = hipMemcpy(h.cblk64, &c64, sizeof(c64), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(h.cblk32, &c32, sizeof(c32), hipMemcpyHostToDevice);
}
#endif

hipError_t HX_DISPATCH_NAME(HX_TOPO)(const HostOp& op, const HostArgs& h, hipStream_t s, bool* ok) {
  if (h.variant != 0 && (HX_TOPO != 0 || h.variant >= kVariants ||
                         (op.kind != OpKind::Apply && op.kind != OpKind::Update))) {
    *ok = false;
    return hipSuccess;
  }
#if HX_TOPO == 1
  // a lattice with stored geometry: the operations that never read the geometry are those of the
  // lattice of trilinear cells
  if (op.kind == OpKind::Diagonal || op.kind == OpKind::DiagonalBlocks ||
      (op.kind == OpKind::Apply && (op.mode == HX_STORE_TANGENT || op.mode == HX_STORE_SPATIAL)))
    return HX_DISPATCH_NAME(0)(op, h, s, ok);
#endif
#if HX_TOPO == 2
  // the diagonal kernel addresses lattices only (general meshes have no multigrid)
  if (op.kind == OpKind::Diagonal || op.kind == OpKind::DiagonalBlocks) {
    *ok = false;
    return hipSuccess;
  }
#endif
#if HX_TOPO == 0
  if (op.kind == OpKind::Diagonal || op.kind == OpKind::DiagonalBlocks) return diagonal(op, h, s, ok);
#endif
#if HX_TOPO != 1
  if (op.kind == OpKind::Apply && op.mode == HX_STORE_TANGENT) return apply_tangent_mode(op, h, s, ok);
#endif
  switch (op.law) {
    case HX_LAW_CNH: return by_law<kCNH>(op, h, s, ok);
    case HX_LAW_INH: return by_law<kINH>(op, h, s, ok);
    case HX_LAW_FIBER:
      return h.fib64 ? by_law<kFIBERC>(op, h, s, ok) : by_law<kFIBER>(op, h, s, ok);
  }
  *ok = false;
  return hipSuccess;
}

}  // namespace hx
