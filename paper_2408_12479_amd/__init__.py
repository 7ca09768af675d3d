"""Python binding of libhx.so (see include/hx.h): argument marshalling only.

Every operator evaluation runs in the HIP kernels of the library; torch provides device memory and
streams. Importing the package loads the in-tree ``libhx.so`` and fails loudly if it is missing
(build it with ``python paper_2408_12479_amd/build.py`` or ``__graft_entry__.build()``).
"""
import ctypes
import os

import numpy as np
# torch is imported before libhx.so is loaded: torch ships its own HIP runtime, and libhx.so's
# libamdhip64 dependency must resolve to that already-loaded runtime. Loaded the other way round,
# the process holds two HIP runtimes and the library's device calls fail ("no HIP device").
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhx.so")

# enums of hx.h
HX_OK = 0
STATUS = {0: "HX_OK", 1: "HX_E_ARG", 2: "HX_E_HIP", 3: "HX_E_NOMEM", 4: "HX_E_STATE", 5: "HX_E_INVERTED",
          6: "HX_E_NONFINITE", 7: "HX_E_NOT_CONVERGED", 8: "HX_E_UNSUPPORTED"}
LAWS = {"cnh": 0, "inh": 1, "fiber": 2}
MODES = {"none": 0, "finv_j": 1, "tangent": 2, "spatial": 3, "spatial_recompute": 4, "scalars": 5, "tensors": 6,
         "spatial_scalars": 7, "auto": 255}
MODE_NAMES = {v: k for k, v in MODES.items()}
STORAGE_MODES = ("none", "finv_j", "tangent", "spatial", "spatial_recompute", "scalars", "tensors",
                 "spatial_scalars")
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_bf16": 2, "fp32_fp16": 3}


class HxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class _Lattice(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("periodic", ctypes.c_int32), ("vertices", ctypes.POINTER(ctypes.c_double)),
                ("dirichlet_faces", ctypes.c_uint32), ("frames", ctypes.POINTER(ctypes.c_double)),
                ("geom_degree", ctypes.c_int32), ("geom_nodes", ctypes.POINTER(ctypes.c_double))]


class _Mesh(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_cells", ctypes.c_int64),
                ("vertices", ctypes.POINTER(ctypes.c_double)), ("cells", ctypes.POINTER(ctypes.c_int64)),
                ("face_bid", ctypes.POINTER(ctypes.c_uint8)), ("geom_degree", ctypes.c_int32),
                ("geom_nodes", ctypes.POINTER(ctypes.c_double)), ("frames", ctypes.POINTER(ctypes.c_double))]


class _TuneEntry(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("variant", ctypes.c_int32), ("cells_per_workgroup", ctypes.c_int32),
                ("nontemporal", ctypes.c_int32), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {"mode": MODE_NAMES[self.mode], "variant": int(self.variant),
                "cells_per_workgroup": int(self.cells_per_workgroup), "nontemporal": int(self.nontemporal),
                "ms": float(self.ms)}


class _Material(ctypes.Structure):
    _fields_ = [("law", ctypes.c_int), ("mu", ctypes.c_double), ("lam", ctypes.c_double),
                ("kappa", ctypes.c_double), ("k1", ctypes.c_double), ("k2", ctypes.c_double),
                ("H4", ctypes.c_double * 9), ("H6", ctypes.c_double * 9),
                ("M4", ctypes.c_double * 3), ("M6", ctypes.c_double * 3)]


class _Options(ctypes.Structure):
    _fields_ = [("jpow_newton_iters", ctypes.c_int32), ("dirichlet_bid_mask", ctypes.c_uint32),
                ("reserved", ctypes.c_int32 * 6)]


class _MgOptions(ctypes.Structure):
    _fields_ = [("smoother_degree", ctypes.c_int32), ("coarse_degree", ctypes.c_int32),
                ("smoothing_range", ctypes.c_double), ("eig_iters", ctypes.c_int32),
                ("eig_safety", ctypes.c_double), ("precision", ctypes.c_int), ("use_graph", ctypes.c_int32),
                ("level_mode", ctypes.c_int), ("coarse_solver", ctypes.c_int32), ("fuse_smoother", ctypes.c_int32),
                ("smoother_blocks", ctypes.c_int32)]


class _NewtonOpts(ctypes.Structure):
    _fields_ = [("newton_rel_tol", ctypes.c_double), ("newton_abs_tol", ctypes.c_double),
                ("max_newton", ctypes.c_int32), ("krylov_rel_tol", ctypes.c_double),
                ("max_krylov", ctypes.c_int32), ("load_steps", ctypes.c_int32), ("outer_mode", ctypes.c_int),
                ("verbose", ctypes.c_int32), ("predictor", ctypes.c_int32)]


class _NewtonReport(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("krylov_iters", ctypes.c_int32),
                ("vcycles", ctypes.c_int32), ("load_steps_done", ctypes.c_int32),
                ("initial_residual", ctypes.c_double), ("final_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("outer_mode", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_2408_12479_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    sig = {
        "hx_setup": (ctypes.c_int, [ctypes.POINTER(_Mesh), ctypes.c_int32, ctypes.POINTER(_Material),
                                    ctypes.POINTER(_Options), ctypes.POINTER(vp)]),
        "hx_setup_lattice": (ctypes.c_int, [ctypes.POINTER(_Lattice), ctypes.c_int32, ctypes.POINTER(_Material),
                                            ctypes.POINTER(_Options), ctypes.POINTER(vp)]),
        "hx_destroy": (ctypes.c_int, [vp]),
        "hx_num_dofs": (i64, [vp]),
        "hx_num_nodes": (i64, [vp]),
        "hx_num_cells": (i64, [vp]),
        "hx_node_coords": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double)]),
        "hx_constrained_mask": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_uint8)]),
        "hx_residual": (ctypes.c_int, [vp, vp, vp, vp]),
        "hx_residual_spatial": (ctypes.c_int, [vp, vp, vp, vp]),
        "hx_update_linearization": (ctypes.c_int, [vp, vp, ctypes.c_int, ctypes.c_int, vp]),
        "hx_apply_tangent": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp]),
        "hx_apply_tangent_noalloc": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp]),
        "hx_linearization_bytes": (i64, [vp, ctypes.c_int]),
        "hx_autotune_storage": (ctypes.c_int, [vp, vp, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(ctypes.c_int),
                                               ctypes.POINTER(ctypes.c_double), vp]),
        "hx_autotune": (ctypes.c_int, [vp, vp, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(_TuneEntry),
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_TuneEntry),
                                       vp]),
        "hx_set_tuning": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int32, ctypes.c_int32]),
        "hx_cells_per_workgroup": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32]),
        "hx_mg_default_options": (ctypes.c_int, [ctypes.POINTER(_MgOptions)]),
        "hx_mg_level_mode": (ctypes.c_int32, [vp, ctypes.c_int32]),
        "hx_fiber_structure": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double]
                               + [ctypes.POINTER(ctypes.c_double)] * 5),
        "hx_mg_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(_MgOptions),
                                        ctypes.POINTER(vp)]),
        "hx_mg_destroy": (ctypes.c_int, [vp]),
        "hx_mg_last_error": (ctypes.c_char_p, [vp]),
        "hx_mg_update": (ctypes.c_int, [vp, vp, vp]),
        "hx_mg_vcycle": (ctypes.c_int, [vp, vp, vp, vp]),
        "hx_mg_vcycle_count": (i64, [vp]),
        "hx_mg_lambda_max": (ctypes.c_double, [vp, ctypes.c_int32]),
        "hx_mg_transfer": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]),
        "hx_mg_inverse_diagonal": (ctypes.c_int, [vp, ctypes.c_int32, vp, vp]),
        "hx_newton_solve": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(_NewtonOpts),
                                           ctypes.POINTER(_NewtonReport), vp]),
        "hx_surface_load": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
        "hx_qpoint_eval": (ctypes.c_int, [ctypes.POINTER(_Material), ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
                                          i64, vp, vp, vp, vp, vp]),
        "hx_stream_triad": (ctypes.c_int, [i64, vp, vp, vp, ctypes.c_double, vp]),
        "hx_fp64_pipe_probe": (ctypes.c_int, [ctypes.c_int32, i64, vp, vp]),
        "hx_last_error": (ctypes.c_char_p, [vp]),
        "hx_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status, ctx=None):
    if status != HX_OK:
        raise HxError(status, lib.hx_last_error(ctx).decode())


def _dptr(arr):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def fiber_structure(a, b, phi, E=None):
    """(H4, H6, M4, M6) of the two fibre families (library host helper, Section 3)."""
    E = np.ascontiguousarray(np.eye(3) if E is None else E, dtype=np.float64)
    H4, H6 = np.zeros(9), np.zeros(9)
    M4, M6 = np.zeros(3), np.zeros(3)
    _check(lib.hx_fiber_structure(a, b, phi, _dptr(E), _dptr(H4), _dptr(H6), _dptr(M4), _dptr(M6)))
    return H4.reshape(3, 3), H6.reshape(3, 3), M4, M6


def _material(law, mu=1.0, lam=0.0, kappa=0.0, k1=0.0, k2=0.0, H4=None, H6=None, M4=None, M6=None):
    mat = _Material()
    mat.law = LAWS[law]
    mat.mu, mat.lam, mat.kappa, mat.k1, mat.k2 = mu, lam, kappa, k1, k2
    for name, val, n in (("H4", H4, 9), ("H6", H6, 9), ("M4", M4, 3), ("M6", M6, 3)):
        arr = np.zeros(n) if val is None else np.asarray(val, dtype=np.float64).ravel()
        getattr(mat, name)[:] = arr.tolist()
    return mat


def qpoint_eval(H, G, law, form="stable", precision="fp64", jpow_newton_iters=0, stream=None, **mat):
    """P(I + H) and P'(H)[G] for batches H, G (CUDA FP64 tensors [n, 3, 3]) through
    hx_qpoint_eval: returns (P, dP) as CUDA FP64 tensors [n, 3, 3]."""
    import torch
    for t in (H, G):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError("H and G must be contiguous CUDA float64 tensors")
    if H.shape != G.shape or H.shape[-2:] != (3, 3):
        raise ValueError("H and G must have shape [n, 3, 3]")
    n = H.shape[0]
    P, dP = torch.empty_like(H), torch.empty_like(H)
    m = _material(law, **mat)
    _check(lib.hx_qpoint_eval(ctypes.byref(m), {"stable": 0, "standard": 1}[form], PRECISIONS[precision],
                              int(jpow_newton_iters), n, ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                              ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(dP.data_ptr()), _stream_handle(stream)))
    return P, dP


def stream_triad(a, b, c, s, stream=None):
    """a = b + s c on contiguous CUDA float64 tensors of one length (hx_stream_triad, the STREAM
    triad bandwidth probe)."""
    import torch
    for t in (a, b, c):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError("a, b and c must be contiguous CUDA float64 tensors")
    if not a.numel() == b.numel() == c.numel():
        raise ValueError("a, b and c must have the same length")
    _check(lib.hx_stream_triad(a.numel(), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                               ctypes.c_void_p(c.data_ptr()), float(s), _stream_handle(stream)))
    return a


PIPE_PROBE_THREADS = 2048 * 256


def fp64_pipe_probe(kind, iters, out, stream=None):
    """FP64 issue-rate probe (hx_fp64_pipe_probe): kind 0 vector FMAs, 1 16x16x4 matrix
    instructions, 2 both; out a contiguous CUDA float64 tensor of PIPE_PROBE_THREADS values.
    Returns the flops of the call."""
    import torch
    if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float64 \
            or not out.is_contiguous() or out.numel() != PIPE_PROBE_THREADS:
        raise TypeError("out must be a contiguous CUDA float64 tensor of PIPE_PROBE_THREADS values")
    _check(lib.hx_fp64_pipe_probe(int(kind), int(iters), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return 2048 * 4 * int(iters) * (16384 if kind == 2 else 8192)


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _frames_arg(frames, n_cells):
    if frames is None:
        return None
    fr = np.ascontiguousarray(frames, dtype=np.float64)
    if fr.shape != (n_cells, 3, 3):
        raise ValueError("frames must have shape [n_cells, 3, 3]")
    return fr


def _geom_arg(geom_nodes, geom_degree, n_cells):
    if geom_nodes is None:
        if int(geom_degree) != 1:
            raise ValueError("geom_degree > 1 needs geom_nodes")
        return None
    g = int(geom_degree)
    G = np.ascontiguousarray(geom_nodes, dtype=np.float64)
    if G.shape != (n_cells, (g + 1) ** 3, 3):
        raise ValueError(f"geom_nodes must have shape [{n_cells}, {(g + 1) ** 3}, 3]")
    return G


class _Context:
    """A context of the library: mesh, degree, material; owns device memory until close()."""

    def _finish(self, ctx, p):
        self.ctx = ctx
        self.p = int(p)
        self.num_nodes = int(lib.hx_num_nodes(ctx))
        self.num_dofs = int(lib.hx_num_dofs(ctx))
        self.num_cells = int(lib.hx_num_cells(ctx))

    def close(self):
        if getattr(self, "ctx", None):
            lib.hx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def node_coords(self):
        out = np.zeros((self.num_nodes, 3))
        _check(lib.hx_node_coords(self.ctx, _dptr(out)), self.ctx)
        return out

    def constrained_mask(self):
        out = np.zeros(self.num_nodes, dtype=np.uint8)
        _check(lib.hx_constrained_mask(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), self.ctx)
        return out.astype(bool)

    def _vec(self, t, dtype, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}")
        if t.numel() != self.num_dofs or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {self.num_dofs} entries ([3][n_nodes])")
        return ctypes.c_void_p(t.data_ptr())

    def residual(self, u, r=None, stream=None, form="material"):
        """r~(u), integrated over the material (hx_residual) or the spatial configuration
        (hx_residual_spatial)."""
        import torch
        r = torch.empty_like(u) if r is None else r
        fn = {"material": lib.hx_residual, "spatial": lib.hx_residual_spatial}[form]
        _check(fn(self.ctx, self._vec(u, torch.float64, "u"), self._vec(r, torch.float64, "r"), _stream_handle(stream)),
               self.ctx)
        return r

    def update_linearization(self, u, mode="tangent", precision="fp64", stream=None):
        import torch
        _check(lib.hx_update_linearization(self.ctx, self._vec(u, torch.float64, "u"), MODES[mode],
                                           PRECISIONS[precision], _stream_handle(stream)), self.ctx)

    def apply_tangent(self, du, dst=None, precision="fp64", stream=None):
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        dst = torch.empty_like(du) if dst is None else dst
        _check(lib.hx_apply_tangent(self.ctx, self._vec(du, dt, "du"), self._vec(dst, dt, "dst"),
                                    PRECISIONS[precision], _stream_handle(stream)), self.ctx)
        return dst

    def apply_tangent_noalloc(self, du, dst, precision="fp64", stream=None):
        """hx_apply_tangent_noalloc: the apply with the library's static element-vector buffer
        (dst must be given; nothing is allocated)."""
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        _check(lib.hx_apply_tangent_noalloc(self.ctx, self._vec(du, dt, "du"), self._vec(dst, dt, "dst"),
                                            PRECISIONS[precision], _stream_handle(stream)), self.ctx)
        return dst

    def linearization_bytes(self, precision="fp64"):
        return int(lib.hx_linearization_bytes(self.ctx, PRECISIONS[precision]))

    def autotune_storage(self, u, precision="fp64", reps=10, stream=None):
        """Runs the library's storage-mode autotuner at u: (best mode, {mode: ms per apply})."""
        import torch
        best = ctypes.c_int()
        ms = np.zeros(4)
        _check(lib.hx_autotune_storage(self.ctx, self._vec(u, torch.float64, "u"), PRECISIONS[precision], int(reps),
                                       ctypes.byref(best), _dptr(ms), _stream_handle(stream)), self.ctx)
        return MODE_NAMES[best.value], {"none": ms[0], "finv_j": ms[1], "tangent": ms[2], "spatial": ms[3]}

    def autotune(self, u, precision="fp64", reps=20, stream=None):
        """hx_autotune at u: (best configuration, every timed configuration) as dicts with mode,
        variant, cells_per_workgroup, nontemporal and ms per apply. The choice per mode is kept by
        the context for its later updates."""
        import torch
        table = (_TuneEntry * 28)()
        n = ctypes.c_int32()
        best = _TuneEntry()
        _check(lib.hx_autotune(self.ctx, self._vec(u, torch.float64, "u"), PRECISIONS[precision], int(reps),
                               table, 28, ctypes.byref(n), ctypes.byref(best), _stream_handle(stream)), self.ctx)
        return best.as_dict(), [table[i].as_dict() for i in range(n.value)]

    def set_tuning(self, mode, precision="fp64", variant=0, nontemporal=-1):
        """hx_set_tuning: the configuration later updates of (precision class, mode) use."""
        _check(lib.hx_set_tuning(self.ctx, PRECISIONS[precision], MODES[mode], int(variant), int(nontemporal)),
               self.ctx)

    def surface_load(self, face, pressure):
        """Dead-load pressure vector on a lattice boundary face (0..5) or, on a general mesh, on the
        faces with boundary id ``face``; host array (3, n_nodes)."""
        out = np.zeros(3 * self.num_nodes)
        _check(lib.hx_surface_load(self.ctx, int(face), float(pressure), _dptr(out)), self.ctx)
        return out.reshape(3, self.num_nodes)


class Operator(_Context):
    """A context on a structured lattice (hx_setup_lattice)."""

    def __init__(self, nx, ny, nz, vertices, p, law="cnh", mu=1.0, lam=0.0, kappa=0.0, k1=0.0,
                 k2=0.0, H4=None, H6=None, M4=None, M6=None, dirichlet_faces=(),
                 periodic=(False, False, False), jpow_newton_iters=0, frames=None, geom_degree=1,
                 geom_nodes=None):
        """frames: optional [n_cells, 3, 3] local fibre frames (rows E1, E2, E3); H4..M6 are then
        components in each cell's frame. geom_nodes: optional [n_cells, (g+1)^3, 3] curved cells
        (each cell's map at its equispaced points), g = geom_degree; the vertices may then be None."""
        n_cells = int(nx) * int(ny) * int(nz)
        G = _geom_arg(geom_nodes, geom_degree, n_cells)
        V = None
        if vertices is not None:
            V = np.ascontiguousarray(vertices, dtype=np.float64)
            vdims = [int(n) + (0 if periodic[d] else 1) for d, n in enumerate((nx, ny, nz))]
            if V.size != 3 * vdims[0] * vdims[1] * vdims[2]:
                raise ValueError(f"vertices must hold 3 * {vdims[0]} * {vdims[1]} * {vdims[2]} values for this "
                                 f"lattice and periodicity, got {V.size}")
        elif G is None:
            raise ValueError("a lattice needs vertices or geom_nodes")
        fr = _frames_arg(frames, n_cells)
        self._keep = (V, G, fr)
        mesh = _Lattice(int(nx), int(ny), int(nz),
                        int(sum(1 << d for d in range(3) if periodic[d])), None if V is None else _dptr(V),
                        int(sum(1 << f for f in dirichlet_faces)), None if fr is None else _dptr(fr),
                        int(geom_degree), None if G is None else _dptr(G))
        mat = _material(law, mu, lam, kappa, k1, k2, H4, H6, M4, M6)
        opt = _Options()
        opt.jpow_newton_iters = int(jpow_newton_iters)
        ctx = ctypes.c_void_p()
        _check(lib.hx_setup_lattice(ctypes.byref(mesh), int(p), ctypes.byref(mat), ctypes.byref(opt),
                                    ctypes.byref(ctx)))
        self._finish(ctx, p)


class HexOperator(_Context):
    """A context on a general hexahedral mesh given by connectivity (hx_setup)."""

    def __init__(self, vertices, cells, p, face_bid=None, dirichlet_bids=(), geom_degree=1, geom_nodes=None,
                 law="cnh", mu=1.0, lam=0.0, kappa=0.0, k1=0.0, k2=0.0, H4=None, H6=None, M4=None, M6=None,
                 jpow_newton_iters=0, frames=None):
        """vertices [V, 3]; cells [E, 8] vertex ids (corner a + 2b + 4c at reference corner (a, b, c));
        face_bid [E, 6] boundary ids (0 none, 1..31 may be constrained) or None; the faces whose id is
        in dirichlet_bids are constrained; geom_nodes [E, (g+1)^3, 3] curved cells or None."""
        V = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1, 3)
        C = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1, 8)
        n_cells = C.shape[0]
        F = None
        if face_bid is not None:
            F = np.ascontiguousarray(face_bid, dtype=np.uint8).reshape(-1, 6)
            if F.shape[0] != n_cells:
                raise ValueError("face_bid must have shape [n_cells, 6]")
        G = _geom_arg(geom_nodes, geom_degree, n_cells)
        fr = _frames_arg(frames, n_cells)
        self._keep = (V, C, F, G, fr)
        mesh = _Mesh(V.shape[0], n_cells, _dptr(V), C.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                     None if F is None else F.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(geom_degree),
                     None if G is None else _dptr(G), None if fr is None else _dptr(fr))
        mat = _material(law, mu, lam, kappa, k1, k2, H4, H6, M4, M6)
        opt = _Options()
        opt.jpow_newton_iters = int(jpow_newton_iters)
        mask = 0
        for b in dirichlet_bids:
            if not 1 <= int(b) <= 31:
                raise ValueError("constrained boundary ids must be in [1, 31]")
            mask |= 1 << int(b)
        opt.dirichlet_bid_mask = mask
        ctx = ctypes.c_void_p()
        _check(lib.hx_setup(ctypes.byref(mesh), int(p), ctypes.byref(mat), ctypes.byref(opt), ctypes.byref(ctx)))
        self._finish(ctx, p)


def _check_mg(status, mg):
    if status != HX_OK:
        raise HxError(status, lib.hx_mg_last_error(mg).decode())


class Multigrid:
    """p-multigrid V-cycle over operators on the same lattice with decreasing degrees."""

    def __init__(self, levels, smoother_degree=4, coarse_degree=30, smoothing_range=100.0, eig_iters=20,
                 eig_safety=1.2, precision="fp32", use_graph=True, level_mode="tangent", coarse_solver="auto",
                 fuse_smoother=True, smoother_blocks=True):
        """levels: Operators, finest first (see hx_mg_create for the allowed level pairs).
        coarse_solver: "auto" (dense up to 8192 DoFs), "chebyshev" or "dense".
        smoother_blocks: Jacobi with the inverses of the nodal 3x3 blocks (True) or of the diagonal."""
        self.levels = list(levels)
        arr = (ctypes.c_void_p * len(self.levels))(*[op.ctx.value for op in self.levels])
        o = _MgOptions(int(smoother_degree), int(coarse_degree), float(smoothing_range), int(eig_iters),
                       float(eig_safety), PRECISIONS[precision], int(bool(use_graph)), MODES[level_mode],
                       {"auto": 0, "chebyshev": 1, "dense": 2}[coarse_solver], int(bool(fuse_smoother)),
                       int(bool(smoother_blocks)))
        mg = ctypes.c_void_p()
        _check(lib.hx_mg_create(arr, len(self.levels), ctypes.byref(o), ctypes.byref(mg)))
        self.mg = mg
        self.precision = precision
        self.smoother_blocks = bool(smoother_blocks)

    def close(self):
        if getattr(self, "mg", None):
            lib.hx_mg_destroy(self.mg)
            self.mg = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, u, stream=None):
        import torch
        _check_mg(lib.hx_mg_update(self.mg, self.levels[0]._vec(u, torch.float64, "u"), _stream_handle(stream)),
                  self.mg)

    def vcycle(self, r, z=None, stream=None):
        import torch
        dt = torch.float64 if self.precision == "fp64" else torch.float32
        z = torch.empty_like(r) if z is None else z
        _check_mg(lib.hx_mg_vcycle(self.mg, self.levels[0]._vec(r, dt, "r"), self.levels[0]._vec(z, dt, "z"),
                                   _stream_handle(stream)), self.mg)
        return z

    @property
    def vcycle_count(self):
        return int(lib.hx_mg_vcycle_count(self.mg))

    def level_mode(self, level):
        m = int(lib.hx_mg_level_mode(self.mg, int(level)))
        return MODE_NAMES.get(m)

    def lambda_max(self, level):
        return float(lib.hx_mg_lambda_max(self.mg, int(level)))

    def transfer(self, level, kind, x, out, stream=None):
        """kind 0: out += P x (fine <- coarse); 1: out += P^T x (coarse <- fine); 2: out = J x."""
        import torch
        dt = torch.float64 if (kind == 2 or self.precision == "fp64") else torch.float32
        lf, lc = self.levels[level], self.levels[level + 1]
        src_op, dst_op = (lc, lf) if kind == 0 else (lf, lc)
        _check_mg(lib.hx_mg_transfer(self.mg, int(level), int(kind), src_op._vec(x, dt, "x"),
                                     dst_op._vec(out, dt, "out"), _stream_handle(stream)), self.mg)
        return out

    def inverse_diagonal(self, level, stream=None):
        """The smoother's D^-1 on a level: [3 * n_nodes] (point Jacobi) or, with nodal blocks,
        [6 * n_nodes], the planes (00, 11, 22, 01, 02, 12) of the inverse blocks."""
        import torch
        dt = torch.float64 if self.precision == "fp64" else torch.float32
        op = self.levels[level]
        out = torch.empty(op.num_dofs * (2 if self.smoother_blocks else 1), dtype=dt, device="cuda")
        _check_mg(lib.hx_mg_inverse_diagonal(self.mg, int(level), ctypes.c_void_p(out.data_ptr()),
                                             _stream_handle(stream)), self.mg)
        return out

    def newton_solve(self, u, f_ext=None, rel_tol=1e-8, abs_tol=0.0, max_newton=20, krylov_rel_tol=1e-3,
                     max_krylov=500, load_steps=1, outer_mode="tangent", stream=None, check=True, verbose=False,
                     predictor=True):
        """predictor: load steps after the first start from the secant extrapolation of the previous
        two converged displacements unless its residual is not finite (see hx_newton_opts)."""
        import torch
        o = _NewtonOpts(float(rel_tol), float(abs_tol), int(max_newton), float(krylov_rel_tol), int(max_krylov),
                        int(load_steps), MODES[outer_mode], int(bool(verbose)), int(bool(predictor)))
        rep = _NewtonReport()
        f = None if f_ext is None else self.levels[0]._vec(f_ext, torch.float64, "f_ext")
        st = lib.hx_newton_solve(self.mg, self.levels[0]._vec(u, torch.float64, "u"), f, ctypes.byref(o),
                                 ctypes.byref(rep), _stream_handle(stream))
        out = {k: getattr(rep, k) for k, _ in _NewtonReport._fields_}
        out["outer_mode"] = MODE_NAMES.get(out["outer_mode"], out["outer_mode"])
        out["status"] = STATUS.get(st, st)
        if check:
            _check_mg(st, self.mg)
        return out


def cells_per_workgroup(p, variant=0):
    """Cells per workgroup of a degree's variant (hx_cells_per_workgroup), -1 if none."""
    return int(lib.hx_cells_per_workgroup(int(p), int(variant)))


def tuning_key(p, law, precision, mode, mesh="lattice"):
    """Key of a stored autotuner choice: degree, law, precision class, storage mode, mesh kind."""
    return f"p{int(p)}/{law}/{'fp64' if precision == 'fp64' else 'fp32'}/{mode}/{mesh}"


def load_tuning(path):
    """The autotuner table stored at path (JSON {key: {variant, nontemporal, ms, ...}}), or {}."""
    import json
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def store_tuning(path, table):
    """Writes the autotuner table (see load_tuning) to path as JSON."""
    import json
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune_with_table(op, u, law, precision="fp64", reps=20, path=None, mesh="lattice"):
    """Tunes op at u, or, where the table at path holds the choice of every storage mode for this
    (degree, law, precision, mesh kind), sets those choices without timing and updates the slot in
    the stored best mode. Returns (best mode, table entries used) and stores new measurements."""
    table = load_tuning(path)
    keys = {m: tuning_key(op.p, law, precision, m, mesh) for m in STORAGE_MODES}
    if all(k in table for k in keys.values()):
        for m, k in keys.items():
            op.set_tuning(m, precision, table[k]["variant"], table[k]["nontemporal"])
        best = min(keys, key=lambda m: table[keys[m]]["ms"])
        op.update_linearization(u, mode=best, precision=precision)
        return best, {m: table[k] for m, k in keys.items()}
    best, entries = op.autotune(u, precision, reps)
    chosen = {}
    for e in entries:
        k = keys[e["mode"]]
        if k not in chosen or e["ms"] < chosen[k]["ms"]:
            chosen[k] = e
    table.update(chosen)
    if path:
        store_tuning(path, table)
    return best["mode"], {m: chosen[k] for m, k in keys.items()}
