"""Parity at the benchmark's full sizes, through the same library calls and launch shapes that
bench.py times, on sampled rows: the oracle evaluates every cell that touches a sampled node, so
those rows are complete.

* 32^3 perturbed cube, Q2/Q3/Q4/Q6 (0.8 to 21.6 MDoF), cNH mu = 1, lambda = 100, u with largest
  stretch 1.3: the four FP64 storage modes, relative error over the sampled rows <= 1e-12; the
  residual to 1e-12 of its cell-contribution scale (the assembled rows of this smooth state
  cancel to ~1e-4 of it);
* 64x32x32 anisotropic box, Q3, fibre law: FP32 applies <= 1e-5 against the FP64 oracle of the
  FP32-rounded direction;
* the Q6 tube of the multigrid study (16x8x200, per-cell frames, 16.9 MDoF): FP64 spatial and
  tangent applies on sampled rows, and symmetry of the operator on random vectors;
* the anisotropic box's 16-bit data applies against the oracle on sampled rows, with bounds;
* a reduced isoparametric pressurised tube solved by the mixed-precision Newton-multigrid
  solver: its solution satisfies the oracle's residual equation on sampled rows to 1e-8.
Sampled nodes: lattice corners, nodes on the constrained face, edges, interior and random ones.
"""
import math

import numpy as np
import pytest
import torch

import paper_2408_12479_amd as hx
import workloads
from oracle import fem, fiber, material, mesh as omesh
from tests.gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _sample_nodes(m, k, seed):
    Nx, Ny, Nz = m.ndims
    lat = lambda i, j, kk: i + Nx * (j + Ny * kk)  # noqa: E731
    fixed = [lat(0, 0, 0), lat(Nx - 1, Ny - 1, Nz - 1), lat(0, Ny // 2, Nz // 3), lat(Nx - 1, 0, Nz // 2),
             lat(Nx // 2, Ny - 1, 0), lat(Nx // 3, Ny // 2, Nz // 2), lat(m.p, m.p, m.p), lat(m.p + 1, 1, 2)]
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.array(fixed) % m.n_nodes, rng.integers(0, m.n_nodes, k)]))


def _rows(v, nodes, n_nodes):
    return np.asarray(v).reshape(3, n_nodes)[:, nodes]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("p", [2, 3, 4, 6])
def test_cube32_sampled_rows(device, p):
    V = workloads.box_vertices(32, 32, 32, perturb=0.2, seed=2)
    m = omesh.BoxMesh(32, 32, 32, V, p, dirichlet_faces=(0,))
    pb = fem.Problem(m, material.Material("cnh", mu=1.0, lam=100.0), chunk=32)
    u, du = workloads.sweep_fields(m.node_coords, m.constrained)
    nodes = _sample_nodes(m, 16 if p < 6 else 8, seed=p)
    cells = pb.cells_touching(nodes)
    ref_k = _rows(pb.apply_tangent(u, du, cells=cells), nodes, m.n_nodes)
    ref_r = _rows(pb.residual(u, cells=cells), nodes, m.n_nodes)
    # the assembled residual of this smooth state nearly cancels between neighbouring cells; its
    # rounding scale is that of the cell contributions, measured by half of the touching cells
    r_scale = max(np.linalg.norm(ref_r), np.linalg.norm(_rows(pb.residual(u, cells=cells[::2]), nodes, m.n_nodes)))
    op = hx.Operator(32, 32, 32, V, p, law="cnh", mu=1.0, lam=100.0, dirichlet_faces=(0,))
    ud, dud = to_dev(u), to_dev(du)
    r = op.residual(ud).cpu().numpy()
    assert np.linalg.norm(_rows(r, nodes, m.n_nodes) - ref_r) < 1e-12 * r_scale
    for mode in ["none", "finv_j", "tangent", "spatial"]:
        op.update_linearization(ud, mode=mode, precision="fp64")
        y = op.apply_tangent(dud).cpu().numpy()
        assert _rel(_rows(y, nodes, m.n_nodes), ref_k) < 1e-12, mode
    op.close()


def test_fiber_box_fp32_sampled_rows(device):
    V = workloads.box_vertices(64, 32, 32, lengths=(2.0, 1.0, 1.0), perturb=0.0)
    m = omesh.BoxMesh(64, 32, 32, V, 3)
    H4, H6, M4, M6 = fiber.structure_tensors(*np.eye(3), math.radians(45.0), *fiber.dispersion_coefficients(3.62, 34.3))
    mat = material.Material("fiber", mu=2.0, kappa=1e3, k1=1.0, k2=10.0, H4=H4, H6=H6, M4=M4, M6=M6)
    pb = fem.Problem(m, mat, chunk=64)
    u, du = workloads.fiber_fields(m.node_coords)
    nodes = _sample_nodes(m, 16, seed=7)
    cells = pb.cells_touching(nodes)
    ref = _rows(pb.apply_tangent(u, du.astype(np.float32).astype(np.float64), cells=cells), nodes, m.n_nodes)
    op = hx.Operator(64, 32, 32, V, 3, law="fiber", mu=2.0, kappa=1e3, k1=1.0, k2=10.0, H4=H4, H6=H6, M4=M4, M6=M6)
    ud, du32 = to_dev(u), to_dev(du, "float32")
    for mode in hx.STORAGE_MODES:
        op.update_linearization(ud, mode=mode, precision="fp32")
        y = op.apply_tangent(du32, precision="fp32").double().cpu().numpy()
        err = _rel(_rows(y, nodes, m.n_nodes), ref)
        assert err < 1e-5, (mode, err)
    # 16-bit stored data against the oracle at full size: no accuracy target, bounded so that a
    # broken path fails (bfloat16 keeps 8 significant bits, binary16 11 with a per-cell scale)
    for mode, prec, bound in [("tangent", "fp32_bf16", 2e-2), ("tangent", "fp32_fp16", 3e-3),
                              ("spatial", "fp32_bf16", 2e-2), ("finv_j", "fp32_bf16", 2e-2)]:
        op.update_linearization(ud, mode=mode, precision=prec)
        y = op.apply_tangent(du32, precision=prec).double().cpu().numpy()
        err = _rel(_rows(y, nodes, m.n_nodes), ref)
        assert 1e-6 < err < bound, (mode, prec, err)
    op.close()


def test_pressurised_isoparametric_tube_newton(device):
    """A reduced version of the Newton study: the isoparametric tube (curved Q4 cells, 16 x 4 x 40,
    length 10), the tissue fibre law, pressure 0.1 on the inner wall in 5 load steps, levels
    4 -> 2 -> 1 -> coarser lattices, FP32 multigrid with FP64 Newton/CG. The solution satisfies the
    oracle's residual equation r(u) = f on sampled rows to the solve's 1e-8."""
    cells = (16, 4, 40)
    tube = dict(r_in=1.0, wall=0.2, length=10.0, bend=1.0)
    g = 4
    G = workloads.tube_geometry_nodes(*cells, g, **tube)
    frames = workloads.tube_frames(*cells, length=10.0, bend=1.0)
    scale = 2.0 / 62.1
    kw = dict(law="fiber", mu=2.0, kappa=3084.3 * scale, k1=1.4 * scale, k2=22.1)
    _, _, M4, M6 = hx.fiber_structure(1.0, 1.0, math.radians(27.47))
    H4, H6 = np.outer(M4, M4), np.outer(M6, M6)

    def level(c, p):
        Gl = workloads.tube_geometry_nodes(*c, g, **tube)
        fr = workloads.tube_frames(*c, length=10.0, bend=1.0)
        return hx.Operator(*c, None, p, H4=H4, H6=H6, M4=M4, M6=M6, dirichlet_faces=(4, 5),
                           periodic=(True, False, False), frames=fr, geom_degree=g, geom_nodes=Gl, **kw)
    ops = [level(cells, 4), level(cells, 2), level(cells, 1), level((16, 2, 20), 1)]
    f = ops[0].surface_load(2, 0.1)
    mg = hx.Multigrid(ops, precision="fp32", level_mode="auto")
    u = torch.zeros(ops[0].num_dofs, dtype=torch.float64, device="cuda")
    rep = mg.newton_solve(u, to_dev(f), rel_tol=1e-8, krylov_rel_tol=1e-3, load_steps=5, max_newton=30,
                          max_krylov=2000, outer_mode="auto")
    assert rep["status"] == "HX_OK" and rep["load_steps_done"] == 5
    mg.close()
    m = omesh.BoxMesh(*cells, workloads.tube_vertices(*cells, **tube), 4, dirichlet_faces=(4, 5),
                      periodic=(True, False, False), geom_degree=g, geom_nodes=G)
    coef = (1.0, 0.0, 0.0)
    mat = material.Material("fiber", mu=kw["mu"], kappa=kw["kappa"], k1=kw["k1"], k2=kw["k2"])
    pb = fem.Problem(m, mat, chunk=64,
                     cell_fibers=fiber.cell_structure_tensors(frames, math.radians(27.47), *coef))
    np.testing.assert_allclose(ops[0].node_coords(), m.node_coords, rtol=0, atol=1e-12)
    uh = u.cpu().numpy().reshape(3, m.n_nodes)
    fo = f.copy()
    fo[:, m.constrained] = 0.0
    # sampled rows: the free nodes of the inner wall (loaded) and random ones
    rng = np.random.default_rng(21)
    nodes = np.unique(np.concatenate([rng.integers(0, m.n_nodes, 24),
                                      np.nonzero(np.abs(fo).sum(axis=0) > 0)[0][::97]]))
    nodes = nodes[~m.constrained[nodes]]
    cells_t = pb.cells_touching(nodes)
    r = pb.residual(uh, cells=cells_t)[:, nodes]
    # the whole load vector's norm is the scale of the 1e-8 relative tolerance of the solve
    assert np.linalg.norm(r - fo[:, nodes]) < 1e-8 * np.linalg.norm(fo)
    assert np.abs(uh).max() > 1e-3
    for op in ops:
        op.close()


def test_tube_q6_sampled_rows_and_symmetry(device):
    cells = (16, 8, 200)
    tube = dict(r_in=1.0, wall=0.2, length=10.0, bend=1.0)
    V = workloads.tube_vertices(*cells, **tube)
    frames = workloads.tube_frames(*cells, length=10.0, bend=1.0)
    m = omesh.BoxMesh(*cells, V, 6, dirichlet_faces=(4, 5), periodic=(True, False, False))
    coef = fiber.dispersion_coefficients(3.62, 34.3)
    pb = fem.Problem(m, material.Material("fiber", mu=2.0, kappa=50.0, k1=1.0, k2=10.0), chunk=16,
                     cell_fibers=fiber.cell_structure_tensors(frames, math.radians(45.0), *coef))
    X = m.node_coords
    s = X[:, 2]
    phi = 0.05 * np.sin(np.pi * s / 10.0)
    dx, y = X[:, 0] - np.sin(np.pi * s / 10.0), X[:, 1]
    u = np.stack([np.cos(phi) * dx - np.sin(phi) * y - dx, np.sin(phi) * dx + np.cos(phi) * y - y, 0 * s])
    u[:, m.constrained] = 0.0
    du = np.random.default_rng(11).standard_normal((3, m.n_nodes))
    nodes = _sample_nodes(m, 8, seed=11)
    ref = _rows(pb.apply_tangent(u, du, cells=pb.cells_touching(nodes)), nodes, m.n_nodes)
    H4, H6, M4, M6 = fiber.structure_tensors(*np.eye(3), math.radians(45.0), *coef)
    op = hx.Operator(*cells, V, 6, law="fiber", mu=2.0, kappa=50.0, k1=1.0, k2=10.0, H4=H4, H6=H6, M4=M4, M6=M6,
                     dirichlet_faces=(4, 5), periodic=(True, False, False), frames=frames)
    ud, dud = to_dev(u), to_dev(du)
    g = torch.Generator(device="cpu").manual_seed(3)
    v1 = torch.randn(op.num_dofs, generator=g, dtype=torch.float64).cuda()
    v2 = torch.randn(op.num_dofs, generator=g, dtype=torch.float64).cuda()
    for mode in ["spatial", "tangent"]:
        op.update_linearization(ud, mode=mode, precision="fp64")
        yk = op.apply_tangent(dud).cpu().numpy()
        assert _rel(_rows(yk, nodes, m.n_nodes), ref) < 1e-12, mode
        a = torch.dot(v2, op.apply_tangent(v1)).item()
        b = torch.dot(v1, op.apply_tangent(v2)).item()
        assert abs(a - b) < 1e-10 * abs(a), (mode, a, b)
    op.close()
