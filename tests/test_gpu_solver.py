"""GPU checks of the p-multigrid and Newton-Krylov rows against the FP64 oracle.

* transfers: prolongation, restriction (= transpose) and interpolation of the linearisation point
  against the oracle's dense transfer matrices (FP64 hierarchy, element by element);
* inverse diagonal of each level against the diagonal of the oracle's assembled operator;
* V-cycle: symmetric (FP64), convergent as a stationary iteration, graph replay = eager launch;
* dead-load surface vector against the oracle;
* Newton solve: the solution satisfies the oracle's residual equation to the solve tolerance, in
  mixed precision (FP32 V-cycle) and in FP64.
"""
import numpy as np
import pytest
import torch

import paper_2408_12479_amd as hx
import workloads
from oracle import fem, fiber, mesh as omesh
from tests.gpu_helpers import rel, to_dev, to_host
from tests.helpers import make_material

pytestmark = pytest.mark.gpu


def _levels(cells, degrees, law="cnh", faces=(0,), perturb=0.2, tube=None, periodic=(False, False, False),
            frames=None, **matkw):
    nx, ny, nz = cells
    if tube is not None:
        V = workloads.tube_vertices(nx, ny, nz, **tube)
    else:
        V = workloads.box_vertices(nx, ny, nz, perturb=perturb, seed=2)
    mat = make_material(law, **matkw)
    cell_fibers = None
    if frames is not None:
        cell_fibers = fiber.cell_structure_tensors(frames, np.deg2rad(45.0), *fiber.dispersion_coefficients(3.62, 34.3))
    ops, pbs = [], []
    for p in degrees:
        m = omesh.BoxMesh(nx, ny, nz, V, p, dirichlet_faces=faces, periodic=periodic)
        pbs.append(fem.Problem(m, mat, cell_fibers=cell_fibers))
        ops.append(hx.Operator(nx, ny, nz, V, p, law=law, mu=mat.mu, lam=mat.lam, kappa=mat.kappa, k1=mat.k1,
                               k2=mat.k2, H4=mat.H4, H6=mat.H6, M4=mat.M4, M6=mat.M6, dirichlet_faces=faces,
                               periodic=periodic, frames=frames))
    return ops, pbs


def _smooth_u(pb, scale=0.02):
    X = pb.mesh.node_coords
    damp = X[:, 0] - X[:, 0].min()
    u = scale * damp * np.stack([np.sin(X[:, 1] + X[:, 2]), np.cos(X[:, 0] - X[:, 2]), np.sin(2 * X[:, 1])])
    u[:, pb.mesh.constrained] = 0.0
    return u


def test_transfers_match_oracle(device):
    ops, pbs = _levels((2, 2, 2), [4, 2, 1], faces=(0,))
    mg = hx.Multigrid(ops, precision="fp64")
    rng = np.random.default_rng(3)
    for l in range(2):
        P = fem.prolongation_matrix(pbs[l].mesh, pbs[l + 1].mesh)
        J = fem.interpolation_matrix(pbs[l].mesh, pbs[l + 1].mesh)
        nf, nc = ops[l].num_nodes, ops[l + 1].num_nodes
        xc = rng.standard_normal((3, nc))
        yf = rng.standard_normal((3, nf))
        out = torch.zeros(3 * nf, dtype=torch.float64, device="cuda")
        mg.transfer(l, 0, to_dev(xc), out)
        assert rel(to_host(out, nf), (P @ xc.T).T) < 1e-14
        out = torch.zeros(3 * nc, dtype=torch.float64, device="cuda")
        mg.transfer(l, 1, to_dev(yf), out)
        ref = (P.T @ yf.T).T
        ref[:, pbs[l + 1].mesh.constrained] = 0.0
        assert rel(to_host(out, nc), ref) < 1e-13
        out = torch.zeros(3 * nc, dtype=torch.float64, device="cuda")
        mg.transfer(l, 2, to_dev(yf), out)
        assert rel(to_host(out, nc), (J @ yf.T).T) < 1e-14
    mg.close()


@pytest.mark.parametrize("law", ["cnh", "fiber"])
def test_inverse_diagonal_matches_oracle(device, law):
    ops, pbs = _levels((2, 2, 1), [3, 1], law=law, faces=(0,))
    u = _smooth_u(pbs[0])
    mg = hx.Multigrid(ops, precision="fp64")
    mg.update(to_dev(u))
    dinv = to_host(mg.inverse_diagonal(0), ops[0].num_nodes)
    K = pbs[0].tangent_matrix(u)
    assert rel(dinv.ravel(), 1.0 / np.diag(K)) < 1e-12
    # the coarse level is linearised at the fine displacement interpolated onto its nodes
    J = fem.interpolation_matrix(pbs[0].mesh, pbs[1].mesh)
    uc = (J @ u.T).T
    dinv1 = to_host(mg.inverse_diagonal(1), ops[1].num_nodes)
    assert rel(dinv1.ravel(), 1.0 / np.diag(pbs[1].tangent_matrix(uc))) < 1e-12
    mg.close()


def test_vcycle_symmetric_and_convergent(device):
    ops, pbs = _levels((3, 3, 2), [3, 2, 1], faces=(0,))
    u = _smooth_u(pbs[0])
    mg = hx.Multigrid(ops, precision="fp64", coarse_degree=20)
    mg.update(to_dev(u))
    n = ops[0].num_nodes
    rng = np.random.default_rng(5)
    mask = pbs[0].mesh.constrained
    w1, w2 = rng.standard_normal((2, 3, n))
    w1[:, mask] = 0.0
    w2[:, mask] = 0.0
    z1 = to_host(mg.vcycle(to_dev(w1)), n)
    z2 = to_host(mg.vcycle(to_dev(w2)), n)
    a, b = np.vdot(w2, z1), np.vdot(w1, z2)
    assert abs(a - b) < 1e-10 * (abs(a) + abs(b))
    assert np.vdot(w1, z1) > 0
    # stationary iteration x <- x + M (b - K x) on the constrained operator converges
    K = pbs[0].tangent_matrix(u)
    bvec = rng.standard_normal(3 * n)
    bvec[np.tile(mask, 3)] = 0.0
    x = np.zeros(3 * n)
    r0 = np.linalg.norm(bvec)
    for _ in range(6):
        r = bvec - K @ x
        x = x + to_host(mg.vcycle(to_dev(r)), n).ravel()
    factor = (np.linalg.norm(bvec - K @ x) / r0) ** (1.0 / 6.0)
    assert factor < 0.75, factor
    mg.close()


def test_graph_replay_matches_eager(device):
    ops, pbs = _levels((3, 2, 2), [4, 2, 1], faces=(0,))
    u = _smooth_u(pbs[0])
    mg_g = hx.Multigrid(ops, precision="fp32", use_graph=True)
    mg_e = hx.Multigrid(ops, precision="fp32", use_graph=False)
    ud = to_dev(u)
    mg_g.update(ud)
    rng = np.random.default_rng(9)
    n = ops[0].num_nodes
    for it in range(3):
        w = rng.standard_normal((3, n))
        w[:, pbs[0].mesh.constrained] = 0.0
        wd = to_dev(w, "float32")
        zg = mg_g.vcycle(wd).double().cpu().numpy()
        torch.cuda.synchronize()
        mg_e.update(ud)   # eager work between the replays (and the eager hierarchy's own update)
        ze = mg_e.vcycle(wd).double().cpu().numpy()
        assert rel(zg, ze) < 1e-5, it
    mg_g.close()
    mg_e.close()


def test_surface_load_matches_oracle(device):
    ops, pbs = _levels((2, 3, 2), [3], faces=(0,))
    for face in range(6):
        assert rel(ops[0].surface_load(face, 0.3), fem.surface_load(pbs[0], face, 0.3)) < 1e-14
    ops, pbs = _levels((8, 2, 3), [2], faces=(4, 5), tube=dict(length=1.0, bend=0.3), periodic=(True, False, False))
    assert rel(ops[0].surface_load(2, 0.1), fem.surface_load(pbs[0], 2, 0.1)) < 1e-14


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_newton_solve_box(device, precision):
    ops, pbs = _levels((3, 2, 2), [2, 1], faces=(0,), mu=1.0, lam=10.0)
    f = -ops[0].surface_load(1, 0.1)   # outward traction (negative pressure) on +x
    mg = hx.Multigrid(ops, precision=precision)
    u = torch.zeros(ops[0].num_dofs, dtype=torch.float64, device="cuda")
    rep = mg.newton_solve(u, to_dev(f), rel_tol=1e-9, krylov_rel_tol=1e-4, load_steps=2, outer_mode="tangent")
    assert rep["status"] == "HX_OK" and rep["newton_iters"] >= 2
    uh = to_host(u, ops[0].num_nodes)
    fo = f.copy()
    fo[:, pbs[0].mesh.constrained] = 0.0
    res = pbs[0].residual(uh) - fo
    assert np.linalg.norm(res) < 1e-8 * np.linalg.norm(fo)
    assert np.abs(uh).max() > 1e-3
    mg.close()


@pytest.mark.parametrize("law", ["inh", "fiber"])
def test_newton_solve_pressurised_ring_mixed_matches_fp64(device, law):
    tube = dict(r_in=1.0, wall=0.2, length=1.0, bend=0.2)
    frames = workloads.tube_frames(8, 2, 3, length=1.0, bend=0.2) if law == "fiber" else None
    ops, pbs = _levels((8, 2, 3), [2, 1], law=law, faces=(4, 5), tube=tube, periodic=(True, False, False),
                       frames=frames, mu=2.0, kappa=50.0)
    f = ops[0].surface_load(2, 0.05)
    sols = {}
    for precision in ["fp32", "fp64"]:
        mg = hx.Multigrid(ops, precision=precision)
        u = torch.zeros(ops[0].num_dofs, dtype=torch.float64, device="cuda")
        rep = mg.newton_solve(u, to_dev(f), rel_tol=1e-9, krylov_rel_tol=1e-4, load_steps=2)
        assert rep["status"] == "HX_OK"
        sols[precision] = to_host(u, ops[0].num_nodes)
        mg.close()
    fo = f.copy()
    fo[:, pbs[0].mesh.constrained] = 0.0
    for s in sols.values():
        assert np.linalg.norm(pbs[0].residual(s) - fo) < 1e-8 * np.linalg.norm(fo)
    assert rel(sols["fp32"], sols["fp64"]) < 1e-6
