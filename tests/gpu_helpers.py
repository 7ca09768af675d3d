"""Builds matching (library operator, oracle problem) pairs on the same seeded inputs."""
import numpy as np

import workloads
from oracle import fem, fiber, mesh as omesh
from tests.helpers import make_material


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def periodic_x_vertices(V, nx, ny, nz):
    return V.reshape(nz + 1, ny + 1, nx + 1, 3)[:, :, :nx, :].reshape(-1, 3).copy()


def make_pair(cells, p, law, perturb=0.2, seed=2, faces=(0,), lengths=(1.0, 1.0, 1.0),
              periodic=(False, False, False), jpow_newton_iters=0, tube=None, frames=None, **matkw):
    """frames: [cells, 3, 3] local fibre frames (fibre law): the oracle builds each cell's
    structure tensors from its frame, the library rotates the material's local tensors."""
    import paper_2408_12479_amd as hx
    nx, ny, nz = cells
    if tube is not None:
        V = workloads.tube_vertices(nx, ny, nz, **tube)
    else:
        V = workloads.box_vertices(nx, ny, nz, lengths=lengths, perturb=perturb, seed=seed)
    m = omesh.BoxMesh(nx, ny, nz, V, p, dirichlet_faces=faces, periodic=periodic)
    mat = make_material(law, **matkw)
    cell_fibers = None
    if frames is not None:
        disp = matkw.get("dispersion", (3.62, 34.3))
        coef = (1.0, 0.0, 0.0) if disp is None else fiber.dispersion_coefficients(*disp)
        cell_fibers = fiber.cell_structure_tensors(frames, np.deg2rad(45.0), *coef)
    pb = fem.Problem(m, mat, cell_fibers=cell_fibers)
    op = hx.Operator(nx, ny, nz, V, p, law=law, mu=mat.mu, lam=mat.lam, kappa=mat.kappa,
                     k1=mat.k1, k2=mat.k2, H4=mat.H4, H6=mat.H6, M4=mat.M4, M6=mat.M6,
                     dirichlet_faces=faces, periodic=periodic, jpow_newton_iters=jpow_newton_iters,
                     frames=frames)
    return op, pb


def to_dev(x, dtype="float64"):
    import torch
    return torch.tensor(np.ascontiguousarray(x).reshape(-1), dtype=getattr(torch, dtype), device="cuda:0")


def to_host(t, n_nodes):
    return t.detach().double().cpu().numpy().reshape(3, n_nodes)
