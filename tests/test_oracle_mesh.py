"""Pins of the oracle's lattice, node coordinates and geometry."""
import numpy as np
import pytest

import workloads
from oracle import fem, mesh
from tests.helpers import make_material


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_counts_vertices_and_volume(p):
    V = workloads.box_vertices(3, 2, 4, lengths=(2.0, 1.0, 1.5), perturb=0.2, seed=5)
    m = mesh.BoxMesh(3, 2, 4, V, p, dirichlet_faces=(0, 5))
    assert m.n_nodes == (3 * p + 1) * (2 * p + 1) * (4 * p + 1)
    # lattice vertices reappear as nodes at lattice index (vx*p, vy*p, vz*p)
    Nx, Ny, _ = m.ndims
    for v in [0, 5, 17, len(V) - 1]:
        vx, vy, vz = v % 4, (v // 4) % 3, v // 12
        node = vx * p + Nx * (vy * p + Ny * vz * p)
        np.testing.assert_allclose(m.node_coords[node], V[v], atol=1e-15)
    pb = fem.Problem(m, make_material("cnh"))
    _, wdet = pb.geometry(np.arange(m.n_cells))
    # only interior vertices move, so the box volume is exact
    assert abs(wdet.sum() - 3.0) < 1e-13
    np.testing.assert_array_equal(m.constrained, workloads.lattice_dirichlet_mask(m.ndims, (0, 5)))


def test_periodic_identification():
    nx, ny, nz, p = 4, 2, 2, 2
    V = workloads.box_vertices(nx, ny, nz)
    Vp = V.reshape(nz + 1, ny + 1, nx + 1, 3)[:, :, :nx, :].reshape(-1, 3)
    m = mesh.BoxMesh(nx, ny, nz, Vp, p, periodic=(True, False, False))
    assert m.ndims == (nx * p, ny * p + 1, nz * p + 1)
    # the last cell's +x face nodes are the first cell's -x face nodes
    n = p + 1
    last = m.cell_nodes[nx - 1].reshape(n, n, n)[:, :, -1]
    first = m.cell_nodes[0].reshape(n, n, n)[:, :, 0]
    np.testing.assert_array_equal(last, first)


def test_invertibility_check():
    V = workloads.box_vertices(1, 1, 1)
    V[7] = [-1.0, -1.0, -1.0]  # fold the cell through itself
    m = mesh.BoxMesh(1, 1, 1, V, 2)
    with pytest.raises(ValueError):
        fem.Problem(m, make_material("cnh")).geometry(np.arange(1))
