"""Pins of the oracle's surface load and transfer matrices (closed forms and identities)."""
import numpy as np
import pytest

import workloads
from oracle import fem, mesh
from tests.helpers import box_problem


def test_pressure_resultant_on_planar_faces():
    pb = box_problem((2, 3, 2), 2, faces=(), lengths=(2.0, 1.0, 1.5))
    areas = {0: 1.5, 1: 1.5, 2: 3.0, 3: 3.0, 4: 2.0, 5: 2.0}
    for face in range(6):
        f = fem.surface_load(pb, face, 0.7)
        d, side = face // 2, face % 2
        expect = np.zeros(3)
        expect[d] = -0.7 * areas[face] * (1.0 if side else -1.0)
        np.testing.assert_allclose(f.sum(axis=1), expect, atol=1e-13)


def test_pressure_on_a_closed_ring_has_no_resultant():
    V = workloads.tube_vertices(8, 2, 3, length=1.0, bend=0.0)
    m = mesh.BoxMesh(8, 2, 3, V, 2, periodic=(True, False, False))
    pb = fem.Problem(m, fem.material.Material("cnh", mu=1.0, lam=1.0))
    f_in = fem.surface_load(pb, 2, 1.0)
    # resultant of a uniform pressure on the closed inner wall of a straight ring vanishes
    assert np.abs(f_in.sum(axis=1)).max() < 1e-13
    # and the radial load points outward (away from the axis) for internal pressure
    X = m.node_coords
    radial = np.einsum("cn,nc->n", f_in[:2], X[:, :2]) / np.linalg.norm(X[:, :2], axis=1)
    assert radial.sum() > 0


@pytest.mark.parametrize("pf,pc", [(2, 1), (3, 2), (4, 2), (6, 3)])
def test_transfers_reproduce_polynomials(pf, pc):
    V = workloads.box_vertices(2, 2, 1)
    mf = mesh.BoxMesh(2, 2, 1, V, pf)
    mc = mesh.BoxMesh(2, 2, 1, V, pc)
    P = fem.prolongation_matrix(mf, mc)
    J = fem.interpolation_matrix(mf, mc)
    rng = np.random.default_rng(0)
    cx = rng.standard_normal(pc + 1)
    Xf, Xc = mf.node_coords, mc.node_coords
    g = lambda X: np.polyval(cx, X[:, 0]) * (1 + X[:, 1]) ** pc - X[:, 2]  # degree <= pc per variable
    np.testing.assert_allclose(P @ g(Xc), g(Xf), atol=1e-12)
    np.testing.assert_allclose(J @ g(Xf), g(Xc), atol=1e-12)
    np.testing.assert_allclose(J @ P, np.eye(mc.n_nodes), atol=1e-12)
