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


def _coarse_box(nf, nc, lengths=(1.0, 1.0, 1.0), faces=(), perturb=0.0):
    Vf = workloads.box_vertices(*nf, lengths=lengths, perturb=perturb, seed=2)
    Vc = workloads.box_vertices(*nc, lengths=lengths, perturb=0.0)
    return mesh.BoxMesh(*nf, Vf, 1, dirichlet_faces=faces), mesh.BoxMesh(*nc, Vc, 1, dirichlet_faces=faces)


@pytest.mark.parametrize("nf,nc", [((4, 2, 4), (2, 1, 2)), ((4, 3, 2), (2, 3, 1))])
def test_lattice_transfer_is_galerkin_on_affine_body(nf, nc):
    # nested lattices of a uniform box: the coarse trilinear space lies in the fine one, so the
    # rediscretised coarse operator equals P^T K_fine P (linear elasticity at u = 0)
    mf, mc = _coarse_box(nf, nc, lengths=(2.0, 1.0, 1.5))
    mat = fem.material.Material("cnh", mu=1.0, lam=3.0)
    Kf = fem.Problem(mf, mat).tangent_matrix(np.zeros((3, mf.n_nodes)), constrain=False)
    Kc = fem.Problem(mc, mat).tangent_matrix(np.zeros((3, mc.n_nodes)), constrain=False)
    P = fem.lattice_prolongation_matrix(mf, mc)
    P3 = np.kron(np.eye(3), P)
    assert np.abs(P3.T @ Kf @ P3 - Kc).max() < 1e-12 * np.abs(Kc).max()


def test_lattice_transfer_partition_of_unity_and_injection():
    mf, mc = _coarse_box((4, 2, 4), (2, 1, 2))
    P = fem.lattice_prolongation_matrix(mf, mc)
    J = fem.lattice_interpolation_matrix(mf, mc)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(J @ P, np.eye(mc.n_nodes), atol=1e-15)
    # reproduces coarse fields affine in the lattice coordinates
    Xc = mc.node_coords
    Xf = mf.node_coords
    g = np.array([0.3, -1.2, 0.7])
    np.testing.assert_allclose(P @ (Xc @ g + 0.5), Xf @ g + 0.5, atol=1e-14)
    # weights are 1 at coincident nodes and products of 1/2 at midpoints
    assert set(np.round(np.unique(P), 12)) <= {0.0, 0.125, 0.25, 0.5, 1.0}


def test_lattice_transfer_on_a_ring():
    Vf = workloads.tube_vertices(8, 2, 4, length=1.0, bend=0.2)
    Vc = workloads.tube_vertices(4, 2, 2, length=1.0, bend=0.2)
    mf = mesh.BoxMesh(8, 2, 4, Vf, 1, periodic=(True, False, False))
    mc = mesh.BoxMesh(4, 2, 2, Vc, 1, periodic=(True, False, False))
    P = fem.lattice_prolongation_matrix(mf, mc)
    J = fem.lattice_interpolation_matrix(mf, mc)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(J @ P, np.eye(mc.n_nodes), atol=1e-15)
    # the coarse vertices are the fine vertices at even lattice indices
    np.testing.assert_allclose(J @ mf.node_coords, mc.node_coords, atol=1e-14)
