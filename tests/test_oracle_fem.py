"""Pins of the oracle's residual and linearised operator (Section 2 definitions).

* patch test: an affine displacement on a perturbed mesh gives zero interior residual and face
  resultants equal to the constant traction P e_x times the face area (exact integration);
* rigid rotation and translation give zero residual; K annihilates translations;
* the residual is the gradient of the total energy (complex step on Psi);
* the linearised operator is the derivative of the residual (complex step), with the
  constrained rows/columns read as identity;
* symmetry of the assembled constrained operator;
* at u = 0 the operator is isotropic linear elasticity, checked against a stiffness written
  independently in Voigt notation.
"""
import numpy as np
import pytest

from oracle import material
from tests.helpers import box_problem

LAWS = ["cnh", "inh", "fiber"]


def _affine(coords, G, c):
    return (coords @ G.T + c).T.copy()


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("law", LAWS)
def test_patch_test(p, law):
    pb = box_problem(2, p, law=law, faces=())
    m = pb.mesh
    rng = np.random.default_rng(1)
    G = 0.1 * rng.uniform(-1, 1, (3, 3))
    u = _affine(m.node_coords, G, rng.uniform(-1, 1, 3))
    r = pb.residual(u)
    Nx, Ny, Nz = m.ndims
    node = np.arange(m.n_nodes)
    I, J, K = node % Nx, (node // Nx) % Ny, node // (Nx * Ny)
    interior = (I > 0) & (I < Nx - 1) & (J > 0) & (J < Ny - 1) & (K > 0) & (K < Nz - 1)
    P = material.first_pk((np.eye(3) + G)[None], pb.mat)[0]
    scale = np.max(np.abs(P)) + 1.0
    assert np.max(np.abs(r[:, interior])) < 1e-12 * scale
    # resultant on the +x face (area 1, outward normal e_x) = P e_x
    face = I == Nx - 1
    np.testing.assert_allclose(r[:, face].sum(axis=1), P[:, 0], atol=1e-12 * scale)


@pytest.mark.parametrize("law", LAWS)
def test_rigid_motions(law):
    pb = box_problem(2, 2, law=law, faces=())
    m = pb.mesh
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    u = _affine(m.node_coords, Q - np.eye(3), np.array([0.3, -0.1, 0.2]))
    assert np.max(np.abs(pb.residual(u))) < 1e-12
    rng = np.random.default_rng(2)
    u = 0.01 * rng.standard_normal((3, m.n_nodes))
    t = np.tile(np.array([[0.4], [-0.2], [0.9]]), (1, m.n_nodes))
    r0 = pb.residual(u)
    np.testing.assert_allclose(pb.residual(u + t), r0, atol=1e-12 * np.max(np.abs(r0)))
    Kt = pb.apply_tangent(u, t, constrain=False)
    assert np.max(np.abs(Kt)) < 1e-11 * np.max(np.abs(pb.apply_tangent(u, u, constrain=False)))


@pytest.mark.parametrize("law", LAWS)
def test_residual_is_energy_gradient(law):
    pb = box_problem(2, 2, law=law, faces=())
    rng = np.random.default_rng(3)
    u = 0.01 * rng.standard_normal((3, pb.mesh.n_nodes))
    r = pb.residual(u, constrain=False)
    h = 1e-30
    for _ in range(6):
        c, node = rng.integers(3), rng.integers(pb.mesh.n_nodes)
        e = np.zeros_like(u, dtype=complex)
        e[c, node] = 1j * h
        g = pb.energy(u + e).imag / h
        assert abs(g - r[c, node]) < 1e-12 * (1 + np.max(np.abs(r)))


@pytest.mark.parametrize("p", [1, 2, 4])
@pytest.mark.parametrize("law", LAWS)
def test_tangent_is_residual_derivative(p, law):
    pb = box_problem(2, p, law=law, faces=(0,))
    m = pb.mesh
    rng = np.random.default_rng(4)
    u = 0.01 * rng.standard_normal((3, m.n_nodes))
    u[:, m.constrained] = 0.0
    du = rng.standard_normal((3, m.n_nodes))
    Kdu = pb.apply_tangent(u, du)
    du_f = du.copy()
    du_f[:, m.constrained] = 0.0
    h = 1e-30
    d = pb.residual(u + 1j * h * du_f).imag / h   # constrained rows of r are zero
    d[:, m.constrained] = du[:, m.constrained]
    assert np.linalg.norm(Kdu - d) < 1e-13 * np.linalg.norm(Kdu)


@pytest.mark.parametrize("law", LAWS)
def test_symmetry(law):
    pb = box_problem(2, 2, law=law, faces=(0, 3))
    rng = np.random.default_rng(5)
    u = 0.01 * rng.standard_normal((3, pb.mesh.n_nodes))
    u[:, pb.mesh.constrained] = 0.0
    K = pb.tangent_matrix(u)
    assert np.max(np.abs(K - K.T)) < 1e-12 * np.max(np.abs(K))
    v, w = rng.standard_normal((2, 3, pb.mesh.n_nodes))
    a = np.vdot(v, pb.apply_tangent(u, w))
    b = np.vdot(w, pb.apply_tangent(u, v))
    assert abs(a - b) < 1e-12 * (abs(a) + abs(b))
    np.testing.assert_allclose(K @ w.ravel(), pb.apply_tangent(u, w).ravel(), atol=1e-12 * np.abs(K).max())


def _voigt_stiffness(pb, lam, mu):
    """Linear-elasticity operator in Voigt notation, written without the oracle's moduli."""
    m = pb.mesh
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[range(3), range(3)] += 2 * mu
    D[range(3, 6), range(3, 6)] = mu
    nn, n3 = m.n_nodes, (m.p + 1) ** 3
    K = np.zeros((3 * nn, 3 * nn))
    cells = np.arange(m.n_cells)
    Gphi, wdet = pb.physical_gradients(cells)
    for e in cells:
        dof = (np.arange(3)[:, None] * nn + m.cell_nodes[e][None, :]).ravel()
        Ke = np.zeros((3 * n3, 3 * n3))
        for q in range(Gphi.shape[1]):
            g = Gphi[e, q]                  # [n3, 3]
            B = np.zeros((6, 3 * n3))
            for c in range(3):
                B[c, c * n3:(c + 1) * n3] = g[:, c]
            # engineering shear strains yz, xz, xy
            for row, (i, j) in zip(range(3, 6), [(1, 2), (0, 2), (0, 1)]):
                B[row, i * n3:(i + 1) * n3] = g[:, j]
                B[row, j * n3:(j + 1) * n3] = g[:, i]
            Ke += wdet[e, q] * B.T @ D @ B
        K[np.ix_(dof, dof)] += Ke
    return K


@pytest.mark.parametrize("law", LAWS)
def test_identity_state_is_linear_elasticity(law):
    pb = box_problem(2, 2, law=law, faces=())
    mat = pb.mat
    lam_lin = 2.0 * mat.lam if law == "cnh" else mat.kappa - 2.0 * mat.mu / 3.0
    K = pb.tangent_matrix(np.zeros((3, pb.mesh.n_nodes)), constrain=False)
    Kv = _voigt_stiffness(pb, lam_lin, mat.mu)
    assert np.max(np.abs(K - Kv)) < 1e-12 * np.max(np.abs(Kv))


def test_sampled_rows_match_full_apply():
    pb = box_problem(3, 2, law="cnh", faces=(0,))
    rng = np.random.default_rng(6)
    u = 0.01 * rng.standard_normal((3, pb.mesh.n_nodes))
    du = rng.standard_normal((3, pb.mesh.n_nodes))
    full = pb.apply_tangent(u, du)
    rows = rng.choice(pb.mesh.n_nodes, 10, replace=False)
    part = pb.apply_tangent(u, du, cells=pb.cells_touching(rows))
    np.testing.assert_allclose(part[:, rows], full[:, rows], rtol=0, atol=1e-13 * np.abs(full).max())
