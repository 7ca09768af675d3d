"""Pins of the oracle with fibre frames that vary from cell to cell (the tube workloads).

* frames equal to the global axes in every cell reproduce the uniform-material problem;
* a mesh whose cells carry one of two frames gives the sum of the two uniform-frame problems,
  each restricted to its own cells (residual and linearised operator);
* frame indifference: rotating the reference body, its fibre frames and the displacement by one
  rotation Q rotates the residual and the operator's action by Q, while rotating the frames alone
  changes them (so the frames do enter);
* on the tube, the linearised operator is the complex-step derivative of the residual;
* the tube frames are orthonormal and right-handed, E2 follows the centreline and E1 is the
  circumferential direction made normal to it.
"""
import numpy as np

import workloads
from oracle import fem, fiber, material, mesh as omesh

PHI = np.deg2rad(45.0)
DISP = fiber.dispersion_coefficients(3.62, 34.3)


def _fiber_mat(frame=np.eye(3)):
    H4, H6, M4, M6 = fiber.structure_tensors(*frame, PHI, *DISP)
    return material.Material("fiber", mu=2.0, kappa=50.0, k1=1.0, k2=10.0, H4=H4, H6=H6, M4=M4, M6=M6)


def _rotation(axis, angle):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * K @ K


def _box(nc=2, p=2, V=None, faces=()):
    if V is None:
        V = workloads.box_vertices(nc, nc, nc, perturb=0.2, seed=2)
    return omesh.BoxMesh(nc, nc, nc, V, p, dirichlet_faces=faces), V


def _stretch_u(m, rng, amp=0.08):
    X = m.node_coords
    u = amp * np.stack([X[:, 0] * (1 + X[:, 1]), 0.5 * X[:, 1] * X[:, 2], -0.3 * X[:, 2]])
    return u + 0.002 * rng.standard_normal(u.shape)


def test_identity_frames_reproduce_uniform_material():
    m, _ = _box()
    frames = np.tile(np.eye(3), (m.n_cells, 1, 1))
    pb_u = fem.Problem(m, _fiber_mat())
    pb_c = fem.Problem(m, _fiber_mat(), cell_fibers=fiber.cell_structure_tensors(frames, PHI, *DISP))
    rng = np.random.default_rng(0)
    u = _stretch_u(m, rng)
    du = rng.standard_normal(u.shape)
    r = pb_u.residual(u)
    assert np.linalg.norm(pb_c.residual(u) - r) <= 1e-15 * np.linalg.norm(r)
    k = pb_u.apply_tangent(u, du)
    assert np.linalg.norm(pb_c.apply_tangent(u, du) - k) <= 1e-15 * np.linalg.norm(k)


def test_two_frame_groups_sum_of_uniform_problems():
    m, _ = _box()
    R = _rotation([1.0, 2.0, 0.5], 0.9)
    ex = np.arange(m.n_cells) % m.nx
    group_b = ex % 2 == 1
    frames = np.where(group_b[:, None, None], R[None], np.eye(3)[None])
    pb_c = fem.Problem(m, _fiber_mat(), cell_fibers=fiber.cell_structure_tensors(frames, PHI, *DISP))
    pb_a, pb_b = fem.Problem(m, _fiber_mat(np.eye(3))), fem.Problem(m, _fiber_mat(R))
    ca, cb = np.nonzero(~group_b)[0], np.nonzero(group_b)[0]
    rng = np.random.default_rng(1)
    u = _stretch_u(m, rng)
    du = rng.standard_normal(u.shape)
    r = pb_c.residual(u)
    ref = pb_a.residual(u, cells=ca) + pb_b.residual(u, cells=cb)
    assert np.linalg.norm(r - ref) <= 1e-14 * np.linalg.norm(ref)
    k = pb_c.apply_tangent(u, du, constrain=False)
    ref = pb_a.apply_tangent(u, du, cells=ca, constrain=False) + pb_b.apply_tangent(u, du, cells=cb, constrain=False)
    assert np.linalg.norm(k - ref) <= 1e-14 * np.linalg.norm(ref)
    # the two groups really differ: the uniform problem alone does not reproduce the sum
    assert np.linalg.norm(pb_a.residual(u) - r) > 1e-3 * np.linalg.norm(r)


def test_frame_indifference_with_cell_frames():
    m, V = _box()
    rng = np.random.default_rng(2)
    frames = np.stack([_rotation(rng.standard_normal(3), rng.uniform(0, np.pi)) for _ in range(m.n_cells)])
    Q = _rotation([0.3, -1.0, 0.7], 1.1)
    pb = fem.Problem(m, _fiber_mat(), cell_fibers=fiber.cell_structure_tensors(frames, PHI, *DISP))
    m_rot, _ = _box(V=V @ Q.T)
    assert np.allclose(m_rot.node_coords, m.node_coords @ Q.T, atol=1e-14)
    frames_rot = frames @ Q.T
    pb_rot = fem.Problem(m_rot, _fiber_mat(), cell_fibers=fiber.cell_structure_tensors(frames_rot, PHI, *DISP))
    u = _stretch_u(m, rng)
    du = rng.standard_normal(u.shape)
    r = pb.residual(u)
    assert np.linalg.norm(pb_rot.residual(Q @ u) - Q @ r) <= 1e-13 * np.linalg.norm(r)
    k = pb.apply_tangent(u, du)
    assert np.linalg.norm(pb_rot.apply_tangent(Q @ u, Q @ du) - Q @ k) <= 1e-13 * np.linalg.norm(k)
    # rotating only the frames is a different material
    pb_f = fem.Problem(m, _fiber_mat(), cell_fibers=fiber.cell_structure_tensors(frames_rot, PHI, *DISP))
    assert np.linalg.norm(pb_f.residual(u) - r) > 1e-3 * np.linalg.norm(r)


def _tube_problem(p=2):
    cells = (8, 2, 2)
    tube = dict(r_in=1.0, wall=0.2, length=1.0, bend=0.3)
    V = workloads.tube_vertices(*cells, **tube)
    m = omesh.BoxMesh(*cells, V, p, dirichlet_faces=(4, 5), periodic=(True, False, False))
    frames = workloads.tube_frames(*cells, length=tube["length"], bend=tube["bend"])
    pb = fem.Problem(m, _fiber_mat(), cell_fibers=fiber.cell_structure_tensors(frames, PHI, *DISP))
    return pb, frames


def test_tube_tangent_is_residual_derivative():
    pb, _ = _tube_problem()
    m = pb.mesh
    rng = np.random.default_rng(3)
    X = m.node_coords
    u = 0.05 * np.stack([X[:, 0], X[:, 1], np.zeros(m.n_nodes)]) + 0.002 * rng.standard_normal((3, m.n_nodes))
    u[:, m.constrained] = 0.0
    du = rng.standard_normal((3, m.n_nodes))
    Kdu = pb.apply_tangent(u, du)
    du_f = du.copy()
    du_f[:, m.constrained] = 0.0
    h = 1e-30
    d = pb.residual(u + 1j * h * du_f).imag / h
    d[:, m.constrained] = du[:, m.constrained]
    assert np.linalg.norm(Kdu - d) < 1e-13 * np.linalg.norm(Kdu)


def test_tube_frames_geometry():
    n_theta, n_wall, n_axial, length, bend = 12, 2, 5, 10.0, 1.0
    F = workloads.tube_frames(n_theta, n_wall, n_axial, length=length, bend=bend)
    assert F.shape == (n_theta * n_wall * n_axial, 3, 3)
    assert np.abs(np.einsum("eai,ebi->eab", F, F) - np.eye(3)).max() < 1e-14
    assert np.all(np.linalg.det(F) > 0.999999)
    e = np.arange(len(F))
    i, k = e % n_theta, e // (n_theta * n_wall)
    s = length * (k + 0.5) / n_axial
    th = -2.0 * np.pi * (i + 0.5) / n_theta
    # E2 along the centreline tangent (bend pi/L cos(pi s/L), 0, 1)
    t = np.stack([bend * np.pi / length * np.cos(np.pi * s / length), np.zeros_like(s), np.ones_like(s)], 1)
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    assert np.abs(F[:, 1] - t).max() < 1e-14
    # E1: the circumferential direction of increasing angle, projected normal to E2
    er = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], 1)
    eth = np.stack([-np.sin(th), np.cos(th), np.zeros_like(th)], 1)
    assert np.abs(np.sum(F[:, 0] * np.cross(eth, t), axis=1)).max() < 1e-14
    assert np.all(np.sum(F[:, 0] * eth, axis=1) > 0.9)
    # straight tube: E3 is the outward radial direction
    F0 = workloads.tube_frames(n_theta, n_wall, n_axial, length=length, bend=0.0)
    assert np.abs(F0[:, 2] - er).max() < 1e-14
